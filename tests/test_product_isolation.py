"""The product path does not route through the oracle: no module of the
package imports it, the native sources do not reach it, and the benchmark
imports it only inside its CPU-baseline leg."""
import ast
import glob
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _imports(path):
    tree = ast.parse(open(path).read())
    out = []
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out += [(a.name, node) for a in node.names]
        elif isinstance(node, ast.ImportFrom) and node.module:
            out.append((node.module, node))
    return tree, out


def test_package_does_not_import_the_oracle():
    for path in glob.glob(os.path.join(ROOT, "paper_1811_00484_amd", "**", "*.py"), recursive=True):
        _, imps = _imports(path)
        assert not any(name == "oracle" or name.startswith("oracle.") for name, _ in imps), path


def test_native_sources_do_not_reach_the_oracle():
    for path in glob.glob(os.path.join(ROOT, "paper_1811_00484_amd", "csrc", "*")):
        text = open(path, errors="replace").read()
        assert "oracle/" not in text and "oracle." not in text, path


def test_benchmark_uses_the_oracle_only_for_the_cpu_baseline():
    path = os.path.join(ROOT, "bench.py")
    tree, imps = _imports(path)
    funcs = {id(n): f.name for f in ast.walk(tree) if isinstance(f, ast.FunctionDef) for n in ast.walk(f)}
    for name, node in imps:
        if name == "oracle" or name.startswith("oracle."):
            assert funcs.get(id(node)) == "cpu_baseline", "oracle imported outside cpu_baseline"
