"""CPU checks of the benchmark's contract that need no GPU: more than one
GPU is refused with a message, and the algorithmic byte and flop counts the
roofline uses follow from the pass structure."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_algorithmic_counts():
    import bench
    # X+ 3+6, Y+ 6+12, Z 12+12, Y- 12+6, X- 6+3+1+3 complex elements per
    # voxel (eps_c read once, chi = eps_c - 1 formed in the kernel): 82V,
    # 656 bytes per voxel at complex64
    assert sum(bench.PASS_ELEMS_V) == 82
    n = (256, 256, 256)
    ranks = [(15, 15, 15)] * 3 + [(17, 17, 16)] * 3
    f = bench.z_pass_flops(n, ranks)
    L = 512
    fft = 2 * 3 * L * L * 5 * L * np.log2(L)
    assert f > fft + 72.0 * L ** 3
    # the Tucker+CP count drops the core contractions but keeps the tables
    fcp = bench.z_pass_flops(n, [(15, 15, 15)] * 6, cp=True)
    ft = bench.z_pass_flops(n, [(15, 15, 15)] * 6)
    assert fcp < ft
    assert ft - fcp < 0.2 * (ft - fft - 72.0 * L ** 3)
