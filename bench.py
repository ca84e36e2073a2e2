"""Benchmark of the Tucker-compressed FFT-VIE matvec on one MI355X.

Default workload: the 256^3 grid at 1 mm (512^3 circulant embedding) with
the nested-ellipsoid head phantom (seed 2) at 298 MHz, HOSVD tolerance 1e-6,
complex64 vectors (FP32 FFTs, FP32 Tucker reconstruction), one right-hand
side (the x-polarised plane-wave excitation).  A step is one application of
the full operator A = M_eps - M_chi N (all five passes).  Prints one JSON
line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--grid 256]
                    [--no-dense] [--no-solve] [--no-cpu-baseline]
"""
import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# algorithmic complex elements moved per pass and right-hand side, in units
# of V = n1 n2 n3 (reads + writes, pruned padding)
PASS_NAMES = ["x_fwd", "y_fwd", "z_fused", "y_inv", "x_inv"]
PASS_ELEMS_V = [3 + 6, 6 + 12, 12 + 12, 12 + 6, 6 + 3 + 1 + 3]


COPY_CAL_BYTES = 1 << 30   # plain copy used to calibrate the HBM byte counters


def kernel_sources_sha256():
    """Hash of every native source: a recorded counter measurement is only
    used while the code it was taken on is unchanged."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1811_00484_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel, grid):
    """HBM bytes per launch of ``kernel`` from the committed FETCH_SIZE /
    WRITE_SIZE counter summary (scaled by a plain copy of known size), or
    None when there is none for this workload or the sources have changed
    since it was taken."""
    want = kernel_sources_sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*hbm_traffic*.md"))):
        text = open(f).read()
        kv = dict(re.findall(r"^([\w.]+):\s*(\S+)\s*$", text, re.M))
        if kv.get("kernel") != kernel or kv.get("grid") != str(grid):
            continue
        if kv.get("sources_sha256") != want:
            log("traffic: %s was taken on other sources; reporting null" % os.path.basename(f))
            return None
        return float(kv["traffic_bytes_per_launch"])
    return None


def cpu_baseline(G, epsc, u, budget_s=60.0):
    """The FP64 oracle's matvec (dense Fourier-domain tensor, FFT
    convolution) timed on this host at the same workload, one application."""
    from oracle import operator as opm
    cores = len(os.sched_getaffinity(0))
    t0 = time.time()
    op = opm.dense_operator(G)
    t_setup = time.time() - t0
    log("cpu baseline: oracle dense operator built in %.1f s" % t_setup)
    t0 = time.time()
    y = opm.matvec(op, epsc, u, "A")
    t = time.time() - t0
    del op
    return {"value": 1.0 / t, "unit": "matvecs/s", "cores": cores, "kind": "oracle",
            "sample": "one FP64 oracle application of A (dense Fourier-domain tensor precomputed, "
                      "scipy.fft with %d workers) on the full workload; %.2f s" % (cores, t)}, y


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy of 1 GiB (untimed) so that counter runs can "
                         "calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (the path is single-GPU; "
              "see DESIGN.md for how it would shard)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import vie_inputs as vi
    from paper_1811_00484_amd import vie

    dev = torch.device("cuda:0")
    f = 298e6
    N = args.grid
    n = (N, N, N)
    h = 0.256 / N
    k0 = vi.wavenumber(f)
    t0 = time.time()
    er, sg, label = vi.head_phantom(n, h, seed=2)
    epsc = vi.complex_permittivity(er, sg, f)
    e_inc = vi.plane_wave(n, h, f)
    b = vi.rhs_from_field(epsc, e_inc, f)
    log("inputs: phantom + rhs %.1f s" % (time.time() - t0))
    t0 = time.time()
    G = vi.green_tensor(n, h, k0)
    log("inputs: Green's tensor %s in %.1f s" % (str(n), time.time() - t0))
    t0 = time.time()
    op = vie.compress(G, tol=args.tol)
    log("vie_compress: %.1f s, ranks %s" % (time.time() - t0, op.ranks))

    V = N ** 3
    x = torch.from_numpy(b.astype(np.complex64)).to(dev)
    e = torch.from_numpy(epsc.astype(np.complex64)).to(dev)
    y = torch.empty_like(x)

    def run(steps):
        for _ in range(steps):
            vie.matvec(op, x, e, out=y)

    run(args.warmup)
    torch.cuda.synchronize()
    if args.copy_calibration:
        src = torch.ones(COPY_CAL_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)   # one elementwise kernel: reads and writes COPY_CAL_BYTES each
        torch.cuda.synchronize()
        del src, dst
    vie.profile_enable(True)
    st = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.time()
    ev0.record(st)
    run(args.steps)
    ev1.record(st)
    torch.cuda.synchronize()
    wall = time.time() - w0
    vie.profile_enable(False)
    pass_ms, pass_cnt = vie.profile_collect()
    ms = ev0.elapsed_time(ev1) / args.steps
    value = 1000.0 / ms
    alg_bytes = 8.0 * V * sum(PASS_ELEMS_V)
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    avg = [pass_ms[p] / max(1, pass_cnt[p]) for p in range(5)]
    dom = int(np.argmax(avg))
    dom_bytes = 8.0 * V * PASS_ELEMS_V[dom]
    dom_gbs = dom_bytes / (avg[dom] * 1e-3) / 1e9
    log("matvec: %.3f ms (%.1f matvecs/s, %.0f GB/s algorithmic); passes %s ms" %
        (ms, value, gbs, ["%.3f" % a for a in avg]))

    extra = {}
    if not args.no_dense:
        vie.densify(op)
        vie.set_nhat(op, "dense")
        run(args.warmup)
        torch.cuda.synchronize()
        d0 = torch.cuda.Event(enable_timing=True)
        d1 = torch.cuda.Event(enable_timing=True)
        d0.record(st)
        run(args.steps)
        d1.record(st)
        torch.cuda.synchronize()
        dms = d0.elapsed_time(d1) / args.steps
        vie.set_nhat(op, "tucker")
        dense_half_bytes = 6 * (N + 1) ** 3 * 8
        extra["dense"] = {"ms_per_matvec": dms, "matvecs_per_s": 1000.0 / dms,
                          "alg_GBps": (alg_bytes + dense_half_bytes) / (dms * 1e-3) / 1e9,
                          "operator_bytes_half_spectrum_c64": dense_half_bytes,
                          "operator_bytes_full_spectrum_c64": op.dense_bytes_c64}
        log("dense-spectrum matvec: %.3f ms" % dms)
    extra["memory"] = {"tucker_operator_bytes_c64": op.tucker_bytes_c64,
                       "dense_operator_bytes_c64": op.dense_bytes_c64,
                       "compression_factor": op.dense_bytes_c64 / op.tucker_bytes_c64}

    if not args.no_solve:
        extra["solve"] = solves(op, b, epsc, dev, vie, torch)

    result = {
        "metric": "VIE matvecs/s (256^3 head phantom, Tucker-compressed operator, 1 rhs)",
        "value": value,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "nested-ellipsoid head phantom (seed 2), %d^3 grid at %.2f mm, 298 MHz, "
                               "HOSVD tol %g, complex64 (FP32 FFT + FP32 Tucker reconstruction), 1 rhs "
                               "(x-polarised plane wave)" % (N, h * 1e3, args.tol),
                   "grid": list(n), "ranks": op.ranks, "alg_bytes_per_matvec": alg_bytes,
                   "alg_GBps": gbs, "wall_s_timed": wall},
        "roofline": {"bound": "hbm", "kernel": PASS_NAMES[dom], "achieved": dom_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dom_gbs / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(PASS_NAMES[dom], N),
                     "avg_ms": avg[dom], "alg_bytes_per_launch": dom_bytes,
                     "pass_avg_ms": dict(zip(PASS_NAMES, avg))},
    }
    result.update(extra)
    if not args.no_cpu_baseline:
        u = b
        log("cpu baseline: timing the FP64 oracle matvec ...")
        cb, y_ref = cpu_baseline(G, epsc, u)
        result["cpu_baseline"] = cb
        yg = y.cpu().numpy().astype(np.complex128)
        result["config"]["matvec_rel_err_vs_oracle_dense"] = float(np.linalg.norm(yg - y_ref) /
                                                                   np.linalg.norm(y_ref))
    print(json.dumps(result), flush=True)


def solves(op, b, epsc, dev, vie, torch):
    """Seconds per solve to an FP64 true residual of 1e-6: refined
    (FP64 residual + FP64 Arnoldi, FP32-computed operator) and plain FP32."""
    out = {}
    bb = torch.from_numpy(b).to(dev)
    ee = torch.from_numpy(epsc).to(dev)
    torch.cuda.synchronize()
    t0 = time.time()
    x, info, st = vie.solve(op, bb, ee, tol=1e-6, restart=50, max_outer=20, refine=True, inner_tol=1e-5)
    torch.cuda.synchronize()
    t_ref = time.time() - t0
    out["refined_fp64_residual"] = {"seconds": t_ref, "converged": info[0]["converged"],
                                    "rel_residual_fp64": info[0]["rel_residual"],
                                    "matvecs_fp32": info[0]["matvecs"], "matvecs_fp64": info[0]["matvecs_fp64"]}
    log("refined solve: %.2f s, %s" % (t_ref, info[0]))
    b32 = bb.to(torch.complex64)
    e32 = ee.to(torch.complex64)
    torch.cuda.synchronize()
    t0 = time.time()
    x32, info32, st32 = vie.solve(op, b32, e32, tol=1e-6, restart=50, max_outer=20)
    torch.cuda.synchronize()
    t_32 = time.time() - t0
    r = vie.matvec(op, x32.to(torch.complex128), ee)
    res64 = (torch.linalg.vector_norm(bb - r) / torch.linalg.vector_norm(bb)).item()
    out["plain_fp32"] = {"seconds": t_32, "converged_fp32_residual": info32[0]["converged"],
                         "rel_residual_fp32": info32[0]["rel_residual"], "rel_residual_fp64": res64,
                         "reached_1e-6_fp64": res64 <= 1e-6, "matvecs": info32[0]["matvecs"]}
    log("plain fp32 solve: %.2f s, fp64 residual %.3e, %s" % (t_32, res64, info32[0]))
    return out


if __name__ == "__main__":
    main()
