"""Benchmark of the Tucker-compressed FFT-VIE matvec on one MI355X.

Default workload: the 256^3 grid at 1 mm (512^3 circulant embedding) with
the nested-ellipsoid head phantom (seed 2) at 298 MHz, HOSVD tolerance 1e-6,
complex64 vectors (FP32 FFTs, FP32 Tucker reconstruction), one right-hand
side (the x-polarised plane-wave excitation).  A step is one application of
the full operator A = M_eps - M_chi N (all five passes).  Prints one JSON
line on stdout; progress goes to stderr.

Beside the headline the line carries: the HIP-graph replay, the BF16
reconstruction, the complex128 matvec, the dense-spectrum (uncompressed)
matvec and solve, the cross-Tucker compression (256^3 and the 270 x 141 x 902
body domain), the per-component decompress-and-multiply timings of Table IV's
sizes, the refined and plain solves, the Tucker+CP operator (compression,
matvec, solve, accuracy and the observables of eq. 18 against the HOSVD
solution), the magnetic operator K with |b1+| and the coupled JMVIE operator
and solves, the batching workload (6 phantoms x 16 dipole fields), the
differentiation workload (128^3 adjoint gradient against central
differences), the piecewise-linear basis on the sphere refinement series of
Fig. 9, and the FP64 oracle timed on the host (cpu_baseline).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--grid 256]
                    [--no-dense] [--no-solve] [--no-cpu-baseline] [--no-cp]
                    [--no-magnetic] [--no-cross] [--no-table4] [--no-fig7] [--no-batch]
                    [--no-grad] [--no-pwl] [--pwl-grids 30,60,90,120] [--copy-calibration]
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
FP32_PEAK_TFLOPS = 157.3   # MI355X vector / dense-MFMA FP32


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# algorithmic complex elements moved per pass and right-hand side, in units
# of V = n1 n2 n3 (reads + writes, pruned padding)
PASS_NAMES = ["x_fwd", "y_fwd", "z_fused", "y_inv", "x_inv"]
PASS_ELEMS_V = [3 + 6, 6 + 12, 12 + 12, 12 + 6, 6 + 3 + 1 + 3]


COPY_CAL_BYTES = 1 << 30   # plain copy used to calibrate the HBM byte counters


def z_pass_flops(n, ranks, cp=False):
    """Algorithmic FP32 flops of one Z-pass launch (one rhs): forward and
    inverse length-2n3 FFTs of 3 components over the (2n1)(2n2) pencils at
    5 L log2 L each, the 3x3 complex product (9 complex MACs = 72 flops) at
    every Fourier point, and the Tucker reconstruction of the half spectrum
    (N^ tables: (n1+1)(n2+1)(n3+1) r3 complex MACs per component, plus the
    per-(k1,k2) and per-k2 core contractions; a Tucker+CP operator, ``cp``,
    has R-term products there instead of contractions)."""
    n1, n2, n3 = n
    L1, L2, L3 = 2 * n1, 2 * n2, 2 * n3
    fft = 2 * 3 * L1 * L2 * 5 * L3 * np.log2(L3)
    prod = 72.0 * L1 * L2 * L3
    rec = 0.0
    for r1, r2, r3 in ranks:
        rec += 8.0 * (n1 + 1) * (n2 + 1) * (n3 + 1) * r3
        if cp:
            rec += 6.0 * ((n1 + 1) * (n2 + 1) * r1 + (n2 + 1) * r1)
        else:
            rec += 8.0 * ((n1 + 1) * (n2 + 1) * r1 * r3 + (n2 + 1) * r1 * r2 * r3)
    return float(fft + prod + rec)


def copy_bandwidth(torch, dev, reps=5):
    """Measured device copy rate (GB/s, read + write) of one elementwise
    kernel over 1 GiB: what HBM delivers to a plain streaming kernel."""
    src = torch.ones(COPY_CAL_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * COPY_CAL_BYTES / (ms * 1e-3) / 1e9


# sources of the five matvec passes' kernels (and what they include)
MATVEC_KERNEL_SOURCES = ["matvec.hip", "matvec_fast.hip", "reg_fft.h", "fft_device.h", "dev_common.h",
                         "vie_internal.h"]


def kernel_sources_sha256():
    """Hash of the matvec kernels' sources: a recorded counter measurement is
    only used while the code it was taken on is unchanged."""
    h = hashlib.sha256()
    for f in sorted(os.path.join(ROOT, "paper_1811_00484_amd", "csrc", b) for b in MATVEC_KERNEL_SOURCES):
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


def cpu_baseline(G, epsc, u, budget_s=60.0, pwl_check=None):
    """The FP64 oracle's matvec (dense Fourier-domain tensor, FFT
    convolution) timed on this host at the same workload, one application.
    ``pwl_check`` = (tensors, eps_c, u, device result, tol) of the smallest
    piecewise-linear grid: returns also the device result's relative error
    against the oracle's PWL matvec on the same HOSVD tensors, in the
    mass-normalised basis (None without it)."""
    from oracle import operator as opm
    from oracle import pwl as opwl
    pwl_err = None
    if pwl_check is not None:
        G0, eps0, u0, y0, tol0 = pwl_check
        kh0, _ = opwl.tucker_kernels(G0, tol0)
        yr = opwl.to_normalised(lambda w: opwl.matvec(kh0, eps0, w, "A"), u0)
        pwl_err = float(np.linalg.norm(y0 - yr) / np.linalg.norm(yr))
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
                      "scipy.fft with %d workers) on the full workload; %.2f s" % (cores, t)}, y, pwl_err


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
    ap.add_argument("--no-cp", action="store_true", help="skip the Tucker+CP leg")
    ap.add_argument("--no-magnetic", action="store_true", help="skip the K operator / b1+ leg")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batching workload: 6 head phantoms of seeded sizes at 2 mm, 16 dipole "
                         "fields each, multi-instance matvec and lockstep GMRES")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the differentiation workload: 128^3 adjoint gradient vs central differences")
    ap.add_argument("--no-table4", action="store_true",
                    help="skip the per-component decompress-and-multiply timings (n = 100, 200, 300, r = 25)")
    ap.add_argument("--no-fig7", action="store_true",
                    help="skip the p_abs / |b1+| error sweep over SVD tolerances (64^3 head, HOSVD and Tucker+CP)")
    ap.add_argument("--no-cross", action="store_true",
                    help="skip the cross-Tucker compression leg (256^3 and the 270 x 141 x 902 body domain)")
    ap.add_argument("--no-pwl", action="store_true", help="skip the piecewise-linear basis leg")
    ap.add_argument("--pwl-grids", default="30,60,90,120",
                    help="edges of the piecewise-linear refinement series (0.3 m cube)")
    ap.add_argument("--pwl-tol", type=float, default=1e-6)
    ap.add_argument("--pwl-jm-grids", default="",
                    help="PWL grids on which the coupled JM system (magnetic sphere) is timed and solved")
    ap.add_argument("--pwl-k-grids", default="120",
                    help="PWL grids on which the magnetic operator K is compressed and timed too")
    ap.add_argument("--pwl-rhs", type=int, default=4,
                    help="vectors per call in the multi-RHS timing on the last PWL grid")
    ap.add_argument("--pwl-head", type=int, default=1,
                    help="1: also solve the plane wave on the 96 x 120 x 126 PWL head (Table V analogue)")
    ap.add_argument("--pwl-solve-grids", default="60,120",
                    help="grids of the series on which the plane-wave problem is solved")
    ap.add_argument("--table3", default="",
                    help="comma-separated HOSVD tolerances: compress the sixty PWL components of the 270 x 141 x "
                         "902 body domain by cross-Tucker on the host (Table III; minutes per tolerance)")
    ap.add_argument("--table3-ops", default="NK", help="operators of the Table III leg (N, K or NK)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy of 1 GiB (untimed) so that counter runs can "
                         "calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (the path runs on one GPU; "
              "no multi-GPU sharding is built)" % args.gpus, file=sys.stderr)
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

    st = torch.cuda.current_stream()

    def run(steps, recon):
        for _ in range(steps):
            vie.matvec(op, x, e, out=y, recon=recon)

    def timed(recon, profile):
        """ms per matvec over the timed steps (HIP events on the library's
        stream) and, with ``profile``, the per-pass kernel averages."""
        run(args.warmup, recon)
        torch.cuda.synchronize()
        if profile:
            vie.profile_enable(True)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.time()
        ev0.record(st)
        run(args.steps, recon)
        ev1.record(st)
        torch.cuda.synchronize()
        wall = time.time() - w0
        avg = None
        if profile:
            vie.profile_enable(False)
            pass_ms, pass_cnt = vie.profile_collect()
            avg = [pass_ms[p] / max(1, pass_cnt[p]) for p in range(5)]
        return ev0.elapsed_time(ev1) / args.steps, avg, wall

    tuned, tune_ms = vie.autotune(op, torch.complex64, 1)
    log("autotune: %d quads per z workgroup (%s ms)" % (tuned, tune_ms))
    run(args.warmup, "fp32")
    torch.cuda.synchronize()
    if args.copy_calibration:
        src = torch.ones(COPY_CAL_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)   # one elementwise kernel: reads and writes COPY_CAL_BYTES each
        torch.cuda.synchronize()
        del src, dst
    ms, avg, wall = timed("fp32", True)
    y32 = y.clone()
    value = 1000.0 / ms
    alg_bytes = 8.0 * V * sum(PASS_ELEMS_V)
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    dom = int(np.argmax(avg))
    dom_bytes = 8.0 * V * PASS_ELEMS_V[dom]
    dom_gbs = dom_bytes / (avg[dom] * 1e-3) / 1e9
    log("matvec: %.3f ms (%.1f matvecs/s, %.0f GB/s algorithmic); passes %s ms" %
        (ms, value, gbs, ["%.3f" % a for a in avg]))
    # the same matvec captured once into a HIP graph and replayed
    graph = vie.MatvecGraph(op, x, e)
    for _ in range(args.warmup):
        graph.launch()
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    g0.record(st)
    for _ in range(args.steps):
        graph.launch()
    g1.record(st)
    torch.cuda.synchronize()
    graph_ms = g0.elapsed_time(g1) / args.steps
    graph_same = bool(torch.equal(graph.y[0], y32))
    graph.close()
    log("graph-replayed matvec: %.3f ms (identical to eager: %s)" % (graph_ms, graph_same))
    zflops = z_pass_flops(n, op.ranks)
    copy_gbs = copy_bandwidth(torch, dev)
    log("device copy: %.0f GB/s" % copy_gbs)

    extra = {}
    # BF16 MFMA reconstruction (the inner operator of the refined solve)
    ms16, avg16, _ = timed("bf16", True)
    y16 = y.clone()
    extra["bf16_recon"] = {"ms_per_matvec": ms16, "matvecs_per_s": 1000.0 / ms16,
                           "alg_GBps": alg_bytes / (ms16 * 1e-3) / 1e9,
                           "pass_avg_ms": dict(zip(PASS_NAMES, avg16)),
                           "rel_diff_vs_fp32_recon": float(torch.linalg.vector_norm(y16 - y32) /
                                                           torch.linalg.vector_norm(y32))}
    log("bf16-reconstruction matvec: %.3f ms; passes %s ms" % (ms16, ["%.3f" % a for a in avg16]))
    if not args.no_dense:
        vie.densify(op)
        vie.set_nhat(op, "dense")
        dms, davg, _ = timed("fp32", True)
        vie.set_nhat(op, "tucker")
        dense_half_bytes = 6 * (N + 1) ** 3 * 8
        extra["dense"] = {"ms_per_matvec": dms, "matvecs_per_s": 1000.0 / dms,
                          "alg_GBps": (alg_bytes + dense_half_bytes) / (dms * 1e-3) / 1e9,
                          "operator_bytes_half_spectrum_c64": dense_half_bytes,
                          "operator_bytes_full_spectrum_c64": op.dense_bytes_c64,
                          "pass_avg_ms": dict(zip(PASS_NAMES, davg))}
        log("dense-spectrum matvec: %.3f ms" % dms)
        if not args.no_solve:
            # the uncompressed method's refined solve on the same GPU (dense
            # half spectra of the six components, FP64 and FP32 copies)
            try:
                vie.densify(op, with_c128=True)
                vie.set_nhat(op, "dense")
                bb = torch.from_numpy(b).to(dev)
                ee = torch.from_numpy(epsc).to(dev)
                torch.cuda.synchronize()
                t0 = time.time()
                xd, infod, _ = vie.solve(op, bb, ee, tol=1e-6, restart=50, max_outer=20, refine=True, inner_tol=1e-5)
                torch.cuda.synchronize()
                extra["dense"]["refined_solve"] = {"seconds": time.time() - t0,
                                                   "converged": bool(infod[0]["converged"]),
                                                   "matvecs_inner": infod[0]["matvecs"],
                                                   "matvecs_fp64": infod[0]["matvecs_fp64"]}
                log("dense-spectrum refined solve: %.2f s, %s" % (extra["dense"]["refined_solve"]["seconds"],
                                                                 infod[0]))
                del xd, bb, ee
            except Exception as exc:
                log("dense-spectrum solve failed: %r" % (exc,))
                extra["dense"]["refined_solve"] = {"error": repr(exc)}
            vie.set_nhat(op, "tucker")
    extra["memory"] = {"tucker_operator_bytes_c64": op.tucker_bytes_c64,
                       "dense_operator_bytes_c64": op.dense_bytes_c64,
                       "compression_factor": op.dense_bytes_c64 / op.tucker_bytes_c64,
                       "operator_device_bytes_all_copies": op.device_bytes,
                       "workspace_bytes_per_rhs_c64": vie.workspace_bytes(op, torch.complex64, 1),
                       "vector_bytes_c64": 3 * V * 8}

    # the complex128 matvec (FP64 FFTs and reconstruction: Table IV's precision)
    try:
        x64 = x.to(torch.complex128)
        e64 = e.to(torch.complex128)
        y64 = torch.empty_like(x64)
        for _ in range(args.warmup):
            vie.matvec(op, x64, e64, out=y64)
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        vie.profile_enable(True)
        c0.record(st)
        for _ in range(args.steps):
            vie.matvec(op, x64, e64, out=y64)
        c1.record(st)
        torch.cuda.synchronize()
        vie.profile_enable(False)
        pm, pc = vie.profile_collect()
        ms128 = c0.elapsed_time(c1) / args.steps
        extra["c128"] = {"ms_per_matvec": ms128, "matvecs_per_s": 1000.0 / ms128,
                         "alg_bytes_per_matvec": 2 * alg_bytes,
                         "alg_GBps": 2 * alg_bytes / (ms128 * 1e-3) / 1e9,
                         "pass_avg_ms": dict(zip(PASS_NAMES, [pm[p] / max(1, pc[p]) for p in range(5)])),
                         "rel_diff_vs_c64": float(torch.linalg.vector_norm(y64.to(torch.complex64) - y32) /
                                                  torch.linalg.vector_norm(y32))}
        log("complex128 matvec: %.3f ms" % ms128)
        del x64, e64
    except Exception as exc:   # the headline line is printed regardless
        log("complex128 matvec failed: %r" % (exc,))
        extra["c128"] = {"error": repr(exc)}
        y64 = None

    if not args.no_cross:
        try:
            extra["cross"] = cross_leg(G, op, x, e, y32, n, h, k0, args, vie, torch, dev)
        except Exception as exc:   # the headline line is printed regardless
            log("cross leg failed: %r" % (exc,))
            extra["cross"] = {"error": repr(exc)}
    if not args.no_fig7:
        try:
            extra["fig7"] = fig7_leg(args, vie, torch, dev)
        except Exception as exc:   # the headline line is printed regardless
            log("fig7 leg failed: %r" % (exc,))
            extra["fig7"] = {"error": repr(exc)}
    if not args.no_table4:
        try:
            extra["table4"] = table4_leg(args, vie, torch, dev)
        except Exception as exc:   # the headline line is printed regardless
            log("table4 leg failed: %r" % (exc,))
            extra["table4"] = {"error": repr(exc)}

    if args.table3:
        try:
            extra["table3"] = table3_leg(args, vie)
        except Exception as exc:   # the headline line is printed regardless
            log("table3 leg failed: %r" % (exc,))
            extra["table3"] = {"error": repr(exc)}
    if not args.no_pwl:
        try:
            extra["pwl"] = pwl_leg(args, vie, torch, dev)
        except Exception as exc:   # the headline line is printed regardless
            log("pwl leg failed: %r" % (exc,))
            extra["pwl"] = {"error": repr(exc)}

    x_sol = None
    opk = None
    if not args.no_solve:
        extra["solve"], x_sol = solves(op, b, epsc, dev, vie, torch)
    if not args.no_magnetic:
        try:
            extra["magnetic"], opk = magnetic_leg(n, h, f, k0, x_sol, op, args, vie, torch, dev)
        except Exception as exc:   # the headline line is printed regardless
            log("magnetic leg failed: %r" % (exc,))
            extra["magnetic"] = {"error": repr(exc)}

    y_cp = None
    if not args.no_cp:
        try:
            extra["tucker_cp"], y_cp = tucker_cp_leg(G, op, x, e, y32, b, epsc, n, args, vie, torch, dev,
                                                     obs=(x_sol, opk, sg, label, h, f))
        except Exception as exc:   # the headline line is printed regardless
            log("tucker_cp leg failed: %r" % (exc,))
            extra["tucker_cp"] = {"error": repr(exc)}
    del x_sol
    if opk is not None:
        opk.close()

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
                   "alg_GBps": gbs, "wall_s_timed": wall, "device_copy_GBps_measured": copy_gbs,
                   "alg_GBps_frac_of_measured_copy": gbs / copy_gbs,
                   "z_quads_per_workgroup_autotuned": tuned, "autotune_z_ms": tune_ms,
                   "graph_ms_per_matvec": graph_ms, "graph_equals_eager": graph_same},
        # The dominant kernel is the fused z pass; at 18 flop per HBM byte with
        # packed FP32 disabled (vector FP32 then issues 78.6 TFLOP/s at most)
        # it is bound by the vector ALUs, so that is the primary figure; its
        # HBM rate is reported beside it.
        "roofline": {"bound": "alu", "kernel": PASS_NAMES[dom],
                     "achieved": zflops / (avg[dom] * 1e-3) / 1e12 if dom == 2 else None,
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": zflops / (avg[dom] * 1e-3) / 1e12 / FP32_PEAK_TFLOPS if dom == 2 else None,
                     "traffic": recorded_traffic(PASS_NAMES[dom], N),
                     "avg_ms": avg[dom], "alg_flops_per_launch": zflops if dom == 2 else None,
                     "frac_of_nonpacked_fp32_peak": (zflops / (avg[dom] * 1e-3) / 1e12 / (FP32_PEAK_TFLOPS / 2)
                                                     if dom == 2 else None),
                     "hbm": {"achieved": dom_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": dom_gbs / HBM_PEAK_GBS, "alg_bytes_per_launch": dom_bytes,
                             "frac_of_measured_copy": dom_gbs / copy_gbs},
                     "pass_avg_ms": dict(zip(PASS_NAMES, avg)),
                     "pass_hbm_GBps": {p: 8.0 * V * PASS_ELEMS_V[i] / (avg[i] * 1e-3) / 1e9
                                       for i, p in enumerate(PASS_NAMES)}},
    }
    result.update(extra)
    for flag, key, fn in ((not args.no_batch, "batch_workload", batch_workload),
                          (not args.no_grad, "grad_workload", grad_workload)):
        if flag:
            try:
                result[key] = fn(vie, torch, dev, args)
            except Exception as exc:   # the headline line is printed regardless
                log("%s failed: %r" % (key, exc))
                result[key] = {"error": repr(exc)}
    if not args.no_cpu_baseline:
        u = b
        log("cpu baseline: timing the FP64 oracle matvec ...")
        cb, y_ref, pwl_err = cpu_baseline(G, epsc, u, pwl_check=result.get("pwl", {}).get("_check"))
        result["cpu_baseline"] = cb
        for key, yy in (("matvec_rel_err_vs_oracle_dense", y32), ("bf16_matvec_rel_err_vs_oracle_dense", y16)):
            yg = yy.cpu().numpy().astype(np.complex128)
            result["config"][key] = float(np.linalg.norm(yg - y_ref) / np.linalg.norm(y_ref))
        if y64 is not None and "error" not in result.get("c128", {"error": 1}):
            yg = y64.cpu().numpy()
            result["c128"]["rel_err_vs_oracle_dense"] = float(np.linalg.norm(yg - y_ref) / np.linalg.norm(y_ref))
        ycr = result.get("cross", {}).get("_y")
        if ycr is not None:
            yg = ycr.cpu().numpy().astype(np.complex128)
            result["cross"]["matvec_rel_err_vs_oracle_dense"] = float(np.linalg.norm(yg - y_ref) /
                                                                      np.linalg.norm(y_ref))
        if pwl_err is not None:
            result["pwl"]["rel_err_vs_oracle_smallest_grid"] = pwl_err
    if isinstance(result.get("pwl"), dict):
        result["pwl"].pop("_check", None)
    if isinstance(result.get("cross"), dict):
        result["cross"].pop("_y", None)
        if y_cp is not None:
            yg = y_cp.cpu().numpy().astype(np.complex128)
            result["tucker_cp"]["matvec_rel_err_vs_oracle_dense"] = float(np.linalg.norm(yg - y_ref) /
                                                                          np.linalg.norm(y_ref))
    print(json.dumps(result), flush=True)


def pwl_z_flops(n, ranks):
    """Algorithmic FP32 flops of the piecewise-linear z pass: forward and
    inverse length-2n3 FFTs of 12 components, the 16 blocks of 3x3 complex
    products (144 complex MACs) at every Fourier point, and the Tucker
    reconstruction of the sixty components' half spectra (as z_pass_flops)."""
    n1, n2, n3 = n
    L1, L2, L3 = 2 * n1, 2 * n2, 2 * n3
    fft = 2 * 12 * L1 * L2 * 5 * L3 * np.log2(L3)
    prod = 8.0 * 144 * L1 * L2 * L3
    rec = 0.0
    for r1, r2, r3 in np.asarray(ranks).reshape(-1, 3):
        rec += 8.0 * (n1 + 1) * (n2 + 1) * (n3 + 1) * r3
        rec += 8.0 * ((n1 + 1) * (n2 + 1) * r1 * r3 + (n2 + 1) * r1 * r2 * r3)
    return float(fft + prod + rec)


# algorithmic complex elements per pass of the piecewise-linear matvec, units
# of V: twelve components through the five passes, the contrast read once
PWL_PASS_ELEMS_V = [12 + 24, 24 + 48, 48 + 48, 48 + 24, 24 + 12 + 1 + 12]


def pwl_jm_solve(vie, vi, torch, dev, op, opk, n, h, f, epsc):
    """The JMVIE system of eq. 4 in the piecewise-linear basis on the sphere
    of the refinement series made magnetic (synthetic mu_r = 1.5, loss 0.1
    inside), x-polarised plane wave (its voxel moments; H = z x E / eta0),
    mass-normalised basis: one coupled product timed, then GMRES(50) to 1e-5
    in complex64."""
    N1, N2, N3 = n
    inside = np.abs(epsc - 1.0) > 0
    mu = np.where(inside, 1.5 - 0.1j, 1.0 + 0j)
    S = np.array([1.0, np.sqrt(12.0), np.sqrt(12.0), np.sqrt(12.0)])[:, None, None, None, None]
    Em = vi.plane_wave_pwl(n, h, f)
    Hm = np.zeros_like(Em)
    eta0 = np.sqrt(vi.MU0 / vi.EPS0)
    Hm[:, 0] = -Em[:, 1] / eta0
    Hm[:, 1] = Em[:, 0] / eta0
    w = 2 * np.pi * f
    b = np.stack([S * (1j * w * vi.EPS0) * (epsc - 1.0)[None, None] * Em,
                  S * (1j * w * vi.MU0) * (mu - 1.0)[None, None] * Hm])
    bd = torch.from_numpy(b.reshape(2, 12, N3, N2, N1)).to(dev, torch.complex64)
    e = torch.from_numpy(epsc).to(dev, torch.complex64)
    m = torch.from_numpy(mu).to(dev, torch.complex64)
    vie.matvec_jm_pwl(op, opk, bd, e, m, h, f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        yd = vie.matvec_jm_pwl(op, opk, bd, e, m, h, f)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / 5 * 1e3
    del yd
    t0 = time.perf_counter()
    xs, info, st_ = vie.solve_jm_pwl(op, opk, bd, e, m, h, f, tol=1e-5, restart=50, max_outer=200)
    torch.cuda.synchronize()
    t_sol = time.perf_counter() - t0
    out = {"ms_per_jm_matvec": ms, "solve_c64_tol1e-5": {"seconds": t_sol, "matvecs": info["matvecs"],
                                                         "converged": info["converged"],
                                                         "rel_residual": info["rel_residual"]},
           "unknowns": 24 * N1 * N2 * N3}
    log("pwl %d^3 JM: %.3f ms per coupled product, plane-wave solve %.2f s, %d matvecs, residual %.2e"
        % (N1, ms, t_sol, info["matvecs"], info["rel_residual"]))
    del xs, bd
    return out


def pwl_leg(args, vie, torch, dev):
    """Piecewise-linear basis (eq. 7a-7b, twelve unknowns per voxel) on the
    refinement series of Sec. VI-C (Fig. 9): a homogeneous sphere of radius
    0.15 m, eps_r = 65, sigma = 0.6 S/m, centred in a 0.3 m cube, 298 MHz,
    edges 30, 60, 90, 120 (and 150) voxels = 10, 5, 3.3, 2.5 (2) mm, i.e.
    0.3, 2.6, 8.7, 20.7 (40.5) million unknowns; HOSVD of the sixty tensors
    at tol 1e-6 (--pwl-tol; the figure's 1e-8 makes the host HOSVD take the
    slow Jacobi refinement, 109 s at 120^3), complex64 matvec A
    (mass-normalised basis) on a seeded random vector, timed over the step
    count; the memory of the compressed and of the dense circulant tensors
    (complex128, as Sec. VI quotes it); on --pwl-solve-grids the x-polarised
    plane wave (its voxel moments against the basis) solved by GMRES(50) to
    1e-5 in complex64 (Sec. VI-C's solver settings); on --pwl-k-grids the
    magnetic operator K of eq. 5 in the same basis (thirty tensors) compressed
    at the same tolerance and its product timed; on the last grid --pwl-rhs
    vectors in one call."""
    import vie_inputs as vi
    out = {}
    f = 298e6
    k0 = vi.wavenumber(f)
    st = torch.cuda.current_stream()
    grids = [int(g) for g in args.pwl_grids.split(",") if g.strip()]
    solve_grids = {int(g) for g in args.pwl_solve_grids.split(",") if g.strip()}
    jm_grids = {int(g) for g in args.pwl_jm_grids.split(",") if g.strip()}
    k_grids = {int(g) for g in args.pwl_k_grids.split(",") if g.strip()} | jm_grids
    for idx, N in enumerate(grids):
        n = (N, N, N)
        h = 0.3 / N
        V = N ** 3
        t0 = time.perf_counter()
        G = vi.green_pwl_tensor(n, h, k0)
        t_gen = time.perf_counter() - t0
        er, sg, _ = vi.sphere_phantom(n, h, 0.15, 65.0, 0.6)
        epsc = vi.complex_permittivity(er, sg, f)
        t0 = time.perf_counter()
        op = vie.compress_pwl(G, tol=args.pwl_tol)
        t_cmp = time.perf_counter() - t0
        rng = np.random.default_rng(300 + N)
        u = rng.standard_normal((4, 3, N, N, N)) + 1j * rng.standard_normal((4, 3, N, N, N))
        x = torch.from_numpy(u.reshape(12, N, N, N)).to(dev, torch.complex64)
        e = torch.from_numpy(epsc).to(dev, torch.complex64)
        y = torch.empty_like(x)
        for _ in range(3):
            vie.matvec_pwl(op, x, e, out=y)
        steps = max(1, min(args.steps, 20))
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        c0.record(st)
        for _ in range(steps):
            vie.matvec_pwl(op, x, e, out=y)
        c1.record(st)
        torch.cuda.synchronize()
        ms = c0.elapsed_time(c1) / steps
        alg = 8.0 * V * sum(PWL_PASS_ELEMS_V)
        row = {"grid": list(n), "h_mm": h * 1e3, "unknowns": 12 * V, "ms_per_matvec": ms,
               "matvecs_per_s": 1000.0 / ms, "Munknowns_per_s": 12 * V / (ms * 1e-3) / 1e6,
               "alg_bytes_per_matvec": alg, "alg_GBps": alg / (ms * 1e-3) / 1e9,
               "z_alg_flops": pwl_z_flops(n, op.ranks), "z_alg_bytes": 8.0 * V * PWL_PASS_ELEMS_V[2],
               "max_rank": int(op.ranks.max()), "tucker_bytes_c64": op.tucker_bytes_c64,
               "dense_circulant_bytes_c128": 60 * 8 * V * 16,
               "green_seconds": t_gen, "compress_seconds": t_cmp}
        out["n%d" % N] = row
        log("pwl %d^3: %.3f ms/matvec (%.1f Munknowns/s), ranks <= %d, compress %.1f s, green %.1f s"
            % (N, ms, row["Munknowns_per_s"], row["max_rank"], t_cmp, t_gen))
        if idx == len(grids) - 1 and args.pwl_rhs > 1:
            # several excitations of the same phantom in one call
            R = args.pwl_rhs
            xr = x.unsqueeze(0).repeat(R, 1, 1, 1, 1)
            yr = torch.empty_like(xr)
            vie.matvec_pwl(op, xr, e, out=yr)
            torch.cuda.synchronize()
            c0.record(st)
            for _ in range(steps):
                vie.matvec_pwl(op, xr, e, out=yr)
            c1.record(st)
            torch.cuda.synchronize()
            msr = c0.elapsed_time(c1) / steps
            row["multi_rhs"] = {"nrhs": R, "ms_per_call": msr, "ms_per_vector": msr / R,
                                "Munknowns_per_s": R * 12 * V / (msr * 1e-3) / 1e6}
            log("pwl %d^3 x %d rhs: %.3f ms per vector" % (N, R, msr / R))
            del xr, yr
        if N in k_grids:
            # the magnetic operator K in the same basis (thirty components)
            t0 = time.perf_counter()
            Kt = vi.green_pwl_k_tensor(n, h, k0)
            t_kgen = time.perf_counter() - t0
            t0 = time.perf_counter()
            opk = vie.compress_pwl_k(Kt, tol=args.pwl_tol)
            t_kcmp = time.perf_counter() - t0
            del Kt
            for _ in range(2):
                vie.matvec_pwl(opk, x, kind="N", out=y)
            torch.cuda.synchronize()
            c0.record(st)
            for _ in range(steps):
                vie.matvec_pwl(opk, x, kind="N", out=y)
            c1.record(st)
            torch.cuda.synchronize()
            msk = c0.elapsed_time(c1) / steps
            row["k_operator"] = {"ms_per_matvec": msk, "Munknowns_per_s": 12 * V / (msk * 1e-3) / 1e6,
                                 "max_rank": int(opk.ranks[:, 3:].max()), "tucker_bytes_c64": opk.tucker_bytes_c64,
                                 "dense_circulant_bytes_c128": 30 * 8 * V * 16,
                                 "green_seconds": t_kgen, "compress_seconds": t_kcmp}
            log("pwl %d^3 K: %.3f ms/matvec, ranks <= %d, compress %.1f s, green %.1f s"
                % (N, msk, row["k_operator"]["max_rank"], t_kcmp, t_kgen))
            if N in jm_grids:
                row["jm"] = pwl_jm_solve(vie, vi, torch, dev, op, opk, n, h, f, epsc)
            opk.close()
        if N in solve_grids:
            S = np.array([1.0, np.sqrt(12.0), np.sqrt(12.0), np.sqrt(12.0)])[:, None, None, None, None]
            bn = S * vi.rhs_from_field(epsc, vi.plane_wave_pwl(n, h, f), f)
            bd = torch.from_numpy(bn.reshape(12, N, N, N)).to(dev, torch.complex64)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xs, info, st_ = vie.solve_pwl(op, bd, e, tol=1e-5, restart=50, max_outer=200)
            torch.cuda.synchronize()
            t_sol = time.perf_counter() - t0
            row["solve_c64_tol1e-5"] = {"seconds": t_sol, "matvecs": info["matvecs"], "restarts": info["restarts"],
                                        "converged": info["converged"], "rel_residual": info["rel_residual"]}
            log("pwl %d^3 plane-wave solve: %.2f s, %d matvecs, residual %.2e"
                % (N, t_sol, info["matvecs"], info["rel_residual"]))
            del xs, bd
        if idx == 0:
            out["_check"] = (G, epsc, u, y.cpu().numpy().astype(np.complex128).reshape(u.shape), args.pwl_tol)
        op.close()
        del x, e, y, G
    if args.pwl_head:
        out["head"] = pwl_head_solve(args, vie, torch, dev)
    return out


def pwl_head_solve(args, vie, torch, dev):
    """Table V analogue: the x-polarised plane wave on the nested-ellipsoid
    head phantom (seed 2) at 2 mm, 96 x 120 x 126 voxels (the FFT-friendly
    grid nearest the paper's 93 x 119 x 125; 17.4 M PWL unknowns), 298 MHz,
    HOSVD tol 1e-6, GMRES(50) to 1e-5 with at most 200 restarts (the paper's
    settings): complex64, and complex128 refined around FP32 products."""
    import vie_inputs as vi
    n, h, f = (96, 120, 126), 0.002, 298e6
    k0 = vi.wavenumber(f)
    t0 = time.perf_counter()
    G = vi.green_pwl_tensor(n, h, k0)
    er, sg, _ = vi.head_phantom(n, h, 2)
    epsc = vi.complex_permittivity(er, sg, f)
    op = vie.compress_pwl(G, tol=args.pwl_tol)
    t_prep = time.perf_counter() - t0
    del G
    S = np.array([1.0, np.sqrt(12.0), np.sqrt(12.0), np.sqrt(12.0)])[:, None, None, None, None]
    bn = (S * vi.rhs_from_field(epsc, vi.plane_wave_pwl(n, h, f), f)).reshape(12, n[2], n[1], n[0])
    out = {"grid": list(n), "unknowns": 12 * n[0] * n[1] * n[2], "prep_seconds": t_prep,
           "max_rank": int(op.ranks.max()), "paper_table5_s": {"FFT-JVIE CPU": 9598, "HOSVD GPU": 851,
                                                               "Tucker+CP GPU": 961}}
    for name, dt, refine in (("c64", torch.complex64, False), ("c128_refined", torch.complex128, True)):
        bd = torch.from_numpy(bn).to(dev, dt)
        e = torch.from_numpy(epsc).to(dev, dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, info, st_ = vie.solve_pwl(op, bd, e, tol=1e-5, restart=50, max_outer=200, refine=refine)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[name] = {"seconds": sec, "matvecs": info["matvecs"], "matvecs_fp64": info["matvecs_fp64"],
                     "converged": info["converged"], "rel_residual": info["rel_residual"]}
        log("pwl head %s solve: %.2f s, %d + %d matvecs, residual %.2e" % (name, sec, info["matvecs"],
                                                                          info["matvecs_fp64"], info["rel_residual"]))
        del xs, bd, e
    op.close()
    return out


# Table III of the paper: memory (MB) of the HOSVD-compressed sixty PWL N
# components of the 270 x 141 x 902 body domain at 2 mm, 298 MHz
PAPER_TABLE3_N_MB = {1e-4: 18.04, 1e-5: 24.16, 1e-6: 32.10, 1e-7: 40.94, 1e-8: 50.82, 1e-9: 60.90, 1e-10: 71.71}
PAPER_TABLE3_K_MB = {1e-4: 12.06, 1e-5: 16.26, 1e-6: 21.24, 1e-7: 26.15, 1e-8: 31.03, 1e-9: 35.69, 1e-10: 40.96}


def table3_leg(args, vie):
    """Table III analogue: the sixty piecewise-linear components of N and the
    thirty of K on the paper's body domain (270 x 141 x 902 voxels at 2 mm,
    298 MHz) compressed one by one by the host cross-Tucker
    (vie_tucker_cross_pwl, entries from
    vie_inputs.GreenPwlEntryCallback; the dense tensors, 33 GB as complex128,
    are never formed) at each tolerance of --table3; memory of the Tucker
    forms in complex128, core + n_i x r_i factors and core + 2 n_i x r_i
    factors (the circulant forms' multilinear ranks are the same), against
    the dense circulant forms (245.6 GB) and the paper's Table III."""
    import vie_inputs as vi
    n = (270, 141, 902)
    h, f = 0.002, 298e6
    cb = vi.GreenPwlEntryCallback(h, vi.wavenumber(f))
    out = {"grid": list(n), "dense_circulant_GB_c128": 60 * 8 * n[0] * n[1] * n[2] * 16 / 2 ** 30}
    for tol in [float(t) for t in args.table3.split(",") if t.strip()]:
        for op_name, comps, paper in (("N", range(60), PAPER_TABLE3_N_MB), ("K", range(60, 90), PAPER_TABLE3_K_MB)):
            if op_name not in args.table3_ops:
                continue
            t0 = time.perf_counter()
            tot, tot2, rmax, evals, ranks = 0, 0, 0, 0, []
            for comp in comps:
                G, Us, info = vie.tucker_cross(n, cb.fn, cb.ctx_ptr, comp, tol=tol, pwl=True)
                r = G.shape
                ranks.append(list(r))
                tot += (r[0] * r[1] * r[2] + sum(n[a] * r[a] for a in range(3))) * 16
                tot2 += (r[0] * r[1] * r[2] + sum(2 * n[a] * r[a] for a in range(3))) * 16
                rmax = max(rmax, max(r))
                evals += sum(info["evals"])
            sec = time.perf_counter() - t0
            row = {"MB_c128": tot / 1e6, "MB_c128_circulant_factors": tot2 / 1e6, "max_rank": rmax,
                   "entries_read": evals, "seconds": sec, "paper_MB": paper.get(tol), "ranks": ranks}
            out["%s_tol%g" % (op_name, tol)] = row
            log("table3 %s tol %g: %.2f MB (%.2f MB with factors of the 2n_i circulant forms; paper %s), "
                "ranks <= %d, %.0f s" % (op_name, tol, row["MB_c128"], row["MB_c128_circulant_factors"],
                                        row["paper_MB"], rmax, sec))
    return out


def cross_leg(G, op_t, x, e, y_t, n, h, k0, args, vie, torch, dev):
    """Cross-Tucker compression (the fiber-sampling alternative to the
    HOSVD named in Sec. IV-A): the defining tensors are read only through
    the input generator's entry callback.  At the headline workload and
    tolerance (against the HOSVD's compression time):
    time, entries read against n^3, ranks, the sampled Frobenius error, the
    matvec against the HOSVD operator's (and, in the CPU-baseline leg,
    against the FP64 oracle's dense operator); then the
    paper's 270 x 141 x 902 body domain at 2 mm (Sec. VI-A; the HOSVD would
    need its 6 x 549 MB dense tensors), compressed on the host only: ranks,
    storage and the sampled error."""
    import vie_inputs as vi
    out = {}
    V = n[0] * n[1] * n[2]
    cb = vi.GreenEntryCallback(h, k0)
    for tol in (args.tol,):
        t0 = time.time()
        opc, xi = vie.compress_cross(n, cb.fn, cb.ctx_ptr, tol=tol, n_sample=20000, seed=5)
        tc = time.time() - t0
        ent = {"compress_seconds": tc, "ranks": opc.ranks, "entries_read": xi["evals"],
               "entries_read_frac_of_n3": [ev / V for ev in xi["evals"]], "sweeps": xi["sweeps"],
               "sampled_rel_err": xi["sample_rel_err"], "operator_bytes_c64": opc.tucker_bytes_c64,
               "compression_factor": opc.dense_bytes_c64 / opc.tucker_bytes_c64}
        y = torch.empty_like(x)
        vie.matvec(opc, x, e, out=y)
        torch.cuda.synchronize()
        ent["rel_diff_vs_hosvd_matvec"] = float(torch.linalg.vector_norm(y - y_t) / torch.linalg.vector_norm(y_t))
        out["_y"] = y
        out["tol_%g" % tol] = ent
        log("cross compression tol %g: %.1f s, ranks %s, entries read %s (of %d each), matvec vs HOSVD %.2e"
            % (tol, tc, opc.ranks, xi["evals"], V, ent["rel_diff_vs_hosvd_matvec"]))
        opc.close()
    # the body domain of Sec. VI-A (host-only Tucker forms; the matvec's
    # FFT lengths are limited to n_i <= 256)
    nb = (270, 141, 902)
    Vb = nb[0] * nb[1] * nb[2]
    cbb = vi.GreenEntryCallback(0.002, k0)
    body = {"grid": list(nb), "h_mm": 2.0, "tol": 1e-6, "components": []}
    t0 = time.time()
    tot_bytes = 0
    for c in range(6):
        Gc, Us, xi = vie.tucker_cross(nb, cbb.fn, cbb.ctx_ptr, c, tol=1e-6, n_sample=20000, seed=11)
        r = Gc.shape
        fb = sum((nb[a] + 1) * r[a] for a in range(3)) * 8 + r[0] * r[1] * r[2] * 8
        tot_bytes += fb
        body["components"].append({"ranks": list(r), "entries_read": xi["evals"][0],
                                   "sampled_rel_err": xi["sample_rel_err"][0], "bytes_c64": fb})
    body["seconds"] = time.time() - t0
    body["tucker_bytes_c64"] = tot_bytes
    body["dense_bytes_c64"] = 6 * 8 * Vb * 8
    body["dense_tensor_bytes_c128_host"] = 6 * Vb * 16
    body["compression_factor"] = body["dense_bytes_c64"] / tot_bytes
    out["body_270x141x902"] = body
    log("cross compression of the 270x141x902 body domain: %.1f s, %.2f MB vs %.1f GB dense"
        % (body["seconds"], tot_bytes / 1e6, body["dense_bytes_c64"] / 1e9))
    return out


def table4_leg(args, vie, torch, dev):
    """The per-component step Table IV times (Sec. VI-B): one component of
    random Tucker rank (25, 25, 25) (core and factors seed 12) or CP rank 25
    decompressed and multiplied element-wise with a random n^3 vector, for
    n = 100, 200, 300, complex128 and complex64 (vie_tucker_hadamard: one
    pass, no buffer for the component), beside the n^3 3D FFT of the same
    vector by the vendor library (rocFFT through torch.fft, not this
    project's kernels; context only)."""
    out = {}
    st = torch.cuda.current_stream()
    for nn in (100, 200, 300):
        rng = np.random.default_rng(12)
        r = 25
        core = rng.standard_normal((r, r, r)) + 1j * rng.standard_normal((r, r, r))
        lam = rng.standard_normal(r) + 1j * rng.standard_normal(r)
        Us = [rng.standard_normal((nn, r)) + 1j * rng.standard_normal((nn, r)) for _ in range(3)]
        xr = rng.standard_normal((nn, nn, nn)) + 1j * rng.standard_normal((nn, nn, nn))
        row = {}
        for dt, name in ((torch.complex128, "c128"), (torch.complex64, "c64")):
            xd = torch.from_numpy(xr).to(dev, dt)
            yd = torch.empty_like(xd)
            Ud = [torch.from_numpy(U).to(dev, dt) for U in Us]
            for key, cf, cp in (("tucker", core, False), ("cp", lam, True)):
                cd_ = torch.from_numpy(cf).to(dev, dt)

                def run():
                    vie.tucker_hadamard(cd_, Ud, xd, cp=cp, out=yd)
                for _ in range(3):
                    run()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record(st)
                for _ in range(10):
                    run()
                e1.record(st)
                torch.cuda.synchronize()
                row["%s_%s_ms" % (key, name)] = e0.elapsed_time(e1) / 10
            for _ in range(2):
                torch.fft.fftn(xd)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(st)
            for _ in range(10):
                torch.fft.fftn(xd)
            e1.record(st)
            torch.cuda.synchronize()
            row["fft3d_rocfft_%s_ms" % name] = e0.elapsed_time(e1) / 10
            del xd, yd, Ud
        out["n%d_r25" % nn] = row
        log("table4 analogue n=%d: %s" % (nn, {k: "%.3f" % v for k, v in row.items()}))
    out["paper_k40m_ms_c128"] = {"n100": {"hosvd_decomp": 0.96, "cp_decomp": 0.79, "cp_loops": 1.28, "fft3d": 0.58},
                                 "n200": {"hosvd_decomp": 6.03, "cp_decomp": 5.79, "cp_loops": 8.9, "fft3d": 5.68},
                                 "n300": {"hosvd_decomp": 17.4, "cp_decomp": 20.1, "cp_loops": 29.4, "fft3d": 26.9}}
    return out


def fig7_leg(args, vie, torch, dev):
    """Fig. 7 analogue: the relative L2 errors of the absorbed power
    p_abs = sigma |E|^2 / 2 and of |b1+| (eq. 18) over the head's voxels,
    between the compressed operators (HOSVD; Tucker+CP with 1000 ALS sweeps
    and R = min r_i terms, and with R = 2 min r_i) and the uncompressed
    operator (dense spectra of the same Galerkin tensors), for SVD
    tolerances 1e-6, 1e-8, 1e-10, under the x-polarised plane wave.  Head
    phantom (seed 2) on a 64^3 grid at 4 mm, 298 MHz; every solve refined in
    FP64 to 1e-10, so the differences are the compressions' alone."""
    import vie_inputs as vi
    f = 298e6
    n = (64, 64, 64)
    h = 0.004
    k0 = vi.wavenumber(f)
    t_all = time.time()
    G = vi.green_tensor(n, h, k0)
    er, sg, label = vi.head_phantom(n, h, seed=2)
    epsc = vi.complex_permittivity(er, sg, f)
    einc_np = vi.plane_wave(n, h, f)
    b = torch.from_numpy(vi.rhs_from_field(epsc, einc_np, f)).to(dev)
    ee = torch.from_numpy(epsc).to(dev)
    einc = torch.from_numpy(einc_np).to(dev)
    hinc = torch.from_numpy(vi.plane_wave_h(n, h, f)).to(dev)
    mask = torch.from_numpy(label >= 0).to(dev)
    sig = torch.from_numpy(sg).to(dev)
    opk = vie.compress_k(vi.green_k_tensor(n, h, k0), tol=1e-12)

    def observables(op):
        x, info, _ = vie.solve(op, b, ee, tol=1e-10, restart=50, max_outer=40, refine=True, inner_tol=1e-5)
        E = vie.total_field(op, einc, x, vie.matvec(op, x, kind="N"), f)
        p = 0.5 * sig * (E.abs() ** 2).sum(dim=0)
        _, b1 = vie.magnetic_field(opk, x, hinc, h)
        return p[mask], b1[mask], bool(info[0]["converged"])

    # reference: the uncompressed operator, i.e. the dense spectra of the
    # tensors (materialised from their HOSVD at tol 1e-14, ranks up to the
    # full 64: the form is exact to rounding)
    ref_op = vie.compress(G, tol=1e-14)
    vie.densify(ref_op, with_c128=True)
    vie.set_nhat(ref_op, "dense")
    p_ref, b_ref, ok_ref = observables(ref_op)
    ref_op.close()

    def rel(a, r):
        return float(torch.linalg.vector_norm(a - r) / torch.linalg.vector_norm(r))

    rows = []
    for tol in (1e-6, 1e-8, 1e-10):
        row = {"tol": tol}
        op = vie.compress(G, tol=tol)
        p, b1, ok = observables(op)
        row["hosvd"] = {"p_abs": rel(p, p_ref), "b1_plus": rel(b1, b_ref), "ranks_max": max(max(r) for r in op.ranks),
                        "converged": ok}
        rmin = [min(r) for r in op.ranks]
        op.close()
        for key, mult in (("tucker_cp_R_min_r", 1), ("tucker_cp_R_2min_r", 2)):
            R = min(64, mult * min(rmin))
            opc = vie.compress_cp(G, tol=tol, cp_rank=R if mult > 1 else 0, cp_iters=1000)
            p, b1, ok = observables(opc)
            row[key] = {"p_abs": rel(p, p_ref), "b1_plus": rel(b1, b_ref), "cp_rank": R if mult > 1 else min(rmin),
                        "cp_fit_err_max": max(opc.cp_rel_err), "converged": ok}
            opc.close()
        rows.append(row)
        log("fig7 analogue tol %g: HOSVD p_abs %.2e b1 %.2e | CP(R=min r) %.2e %.2e | CP(R=2 min r) %.2e %.2e"
            % (tol, row["hosvd"]["p_abs"], row["hosvd"]["b1_plus"], row["tucker_cp_R_min_r"]["p_abs"],
               row["tucker_cp_R_min_r"]["b1_plus"], row["tucker_cp_R_2min_r"]["p_abs"],
               row["tucker_cp_R_2min_r"]["b1_plus"]))
    opk.close()
    return {"grid": list(n), "h_mm": 4.0, "reference": "dense spectra of the same Galerkin tensors",
            "reference_converged": ok_ref, "rows": rows, "seconds": time.time() - t_all}


def tucker_cp_leg(G, op_t, x, e, y_t, b, epsc, n, args, vie, torch, dev, obs=None):
    """The same workload with the Tucker+CP operator (Alg. 2: HOSVD at the
    same tolerance, then CP of each core with R = 2 min r_i terms, 1000 ALS
    sweeps): compression time and fits, operator bytes, matvec time on the
    z pass's CP branch, its distance from the HOSVD operator's matvec, a
    refined solve and the observables of eq. 18 against the HOSVD
    solution's."""
    # R = 2 min r_i CP terms: with R = min r_i (the rank Sec. V-B assumes)
    # the fits stall near 1e-3 and a smooth excitation sees 0.2 of error (the
    # fig7 leg shows both ranks against the uncompressed operator)
    R = min(64, 2 * min(min(r) for r in op_t.ranks))
    log("vie_compress_cp: HOSVD at tol %g, then CP-ALS (1000 sweeps, R = %d) of each core ..." % (args.tol, R))
    t0 = time.time()
    op = vie.compress_cp(G, tol=args.tol, cp_rank=R)
    t_c = time.time() - t0
    log("vie_compress_cp: %.1f s, CP ranks %s, fit errors %s"
        % (t_c, [r[0] for r in op.ranks], ["%.2e" % v for v in op.cp_rel_err]))
    y = torch.empty_like(x)
    vie.autotune(op, torch.complex64, 1)
    st = torch.cuda.current_stream()
    for _ in range(args.warmup):
        vie.matvec(op, x, e, out=y)
    torch.cuda.synchronize()
    vie.profile_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(st)
    for _ in range(args.steps):
        vie.matvec(op, x, e, out=y)
    ev1.record(st)
    torch.cuda.synchronize()
    vie.profile_enable(False)
    pass_ms, pass_cnt = vie.profile_collect()
    avg = [pass_ms[p] / max(1, pass_cnt[p]) for p in range(5)]
    ms = ev0.elapsed_time(ev1) / args.steps
    zfl = z_pass_flops(n, op.ranks, cp=True)
    out = {"compress_seconds": t_c, "cp_rank": R, "cp_ranks": [r[0] for r in op.ranks],
           "hosvd_ranks": op_t.ranks, "cp_rel_err": list(op.cp_rel_err),
           "ms_per_matvec": ms, "matvecs_per_s": 1000.0 / ms, "pass_avg_ms": dict(zip(PASS_NAMES, avg)),
           "z_fused_TFLOPs": zfl / (avg[2] * 1e-3) / 1e12, "z_fused_alg_flops": zfl,
           "operator_bytes_c64": op.tucker_bytes_c64, "compression_factor": op.dense_bytes_c64 / op.tucker_bytes_c64,
           "rel_diff_vs_hosvd_matvec": float(torch.linalg.vector_norm(y - y_t) / torch.linalg.vector_norm(y_t))}
    # the same comparison on a random (non-smooth) field: the CP fit error
    # shows at its own size there, while the smooth excitation above sits
    # where the CP error of the Fourier-domain tensor is concentrated
    import vie_inputs as vi
    ur = torch.from_numpy(vi.random_field(n, 5).astype(np.complex64)).to(dev)
    nr_c = vie.matvec(op, ur, kind="N")
    nr_t = vie.matvec(op_t, ur, kind="N")
    out["rel_diff_vs_hosvd_N_random_field"] = float(torch.linalg.vector_norm(nr_c - nr_t) /
                                                    torch.linalg.vector_norm(nr_t))
    del ur, nr_c, nr_t
    log("tucker+cp matvec: %.3f ms; passes %s ms; rel diff to HOSVD %.3e"
        % (ms, ["%.3f" % a for a in avg], out["rel_diff_vs_hosvd_matvec"]))
    if not args.no_solve:
        bb = torch.from_numpy(b).to(dev)
        ee = torch.from_numpy(epsc).to(dev)
        torch.cuda.synchronize()
        t0 = time.time()
        xs, info, st_ = vie.solve(op, bb, ee, tol=1e-6, restart=50, max_outer=20, refine=True, inner_tol=1e-5)
        torch.cuda.synchronize()
        t = time.time() - t0
        out["refined_solve"] = {"seconds": t, "converged": bool(info[0]["converged"]),
                                "rel_residual_fp64": info[0]["rel_residual"], "matvecs_inner": info[0]["matvecs"],
                                "matvecs_fp64": info[0]["matvecs_fp64"]}
        log("tucker+cp refined solve: %.2f s, %s" % (t, info[0]))
        x_t, opk, sg, label, h, f = obs if obs is not None else (None,) * 6
        if x_t is not None and opk is not None:
            # the observables of eq. 18 from the Tucker+CP solution against the
            # HOSVD solution (whose operator is within 5e-6 of the dense one):
            # p_abs = sigma |E|^2 / 2 and |b1+| over the head's voxels
            import vie_inputs as vi
            mask = torch.from_numpy(label >= 0).to(dev)
            sig = torch.from_numpy(sg).to(dev)
            einc = torch.from_numpy(vi.plane_wave(n, h, f)).to(dev)
            hinc = torch.from_numpy(vi.plane_wave_h(n, h, f)).to(dev)
            obs_v = {}
            for key, o_, xx in (("hosvd", op_t, x_t), ("tucker_cp", op, xs)):
                E = vie.total_field(o_, einc, xx, vie.matvec(o_, xx, kind="N"), f)
                p = 0.5 * sig * (E.abs() ** 2).sum(dim=0)
                _, b1 = vie.magnetic_field(opk, xx, hinc, h)
                obs_v[key] = (p[mask], b1[mask])
                del E
            for i, nm in ((0, "p_abs"), (1, "b1_plus")):
                a_, r_ = obs_v["tucker_cp"][i], obs_v["hosvd"][i]
                out[nm + "_rel_l2_err_vs_hosvd"] = float(torch.linalg.vector_norm(a_ - r_) /
                                                         torch.linalg.vector_norm(r_))
            log("tucker+cp observables vs HOSVD: p_abs %.3e, |b1+| %.3e"
                % (out["p_abs_rel_l2_err_vs_hosvd"], out["b1_plus_rel_l2_err_vs_hosvd"]))
            del obs_v, einc, hinc
        del xs
    op.close()
    return out, y


def magnetic_leg(n, h, f, k0, x_sol, opn_for_jm, args, vie, torch, dev):
    """The magnetic operator K (eq. 5) at the same grid: compression of its
    three components, the K product (same five passes, antisymmetric 3x3
    product), the full JMVIE operator of eq. 4 with a synthetic magnetic
    contrast, and |b1+| (eq. 18) of the refined solution's current."""
    import vie_inputs as vi
    t0 = time.time()
    kt = vi.green_k_tensor(n, h, k0)
    t_in = time.time() - t0
    t0 = time.time()
    opk = vie.compress_k(kt, tol=args.tol)
    t_c = time.time() - t0
    del kt
    log("K tensor %.1f s, vie_compress_k %.1f s, ranks %s" % (t_in, t_c, opk.k_ranks))
    u = torch.from_numpy(vi.random_field(n, 5).astype(np.complex64)).to(dev)
    y = torch.empty_like(u)
    st = torch.cuda.current_stream()
    for _ in range(args.warmup):
        vie.matvec(opk, u, kind="N", out=y)
    torch.cuda.synchronize()
    vie.profile_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(st)
    for _ in range(args.steps):
        vie.matvec(opk, u, kind="N", out=y)
    ev1.record(st)
    torch.cuda.synchronize()
    vie.profile_enable(False)
    pass_ms, pass_cnt = vie.profile_collect()
    avg = [pass_ms[p] / max(1, pass_cnt[p]) for p in range(5)]
    ms = ev0.elapsed_time(ev1) / args.steps
    out = {"k_tensor_seconds": t_in, "compress_seconds": t_c, "ranks": [list(r) for r in opk.k_ranks],
           "operator_bytes_c64": opk.tucker_bytes_c64, "ms_per_k_matvec": ms,
           "pass_avg_ms": dict(zip(PASS_NAMES, avg))}
    log("K matvec: %.3f ms; passes %s ms" % (ms, ["%.3f" % a for a in avg]))
    del u, y
    # the full JMVIE operator of eq. 4 with a magnetic contrast (synthetic:
    # mu_r = 1.5, loss 0.1 inside the head) beside the head's permittivity
    er, sg, label = vi.head_phantom(n, h, seed=2)
    eps_c = torch.from_numpy(vi.complex_permittivity(er, sg, f).astype(np.complex64)).to(dev)
    mu_c = torch.from_numpy(np.where(label >= 0, 1.5 - 0.1j, 1.0 + 0j).astype(np.complex64)).to(dev)
    xj = torch.from_numpy(np.stack([vi.random_field(n, 6), vi.random_field(n, 7)]).astype(np.complex64)).to(dev)
    for _ in range(args.warmup):
        vie.matvec_jm(opn_for_jm, opk, xj, eps_c, mu_c, h, f)
    torch.cuda.synchronize()
    ev0.record(st)
    for _ in range(args.steps):
        yj = vie.matvec_jm(opn_for_jm, opk, xj, eps_c, mu_c, h, f)
    ev1.record(st)
    torch.cuda.synchronize()
    out["ms_per_jm_matvec"] = ev0.elapsed_time(ev1) / args.steps
    log("JM matvec (eq. 4, N and K on [J; M] + combine): %.3f ms" % out["ms_per_jm_matvec"])
    del xj, yj
    if not args.no_solve:
        # the JM system with this magnetic contrast, plane-wave excitation
        ce = 1j * 2 * np.pi * f * vie.EPS0
        cm = 1j * 2 * np.pi * f * vie.MU0
        e_inc = torch.from_numpy(vi.plane_wave(n, h, f).astype(np.complex64)).to(dev)
        h_inc = torch.from_numpy(vi.plane_wave_h(n, h, f).astype(np.complex64)).to(dev)
        bj = torch.stack([ce * (eps_c - 1)[None] * e_inc, cm * (mu_c - 1)[None] * h_inc]).contiguous()
        del e_inc, h_inc
        # refined: complex128 vectors, FP32 products in the Arnoldi steps,
        # FP64 restart residuals, to 1e-6
        e64, m64 = eps_c.to(torch.complex128), mu_c.to(torch.complex128)
        b64 = bj.to(torch.complex128)
        torch.cuda.synchronize()
        t0 = time.time()
        xs, info, st_ = vie.solve_jm(opn_for_jm, opk, b64, e64, m64, h, f, tol=1e-6, restart=30, max_outer=30,
                                     refine=True, inner_tol=1e-5)
        torch.cuda.synchronize()
        out["jm_solve_refined"] = {"seconds": time.time() - t0, "converged": info["converged"],
                                   "matvecs_fp32_products": info["matvecs"], "matvecs_fp64": info["matvecs_fp64"],
                                   "rel_residual": info["rel_residual"], "tol": 1e-6}
        log("JM solve (refined, tol 1e-6): %.2f s, %s" % (out["jm_solve_refined"]["seconds"], info))
        del xs, bj, b64, e64, m64
    del eps_c, mu_c
    if x_sol is not None:
        hinc = torch.from_numpy(vi.plane_wave_h(n, h, f)).to(dev)
        torch.cuda.synchronize()
        t0 = time.time()
        H, b1 = vie.magnetic_field(opk, x_sol[0] if x_sol.dim() == 5 else x_sol, hinc, h)
        torch.cuda.synchronize()
        out["b1_seconds_complex128"] = time.time() - t0
        b1n = b1 * vie.C0     # |b1+| in units of the incident plane wave's mu0 |H|
        out["b1_over_incident"] = {"min": float(b1n.min()), "max": float(b1n.max()), "mean": float(b1n.mean())}
        log("b1+ of the refined solution: %.3f s, |b1+| / incident in [%.3f, %.3f]"
            % (out["b1_seconds_complex128"], out["b1_over_incident"]["min"], out["b1_over_incident"]["max"]))
        del H, b1, hinc
    return out, opk


def solves(op, b, epsc, dev, vie, torch):
    """Seconds per solve to an FP64 true residual of 1e-6: refined (FP64
    residual + FP64 Arnoldi around the FP32-computed operator, with FP32 or
    BF16-MFMA reconstruction) and plain FP32 (FP32 Arnoldi and residual,
    checked afterwards in FP64)."""
    out = {}
    bb = torch.from_numpy(b).to(dev)
    ee = torch.from_numpy(epsc).to(dev)
    # the refined solve with FP32 and with BF16 reconstruction at GMRES
    # restart lengths 50 and 30 (the FP64 Gram-Schmidt over 805 MB vectors
    # costs ~2 (j + 1) vector reads per Arnoldi step, so a shorter restart
    # trades Krylov traffic against iterations; restart 20 was slower); the time
    # inside the matvec kernels (per-pass HIP events) against the rest
    # (Gram-Schmidt, residuals, host Givens and round trips)
    x_keep = None
    for key, rc, itol, rs in (("refined_fp32_recon", "fp32", 1e-5, 50), ("refined_fp32_recon_restart30", "fp32", 1e-5, 30),
                              ("refined_bf16_recon", "bf16", 1e-3, 50), ("refined_bf16_recon_restart30", "bf16", 1e-3, 30)):
        torch.cuda.synchronize()
        vie.profile_enable(True)
        t0 = time.time()
        x, info, st = vie.solve(op, bb, ee, tol=1e-6, restart=rs, max_outer=30, refine=True, inner_tol=itol,
                                inner_recon=rc)
        torch.cuda.synchronize()
        t = time.time() - t0
        vie.profile_enable(False)
        pm, pc = vie.profile_collect()
        mv = sum(pm) * 1e-3
        out[key] = {"seconds": t, "converged": bool(info[0]["converged"]), "inner_tol": itol, "restart": rs,
                    "rel_residual_fp64": info[0]["rel_residual"], "matvecs_inner": info[0]["matvecs"],
                    "matvecs_fp64": info[0]["matvecs_fp64"], "refine_steps": info[0]["refine_steps"],
                    "matvec_kernel_seconds": mv, "krylov_and_host_seconds": t - mv}
        log("refined solve (%s reconstruction, restart %d): %.2f s (matvec kernels %.2f s), %s"
            % (rc, rs, t, mv, info[0]))
        if key == "refined_fp32_recon":
            x_keep = x
        del x
    best = min(((v["seconds"], k) for k, v in out.items() if v["converged"]), default=(None, None))
    out["best_refined"] = {"key": best[1], "seconds": best[0]}
    b32 = bb.to(torch.complex64)
    e32 = ee.to(torch.complex64)
    torch.cuda.synchronize()
    t0 = time.time()
    x32, info32, st32 = vie.solve(op, b32, e32, tol=1e-6, restart=50, max_outer=20)
    torch.cuda.synchronize()
    t_32 = time.time() - t0
    r = vie.matvec(op, x32.to(torch.complex128), ee)
    res64 = (torch.linalg.vector_norm(bb - r) / torch.linalg.vector_norm(bb)).item()
    out["plain_fp32"] = {"seconds": t_32, "converged_fp32_residual": bool(info32[0]["converged"]),
                         "rel_residual_fp32": info32[0]["rel_residual"], "rel_residual_fp64": res64,
                         "reached_1e-6_fp64": res64 <= 1e-6, "matvecs": info32[0]["matvecs"]}
    log("plain fp32 solve: %.2f s, fp64 residual %.3e, %s" % (t_32, res64, info32[0]))
    return out, x_keep


def batch_workload(vie, torch, dev, args):
    """Six nested-ellipsoid head phantoms (jitter seeds 100+i) with grid
    sizes drawn by default_rng(4) from {48^3, 64x80x96, 96x112x128, 128^3}
    at 2 mm, 16 z-dipole fields each on a 150 mm cylinder (seeds 400+i,
    z within half the skin semi-axis), complex64, HOSVD tol 1e-6.  Operators
    depend only on the grid, so each distinct grid is compressed once and
    shared.  Reports batched matvecs/s (all 96 right-hand sides, one launch
    per pass over every instance) beside per-instance launches, and the
    lockstep GMRES solve of all 96 systems to 1e-6."""
    import vie_inputs as vi
    f = 298e6
    h = 0.002
    k0 = vi.wavenumber(f)
    sizes = [(48, 48, 48), (64, 80, 96), (96, 112, 128), (128, 128, 128)]
    draw = np.random.default_rng(4).integers(0, 4, 6)
    ops = {}
    items = []
    t0 = time.time()
    for i, k in enumerate(draw):
        n = sizes[int(k)]
        if n not in ops:
            ops[n] = vie.compress(vi.green_tensor(n, h, k0), tol=1e-6)
            vie.autotune(ops[n], torch.complex64, 16)
        er, sg, label = vi.head_phantom(n, h, seed=100 + i)
        epsc = vi.complex_permittivity(er, sg, f)
        mask = label >= 0
        half_z = vi.head_semi_axes(n, h, 100 + i)[0, 2] / 2
        dips = vi.dipole_cylinder(16, 0.15, half_z, seed=400 + i)
        b = np.stack([vi.rhs_from_field(epsc, vi.dipole_field(n, h, f, p, mask), f) for p in dips])
        items.append((ops[n], torch.from_numpy(b.astype(np.complex64)).to(dev),
                      torch.from_numpy(epsc.astype(np.complex64)).to(dev)))
    log("batch workload: inputs for grids %s in %.1f s" % ([sizes[int(k)] for k in draw], time.time() - t0))
    nrhs = sum(it[1].shape[0] for it in items)
    st = torch.cuda.current_stream()

    def timed(fn, steps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    steps = max(3, args.steps // 4)
    # default: one register-FFT launch per pass and FFT length over every
    # instance (7 launches per step here: two x lengths, two y lengths, one z)
    ms_each = timed(lambda: vie.matvec_multi(items), steps)
    vie.set_batch_mode(1)
    try:
        ms_multi = timed(lambda: vie.matvec_multi(items), steps)   # one mixed-radix launch per pass
    finally:
        vie.set_batch_mode(0)
    vox = sum(it[1].shape[0] * it[1][0, 0].numel() for it in items)
    out = {"grids": [list(sizes[int(k)]) for k in draw], "rhs_total": nrhs, "voxels_x_rhs": vox,
           "ranks": {"x".join(map(str, n)): op.ranks for n, op in ops.items()},
           "single_mixed_radix_launch": {"ms_per_step": ms_multi, "matvecs_per_s": nrhs * 1000.0 / ms_multi,
                            "alg_GBps": 664.0 * vox / (ms_multi * 1e-3) / 1e9},
           "grouped_register_fft_launch": {"ms_per_step": ms_each, "matvecs_per_s": nrhs * 1000.0 / ms_each,
                                   "alg_GBps": 664.0 * vox / (ms_each * 1e-3) / 1e9}}
    log("batch workload: %d rhs, single mixed-radix launch per pass %.2f ms/step (%.0f matvecs/s), grouped "
        "register-FFT launches %.2f ms/step (%.0f matvecs/s)" % (nrhs, ms_multi, nrhs * 1000.0 / ms_multi, ms_each,
                                                                  nrhs * 1000.0 / ms_each))
    # GMRES to an FP64 residual of 1e-6 (complex64 operator inside FP64
    # refinement; plain FP32 GMRES stagnates near 1.5e-6 on these systems),
    # in calls of a few refinement steps each, every call warm-started from
    # the previous iterate (the same iteration as one long call: each call
    # re-evaluates the true residual first)
    items = [(op, x.to(torch.complex128), e.to(torch.complex128)) for op, x, e in items]
    torch.cuda.synchronize()
    t0 = time.time()
    x0 = None
    its = [0] * nrhs
    conv = False
    for call in range(40):
        res, stt = vie.solve_multi(items, tol=1e-6, restart=10, max_outer=3, refine=True, inner_tol=1e-5, x0=x0)
        x0 = [x for x, _ in res]
        infos = [i for _, inf in res for i in inf]
        its = [a + i["matvecs"] for a, i in zip(its, infos)]
        conv = all(i["converged"] for i in infos)
        log("batch workload: solve call %d, %.1f s, worst residual %.3e" %
            (call, time.time() - t0, max(i["rel_residual"] for i in infos)))
        if conv:
            break
    torch.cuda.synchronize()
    t = time.time() - t0
    out["solve_all_lockstep"] = {"seconds": t, "tol": 1e-6, "restart": 10, "refined": True, "all_converged": conv,
                                 "matvecs_min": min(its), "matvecs_max": max(its),
                                 "seconds_per_system": t / nrhs}
    log("batch workload: lockstep solve of %d systems in %.1f s (matvecs %d..%d, converged %s)"
        % (nrhs, t, min(its), max(its), conv))
    return out


def grad_workload(vie, torch, dev, args):
    """Differentiation at 128^3, 2 mm, head phantom seed 2, x-polarised plane
    wave: L = sum over 500 tissue targets (seed 50) of |E_x - E*|^2 with E*
    from the 5%-perturbed phantom (seed 51) solved in complex128 to 1e-10.
    The adjoint gradient (complex64 forward and adjoint solves to 1e-6, and
    the refined variant) is compared with central differences (relative step
    1e-4, complex128 correction solves from the unperturbed solution) on 20
    tissue voxels (seed 52) x {eps_r, sigma}."""
    import vie_inputs as vi
    from paper_1811_00484_amd.autograd import total_field
    f = 298e6
    n = (128, 128, 128)
    h = 0.002
    k0 = vi.wavenumber(f)
    op = vie.compress(vi.green_tensor(n, h, k0), tol=1e-6)
    vie.autotune(op, torch.complex64, 1)
    er, sg, label = vi.head_phantom(n, h, seed=2)
    e_inc = vi.plane_wave(n, h, f)
    tissue = np.nonzero(label.ravel() >= 0)[0]
    targets = np.sort(np.random.default_rng(50).choice(tissue, 500, replace=False))
    rng = np.random.default_rng(51)
    tm = label >= 0
    er_t = er * np.where(tm, 1 + 0.05 * rng.uniform(-1, 1, er.shape), 1.0)
    sg_t = sg * np.where(tm, 1 + 0.05 * rng.uniform(-1, 1, sg.shape), 1.0)
    ee = torch.from_numpy(e_inc).to(dev)
    tg = torch.from_numpy(targets).to(dev)

    def field(er_, sg_, tol, dtype=torch.complex128, u0=None):
        """E for (eps_r, sigma); with ``u0`` (the solution at nearby
        parameters) the solve is for the correction d = u - u0 from the
        FP64 residual b - A u0, so the tolerance is relative to that small
        residual and the finite differences see no solver noise."""
        eps_c, b = vie.problem_setup(op, torch.from_numpy(er_).to(dev), torch.from_numpy(sg_).to(dev),
                                     ee.to(dtype), f)
        if u0 is None:
            u, info, _ = vie.solve(op, b, eps_c, tol=tol, restart=60, max_outer=100)
        else:
            r = b - vie.matvec(op, u0, eps_c)
            d, info, _ = vie.solve(op, r, eps_c, tol=tol, restart=60, max_outer=100)
            u = u0 + d
        return vie.total_field(op, ee.to(dtype), u, vie.matvec(op, u, kind="N"), f), u

    E_t = field(er_t, sg_t, 1e-10)[0][0].reshape(-1)[tg]
    _, u_base = field(er, sg, 1e-12)

    def loss_of(E):
        return torch.sum(torch.abs(E[0].reshape(-1)[tg] - E_t.to(E.dtype)) ** 2)

    out = {"grid": list(n), "targets": 500}
    grads = {}
    for key, cdt, rdt, refine in (("c64", torch.complex64, torch.float32, False),
                                  ("c64_refined", torch.complex128, torch.float64, True)):
        e_r = torch.from_numpy(er).to(dev, rdt).requires_grad_(True)
        s_g = torch.from_numpy(sg).to(dev, rdt).requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.time()
        E = total_field(op, e_r, s_g, ee.to(cdt), f, tol=1e-6 if not refine else 1e-10, refine=refine)
        L = loss_of(E)
        L.backward()
        torch.cuda.synchronize()
        grads[key] = (e_r.grad.double().cpu().numpy(), s_g.grad.double().cpu().numpy())
        out[key] = {"seconds_forward_backward": time.time() - t0, "loss": float(L.item())}
    picks = np.random.default_rng(52).choice(tissue, 20, replace=False)
    fd, ad = [], {k: [] for k in grads}
    t0 = time.time()
    for vox in picks:
        idx = np.unravel_index(vox, er.shape)
        for which, base in ((0, er), (1, sg)):
            step = 1e-4 * base[idx]
            p = base.copy()
            m = base.copy()
            p[idx] += step
            m[idx] -= step
            args_p = (p, sg) if which == 0 else (er, p)
            args_m = (m, sg) if which == 0 else (er, m)
            lp = loss_of(field(*args_p, 1e-10, u0=u_base)[0]).item()
            lm = loss_of(field(*args_m, 1e-10, u0=u_base)[0]).item()
            fd.append((lp - lm) / (2 * step))
            for k in grads:
                ad[k].append(grads[k][which][idx])
    fd = np.array(fd)
    out["fd_seconds"] = time.time() - t0
    for k in grads:
        a = np.array(ad[k])
        out[k]["rel_err_vs_fd"] = float(np.linalg.norm(a - fd) / np.linalg.norm(fd))
    log("grad workload: %s" % out)
    return out


if __name__ == "__main__":
    main()
