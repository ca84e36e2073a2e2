"""CPU checks of the C ABI library: it loads, exports every function that
include/vie.h declares, rejects bad arguments before touching a device, and
its host-side HOSVD (the compression half of vie_compress) agrees with the
oracle's SVD-based HOSVD."""
import os
import re

import numpy as np
import pytest

import vie_inputs as vi
from oracle import tucker

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vie.h")


def _lib():
    from paper_1811_00484_amd import vie
    if not os.path.exists(vie.LIB_PATH):
        from paper_1811_00484_amd import build
        build.build()
    return vie


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vie_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("vie_compress", "vie_matvec", "vie_matvec_adjoint", "vie_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    vie = _lib()
    lib = vie.load()
    names = _declared_functions()
    for name in names:
        assert hasattr(lib, name), name
    # the ctypes signature table covers the header exactly
    assert sorted(vie.exported_symbols()) == names


def test_argument_errors_before_any_device_work():
    import ctypes
    vie = _lib()
    lib = vie.load()
    assert lib.vie_compress(None, None, None, None, None) == vie.VIE_E_ARG
    assert b"null" in lib.vie_last_error()
    assert lib.vie_matvec(None, 0, 0, 0, None, None, None, 1, None, 0, None) == vie.VIE_E_ARG
    assert lib.vie_solve(None, 0, None, None, None, 1, None, None, None, 0, None) == vie.VIE_E_ARG
    assert lib.vie_op_destroy(None) == vie.VIE_OK
    assert lib.vie_workspace_bytes(None, 0, 1) == 0
    n = (ctypes.c_int * 3)(4, 4, 300)
    g = np.zeros(12)
    assert lib.vie_compress(n, g.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(ctypes.c_void_p()),
                            None) == vie.VIE_E_UNSUPPORTED
    n = (ctypes.c_int * 3)(11, 4, 4)            # 2 * 11 has the prime factor 11
    g = np.zeros(12 * 11 * 16)
    assert lib.vie_compress(n, g.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(ctypes.c_void_p()),
                            None) == vie.VIE_E_UNSUPPORTED


@pytest.mark.parametrize("c", [0, 3, 5])
@pytest.mark.parametrize("tol", [1e-6, 1e-8])
def test_host_hosvd_matches_oracle(c, tol):
    vie = _lib()
    n = (14, 12, 10)
    G = vi.green_tensor(n, 0.004, vi.wavenumber(298e6))
    A = G[c]
    ranks, sv, rec, tail = vie.debug_hosvd(A, tol)
    Gc, Us, s = tucker.hosvd(tucker.from_storage(A), tol)
    assert list(ranks) == [U.shape[1] for U in Us]
    for a in range(3):
        np.testing.assert_allclose(sv[a], s[a], rtol=0, atol=1e-13 * s[a][0])
    rec_o = tucker.to_storage(tucker.tucker_reconstruct(Gc, *Us))
    assert np.linalg.norm(rec - rec_o) <= 1e-12 * np.linalg.norm(rec_o)
    assert np.linalg.norm(rec - A) <= tol * np.linalg.norm(A)
    assert tail <= tol


def test_host_hosvd_exact_low_rank():
    vie = _lib()
    rng = np.random.default_rng(0)
    n = (9, 8, 7)
    core = rng.standard_normal((3, 4, 2)) + 1j * rng.standard_normal((3, 4, 2))
    Us = [np.linalg.qr(rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r)))[0]
          for m, r in zip(n, core.shape)]
    A = tucker.to_storage(tucker.tucker_reconstruct(core, *Us))
    ranks, sv, rec, tail = vie.debug_hosvd(A, 1e-10)
    assert ranks == (3, 4, 2)
    assert np.linalg.norm(rec - A) <= 1e-13 * np.linalg.norm(A)


def test_literal_truncation_rule():
    vie = _lib()
    G = vi.green_tensor((10, 9, 8), 0.004, vi.wavenumber(298e6))
    ranks, sv, _, _ = vie.debug_hosvd(G[1], 1e-5, rule=1, want_recon=False)
    for a in range(3):
        assert ranks[a] == max(1, int(np.sum(sv[a] >= 1e-5 / np.sqrt(3) * sv[a][0])))


@pytest.mark.parametrize("c", [0, 4])
@pytest.mark.parametrize("iters", [1, 20, 200])
def test_host_cp_als_matches_oracle(c, iters):
    # the CP step of vie_compress_cp on a real Green's-tensor Tucker core: the
    # sweeps are equivariant under the column phases of the SVD start, so the
    # CP tensors of library and oracle agree after every full sweep up to
    # rounding.  That rounding is amplified: the ALS Gram matrices of these
    # near-degenerate fits have condition numbers near 1e13, and the library's
    # pivoted elimination and the oracle's pseudo-inverse round differently,
    # so the two drift apart by up to ~3e-7 relative over 200 sweeps
    from oracle import cp
    vie = _lib()
    n = (14, 12, 10)
    G = vi.green_tensor(n, 0.004, vi.wavenumber(298e6))
    Gc, _, _ = tucker.hosvd(tucker.from_storage(G[c]), 1e-6)
    R = min(Gc.shape)
    Vl, el = vie.debug_cp(Gc, R, iters)
    Vo, eo = cp.cp_als(Gc, R, iters)
    tight = iters == 1
    assert abs(el - eo[-1]) <= (1e-9 if tight else 1e-4) * eo[-1]
    rl, ro = cp.cp_reconstruct(Vl), cp.cp_reconstruct(Vo)
    assert np.linalg.norm(rl - ro) <= (1e-10 if tight else 2e-6) * np.linalg.norm(ro)


@pytest.mark.parametrize("iters", [0, 1, 30])
def test_host_cp_above_the_tucker_rank_matches_oracle(iters):
    # a CP rank above the core's smallest dimension: the extra start columns
    # follow the same definition on both sides, so the sweeps agree
    from oracle import cp
    vie = _lib()
    n = (14, 12, 10)
    G = vi.green_tensor(n, 0.004, vi.wavenumber(298e6))
    Gc, _, _ = tucker.hosvd(tucker.from_storage(G[0]), 1e-6)
    R = int(1.5 * min(Gc.shape))
    Vl, el = vie.debug_cp(Gc, R, iters)
    Vo, eo = cp.cp_als(Gc, R, max(iters, 0))
    if iters == 0:
        for a in range(3):
            assert np.allclose(np.abs(Vl[a]), np.abs(cp.start_columns(np.linalg.svd(tucker.unfold(Gc, a + 1),
                                                                                       full_matrices=False)[0], R)),
                               atol=1e-12)
        return
    rl, ro = cp.cp_reconstruct(Vl), cp.cp_reconstruct(Vo)
    assert np.linalg.norm(rl - ro) <= (1e-9 if iters == 1 else 1e-5) * np.linalg.norm(ro)


def test_host_cp_argument_errors():
    import ctypes
    vie = _lib()
    lib = vie.load()
    G = np.ones((3, 3, 2), dtype=np.complex128)
    r = (ctypes.c_int * 3)(3, 3, 2)
    V = np.empty(64, dtype=np.complex128)
    p = G.ctypes.data_as(ctypes.c_void_p)
    assert lib.vie_debug_cp(r, p, 65, 5, V.ctypes.data_as(ctypes.c_void_p), None) == vie.VIE_E_ARG   # R > 64
    assert lib.vie_debug_cp(r, p, 0, 5, V.ctypes.data_as(ctypes.c_void_p), None) == vie.VIE_E_ARG
    assert lib.vie_debug_cp(r, None, 2, 5, V.ctypes.data_as(ctypes.c_void_p), None) == vie.VIE_E_ARG
    n = (ctypes.c_int * 3)(4, 4, 4)
    g = np.zeros(12 * 64)
    assert lib.vie_compress_cp(n, g.ctypes.data_as(ctypes.c_void_p), None, -1, 0, ctypes.byref(ctypes.c_void_p()),
                               None, None) == vie.VIE_E_ARG


def test_magnetic_and_jm_argument_errors():
    import ctypes
    vie = _lib()
    lib = vie.load()
    p = ctypes.c_void_p
    assert lib.vie_compress_k(None, None, None, None, None) == vie.VIE_E_ARG
    n = (ctypes.c_int * 3)(4, 4, 300)
    g = np.zeros(6 * 4 * 4 * 300)
    assert lib.vie_compress_k(n, g.ctypes.data_as(p), None, ctypes.byref(p()), None) == vie.VIE_E_UNSUPPORTED
    assert lib.vie_magnetic_field(None, 0, None, None, 1.0, 1.0, None, None, None) == vie.VIE_E_ARG
    assert lib.vie_matvec_jm(None, None, 0, 1.0, 1.0, None, None, None, None, None, 0, None) == vie.VIE_E_ARG
    assert lib.vie_jm_workspace_bytes(None, None, 0) == 0
    assert lib.vie_solve_jm_workspace_bytes(None, None, 0, None) == 0
    assert lib.vie_solve_jm(None, None, 0, 1.0, 1.0, None, None, None, None, None, None, None, 0, None) == vie.VIE_E_ARG


def test_host_hosvd_is_independent_of_the_thread_count():
    # the Gram sums of the host SVD are grouped independently of the number
    # of host threads, so the compression is bitwise the same on any machine
    vie = _lib()
    G = vi.green_tensor((64, 48, 40), 0.002, vi.wavenumber(298e6))
    old = os.environ.get("VIE_NUM_THREADS")
    results = []
    try:
        for nt in ("1", "3", "4", "16"):
            os.environ["VIE_NUM_THREADS"] = nt
            results.append([vie.debug_hosvd(G[c], 1e-8) for c in (0, 4)])
    finally:
        if old is None:
            os.environ.pop("VIE_NUM_THREADS", None)
        else:
            os.environ["VIE_NUM_THREADS"] = old
    for other in results[1:]:
        for (r0, s0, rec0, t0), (r1, s1, rec1, t1) in zip(results[0], other):
            assert r0 == r1 and t0 == t1
            for a in range(3):
                assert np.array_equal(s0[a], s1[a])
            assert np.array_equal(rec0, rec1)


def test_debug_pass_entry_points_reject_null_arguments():
    vie = _lib()
    lib = vie.load()
    assert lib.vie_debug_pad(None, 0, None, None, 1, None) == vie.VIE_E_ARG
    assert lib.vie_debug_crop(None, 0, None, None, 1, None) == vie.VIE_E_ARG
    assert lib.vie_debug_pass(None, 0, 0, 0, 0, 0, None, None, None, None, 1, None) == vie.VIE_E_ARG
