/*
 * vie.h -- C ABI of the MI355X (gfx950) Tucker-compressed FFT-VIE library.
 *
 * Operation (Giannakopoulos, Litsarev, Polimeridis, "Memory footprint
 * reduction for the FFT-based volume integral equation method via tensor
 * decompositions"): the electric block of the current-based VIE system
 * (eq. 1-4) on a uniform n1 x n2 x n3 voxel grid with piecewise-constant
 * current coefficients,
 *
 *     (A u)_p(m) = eps_c(m) u_p(m) - chi(m) sum_q sum_m' Nt_pq(m - m') u_q(m'),
 *     chi = eps_c - 1,
 *
 * where the Toeplitz (BTTB, Sec. II-B) defining tensors Nt_c of the six unique
 * components c = xx, yy, zz, xy, xz, yz are held only in Tucker form (HOSVD,
 * Sec. IV-A, Alg. 1), with circulant embedding and FFT applied to the factor
 * columns (Sec. V-A), and are reconstructed on the fly inside the matvec
 * (the "component decompression" of Sec. V-B, done per pencil, never into a
 * dense buffer).
 *
 * Beside it: the cross-Tucker compression named in Sec. IV-A, which reads
 * only fibers of the defining tensors through an entry callback
 * (vie_compress_cross, vie_tucker_cross), the Tucker+CP form of Alg. 2 /
 * eq. 17 (vie_compress_cp), the
 * magnetic operator K of eq. 5 as a compressed operator of its own
 * (vie_compress_k) with the field and |b1+| of eq. 18
 * (vie_magnetic_field), and the full JMVIE system of eq. 4 with electric
 * and magnetic contrasts (vie_matvec_jm, vie_solve_jm).
 *
 * Conventions shared by every call:
 *  - Complex numbers are interleaved (re, im); complex64 = 2 x float,
 *    complex128 = 2 x double.
 *  - Vector layout [nrhs][3][n3][n2][n1], x fastest (component q = x, y, z).
 *    Scalar maps [n3][n2][n1].
 *  - DEVICE pointers are HIP device allocations owned by the caller; HOST
 *    pointers are ordinary host memory owned by the caller.  The library owns
 *    only the memory of a vie_op.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *    enqueued asynchronously on it; vie_solve synchronises it internally.
 *  - Return value: VIE_OK (0), a positive warning (result valid), or a
 *    negative error.  On an argument error nothing is enqueued and outputs are
 *    untouched; on VIE_E_HIP outputs are undefined.  vie_last_error() gives a
 *    thread-local message for the last negative status.
 */
#ifndef VIE_H
#define VIE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int vie_status;
enum {
    VIE_OK = 0,
    VIE_NOT_CONVERGED = 1,   /* solve ended at its iteration limit; x holds the last iterate */
    VIE_E_ARG = -1,          /* invalid argument (null pointer, bad size, aliasing, small workspace) */
    VIE_E_NOMEM = -2,        /* device or host allocation failed */
    VIE_E_HIP = -3,          /* a HIP runtime call failed */
    VIE_E_NONFINITE = -4,    /* NaN or Inf met in an input norm or a Krylov quantity */
    VIE_E_UNSUPPORTED = -5   /* size, rank or option outside what the kernels implement */
};

/* vector / FFT precision */
enum { VIE_C64 = 0, VIE_C128 = 1 };
/* arithmetic of the on-the-fly Tucker reconstruction */
enum { VIE_RECON_AUTO = 0,   /* FP32 for VIE_C64, FP64 for VIE_C128 */
       VIE_RECON_FP32 = 1,
       VIE_RECON_BF16 = 2,   /* BF16 factors and core on MFMA, FP32 accumulate (VIE_C64 only) */
       VIE_RECON_FP64 = 3 };
/* which operator a matvec applies */
enum { VIE_OP_A = 0,         /* eps_c u - chi (N u)             (eq. 4, electric block) */
       VIE_OP_N = 1 };       /* N u (bare Green's operator)                              */
/* source of the Fourier-domain Green's tensor inside the matvec */
enum { VIE_NHAT_TUCKER = 0,  /* reconstructed per pencil from core + factors (default) */
       VIE_NHAT_DENSE = 1 }; /* read from a dense half-spectrum store (the uncompressed
                                method, for comparison; see vie_op_densify) */

typedef struct vie_op vie_op;   /* opaque; immutable after vie_compress except
                                   vie_op_densify / vie_op_set_nhat; shareable
                                   across streams */

typedef struct {
    double tol;          /* HOSVD tolerance eps (eq. 12); relative Frobenius error bound */
    int trunc_rule;      /* 0: discarded Frobenius tail of each unfolding <= tol/sqrt(3) ||A||_F
                            (default); 1: keep sigma_k >= tol/sqrt(3) sigma_max (Alg. 1 as printed) */
    int max_rank;        /* 0 = no cap; else cap every r_i (VIE_E_UNSUPPORTED if the tail bound
                            then exceeds tol) */
} vie_compress_opts;

typedef struct {
    int ranks[6][3];         /* Tucker ranks (r1, r2, r3) per component */
    double tail_bound[6];    /* sqrt(sum of discarded sigma^2 over the 3 unfoldings) / ||A||_F */
    double fro_norm[6];      /* ||A_c||_F of each defining tensor */
    size_t tucker_bytes_c64; /* bytes of the cores + Fourier factors (rows 0..n_i), each stored
                                once, at complex64: the compressed operator (a superdiagonal
                                Tucker+CP core counts its R diagonal weights only) */
    size_t dense_bytes_c64;  /* bytes of the 6 dense circulant spectra (8 n1 n2 n3 points each)
                                at complex64: what the uncompressed method stores */
    size_t device_bytes;     /* all device memory the operator holds: FP64, FP32 and BF16
                                copies, the kernels' extra z-factor layouts, twiddles */
    double seconds;          /* host time of the compression */
    int cp;                  /* 1 if every core is superdiagonal with r1 = r2 = r3 (a Tucker+CP
                                form, eq. 17; ranks then hold (R, R, R)), 0 otherwise */
} vie_compress_info;

/*
 * vie_compress -- HOSVD (Alg. 1) of each defining tensor on the host in FP64,
 * then circulant embedding + DFT of the factor columns (Sec. V-A), upload of
 * cores and Fourier factors to the current device in FP64, FP32 and BF16.
 *   n      HOST int[3]: grid (n1, n2, n3), 1 <= n_i <= 256.
 *   green  HOST complex128 [6][n3][n2][n1]: Nt_c(offset (i, j, k)), component order
 *          xx, yy, zz, xy, xz, yz, normalised so that the identity part of N has
 *          unit diagonal (Galerkin rows divided by the voxel volume).  xy, xz, yz
 *          must be odd along their two axes (zero at offset 0 along them); the
 *          negative offsets are implied by that parity.
 *   opts   HOST, may be NULL (tol 1e-6, rule 0, no cap).
 *   out    receives the new operator (library-owned device memory).
 *   info   HOST, may be NULL.
 * Synchronous.  Errors: VIE_E_ARG, VIE_E_NOMEM, VIE_E_HIP, VIE_E_UNSUPPORTED.
 */
vie_status vie_compress(const int n[3], const double* green, const vie_compress_opts* opts,
                        vie_op** out, vie_compress_info* info);

/*
 * vie_compress_cp -- Tucker+CP compression (Alg. 2): the HOSVD of vie_compress
 * (same n, green, opts), then a CP decomposition of each core with cp_rank
 * terms (0 = the smallest of that core's Tucker ranks; up to 64, also above
 * the Tucker ranks, where more terms fit the core better) by alternating
 * least squares, cp_iters sweeps (0 = 1000), started from the leading left
 * singular vectors of the core's unfoldings (columns beyond a mode's Tucker
 * rank r: exp(2 pi i frac(g (i + 1) (l + 1))) / sqrt(r), g = (sqrt 5 - 1) / 2);
 * the operator holds the Tucker+CP factors W^i = U^i V^i (eq. 17) and the z
 * pass builds each N^ pencil from them with no core contraction.
 *   cp_rel_err  HOST double[6] out (may be NULL): ||G_c - CP(G_c)||_F / ||G_c||_F.
 * Errors as vie_compress; VIE_E_UNSUPPORTED for a CP rank above 64.
 */
vie_status vie_compress_cp(const int n[3], const double* green, const vie_compress_opts* opts, int cp_rank,
                           int cp_iters, vie_op** out, vie_compress_info* info, double cp_rel_err[6]);

/*
 * vie_compress_k -- the magnetic operator K of eq. 5 (curl of the
 * single-layer potential) as a compressed operator: HOSVD (Alg. 1) of its
 * three defining tensors and the embedded-factor DFT of Sec. V-A, as
 * vie_compress.  K's component pair is antisymmetric (K_qp = -K_pq, zero
 * diagonal) and each component is odd along one axis (xy along z, xz along
 * y, yz along x); the operator applies
 *   y_p(m) = sum_q sum_m' K_pq(m - m') x_q(m')
 * through vie_matvec with kind VIE_OP_N only (no contrast epilogue, no
 * adjoint: other calls return VIE_E_UNSUPPORTED; it is not accepted by the
 * solvers, multi-instance calls or vie_autotune).  Its z pass has its own
 * variant of the register-FFT kernel (z lengths 128, 256, 512) and of the
 * mixed-radix one.
 *   green_k HOST complex128 [3][n3][n2][n1]: K_c(offset (i, j, k)) for
 *           c = xy, xz, yz, observation voxel at the offset, source at 0.
 *   n, opts, out as vie_compress; info (may be NULL): ranks[0..2] are the
 *   zero diagonal slots (1, 1, 1), ranks[3..5] the Tucker ranks of xy, xz, yz.
 */
vie_status vie_compress_k(const int n[3], const double* green_k, const vie_compress_opts* opts, vie_op** out,
                          vie_compress_info* info);

/*
 * vie_op_from_tucker -- build an operator from a Tucker form of the six
 * defining tensors computed elsewhere (eq. 13-14: another truncation, a cross
 * approximation, a stored decomposition).  The factor columns are embedded
 * and transformed (Sec. V-A) and uploaded exactly as in vie_compress.
 *   n        HOST int[3], 1 <= n_i <= 256, 2 n_i a product of 2, 3, 5, 7.
 *   ranks    HOST int[6][3], 1 <= r_a <= min(n_a, 64).
 *   cores    HOST complex128, the six cores one after another, each
 *            [r1][r2][r3] (r3 fastest), unscaled (Nt_c = G x1 U1 x2 U2 x3 U3).
 *   factors  HOST complex128, for c = 0..5 and a = 0..2 in that order the
 *            real-space factor U_a of component c, n_a x r_a row-major.
 *            For xy, xz, yz the factors along their two odd axes must have a
 *            zero row 0 (the odd tensor vanishes at zero offset; VIE_E_ARG).
 *   out      receives the new operator; info (may be NULL) as in vie_compress
 *            with tail_bound and fro_norm set to 0.
 * Superdiagonal cores with r1 = r2 = r3 (a Tucker+CP form) take the same
 * core-free z-pass branch as vie_compress_cp.
 */
vie_status vie_op_from_tucker(const int n[3], const int ranks[6][3], const double* cores, const double* factors,
                              vie_op** out, vie_compress_info* info);

/*
 * Entry callback of the cross compressions: write Nt_comp at `count` offsets
 * idx[3 t], idx[3 t + 1], idx[3 t + 2] = (i, j, k), 0 <= i < n1, 0 <= j < n2,
 * 0 <= k < n3 (the defining tensor of vie_compress), into out[2 t],
 * out[2 t + 1] (complex128 interleaved).  Return 0, nonzero on failure.  The
 * library calls it from one host thread at a time with whole batches of
 * fibers (up to n_a times a few hundred entries); it may parallelise inside.
 */
typedef int (*vie_entry_fn)(void* ctx, int comp, long count, const int* idx, double* out);

typedef struct {
    double tol;          /* truncation tolerance, with trunc_rule and max_rank as in
                            vie_compress_opts (applied to the fiber matrices and to the
                            recompression of the cross core) */
    int trunc_rule;
    int max_rank;        /* 0 = no cap */
    int oversample;      /* p: index-set size beyond the rank found (0 = 8) */
    int max_sweeps;      /* sweep limit over the three modes (0 = 8) */
    int n_sample;        /* extra random entries for an a-posteriori error estimate (0 = none) */
    unsigned long long seed;   /* positions of those sample entries */
} vie_cross_opts;

typedef struct {
    long evals[6];           /* entries read to build each component's Tucker form */
    long evals_sample[6];    /* entries read for the error estimate */
    int sweeps[6];           /* sweeps until the index sets stopped changing */
    double sample_rel_err[6];/* estimate of ||A - A~||_F / ||A~||_F from the sample entries
                                (V times their mean squared error) */
    double seconds;          /* host time */
} vie_cross_info;

/*
 * vie_compress_cross -- Tucker cross approximation (the cross-Tucker
 * alternative to the HOSVD named in Sec. IV-A, cost linear in n) of each
 * defining tensor from its entries, without the dense tensor: only mode
 * fibers through index sets chosen by maxvol (alternating over the modes
 * until the sets stop changing) and the entries at the sets' crossings are
 * read through `fn`; the interpolation form is recompressed (QR of the
 * factors, HOSVD of the small core at tol) to orthonormal factors and
 * tolerance-based ranks, then embedded, transformed and uploaded as in
 * vie_compress.  The parity zeros of xy, xz, yz (offset 0 along their odd
 * axes) are taken as exact zeros whatever fn returns there.
 *   n      HOST int[3], 1 <= n_i <= 256, 2 n_i a product of 2, 3, 5, 7.
 *   fn, ctx  entry callback (see vie_entry_fn), components 0..5 = xx .. yz.
 *   opts   HOST, may be NULL (tol 1e-6, rule 0, p 8, 8 sweeps, no sample).
 *   out    receives the new operator; info (may be NULL) as vie_compress,
 *          tail_bound and fro_norm of the recompressed core; xinfo (may be
 *          NULL) the entry counts and the sampled error.
 * Synchronous.  Errors: VIE_E_ARG (also a failing callback), VIE_E_NONFINITE,
 * VIE_E_UNSUPPORTED, VIE_E_NOMEM, VIE_E_HIP.
 */
vie_status vie_compress_cross(const int n[3], vie_entry_fn fn, void* ctx, const vie_cross_opts* opts,
                              vie_op** out, vie_compress_info* info, vie_cross_info* xinfo);

/*
 * vie_tucker_cross -- the same cross approximation of one component `comp`
 * (0..5, with that component's parity zeros) on the host only, returned as
 * a Tucker form: for grids of any size (1 <= n_i <= 65536; no FFT plan is
 * needed) and for checking the compression by itself.
 *   ranks    HOST int[3] out.
 *   core     HOST complex128 out, [r1][r2][r3] (r3 fastest), core_cap complex
 *            entries available (NULL: not returned).
 *   factors  HOST complex128 out, U1 (n1 x r1), U2, U3 row-major one after
 *            another, fac_cap complex entries available (NULL: not returned).
 *   xinfo    HOST, may be NULL; the counts of this component sit at [comp].
 * VIE_E_ARG if a given output is too small (ranks are still set).
 */
vie_status vie_tucker_cross(const int n[3], vie_entry_fn fn, void* ctx, int comp, const vie_cross_opts* opts,
                            int ranks[3], double* core, size_t core_cap, double* factors, size_t fac_cap,
                            vie_cross_info* xinfo);

/* ---------------- piecewise-linear basis (eq. 7a-7b) ----------------
 *
 * Twelve unknowns per voxel: for each current component q the coefficients
 * of the pulse (l = 0) and of the pulse times the normalised local
 * coordinates (x - x_m)/h, (y - y_m)/h, (z - z_m)/h (l = 1, 2, 3).  The sixty
 * unique defining tensors of Sec. II-B are ten basis pairs (l, l'), l <= l',
 * in the order (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3),
 * of six dyadic components each (xx, yy, zz, xy, xz, yz): the Galerkin entry
 * (eq. 8a-8b) of test function (p, l) in voxel 0 against basis function
 * (q, l') in the voxel at offset D, rows divided by the voxel volume (so the
 * self products of the basis are 1 and 1/12).  The other pairs and negative
 * offsets are implied: Nt^(l',l) = -Nt^(l,l') when exactly one of l, l' is
 * 0 (else +), and component (l, l', p, q) is odd along axis a when
 * [p = a] + [q = a] + [l = a + 1] + [l' = a + 1] is odd.
 *
 * The operator acts on coefficients of the mass-normalised basis (linear
 * functions scaled by sqrt 12, unit self products): with S = diag(1, sqrt 12,
 * sqrt 12, sqrt 12) over l it applies S A S, A the paper-basis block
 *   (A u)^{pl}(m) = eps_c(m) m_l u^{pl}(m) - chi(m) sum Nt^{(l,l')}_pq(m' - m) u^{ql'}(m').
 * Vectors: [l][q][n3][n2][n1] (12 components, x fastest).
 */
typedef struct vie_pwl_op vie_pwl_op;

/*
 * vie_compress_pwl -- HOSVD (Alg. 1) of the sixty defining tensors, or
 * Tucker+CP (Alg. 2) when cp_rank >= 0 (as vie_compress_cp, cp_iters 0 =
 * 1000), ten six-component blocks on the current device.
 *   n          HOST int[3], 1 <= n_i <= 256, 2 n_i factoring into 2, 3, 5, 7.
 *   green_pwl  HOST complex128 [10][6][n3][n2][n1] in the pair order above.
 *   opts       HOST, may be NULL (tol 1e-6); the tolerance applies to each
 *              component.
 *   cp_rank    -1 = Tucker (HOSVD) only.
 *   info       HOST vie_compress_info[10] out (one per pair), may be NULL.
 * Errors as vie_compress.
 */
vie_status vie_compress_pwl(const int n[3], const double* green_pwl, const vie_compress_opts* opts, int cp_rank,
                            int cp_iters, vie_pwl_op** out, vie_compress_info* info);

vie_status vie_pwl_op_destroy(vie_pwl_op* op);

/*
 * vie_compress_pwl_k -- the magnetic operator K of eq. 5 (curl of the
 * single-layer potential) in the piecewise-linear basis: HOSVD (Alg. 1) of
 * its thirty defining tensors, ten pairs (l, l') in the order above times the
 * components xy, xz, yz, each the Galerkin entry of test function (p, l) in
 * the observation voxel at offset D against basis function (q, l') in the
 * source voxel 0, rows divided by the voxel volume.  Implied entries:
 * Kt_qp = -Kt_pq (zero diagonal), Kt^(l',l) = sigma Kt^(l,l') with the sigma
 * of N, and component xy / xz / yz (derivative axis s = z / y / x) is odd
 * along axis a when [s = a] + [l = a + 1] + [l' = a + 1] is odd.  The
 * operator applies, in the mass-normalised basis, S K S with
 *   (K u)^{pl}(m) = sum_{q, l', m'} Kt^{(l,l')}_pq(m - m') u^{ql'}(m')
 * through vie_matvec_pwl with kind VIE_OP_N and adjoint 0 only (other calls
 * and vie_solve_pwl return VIE_E_UNSUPPORTED).
 *   n            HOST int[3] as vie_compress_pwl.
 *   green_pwl_k  HOST complex128 [10][3][n3][n2][n1].
 *   opts         HOST, may be NULL (tol 1e-6), per component.
 *   info         HOST vie_compress_info[10] out, may be NULL: per pair as
 *                vie_compress_k (slots 0..2 the zero diagonal).
 * Errors as vie_compress_k.
 */
vie_status vie_compress_pwl_k(const int n[3], const double* green_pwl_k, const vie_compress_opts* opts,
                              vie_pwl_op** out, vie_compress_info* info);

/* grid and the Tucker ranks [pair][component][mode]; either may be NULL (a K
 * operator: components 3..5 = xy, xz, yz, 0..2 the zero diagonal (1, 1, 1)) */
vie_status vie_pwl_op_query(const vie_pwl_op* op, int n[3], int ranks[10][6][3]);

/* DEVICE workspace of vie_matvec_pwl in bytes for nrhs vectors: their 12
 * padded components through the five passes and the core products
 * W_c(k2) = G_c x2 U2_c(k2, :) of the sixty (K: thirty) components for k2 in
 * [0, n2] (shared by the vectors) */
size_t vie_pwl_workspace_bytes(const vie_pwl_op* op, int dtype, int nrhs);

/*
 * vie_matvec_pwl -- y = S A S x (kind VIE_OP_A, needs eps_c) or the bare
 * Galerkin sum S N S x (VIE_OP_N), or their adjoints (adjoint = 1), in the
 * mass-normalised basis: the five passes of vie_matvec with the twelve
 * components as four groups of three and a z pass that adds the sixteen
 * (l, l') blocks per Fourier-domain position, each block's six N^ tables
 * rebuilt from its Tucker form per pencil group (Sec. V-A/B).  For an
 * operator of vie_compress_pwl_k: y = S K S x (VIE_OP_N, adjoint 0), the
 * same passes with each block's three K^ tables and the antisymmetric
 * product.
 *   dtype  VIE_C64 (FP32 compute) or VIE_C128 (FP64) for x, y, eps_c.
 *   eps_c  DEVICE [n3][n2][n1]; x, y DEVICE [nrhs][12][n3][n2][n1], not
 *          overlapping; nrhs in [1, 4096] vectors with the same contrast.
 *   ws     DEVICE, vie_pwl_workspace_bytes(op, dtype, nrhs).
 * Asynchronous on `stream`.  VIE_E_UNSUPPORTED when the z pass does not fit
 * in LDS (2 n3 and the ranks too large).
 */
vie_status vie_matvec_pwl(const vie_pwl_op* op, int kind, int adjoint, int dtype, const void* eps_c, const void* x,
                          void* y, int nrhs, void* ws, size_t ws_bytes, void* stream);

/*
 * vie_tucker_cross_pwl -- vie_tucker_cross for one piecewise-linear
 * component: comp 0..59 the N components 6 P + c (pair P in the order of
 * vie_compress_pwl, dyadic component c), comp 60..89 the thirty K components
 * 60 + 3 P + c (c = xy, xz, yz of the magnetic operator, test function in
 * the observation voxel; each odd along the axis of K's pulse component,
 * flipped by the pair as for N).  The callback receives comp unchanged; the
 * parity zeros follow the component's parities; the counts go to slot c of
 * xinfo (K: slot 3 + c).  Host only, grids up to 65536 per axis (the paper's
 * 270 x 141 x 902 body domain, Table III).
 */
vie_status vie_tucker_cross_pwl(const int n[3], vie_entry_fn fn, void* ctx, int comp, const vie_cross_opts* opts,
                                int ranks[3], double* core, size_t core_cap, double* factors, size_t fac_cap,
                                vie_cross_info* xinfo);

/*
 * vie_tucker_hadamard -- one compressed component applied element-wise on
 * its own grid: y = D .* x with D = G x1 U1 x2 U2 x3 U3 (Tucker, eq. 14) or
 * D(i,j,k) = sum_l lambda_l U1(i,l) U2(j,l) U3(k,l) (Tucker+CP, eq. 17 with
 * the CP weights folded into a diagonal core): the "decompression and
 * element-wise product" of Sec. V-B that Table IV times (and, for CP, its
 * 4-D loop), done in one pass with no buffer for D.  Building block and
 * benchmark of the per-component step; the matvec itself reconstructs its
 * Fourier-domain components inside the z pass.
 *   n      HOST int[3] grid; r HOST int[3] ranks, 1 <= r_a <= 32 (cp: r1 = r2 = r3).
 *   cp     0: core = G [r1][r2][r3] (r3 fastest); 1: core = lambda [r1].
 *   dtype  VIE_C64 or VIE_C128 for every array.
 *   core, u1, u2, u3  DEVICE; U_a is n_a x r_a row-major.
 *   x, y   DEVICE [n3][n2][n1]; y may equal x (in place) but not partly overlap it.
 *   ws     DEVICE workspace of vie_tucker_hadamard_ws_bytes: U1 transposed
 *          (n1 r1 complex), V (n3 n2 r1 complex) and, for Tucker, W (n3 r1 r2
 *          complex).
 * Asynchronous on `stream`.  Errors: VIE_E_ARG, VIE_E_UNSUPPORTED, VIE_E_HIP.
 */
size_t vie_tucker_hadamard_ws_bytes(const int n[3], const int r[3], int cp, int dtype);
vie_status vie_tucker_hadamard(const int n[3], const int r[3], int cp, int dtype, const void* core, const void* u1,
                               const void* u2, const void* u3, const void* x, void* y, void* ws, size_t ws_bytes,
                               void* stream);

/* Release the operator's device memory.  NULL is accepted. */
vie_status vie_op_destroy(vie_op* op);

/* Grid and ranks of an operator (HOST outputs, any may be NULL). */
vie_status vie_op_query(const vie_op* op, int n[3], int ranks[6][3]);

/*
 * vie_op_densify -- materialise the Fourier-domain tensor of every component
 * densely from the Tucker form on the device (half spectrum
 * (n1+1)(n2+1)(n3+1) points per component, the rest follows from parity), at
 * complex64 and, if with_c128, complex128.  Enables VIE_NHAT_DENSE for
 * comparison runs; memory is released by vie_op_destroy.
 */
vie_status vie_op_densify(vie_op* op, int with_c128);
/* Select VIE_NHAT_TUCKER or VIE_NHAT_DENSE for subsequent matvecs. */
vie_status vie_op_set_nhat(vie_op* op, int source);

/* Device workspace (bytes) that vie_matvec / vie_matvec_adjoint need for
 * `nrhs` right-hand sides at precision `dtype` (18 n1 n2 n3 complex per rhs). */
size_t vie_workspace_bytes(const vie_op* op, int dtype, int nrhs);

/*
 * vie_matvec -- y = A x (kind VIE_OP_A) or y = N x (kind VIE_OP_N) for nrhs
 * right-hand sides sharing one operator and one eps_c.
 *   dtype   VIE_C64 or VIE_C128: element type of eps_c, x, y and of the FFTs.
 *   recon   VIE_RECON_*: arithmetic of the Tucker reconstruction (eq. 14 per
 *           k-pencil).  VIE_RECON_BF16 (VIE_C64 only): the z-factor contraction
 *           runs on MFMA with BF16 inputs and FP32 accumulation, about 1e-3
 *           relative error in N^; needs 2 n3 in {128, 256, 512} and z ranks
 *           <= 32, else VIE_E_UNSUPPORTED.
 *   eps_c   DEVICE [n3][n2][n1] complex relative permittivity
 *           eps_r - i sigma/(omega eps0); ignored (may be NULL) for VIE_OP_N.
 *   x       DEVICE [nrhs][3][n3][n2][n1] input.
 *   y       DEVICE, same shape; must not overlap x.
 *   ws      DEVICE workspace of at least vie_workspace_bytes(op, dtype, nrhs).
 * Asynchronous on `stream`.  Errors: VIE_E_ARG, VIE_E_UNSUPPORTED, VIE_E_HIP.
 */
vie_status vie_matvec(const vie_op* op, int kind, int dtype, int recon, const void* eps_c,
                      const void* x, void* y, int nrhs, void* ws, size_t ws_bytes, void* stream);

/*
 * vie_matvec_adjoint -- y = A^H x (VIE_OP_A): conj(eps_c) x - N^H(conj(chi) x),
 * or y = N^H x (VIE_OP_N).  N is complex symmetric (Nt_pq = Nt_qp and every
 * embedded component is even in the full offset), so N^H applies conj(N^).
 * Same arguments and errors as vie_matvec.
 */
vie_status vie_matvec_adjoint(const vie_op* op, int kind, int dtype, int recon, const void* eps_c,
                              const void* x, void* y, int nrhs, void* ws, size_t ws_bytes,
                              void* stream);

/*
 * vie_matvec_noalloc -- the product of vie_matvec (adjoint = 0) or
 * vie_matvec_adjoint (adjoint = 1) for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It allocates nothing and takes no workspace argument:
 * the five passes run in a fixed scratch array of VIE_NOALLOC_SCRATCH_BYTES
 * (256 MiB) that the library holds on each device it runs on until the
 * process ends.  The caller still passes eps_c, x and y as for vie_matvec
 * (same layouts, kinds, dtypes, recon values and results: the same kernels
 * run).  The current device must be the operator's device.
 * Limit: vie_workspace_bytes(op, dtype, nrhs) <= VIE_NOALLOC_SCRATCH_BYTES
 * (e.g. a 96 x 112 x 128 grid with one complex64 right-hand side, 198 MB);
 * larger requests return VIE_E_ARG before any launch.  No part of the
 * scratch needs to start at zero: every pass writes all of what the next
 * pass reads.  Every call on one device shares that device's array, so calls
 * that overlap in time on one device (different streams or host threads)
 * race and give undefined results; calls on one stream are ordered and safe.
 * Not available while per-pass profiling is on (VIE_E_UNSUPPORTED).
 * Asynchronous on `stream`.  Errors: VIE_E_ARG, VIE_E_UNSUPPORTED, VIE_E_HIP.
 */
#define VIE_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
size_t vie_noalloc_scratch_bytes(void);
vie_status vie_matvec_noalloc(const vie_op* op, int kind, int adjoint, int dtype, int recon, const void* eps_c,
                              const void* x, void* y, int nrhs, void* stream);

typedef struct {
    double tol;        /* target relative residual ||b - A x|| / ||b|| (true residual) */
    int restart;       /* GMRES restart length m (inner iterations per cycle), 1..200 */
    int max_outer;     /* maximum restart cycles (plain) or refinement steps (refine = 1) */
    int adjoint;       /* 0: solve A x = b;  1: solve A^H x = b */
    int refine;        /* 0: plain GMRES in `dtype`; 1: iterative refinement: FP64 true
                          residual with the FP64 operator, inner GMRES(m) cycles with FP64
                          Arnoldi on the `inner_recon` operator computed in FP32 (dtype must
                          be VIE_C128) */
    int inner_recon;   /* refine = 1: VIE_RECON_FP32 or VIE_RECON_BF16 (single-instance
                          solves; the FP64 residual recovers the BF16 error) */
    double inner_tol;  /* refine = 1: relative reduction asked of each inner cycle */
} vie_solve_opts;

typedef struct {
    int matvecs;          /* operator applications in the working precision */
    int matvecs_fp64;     /* FP64 residual matvecs (refine = 1) */
    int restarts;         /* completed GMRES cycles */
    int refine_steps;     /* refinement steps (refine = 1) */
    int converged;        /* 1 if the true relative residual reached tol */
    double rel_residual;  /* final true relative residual (in the solve's dtype) */
    double* history;      /* HOST, optional: true relative residual per cycle/step */
    int hist_cap;         /* capacity of history */
    int hist_len;         /* entries written */
} vie_solve_info;

/* Device workspace (bytes) for vie_solve with these options. */
size_t vie_solve_workspace_bytes(const vie_op* op, int dtype, int nrhs, const vie_solve_opts* opts);

/*
 * vie_solve -- restarted GMRES (the paper's solver, Sec. VI-C) on
 * A x = b (or A^H x = b) for nrhs independent right-hand sides.
 *   eps_c   DEVICE [n3][n2][n1] complex (dtype).
 *   b       DEVICE [nrhs][3][n3][n2][n1] complex (dtype).
 *   x       DEVICE, same shape: in = initial guess (zeros for a cold start),
 *           out = solution.  Must not overlap b.
 *   opts    HOST (NULL = tol 1e-6, restart 50, max_outer 200, plain).
 *   info    HOST array of nrhs entries, may be NULL.
 * Arnoldi (classical Gram-Schmidt with one re-orthogonalisation) runs in the
 * precision of dtype; the small Hessenberg least-squares problem is solved on
 * the host.  Systems that converge are dropped from further matvecs.
 * Returns VIE_OK if every system converged, VIE_NOT_CONVERGED if one did not
 * (x is still the last iterate), VIE_E_NONFINITE on a NaN/Inf residual.
 * Synchronises `stream`.
 */
vie_status vie_solve(const vie_op* op, int dtype, const void* eps_c, const void* b, void* x,
                     int nrhs, const vie_solve_opts* opts, vie_solve_info* info, void* ws,
                     size_t ws_bytes, void* stream);

/*
 * vie_solve_pwl -- GMRES(m) solve of S A S x = b (or its adjoint, opts
 * adjoint = 1) for the piecewise-linear operator, one system, x starting at
 * zero: the device Krylov basis and classical Gram-Schmidt of vie_solve_jm
 * (two passes, FP64 dots), restart on the true residual.  With opts refine
 * (VIE_C128 vectors only) the Arnoldi steps apply the operator with FP32
 * products on the FP64 vectors and each restart takes the FP64 residual
 * (inner_tol per cycle).  b, x DEVICE [12][n3][n2][n1] (not overlapping),
 * eps_c DEVICE [n3][n2][n1]; ws DEVICE, vie_solve_pwl_workspace_bytes.
 * Returns VIE_NOT_CONVERGED (x holds the last iterate) when max_outer
 * restarts do not reach tol.  Synchronous on `stream`.
 */
size_t vie_solve_pwl_workspace_bytes(const vie_pwl_op* op, int dtype, const vie_solve_opts* opts);
vie_status vie_solve_pwl(const vie_pwl_op* op, int dtype, const void* eps_c, const void* b, void* x,
                         const vie_solve_opts* opts, vie_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/*
 * vie_matvec_jm_pwl -- the full JMVIE operator of eq. 4 in the
 * piecewise-linear basis, as vie_matvec_jm with twelve coefficients per
 * current and voxel (mass-normalised basis, whose mass term is the identity):
 *     y_J = eps_c J - chi_e (S N S) J + c_e h chi_e (S K S) M,
 *     y_M = mu_c M  - chi_h (S N S) M - c_m h chi_h (S K S) J,
 *   the contrasts constant per voxel multiplying whole Galerkin rows;
 *   op_n from vie_compress_pwl, op_k from vie_compress_pwl_k, same grid
 *   (VIE_E_ARG otherwise).  J and M go through each operator as two
 *   right-hand sides of vie_matvec_pwl, then one kernel combines.
 *   x, y DEVICE complex [2][12][n3][n2][n1] (J then M, not overlapping);
 *   eps_c, mu_c DEVICE complex [n3][n2][n1]; ws DEVICE scratch of
 *   vie_jm_pwl_workspace_bytes(op_n, op_k, dtype) bytes (0 for a null
 *   operator or a bad dtype), owned by the caller.  Asynchronous on
 *   `stream`; VIE_E_ARG for a null pointer, h or omega not positive, a bad
 *   dtype, too small a workspace or overlapping x and y.
 */
size_t vie_jm_pwl_workspace_bytes(const vie_pwl_op* op_n, const vie_pwl_op* op_k, int dtype);
vie_status vie_matvec_jm_pwl(const vie_pwl_op* op_n, const vie_pwl_op* op_k, int dtype, double h, double omega,
                             const void* eps_c, const void* mu_c, const void* x, void* y, void* ws, size_t ws_bytes,
                             void* stream);

/*
 * vie_solve_jm_pwl -- GMRES(m) on vie_matvec_jm_pwl's operator, one system,
 * as vie_solve_jm (forward only, x starting at zero, opts refine with FP32
 * products on VIE_C128 vectors and FP64 restart residuals).  b, x DEVICE
 * [2][12][n3][n2][n1] in the mass-normalised basis (not overlapping);
 * ws DEVICE, vie_solve_jm_pwl_workspace_bytes (0 when the options or the
 * operators are rejected).  Returns VIE_OK, VIE_NOT_CONVERGED with x the
 * last iterate, VIE_E_UNSUPPORTED for opts->adjoint, VIE_E_ARG for bad
 * arguments.  Synchronous on `stream`.
 */
size_t vie_solve_jm_pwl_workspace_bytes(const vie_pwl_op* op_n, const vie_pwl_op* op_k, int dtype,
                                        const vie_solve_opts* opts);
vie_status vie_solve_jm_pwl(const vie_pwl_op* op_n, const vie_pwl_op* op_k, int dtype, double h, double omega,
                            const void* eps_c, const void* mu_c, const void* b, void* x, const vie_solve_opts* opts,
                            vie_solve_info* info, void* ws, size_t ws_bytes, void* stream);


/*
 * Batches of several grids (instances) of uneven size: every pass of the
 * matvec runs as ONE launch over all instances' tiles (the work of each
 * block is looked up in a device table of instances).  Each instance has its
 * own operator, eps_c, vectors and right-hand-side count.
 */
typedef struct {
    const vie_op* op;     /* operator of this instance's grid */
    const void* eps_c;    /* DEVICE [n3][n2][n1] complex (dtype); may be NULL for VIE_OP_N */
    const void* x;        /* DEVICE [nrhs][3][n3][n2][n1] */
    void* y;              /* DEVICE, same shape, no overlap with x */
    int nrhs;
} vie_instance;

/* Workspace (bytes) of vie_matvec_multi for this batch. */
size_t vie_matvec_multi_workspace_bytes(const vie_instance* inst, int count, int dtype);
/* y = A x (kind VIE_OP_A) or N x (VIE_OP_N), or their adjoints (adjoint = 1),
 * for every instance; asynchronous on `stream`.  Mixed-radix kernels, any
 * supported grid per instance; Tucker operators only. */
vie_status vie_matvec_multi(const vie_instance* inst, int count, int kind, int adjoint, int dtype, void* ws,
                            size_t ws_bytes, void* stream);

typedef struct {
    const vie_op* op;
    const void* eps_c;      /* DEVICE [n3][n2][n1] complex (dtype) */
    const void* b;          /* DEVICE [nrhs][3][n3][n2][n1] */
    void* x;                /* DEVICE, same shape: initial guess in, solution out */
    int nrhs;
    vie_solve_info* info;   /* HOST array of nrhs, may be NULL */
} vie_solve_instance;

/* Workspace (bytes) of vie_solve_multi. */
size_t vie_solve_multi_workspace_bytes(const vie_solve_instance* inst, int count, int dtype, const vie_solve_opts* opts);
/* GMRES on every system of every instance in lockstep (as vie_solve): each
 * Arnoldi step issues one multi-instance matvec for all unconverged systems.
 * Returns VIE_OK if every system converged, else VIE_NOT_CONVERGED. */
vie_status vie_solve_multi(const vie_solve_instance* inst, int count, int dtype, const vie_solve_opts* opts, void* ws,
                           size_t ws_bytes, void* stream);

/*
 * Helpers of the differentiable forward model (voxel-wise, asynchronous on
 * `stream`; dtype VIE_C64 with float real maps or VIE_C128 with double).
 * omega_eps0 = 2 pi f eps0 > 0.
 *
 * vie_problem_setup -- eps_c = eps_r - i sigma / (omega eps0) (exp(+i omega t)
 *   convention) and the right-hand side b = c_e chi e_inc, c_e = i omega eps0,
 *   chi = eps_c - 1 (eq. 1-2).  eps_r, sigma DEVICE real [n3][n2][n1];
 *   e_inc, b DEVICE complex [3][n3][n2][n1]; eps_c DEVICE complex [n3][n2][n1].
 */
vie_status vie_problem_setup(const vie_op* op, int dtype, const void* eps_r, const void* sigma, const void* e_inc,
                             double omega_eps0, void* eps_c, void* b, void* stream);
/*
 * vie_total_field -- E = e_inc + (N u - u) / c_e: the total field of the
 *   polarisation current u = c_e chi E (eq. 3).  Nu = vie_matvec(VIE_OP_N, u).
 *   All DEVICE complex [3][n3][n2][n1].
 */
vie_status vie_total_field(const vie_op* op, int dtype, const void* e_inc, const void* u, const void* Nu,
                           double omega_eps0, void* E, void* stream);
/*
 * vie_matvec_jm -- the full JMVIE operator of eq. 4 on x = [J; M] (electric
 *   and magnetic polarisation currents):
 *     y_J = eps_c J - chi_e N J + c_e chi_e K M,
 *     y_M = mu_c M  - chi_h N M - c_m chi_h K J,
 *   chi_e = eps_c - 1, chi_h = mu_c - 1, c_e = i omega eps0, c_m = i omega mu0
 *   (eq. 2), with the N operator op_n (vie_compress) and the K operator op_k
 *   (vie_compress_k) of the same grid, h the voxel edge (the physical K is h
 *   times its dimensionless tensor).  J and M go through each operator as
 *   two right-hand sides (two five-pass products), then one kernel combines.
 *   x, y DEVICE complex [2][3][n3][n2][n1] (J then M, must not overlap);
 *   eps_c, mu_c DEVICE complex [n3][n2][n1]; ws DEVICE scratch of at least
 *   vie_jm_workspace_bytes(op_n, op_k, dtype) bytes.  Asynchronous on stream.
 */
size_t vie_jm_workspace_bytes(const vie_op* op_n, const vie_op* op_k, int dtype);
vie_status vie_matvec_jm(const vie_op* op_n, const vie_op* op_k, int dtype, double h, double omega, const void* eps_c,
                         const void* mu_c, const void* x, void* y, void* ws, size_t ws_bytes, void* stream);

/*
 * vie_solve_jm -- GMRES(m) for the full JMVIE system of eq. 4,
 *   A [J; M] = b, one system, A as in vie_matvec_jm.  The right-hand side of
 *   eq. 1 is b = [c_e chi_e E_inc; c_m chi_h H_inc].  Forward solves only
 *   (opts->adjoint = 1 gives VIE_E_UNSUPPORTED); tol, restart, max_outer as
 *   in vie_solve; x0 = 0; every Arnoldi step takes two classical
 *   Gram-Schmidt passes with FP64 dot products; restart on the true residual.
 *   opts->refine = 1 (VIE_C128 vectors, else VIE_E_ARG): the Arnoldi steps
 *   apply the operator with its N and K products computed in FP32, each
 *   cycle asks for a relative reduction opts->inner_tol, and the restart
 *   residual uses the FP64 operator, so the solve reaches FP64 accuracy
 *   (info->matvecs counts the FP32-product applications, matvecs_fp64 the
 *   residuals, refine_steps the cycles).
 *   b, x DEVICE complex [2][3][n3][n2][n1]; eps_c, mu_c DEVICE complex
 *   [n3][n2][n1]; info (may be NULL) as in vie_solve;
 *   ws DEVICE scratch of vie_solve_jm_workspace_bytes bytes.  Returns VIE_OK,
 *   or VIE_NOT_CONVERGED with x the last iterate.  Synchronises the stream.
 */
size_t vie_solve_jm_workspace_bytes(const vie_op* op_n, const vie_op* op_k, int dtype, const vie_solve_opts* opts);
vie_status vie_solve_jm(const vie_op* op_n, const vie_op* op_k, int dtype, double h, double omega, const void* eps_c,
                        const void* mu_c, const void* b, void* x, const vie_solve_opts* opts, vie_solve_info* info,
                        void* ws, size_t ws_bytes, void* stream);

/*
 * vie_magnetic_field -- H = h_inc + h KJ and |b1+| = mu0 |H_x + i H_y|
 *   (eq. 18) for the polarisation current J of the electric equation, where
 *   KJ = vie_matvec(op_k, VIE_OP_N, J) with op_k from vie_compress_k and h
 *   the voxel edge (the physical K is h times the dimensionless tensor).
 *   h_inc, KJ, H DEVICE complex [3][n3][n2][n1] (dtype); b1 DEVICE real
 *   [n3][n2][n1] (float for VIE_C64, double for VIE_C128).
 */
vie_status vie_magnetic_field(const vie_op* op_k, int dtype, const void* h_inc, const void* KJ, double h, double mu0,
                              void* H, void* b1, void* stream);
/*
 * vie_adjoint_source -- t = N^H g - g, the right-hand side A^H z = (N - I)^H g
 *   of the adjoint solve for an objective gradient g = dL/dRe(E) + i dL/dIm(E).
 */
vie_status vie_adjoint_source(const vie_op* op, int dtype, const void* g, const void* NHg, void* t, void* stream);
/*
 * vie_field_gradient -- with X_n = sum_q conj(z_q(n)) E_q(n):
 *   g_eps[n] = Re X_n = dL/d eps_r(n),  g_sigma[n] = Im X_n / (omega eps0) = dL/d sigma(n),
 *   where z solves A^H z = N^H g - g (chi_n = eps_r - 1 - i sigma/(omega eps0), so
 *   d chi/d eps_r = 1 and d chi/d sigma = -i/(omega eps0)).
 *   z, E DEVICE complex [3][n3][n2][n1]; g_eps, g_sigma DEVICE real [n3][n2][n1].
 */
vie_status vie_field_gradient(const vie_op* op, int dtype, const void* z, const void* E, double omega_eps0,
                              void* g_eps, void* g_sigma, void* stream);

/*
 * Debug / test entry points (bit-exact checks of indexing).
 * vie_debug_nhat: Fourier-domain tensor values N^_c(k1, k2, k3) at `count`
 *   HOST points idx[4*m .. 4*m+3] = (c, k1, k2, k3), 0 <= k_i < 2 n_i, from the
 *   device-resident Tucker form (precision dtype/recon), written to HOST
 *   out[2*m], out[2*m+1] as double.  Includes the 1/(8 n1 n2 n3) inverse-FFT
 *   normalisation that the device core carries.
 */
vie_status vie_debug_nhat(const vie_op* op, int dtype, int recon, const int* idx, int count,
                          double* out);

/*
 * Single passes of the matvec (Sec. V-A: zero padding, circulant embedding
 * and FFT of the currents, the Fourier-domain product, inverse FFT and
 * cropping), for tests of the index maps and of each transform on its own.
 * Buffers are DEVICE complex (dtype VIE_C64 or VIE_C128), caller-owned, in
 * the layouts the five passes exchange, with L_a = 2 n_a (per right-hand
 * side, index order slowest first):
 *   vector  [3][n3][n2][n1]   (the layout of x and y of vie_matvec)
 *   S1, S3  [3][n3][L1][n2]   (after X+, and after Y-)
 *   S2      [3][L2][L1][n3]   (after Y+ and after the z pass; only the n3
 *                               kept z positions of each (k1, k2) pencil)
 * F_L is the unnormalised DFT sum_m a[m] exp(-2 pi i m k / L) and F_L^* its
 * conjugate-kernel counterpart (also unnormalised: the 1/(8 n1 n2 n3) of the
 * inverse transform is carried by the Fourier-domain tensor, see
 * vie_debug_nhat).  All are asynchronous on `stream`; out must not overlap
 * the inputs (except in == out for pass 2).  Errors: VIE_E_ARG (null or
 * overlapping buffers, bad pass/kind/dtype), VIE_E_UNSUPPORTED, VIE_E_HIP.
 *
 * vie_debug_pad -- the index map of pass X+ with the identity in place of
 *   its transform: S1[b][q][k][i][j] = x[b][q][k][j][i] for i < n1 and 0 for
 *   n1 <= i < L1 (zero padding along x, transposed so that y is contiguous).
 *   Same kernel as the matvec's pass (register-FFT kernel for L1 in 128,
 *   192, 224, 256, 512, mixed-radix kernel otherwise).
 * vie_debug_crop -- the index map of pass X- with the identity in place of
 *   its transform and the bare (VIE_OP_N) epilogue:
 *   y[b][q][k][j][i] = S3[b][q][k][i][j] for i < n1 (rows n1..L1-1 dropped).
 *   vie_debug_crop(vie_debug_pad(x)) = x bit for bit.
 * vie_debug_pass -- pass `pass` of the matvec of kind (VIE_OP_A or VIE_OP_N)
 *   and adjoint flag, exactly as vie_matvec runs it:
 *   0 (X+):  in unused; reads x (and eps_c for the A^H pre-scale x <- conj(chi) x);
 *            out S1[b][q][k][.][j] = F_L1 of x[b][q][k][j][.] padded to L1
 *   1 (Y+):  in S1, out S2[b][q][.][i][k] = F_L2 of S1[b][q][k][i][.] padded to L2
 *   2 (Z*):  in S2, out S2 (in may equal out): per pencil (i, j) and output
 *            component p, the first n3 values of
 *            F_L3^* ( sum_q N^_pq(i, j, .) * F_L3(S2[b][q][j][i][.] padded to L3) )
 *            with N^ reconstructed from the Tucker form (conj(N^) for the adjoint;
 *            recon as in vie_matvec)
 *   3 (Y-):  in S2, out S3[b][q][k][i][.] = first n2 values of F_L2^* of S2[b][q][.][i][k]
 *   4 (X-):  in S3, reads x and eps_c for kind A; r = first n1 values of F_L1^* of
 *            S3[b][q][k][.][j]; out y = r (N), eps_c x - chi r (A),
 *            conj(eps_c) x - r (A^H), chi = eps_c - 1.
 */
vie_status vie_debug_pad(const vie_op* op, int dtype, const void* x, void* s1, int nrhs, void* stream);
vie_status vie_debug_crop(const vie_op* op, int dtype, const void* s3, void* y, int nrhs, void* stream);
vie_status vie_debug_pass(const vie_op* op, int pass, int kind, int adjoint, int dtype, int recon,
                          const void* eps_c, const void* x, const void* in, void* out, int nrhs, void* stream);

/*
 * vie_debug_hosvd: the host part of vie_compress for ONE defining tensor,
 * with no device work (for CPU tests of the compression logic).
 *   n       HOST int[3]; tensor HOST complex128 [n3][n2][n1].
 *   ranks   HOST int[3] out: truncation ranks (tol, rule as in vie_compress_opts).
 *   svals   HOST double[n1 + n2 + n3] out (may be NULL): singular values of the
 *           mode-1, mode-2, mode-3 unfoldings, each block descending.
 *   recon   HOST complex128 [n3][n2][n1] out (may be NULL): the Tucker
 *           reconstruction G x1 U1 x2 U2 x3 U3 (eq. 14) of the result.
 *   tail    HOST double out (may be NULL): the discarded-tail bound / ||A||_F.
 */
vie_status vie_debug_hosvd(const int n[3], const double* tensor, double tol, int rule, int ranks[3],
                           double* svals, double* recon, double* tail);

/*
 * vie_debug_cp: the CP step of vie_compress_cp (Alg. 2) for ONE core, with no
 * device work.
 *   r       HOST int[3], 1 <= r_i <= 64; core HOST complex128 [r1][r2][r3].
 *   R       CP rank, 1 <= R <= 64; iters: ALS sweeps (0 = start only).
 *   V       HOST complex128 out, V1 [r1][R] then V2 [r2][R] then V3 [r3][R],
 *           so that core ~ sum_l V1[:, l] (x) V2[:, l] (x) V3[:, l].
 *   rel_err HOST double out (may be NULL): ||core - CP||_F / ||core||_F.
 */
vie_status vie_debug_cp(const int r[3], const double* core, int R, int iters, double* V, double* rel_err);

/*
 * Per-pass timing of the matvec pipeline (for benchmarks).  While enabled,
 * every matvec records a HIP event pair on its stream around each of its five
 * passes (0 = pad + x FFT, 1 = y FFT, 2 = fused z pass with the Tucker
 * reconstruction and component product, 3 = inverse y FFT + crop, 4 =
 * inverse x FFT + crop + contrast).  vie_profile_collect waits for the
 * recorded events, returns the summed milliseconds and launch counts per
 * pass (HOST double[5], int[5]) and clears the record.  Process-wide, not
 * thread-safe; the recording costs two event records per pass.
 */
vie_status vie_profile_enable(int on);
vie_status vie_profile_collect(double ms[5], int counts[5]);

/*
 * Kernel selection (for tests that compare the two implementations): 0 =
 * default (register-FFT kernels for FFT lengths 128, 256, 512, LDS-staged
 * mixed-radix kernels otherwise), 1 = mixed-radix kernels for every pass.
 * Process-wide.
 */
vie_status vie_set_kernel_path(int path);

/*
 * Execution of multi-instance batches (vie_matvec_multi, vie_solve_multi,
 * and every matvec step of their solves): 0 = default: when every instance
 * has register-FFT kernels for its lengths (2 n1, 2 n2 in 128, 192, 224, 256,
 * 512; 2 n3 in 128, 256, 512), one launch per pass and FFT length covers all
 * instances of that length (descriptors in the kernel arguments, up to 24 / 8
 * instances per x-y / z launch), bitwise equal to single-instance calls;
 * otherwise each instance's passes run on their own launches.  1 = one launch
 * per pass covering every instance with the mixed-radix LDS kernels
 * (per-instance plans from a device table).  Process-wide.
 */
vie_status vie_set_batch_mode(int mode);

/*
 * vie_autotune -- pick the launch shape of the fused z pass for this operator
 * by timing the candidates on the device: the number of consecutive k1
 * mirror quads a workgroup takes (4, 8, 16 or 32; fewer means more
 * workgroups, more means the per-k2 core contraction W_c(k2) is shared by
 * more quads).  The choice is stored in the operator and used by every later
 * matvec and solve on it.
 *   dtype   VIE_C64 or VIE_C128 (the arithmetic tuned for).
 *   nrhs    right-hand sides per launch to tune for.
 *   ws      DEVICE workspace of at least vie_workspace_bytes(op, dtype, nrhs);
 *           overwritten (zeroed, then used as the z-pass buffer).
 *   ms      HOST double[4] out (may be NULL): milliseconds per z pass of the
 *           candidates 4, 8, 16, 32 (0 where not applicable).
 *   chosen  HOST int out (may be NULL): the chosen quads per workgroup.
 * Synchronous.  Only the register-FFT z pass (2 n3 = 128, 256, 512) has a
 * tunable shape; for other lengths it returns VIE_OK and changes nothing.
 */
vie_status vie_autotune(vie_op* op, int dtype, int nrhs, void* ws, size_t ws_bytes, void* stream,
                        double ms[4], int* chosen);

/*
 * Captured matvecs: vie_matvec_graph records one vie_matvec /
 * vie_matvec_adjoint (same arguments; adjoint selects which) into a HIP graph
 * on a private stream and instantiates it; vie_graph_launch replays it on
 * `stream` — the same five launches on the same buffers, with one launch
 * call.  The buffers (eps_c, x, y, ws) must stay allocated while the graph
 * exists and their contents are read at replay time.  The operator must not
 * be destroyed or re-tuned while the graph exists.  Per-pass profiling must
 * be off while capturing.
 */
typedef struct vie_graph vie_graph;
vie_status vie_matvec_graph(const vie_op* op, int kind, int adjoint, int dtype, int recon, const void* eps_c,
                            const void* x, void* y, int nrhs, void* ws, size_t ws_bytes, vie_graph** out);
vie_status vie_graph_launch(vie_graph* g, void* stream);
vie_status vie_graph_destroy(vie_graph* g);

const char* vie_last_error(void);
/* library version string */
const char* vie_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VIE_H */
