// Piecewise-linear (PWL) basis, eq. 7a-7b: twelve unknowns per voxel (the
// pulse and three linear functions per current component) and the sixty
// unique defining tensors of Sec. II-B (ten basis pairs l <= l' of six
// dyadic components each), every one held in Tucker form.
//
// The matvec is the five-pass scheme of the pulse basis with the twelve
// components as four groups of three:
//   X+, Y+   the pulse kernels on (l, q) = 4 right-hand sides of 3 components
//   Z        this file: per pencil group, the forward z FFT of all twelve
//            components, the Fourier-domain sum over the sixteen (l, l')
//            blocks, the inverse z FFT
//   Y-, X-   the pulse kernels, X- with the contrast epilogue
//            y = eps_c x - chi (N x)
// The operator acts on coefficients of the mass-normalised basis (linear
// functions scaled by sqrt 12, unit self products), in which that epilogue is
// exact; the blocks carry the factor sqrt 12 per linear function in their
// cores.
//
// The Fourier-domain sum.  Block (l, l') of the Galerkin sum is a convolution
// with K_ll'(E) = Nt^(l,l')(-E).  For a stored pair (a, b), a <= b, with
// T = the transform of the parity-embedded Nt^(a,b) (eq. 13-14 per pencil):
//   K^_ab = sigma T,   K^_ba = T,   sigma = -1 iff exactly one of a, b is 0,
// because reflecting every axis multiplies Nt^(a,b) by sigma and
// Nt^(a,b)(-E) = Nt^(b,a)(E).  The adjoint takes conj(T) with sigma moved to
// the (b, a) block.  T is symmetric over the dyadic pair (p, q), so each
// block is the 3 x 3 product of the pulse basis.
//
// Kernel layout: one workgroup per mirror group of pencils (as the generic z
// pass), the twelve pencils of each in LDS; every thread owns up to EPT
// Fourier-domain positions and keeps their twelve output components in
// registers while the ten pairs go by, each pair's six tables rebuilt from
// the Tucker form into LDS (W = G x3 U3 contracted with the y row, then the
// x row, then the z factor per k3).
#include <hip/hip_runtime.h>

#include <string>

#include "fft_device.h"

#include "vie.h"
#include "vie_internal.h"

namespace vie {
vie_status fail(vie_status st, const std::string& msg);
vie_status hip_fail(hipError_t e, const char* where);
}  // namespace vie

namespace {

using namespace vie;

constexpr int kNT = 256;

struct PwlZArgs {
    int n[3];
    int L[3];
    int G;       // pencils per workgroup (mirror group size: 1, 2 or 4)
    int conj;    // adjoint
    int rmax;    // largest Tucker rank over the ten blocks
};

template <typename T>
__device__ __forceinline__ void sym3(const c2<T> (&N)[6], const c2<T> (&x)[3], c2<T> (&y)[3])
{
    y[0] = N[0] * x[0] + N[3] * x[1] + N[4] * x[2];
    y[1] = N[3] * x[0] + N[1] * x[1] + N[5] * x[2];
    y[2] = N[4] * x[0] + N[5] * x[1] + N[2] * x[2];
}

template <typename T, int MAXE, int EPT>
__global__ void __launch_bounds__(kNT) k_pwl_z(c2<T>* __restrict__ S2, FftPlan pl, const c2<T>* __restrict__ tw,
                                               PwlZArgs a, const PwlBlock<T>* __restrict__ blk)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n1 = a.n[0], n2 = a.n[1], n3 = a.n[2];
    const int L1 = a.L[0], L2 = a.L[1], L3 = a.L[2];
    const int rmax = a.rmax;
    const int tid = threadIdx.x;

    // ---- the pencils of this workgroup: (k1, k2) and its mirrors
    int k1, k2, f1base = 0, f2base = 0;
    int P = 0;
    int pk1[4], pk2[4], pf1[4], pf2[4];
    {
        const int bidx = blockIdx.x;
        if (a.G == 4) {
            k1 = bidx % (n1 + 1);
            k2 = bidx / (n1 + 1);
        } else if (a.G == 2) {
            k1 = bidx % (n1 + 1);
            const int kk2 = bidx / (n1 + 1);
            k2 = kk2 <= n2 ? kk2 : L2 - kk2;
            f2base = kk2 > n2;
        } else {
            const int kk1 = bidx % L1, kk2 = bidx / L1;
            k1 = kk1 <= n1 ? kk1 : L1 - kk1;
            f1base = kk1 > n1;
            k2 = kk2 <= n2 ? kk2 : L2 - kk2;
            f2base = kk2 > n2;
        }
        const bool m1 = (a.G >= 2) && k1 > 0 && k1 < n1;
        const bool m2 = (a.G == 4) && k2 > 0 && k2 < n2;
        for (int s2 = 0; s2 <= (m2 ? 1 : 0); ++s2)
            for (int s1 = 0; s1 <= (m1 ? 1 : 0); ++s1) {
                const int f1 = f1base | s1, f2 = f2base | s2;
                pk1[P] = f1 ? L1 - k1 : k1;
                pk2[P] = f2 ? L2 - k2 : k2;
                pf1[P] = f1;
                pf2[P] = f2;
                ++P;
            }
    }

    // ---- LDS: pencils [12 * G][L3] (sequence (3 l + q) * P + pencil), the
    // six N^ tables of the current pair, W, V, twiddles
    c2<T>* X = reinterpret_cast<c2<T>*>(smem_raw);
    c2<T>* NT6 = X + (size_t)12 * a.G * L3;        // [6][n3 + 1]
    c2<T>* Wc = NT6 + (size_t)6 * (n3 + 1);        // [rmax * rmax]
    c2<T>* Vc = Wc + (size_t)rmax * rmax;          // [6][rmax]
    c2<T>* tws = Vc + (size_t)6 * rmax;            // [L3]
    for (int m = tid; m < L3; m += kNT) tws[m] = tw[m];

    for (int e = tid; e < 12 * P * L3; e += kNT) {
        const int s = e / L3, m = e - s * L3;
        const int comp = s / P, pe = s - comp * P;
        c2<T> val = mk<T>(0, 0);
        if (m < n3) val = S2[(((long)comp * L2 + pk2[pe]) * L1 + pk1[pe]) * n3 + m];
        X[s * L3 + m] = val;
    }
    __syncthreads();
    fft_lds<-1, false, MAXE>(X, 12 * P, L3, 1, pl, tws, tid, kNT);

    c2<T> acc[12][EPT];
#pragma unroll
    for (int c = 0; c < 12; ++c)
#pragma unroll
        for (int j = 0; j < EPT; ++j) acc[c][j] = mk<T>(0, 0);

#pragma unroll 1
    for (int b = 0; b < 10; ++b) {
        const OpView& v = blk[b].v;
        const c2<T>* core = blk[b].core;
        const c2<T>* fac = blk[b].fac;
        // ---- N^_c(k1, k2, k3) of this pair for k3 in [0, n3]
        for (int c = 0; c < 6; ++c) {
            const int r1 = v.r[c][0], r2 = v.r[c][1], r3 = v.r[c][2];
            const c2<T>* Gc = core + v.core_off[c];
            const c2<T>* U1 = fac + v.fac_off[c][0] + (long)k1 * r1;
            const c2<T>* U2 = fac + v.fac_off[c][1] + (long)k2 * r2;
            for (int e = tid; e < r1 * r3; e += kNT) {
                const int al = e / r3, ga = e - al * r3;
                c2<T> s = mk<T>(0, 0);
                for (int be = 0; be < r2; ++be) fma_c(s, Gc[((long)al * r2 + be) * r3 + ga], U2[be]);
                Wc[e] = s;
            }
            __syncthreads();
            for (int ga = tid; ga < r3; ga += kNT) {
                c2<T> s = mk<T>(0, 0);
                for (int al = 0; al < r1; ++al) fma_c(s, U1[al], Wc[al * r3 + ga]);
                Vc[c * rmax + ga] = s;
            }
            __syncthreads();
        }
        for (int e = tid; e < 6 * (n3 + 1); e += kNT) {
            const int c = e / (n3 + 1), kk = e - c * (n3 + 1);
            const int r3 = v.r[c][2];
            const c2<T>* U3 = fac + v.fac_off[c][2] + (long)kk * r3;
            c2<T> s = mk<T>(0, 0);
            for (int ga = 0; ga < r3; ++ga) fma_c(s, Vc[c * rmax + ga], U3[ga]);
            NT6[e] = s;
        }
        __syncthreads();

        // ---- the (a, b) and (b, a) blocks on every owned position
        const int la = kPwlPairs[b][0], lb = kPwlPairs[b][1];
        const T sig = ((la == 0) != (lb == 0)) ? (T)-1 : (T)1;
        const T sab = a.conj ? (T)1 : sig;     // factor of the (a, b) block
        const T sba = a.conj ? sig : (T)1;     // factor of the (b, a) block
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = tid + j * kNT;
            if (e < P * L3) {
                const int pe = e / L3, m = e - pe * L3;
                const int f3 = m > n3;
                const int kk = f3 ? L3 - m : m;
                c2<T> Nc[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    c2<T> t = NT6[c * (n3 + 1) + kk];
                    const int neg = (view_odd(0, v.lmask, c, 0) & pf1[pe]) ^ (view_odd(0, v.lmask, c, 1) & pf2[pe]) ^
                                    (view_odd(0, v.lmask, c, 2) & f3);
                    if (neg) t = mk<T>(-t.x, -t.y);
                    Nc[c] = a.conj ? vie::conj(t) : t;
                }
                c2<T> xa[3], xb[3], y[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    xa[q] = X[((3 * la + q) * P + pe) * L3 + m];
                    xb[q] = X[((3 * lb + q) * P + pe) * L3 + m];
                }
                sym3(Nc, xb, y);
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    // register arrays need compile-time indices: select the row
#pragma unroll
                    for (int l = 0; l < 4; ++l)
                        if (l == la) acc[3 * l + q][j] = acc[3 * l + q][j] + sab * y[q];
                }
                if (la != lb) {
                    sym3(Nc, xa, y);
#pragma unroll
                    for (int q = 0; q < 3; ++q)
#pragma unroll
                        for (int l = 0; l < 4; ++l)
                            if (l == lb) acc[3 * l + q][j] = acc[3 * l + q][j] + sba * y[q];
                }
            }
        }
        __syncthreads();
    }

    // ---- outputs back into the pencils, inverse FFT, cropped store
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int e = tid + j * kNT;
        if (e < P * L3) {
            const int pe = e / L3, m = e - pe * L3;
#pragma unroll
            for (int c = 0; c < 12; ++c) X[(c * P + pe) * L3 + m] = acc[c][j];
        }
    }
    __syncthreads();
    fft_lds<1, false, MAXE>(X, 12 * P, L3, 1, pl, tws, tid, kNT);
    for (int e = tid; e < 12 * P * n3; e += kNT) {
        const int s = e / n3, m = e - s * n3;
        const int comp = s / P, pe = s - comp * P;
        S2[(((long)comp * L2 + pk2[pe]) * L1 + pk1[pe]) * n3 + m] = X[s * L3 + m];
    }
}

template <typename T>
constexpr int pwl_ept()
{
    return 2;   // owned positions per thread: G * L3 <= EPT * 256
}

template <typename T>
size_t pwl_z_lds(const OpView& v, int rmax, int G)
{
    return sizeof(c2<T>) * ((size_t)12 * G * v.L[2] + 6 * (size_t)(v.n[2] + 1) + (size_t)rmax * rmax +
                            6 * (size_t)rmax + v.L[2]);
}

// pencils per workgroup for the z pass; 0 = does not fit
template <typename T>
int pwl_z_group(const DeviceOp& op, int rmax)
{
    for (int G = 4; G >= 1; G /= 2)
        if ((size_t)G * op.view.L[2] <= (size_t)pwl_ept<T>() * kNT && pwl_z_lds<T>(op.view, rmax, G) <= op.max_lds)
            return G;
    return 0;
}

template <typename T>
hipError_t launch_pwl_z(const vie_pwl_op& P, int conj, c2<T>* S2, hipStream_t s, std::string& err)
{
    const DeviceOp& op = P.blk[0]->d;
    const OpView& v = op.view;
    const int G = pwl_z_group<T>(op, P.rmax);
    if (G == 0) {
        err = "the piecewise-linear z pass does not fit in LDS (z length or ranks too large)";
        return hipErrorInvalidValue;
    }
    PwlZArgs za;
    for (int a = 0; a < 3; ++a) {
        za.n[a] = v.n[a];
        za.L[a] = v.L[a];
    }
    za.G = G;
    za.conj = conj;
    za.rmax = P.rmax;
    const int n1 = v.n[0], n2 = v.n[1];
    const int nblk = G == 4 ? (n1 + 1) * (n2 + 1) : (G == 2 ? (n1 + 1) * v.L[1] : v.L[0] * v.L[1]);
    const size_t lds = pwl_z_lds<T>(v, P.rmax, G);
    const c2<T>* tw;
    const PwlBlock<T>* blk;
    if constexpr (sizeof(T) == 8) {
        tw = op.tw64[2];
        blk = P.dev64;
    } else {
        tw = op.tw32[2];
        blk = P.dev32;
    }
    constexpr int EPT = pwl_ept<T>();
    constexpr int MAXE = 12 * EPT;
    auto kern = k_pwl_z<T, MAXE, EPT>;
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(kNT), lds, s, S2, op.plan[2], tw, za, blk);
    return hipGetLastError();
}

template <typename T>
hipError_t pwl_matvec(const vie_pwl_op& P, int mode, const c2<T>* eps, const c2<T>* x, c2<T>* y, c2<T>* ws,
                      hipStream_t s, std::string& err)
{
    const DeviceOp& op = P.blk[0]->d;
    const OpView& v = op.view;
    c2<T>* S2 = ws;
    c2<T>* S1 = ws + (size_t)3 * v.L[1] * v.L[0] * v.n[2] * 4;
    const bool conj = (mode == MODE_AH || mode == MODE_NH);
    // X+ : x -> S1, Y+ : S1 -> S2, Z : S2 in place, Y- : S2 -> S1, X- : S1 -> y
    hipError_t e = run_pass<T, T>(op, 0, mode, 0, eps, x, nullptr, S1, 4, s, nullptr, err, false);
    if (e == hipSuccess) e = run_pass<T, T>(op, 1, mode, 0, eps, x, S1, S2, 4, s, nullptr, err, false);
    if (e == hipSuccess) e = launch_pwl_z<T>(P, conj ? 1 : 0, S2, s, err);
    if (e == hipSuccess) e = run_pass<T, T>(op, 3, mode, 0, eps, x, S2, S1, 4, s, nullptr, err, false);
    if (e == hipSuccess) e = run_pass<T, T>(op, 4, mode, 0, eps, x, S1, y, 4, s, nullptr, err, false);
    return e;
}

}  // namespace

extern "C" {

size_t vie_pwl_workspace_bytes(const vie_pwl_op* op, int dtype)
{
    if (!op || !op->blk[0]) return 0;
    const size_t el = dtype == VIE_C128 ? sizeof(c2<double>) : sizeof(c2<float>);
    return matvec_ws_elems(op->blk[0]->d, 4) * el;
}

vie_status vie_pwl_op_query(const vie_pwl_op* op, int n[3], int ranks[10][6][3])
{
    if (!op || !op->blk[0]) return fail(VIE_E_ARG, "vie_pwl_op_query: null operator");
    const OpView& v0 = op->blk[0]->d.view;
    if (n)
        for (int a = 0; a < 3; ++a) n[a] = v0.n[a];
    if (ranks)
        for (int b = 0; b < 10; ++b)
            for (int c = 0; c < 6; ++c)
                for (int a = 0; a < 3; ++a) ranks[b][c][a] = op->blk[b]->d.view.r[c][a];
    return VIE_OK;
}

vie_status vie_matvec_pwl(const vie_pwl_op* op, int kind, int adjoint, int dtype, const void* eps_c, const void* x,
                          void* y, void* ws, size_t ws_bytes, void* stream)
{
    if (!op || !op->blk[0] || !x || !y || !ws) return fail(VIE_E_ARG, "vie_matvec_pwl: null argument");
    if (kind != VIE_OP_A && kind != VIE_OP_N) return fail(VIE_E_ARG, "vie_matvec_pwl: bad kind");
    if (adjoint != 0 && adjoint != 1) return fail(VIE_E_ARG, "vie_matvec_pwl: adjoint must be 0 or 1");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_matvec_pwl: bad dtype");
    if (kind == VIE_OP_A && !eps_c) return fail(VIE_E_ARG, "vie_matvec_pwl: eps_c is required for VIE_OP_A");
    if (ws_bytes < vie_pwl_workspace_bytes(op, dtype)) return fail(VIE_E_ARG, "vie_matvec_pwl: workspace too small");
    const OpView& v = op->blk[0]->d.view;
    const size_t vbytes = (size_t)12 * v.n[0] * v.n[1] * v.n[2] * (dtype == VIE_C128 ? 16 : 8);
    const char* xb = (const char*)x;
    const char* yb = (const char*)y;
    if (!(xb + vbytes <= yb || yb + vbytes <= xb)) return fail(VIE_E_ARG, "vie_matvec_pwl: x and y overlap");
    const int mode = kind == VIE_OP_A ? (adjoint ? MODE_AH : MODE_A) : (adjoint ? MODE_NH : MODE_N);
    hipStream_t s = (hipStream_t)stream;
    std::string err;
    hipError_t e = dtype == VIE_C128
                       ? pwl_matvec<double>(*op, mode, (const c2<double>*)eps_c, (const c2<double>*)x, (c2<double>*)y,
                                            (c2<double>*)ws, s, err)
                       : pwl_matvec<float>(*op, mode, (const c2<float>*)eps_c, (const c2<float>*)x, (c2<float>*)y,
                                           (c2<float>*)ws, s, err);
    if (e != hipSuccess) {
        if (!err.empty()) return fail(VIE_E_UNSUPPORTED, "vie_matvec_pwl: " + err);
        return hip_fail(e, "vie_matvec_pwl launch");
    }
    return VIE_OK;
}

}  // extern "C"
