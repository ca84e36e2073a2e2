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
// The magnetic operator K (eq. 5) in the same basis runs through the same
// kernels with the operator family as a template argument: thirty stored
// tensors (ten pairs x xy, xz, yz, the block views' slots 3..5), the
// antisymmetric 3 x 3 product Kt_qp = -Kt_pq, and, since K's sum is a
// convolution over m - m' (test function at the observation voxel),
//   K^_ab = T,   K^_ba = sigma T.
// The coupled JM operator of eq. 4 takes [J; M] as two right-hand sides of
// the N and of the K product and combines them per voxel.
//
// Kernel layout: one 512-thread workgroup per mirror group of pencils (as
// the generic z pass), the twelve pencils of each in LDS; every thread owns
// up to EPT Fourier-domain positions and keeps their twelve output
// components in registers while the ten pairs go by, in batches whose
// tables fit the LDS together, each table rebuilt from the Tucker form:
// W_c(k2) = G_c x2 U2_c(k2, :) comes from a small kernel that runs first
// (once per canonical k2, not per pencil group), V_c = U1_c(k1, :) W_c(k2),
// then the z factor per k3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <string>
#include <utility>

#include "fft_device.h"
#include "krylov.h"

#include "vie.h"
#include "vie_internal.h"

namespace vie {
vie_status fail(vie_status st, const std::string& msg);
vie_status hip_fail(hipError_t e, const char* where);
}  // namespace vie

namespace {

using namespace vie;

constexpr int kNT = 256;    // threads of the W kernel
size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr int kNTZ = 512;   // threads of the z kernel

template <typename T>
__device__ __forceinline__ void sym3(const c2<T> (&N)[6], const c2<T> (&x)[3], c2<T> (&y)[3])
{
    y[0] = N[0] * x[0] + N[3] * x[1] + N[4] * x[2];
    y[1] = N[3] * x[0] + N[1] * x[1] + N[5] * x[2];
    y[2] = N[4] * x[0] + N[5] * x[1] + N[2] * x[2];
}

// the antisymmetric 3 x 3 product of K (eq. 5: Kt_pq = eps_psq F_s) from its
// xy, xz, yz entries
template <typename T>
__device__ __forceinline__ void asym3(const c2<T> (&K)[3], const c2<T> (&x)[3], c2<T> (&y)[3])
{
    y[0] = K[0] * x[1] + K[1] * x[2];
    y[1] = K[2] * x[2] - K[0] * x[0];
    y[2] = (T)-1 * (K[1] * x[0] + K[2] * x[1]);
}

// components per stored pair and the first slot of the block views: N keeps
// all six, K the three off-diagonal ones (slots 3..5)
template <int FAM>
constexpr int pwl_nc()
{
    return FAM ? 3 : 6;
}

struct PwlZArgs {
    int n[3];
    int L[3];
    int G;       // pencils per workgroup (mirror group size: 1, 2 or 4)
    int conj;    // adjoint
    int rmax;    // largest Tucker rank over the ten blocks
    int pb;      // pairs whose tables are built and applied together (1..10)
    // for each mirror-flag combination f = f1 | f2 << 1 | f3 << 2, the tables
    // that change sign there: bit b * nc + c of neg[f] is set when component c
    // of pair b is odd along an odd number of the flagged axes
    unsigned long long neg[8];
};

// the sign bit of table t under the flags' mask nm
__device__ __forceinline__ bool pwl_neg(unsigned long long nm, int t)
{
    return (nm >> t) & 1ull;
}

// the (a, b) and (b, a) blocks of stored pair B on one Fourier position,
// pair indices known at compile time (no runtime selection of registers).
// N (FAM 0): K^_ab = sigma T, K^_ba = T (the sum runs over m' - m);
// K (FAM 1): K^_ab = T, K^_ba = sigma T (the sum runs over m - m'); no adjoint
template <int B, int FAM, typename T>
__device__ __forceinline__ void pwl_pair(c2<T> (&acc)[12], const c2<T> (&x)[12], const c2<T>* NTT, int n3p1, int kk,
                                         unsigned long long nm, bool conj)
{
    constexpr int la = kPwlPairs[B][0], lb = kPwlPairs[B][1];
    constexpr bool sig = (la == 0) != (lb == 0);
    constexpr int NC = pwl_nc<FAM>();
    c2<T> N[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        c2<T> t = NTT[(B * NC + c) * n3p1 + kk];
        if (pwl_neg(nm, B * NC + c)) t = mk<T>(-t.x, -t.y);
        N[c] = conj ? vie::conj(t) : t;
    }
    T sab, sba;
    if constexpr (FAM == 0) {
        sab = (sig && !conj) ? (T)-1 : (T)1;
        sba = (sig && conj) ? (T)-1 : (T)1;
    } else {
        sab = (T)1;
        sba = sig ? (T)-1 : (T)1;
    }
    c2<T> y[3];
    const c2<T> xb[3] = {x[3 * lb], x[3 * lb + 1], x[3 * lb + 2]};
    if constexpr (FAM == 0) sym3(N, xb, y);
    else asym3(N, xb, y);
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[3 * la + q] = acc[3 * la + q] + sab * y[q];
    if constexpr (la != lb) {
        const c2<T> xa[3] = {x[3 * la], x[3 * la + 1], x[3 * la + 2]};
        if constexpr (FAM == 0) sym3(N, xa, y);
        else asym3(N, xa, y);
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[3 * lb + q] = acc[3 * lb + q] + sba * y[q];
    }
}

template <int FAM, typename T, int... B>
__device__ __forceinline__ void pwl_all_pairs(c2<T> (&acc)[12], const c2<T> (&x)[12], const c2<T>* NTT, int n3p1,
                                              int kk, unsigned long long nm, bool conj,
                                              std::integer_sequence<int, B...>)
{
    (pwl_pair<B, FAM, T>(acc, x, NTT, n3p1, kk, nm, conj), ...);
}

// mixed-radix LDS transform of the 12 P pencils (sequence-major); LC > 0:
// the length is known at compile time
template <int DIR, int MAXE, int LC, typename T>
__device__ __forceinline__ void pwl_fft(c2<T>* X, int nseq, int L3, const FftPlan& pl, const c2<T>* tws, int tid)
{
    if constexpr (LC == 252) {   // the head grid's z length (126 voxels)
        stage_r<7, DIR, false, MAXE>(X, nseq, LC, 1, LC, 1, tws, tid, kNTZ);
        stage_r<4, DIR, false, MAXE>(X, nseq, LC, 1, LC, 7, tws, tid, kNTZ);
        stage_r<3, DIR, false, MAXE>(X, nseq, LC, 1, LC, 28, tws, tid, kNTZ);
        stage_r<3, DIR, false, MAXE>(X, nseq, LC, 1, LC, 84, tws, tid, kNTZ);
    } else {
        fft_lds_len<DIR, false, MAXE, LC>(X, nseq, L3, 1, pl, tws, tid, kNTZ);
    }
}

// W_c(k2) = G_c x2 U2_c(k2, :) (r1 x r3) for every component of the ten
// blocks and every canonical k2 in [0, n2], once per matvec:
// Wg[((k2 * 10 nc) + nc b + c) * rmax^2 + al * r3 + ga] (nc components per
// block).  The z pass then only contracts the x row and the z factor per
// pencil group.
template <typename T, int FAM>
__global__ void __launch_bounds__(kNT) k_pwl_w(const PwlBlock<T>* __restrict__ blk, int rmax, c2<T>* __restrict__ Wg)
{
    constexpr int NC = pwl_nc<FAM>(), C0 = 6 - NC;
    const int k2 = blockIdx.x, bc = blockIdx.y;
    const int b = bc / NC, c = C0 + bc - NC * b;
    const OpView& v = blk[b].v;
    const int r1 = v.r[c][0], r2 = v.r[c][1], r3 = v.r[c][2];
    const c2<T>* Gc = blk[b].core + v.core_off[c];
    const c2<T>* U2 = blk[b].fac + v.fac_off[c][1] + (long)k2 * r2;
    c2<T>* out = Wg + ((size_t)k2 * 10 * NC + bc) * rmax * rmax;
    for (int e = threadIdx.x; e < r1 * r3; e += kNT) {
        const int al = e / r3, ga = e - al * r3;
        c2<T> s = mk<T>(0, 0);
        for (int be = 0; be < r2; ++be) fma_c(s, Gc[((long)al * r2 + be) * r3 + ga], U2[be]);
        out[e] = s;
    }
}

template <typename T, int MAXE, int EPT, int LC, int FAM>
__global__ void __launch_bounds__(kNTZ) k_pwl_z(c2<T>* __restrict__ S2, FftPlan pl, const c2<T>* __restrict__ tw,
                                               PwlZArgs a, const PwlBlock<T>* __restrict__ blk,
                                               const c2<T>* __restrict__ Wg)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n1 = a.n[0], n2 = a.n[1];
    const int n3 = LC ? LC / 2 : a.n[2];
    const int L1 = a.L[0], L2 = a.L[1], L3 = LC ? LC : a.L[2];
    S2 += (long)blockIdx.y * 12 * L2 * L1 * n3;   // right-hand side
    const int rmax = a.rmax;
    const int tid = threadIdx.x;
    constexpr int NC = pwl_nc<FAM>(), C0 = 6 - NC;

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
    // N^ tables and V of a batch of pairs, twiddles
    c2<T>* X = reinterpret_cast<c2<T>*>(smem_raw);
    c2<T>* NTT = X + (size_t)12 * a.G * L3;         // [pb][NC][n3 + 1]
    c2<T>* Vc = NTT + (size_t)a.pb * NC * (n3 + 1); // [pb][NC][rmax]
    c2<T>* tws = Vc + (size_t)a.pb * NC * rmax;     // [L3]
    unsigned long long* negs = reinterpret_cast<unsigned long long*>(tws + L3);   // [8]
    for (int m = tid; m < L3; m += kNTZ) tws[m] = tw[m];
    if (tid == 0) {
#pragma unroll
        for (int f = 0; f < 8; ++f) negs[f] = a.neg[f];
    }

    for (int e = tid; e < 12 * P * L3; e += kNTZ) {
        const int s = e / L3, m = e - s * L3;
        const int comp = s / P, pe = s - comp * P;
        c2<T> val = mk<T>(0, 0);
        if (m < n3) val = S2[(((long)comp * L2 + pk2[pe]) * L1 + pk1[pe]) * n3 + m];
        X[s * L3 + m] = val;
    }
    __syncthreads();
    pwl_fft<-1, MAXE, LC>(X, 12 * P, L3, pl, tws, tid);

    c2<T> acc[12][EPT];
#pragma unroll
    for (int c = 0; c < 12; ++c)
#pragma unroll
        for (int j = 0; j < EPT; ++j) acc[c][j] = mk<T>(0, 0);

    // ---- the ten pairs in batches of a.pb whose tables fit in LDS together:
    // per batch V_c = U1_c(k1, :) W_c(k2) of every component, then the
    // N^_c(k1, k2, k3) tables for k3 in [0, n3], then the (a, b) and (b, a)
    // blocks of every pair on every owned position
#pragma unroll 1
    for (int b0 = 0; b0 < 10; b0 += a.pb) {
        const int nb = min(a.pb, 10 - b0);
        for (int e = tid; e < nb * NC * rmax; e += kNTZ) {
            const int bc = e / rmax, ga = e - bc * rmax;
            const int b = b0 + bc / NC, c = C0 + bc % NC;
            const OpView& v = blk[b].v;
            const int r1 = v.r[c][0], r3 = v.r[c][2];
            if (ga < r3) {
                const c2<T>* U1 = blk[b].fac + v.fac_off[c][0] + (long)k1 * r1;
                const c2<T>* W = Wg + ((size_t)k2 * 10 * NC + NC * b + c - C0) * rmax * rmax + ga;
                c2<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
                int al = 0;
                for (; al + 4 <= r1; al += 4) {
                    const c2<T> w0 = W[al * r3], w1 = W[(al + 1) * r3], w2 = W[(al + 2) * r3], w3 = W[(al + 3) * r3];
                    fma_c(s0, U1[al], w0);
                    fma_c(s1, U1[al + 1], w1);
                    fma_c(s0, U1[al + 2], w2);
                    fma_c(s1, U1[al + 3], w3);
                }
                for (; al < r1; ++al) fma_c(s0, U1[al], W[al * r3]);
                Vc[e] = s0 + s1;
            }
        }
        __syncthreads();
        for (int e = tid; e < nb * NC * (n3 + 1); e += kNTZ) {
            // z factor read column-major ([g][k3]): consecutive threads take
            // consecutive k3; four rows in flight
            const int bc = e / (n3 + 1), kk = e - bc * (n3 + 1);
            const int b = b0 + bc / NC, c = C0 + bc % NC;
            const OpView& v = blk[b].v;
            const int r3 = v.r[c][2];
            const long st = n3 + 1;
            const c2<T>* U3 = blk[b].fac + v.fac3t_off[c] + kk;
            const c2<T>* vc = Vc + bc * rmax;
            c2<T> s0 = mk<T>(0, 0), s1 = mk<T>(0, 0);
            int ga = 0;
            for (; ga + 4 <= r3; ga += 4) {
                const c2<T> u0 = U3[ga * st], u1 = U3[(ga + 1) * st], u2 = U3[(ga + 2) * st], u3 = U3[(ga + 3) * st];
                fma_c(s0, vc[ga], u0);
                fma_c(s1, vc[ga + 1], u1);
                fma_c(s0, vc[ga + 2], u2);
                fma_c(s1, vc[ga + 3], u3);
            }
            for (; ga < r3; ++ga) fma_c(s0, vc[ga], U3[ga * st]);
            NTT[e] = s0 + s1;
        }
        __syncthreads();

#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = tid + j * kNTZ;
            if (e < P * L3) {
                const int pe = e / L3, m = e - pe * L3;
                const int f3 = m > n3;
                const int kk = f3 ? L3 - m : m;
                c2<T> x[12];
#pragma unroll
                for (int c = 0; c < 12; ++c) x[c] = X[(c * P + pe) * L3 + m];
                const unsigned fb = (unsigned)pf1[pe] | ((unsigned)pf2[pe] << 1) | ((unsigned)f3 << 2);
                const unsigned long long nm = negs[fb];
                if (nb == 10) {
                    c2<T> ac[12];
#pragma unroll
                    for (int c = 0; c < 12; ++c) ac[c] = acc[c][j];
                    pwl_all_pairs<FAM, T>(ac, x, NTT, n3 + 1, kk, nm, a.conj != 0,
                                          std::make_integer_sequence<int, 10>{});
#pragma unroll
                    for (int c = 0; c < 12; ++c) acc[c][j] = ac[c];
                    continue;
                }
#pragma unroll 1
                for (int bi = 0; bi < nb; ++bi) {
                    const int b = b0 + bi;
                    const int la = kPwlPairs[b][0], lb = kPwlPairs[b][1];
                    const T sig = ((la == 0) != (lb == 0)) ? (T)-1 : (T)1;
                    // factors of the (a, b) and (b, a) blocks (as pwl_pair)
                    const T sab = FAM ? (T)1 : (a.conj ? (T)1 : sig);
                    const T sba = FAM ? sig : (a.conj ? sig : (T)1);
                    c2<T> Nc[NC];
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        c2<T> t = NTT[(bi * NC + c) * (n3 + 1) + kk];
                        if (pwl_neg(nm, b * NC + c)) t = mk<T>(-t.x, -t.y);
                        Nc[c] = a.conj ? vie::conj(t) : t;
                    }
                    // register arrays need compile-time indices: select the rows
                    c2<T> xa[3], xb[3], y[3];
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        xa[q] = mk<T>(0, 0);
                        xb[q] = mk<T>(0, 0);
#pragma unroll
                        for (int l = 0; l < 4; ++l) {
                            if (l == la) xa[q] = x[3 * l + q];
                            if (l == lb) xb[q] = x[3 * l + q];
                        }
                    }
                    if constexpr (FAM == 0) sym3(Nc, xb, y);
                    else asym3(Nc, xb, y);
#pragma unroll
                    for (int q = 0; q < 3; ++q)
#pragma unroll
                        for (int l = 0; l < 4; ++l)
                            if (l == la) acc[3 * l + q][j] = acc[3 * l + q][j] + sab * y[q];
                    if (la != lb) {
                        if constexpr (FAM == 0) sym3(Nc, xa, y);
                        else asym3(Nc, xa, y);
#pragma unroll
                        for (int q = 0; q < 3; ++q)
#pragma unroll
                            for (int l = 0; l < 4; ++l)
                                if (l == lb) acc[3 * l + q][j] = acc[3 * l + q][j] + sba * y[q];
                    }
                }
            }
        }
        __syncthreads();
    }

    // ---- outputs back into the pencils, inverse FFT, cropped store
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int e = tid + j * kNTZ;
        if (e < P * L3) {
            const int pe = e / L3, m = e - pe * L3;
#pragma unroll
            for (int c = 0; c < 12; ++c) X[(c * P + pe) * L3 + m] = acc[c][j];
        }
    }
    __syncthreads();
    pwl_fft<1, MAXE, LC>(X, 12 * P, L3, pl, tws, tid);
    for (int e = tid; e < 12 * P * n3; e += kNTZ) {
        const int s = e / n3, m = e - s * n3;
        const int comp = s / P, pe = s - comp * P;
        S2[(((long)comp * L2 + pk2[pe]) * L1 + pk1[pe]) * n3 + m] = X[s * L3 + m];
    }
}

// Fourier positions per thread of the z kernel in complex64 (G L3 <= EPT 512):
// 2 lets four mirror pencils share each table at z lengths up to 256
#ifndef VIE_PWL_EPT32
#define VIE_PWL_EPT32 2
#endif

template <typename T>
constexpr int pwl_ept()
{
    return sizeof(T) == 4 ? VIE_PWL_EPT32 : 1;
}

template <typename T>
size_t pwl_z_lds(const OpView& v, int rmax, int nc, int G, int pb)
{
    return sizeof(c2<T>) * ((size_t)12 * G * v.L[2] + (size_t)pb * nc * ((v.n[2] + 1) + rmax) + v.L[2]) +
           8 * sizeof(unsigned long long);
}

// pencils per workgroup for the z pass (the largest mirror group whose
// pencils fit the threads) and the pairs per table batch (as many as the LDS
// then holds); G = 0: does not fit
template <typename T>
void pwl_z_shape(const DeviceOp& op, int rmax, int nc, int& G, int& pb)
{
    for (G = 4; G >= 1; G /= 2)
        if ((size_t)G * op.view.L[2] <= (size_t)pwl_ept<T>() * kNTZ &&
            pwl_z_lds<T>(op.view, rmax, nc, G, 1) <= op.max_lds)
            break;
    if (G < 1) {
        G = 0;
        return;
    }
    for (pb = 10; pb > 1; --pb)
        if (pwl_z_lds<T>(op.view, rmax, nc, G, pb) <= op.max_lds) break;
}

int pwl_op_nc(const vie_pwl_op& P)
{
    return P.fam ? pwl_nc<1>() : pwl_nc<0>();
}

// complex elements of the W buffer (every k2 of every block component)
size_t pwl_w_elems(const vie_pwl_op& P)
{
    return (size_t)(P.blk[0]->d.view.n[1] + 1) * 10 * pwl_op_nc(P) * P.rmax * P.rmax;
}

template <typename T, int FAM>
auto pwl_z_kernel(int L3)
{
    constexpr int EPT = pwl_ept<T>();
    constexpr int MAXE = 12 * EPT;
    return L3 == 512 ? k_pwl_z<T, MAXE, EPT, 512, FAM>
           : L3 == 256 ? k_pwl_z<T, MAXE, EPT, 256, FAM>
           : L3 == 128 ? k_pwl_z<T, MAXE, EPT, 128, FAM>
           : L3 == 64 ? k_pwl_z<T, MAXE, EPT, 64, FAM>
           : L3 == 300 ? k_pwl_z<T, MAXE, EPT, 300, FAM>
           : L3 == 252 ? k_pwl_z<T, MAXE, EPT, 252, FAM>
           : L3 == 240 ? k_pwl_z<T, MAXE, EPT, 240, FAM>
           : L3 == 180 ? k_pwl_z<T, MAXE, EPT, 180, FAM>
           : L3 == 120 ? k_pwl_z<T, MAXE, EPT, 120, FAM>
           : L3 == 60 ? k_pwl_z<T, MAXE, EPT, 60, FAM>
           : k_pwl_z<T, MAXE, EPT, 0, FAM>;
}

template <typename T>
hipError_t launch_pwl_z(const vie_pwl_op& P, int conj, c2<T>* S2, c2<T>* Wg, int nrhs, hipStream_t s,
                        std::string& err)
{
    const DeviceOp& op = P.blk[0]->d;
    const OpView& v = op.view;
    const int nc = pwl_op_nc(P), c0 = 6 - nc;
    int G = 0, pb = 1;
    pwl_z_shape<T>(op, P.rmax, nc, G, pb);
    // tuning override: at most this many pairs per table batch (same results)
    if (const char* e = getenv("VIE_PWL_PAIRS_PER_BATCH")) pb = std::max(1, std::min(pb, atoi(e)));
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
    za.pb = pb;
    for (int f = 0; f < 8; ++f) za.neg[f] = 0;
    for (int b = 0; b < 10; ++b)
        for (int c = 0; c < nc; ++c) {
            const int lm = P.blk[b]->d.view.lmask;
            const int om = view_odd(P.fam, lm, c0 + c, 0) | (view_odd(P.fam, lm, c0 + c, 1) << 1) |
                           (view_odd(P.fam, lm, c0 + c, 2) << 2);
            for (int f = 0; f < 8; ++f)
                if (__builtin_popcount(om & f) & 1) za.neg[f] |= 1ull << (b * nc + c);
        }
    const int n1 = v.n[0], n2 = v.n[1];
    const int nblk = G == 4 ? (n1 + 1) * (n2 + 1) : (G == 2 ? (n1 + 1) * v.L[1] : v.L[0] * v.L[1]);
    const size_t lds = pwl_z_lds<T>(v, P.rmax, nc, G, pb);
    const c2<T>* tw;
    const PwlBlock<T>* blk;
    if constexpr (sizeof(T) == 8) {
        tw = op.tw64[2];
        blk = P.dev64;
    } else {
        tw = op.tw32[2];
        blk = P.dev32;
    }
    if (P.fam) hipLaunchKernelGGL((k_pwl_w<T, 1>), dim3(n2 + 1, 10 * nc), dim3(kNT), 0, s, blk, P.rmax, Wg);
    else hipLaunchKernelGGL((k_pwl_w<T, 0>), dim3(n2 + 1, 10 * nc), dim3(kNT), 0, s, blk, P.rmax, Wg);
    const int L3 = v.L[2];
    auto kern = P.fam ? pwl_z_kernel<T, 1>(L3) : pwl_z_kernel<T, 0>(L3);
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3(nblk, nrhs), dim3(kNTZ), lds, s, S2, op.plan[2], tw, za, blk, (const c2<T>*)Wg);
    return hipGetLastError();
}

// TV: vector element type, T: compute type (T = float with TV = double: the
// FP32 products on FP64 vectors of a refined solve)
template <typename TV, typename T>
hipError_t pwl_matvec(const vie_pwl_op& P, int mode, const c2<TV>* eps, const c2<TV>* x, c2<TV>* y, c2<T>* ws,
                      int nrhs, hipStream_t s, std::string& err)
{
    const DeviceOp& op = P.blk[0]->d;
    const OpView& v = op.view;
    const int nb = 4 * nrhs;   // groups of three components through the pulse passes
    c2<T>* S2 = ws;
    c2<T>* S1 = ws + (size_t)3 * v.L[1] * v.L[0] * v.n[2] * nb;
    c2<T>* Wg = ws + matvec_ws_elems(op, nb);
    const bool conj = (mode == MODE_AH || mode == MODE_NH);
    // X+ : x -> S1, Y+ : S1 -> S2, Z : S2 in place, Y- : S2 -> S1, X- : S1 -> y
    hipError_t e = run_pass<TV, T>(op, 0, mode, 0, eps, x, nullptr, S1, nb, s, nullptr, err, false);
    if (e == hipSuccess) e = run_pass<TV, T>(op, 1, mode, 0, eps, x, S1, S2, nb, s, nullptr, err, false);
    if (e == hipSuccess) e = launch_pwl_z<T>(P, conj ? 1 : 0, S2, Wg, nrhs, s, err);
    if (e == hipSuccess) e = run_pass<TV, T>(op, 3, mode, 0, eps, x, S2, S1, nb, s, nullptr, err, false);
    if (e == hipSuccess) e = run_pass<TV, T>(op, 4, mode, 0, eps, x, S1, y, nb, s, nullptr, err, false);
    return e;
}

}  // namespace

namespace vie {
// FP32 products on complex128 vectors (refined solves); ws as for VIE_C128
vie_status pwl_apply_mixed(const vie_pwl_op* op, int mode, const void* eps, const void* x, void* y, void* ws,
                           hipStream_t s)
{
    std::string err;
    hipError_t e = pwl_matvec<double, float>(*op, mode, (const c2<double>*)eps, (const c2<double>*)x, (c2<double>*)y,
                                             (c2<float>*)ws, 1, s, err);
    if (e != hipSuccess) {
        if (!err.empty()) return fail(VIE_E_UNSUPPORTED, "vie_solve_pwl: " + err);
        return hip_fail(e, "vie_solve_pwl launch");
    }
    return VIE_OK;
}
}  // namespace vie

extern "C" {

size_t vie_pwl_workspace_bytes(const vie_pwl_op* op, int dtype, int nrhs)
{
    if (!op || !op->blk[0] || nrhs < 1) return 0;
    const size_t el = dtype == VIE_C128 ? sizeof(c2<double>) : sizeof(c2<float>);
    return (matvec_ws_elems(op->blk[0]->d, 4 * nrhs) + pwl_w_elems(*op)) * el;
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
                          void* y, int nrhs, void* ws, size_t ws_bytes, void* stream)
{
    if (!op || !op->blk[0] || !x || !y || !ws) return fail(VIE_E_ARG, "vie_matvec_pwl: null argument");
    if (nrhs < 1 || nrhs > 4096) return fail(VIE_E_ARG, "vie_matvec_pwl: nrhs must be in [1, 4096]");
    if (kind != VIE_OP_A && kind != VIE_OP_N) return fail(VIE_E_ARG, "vie_matvec_pwl: bad kind");
    if (adjoint != 0 && adjoint != 1) return fail(VIE_E_ARG, "vie_matvec_pwl: adjoint must be 0 or 1");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_matvec_pwl: bad dtype");
    if (op->fam != 0 && (kind != VIE_OP_N || adjoint != 0))
        return fail(VIE_E_UNSUPPORTED, "vie_matvec_pwl: a K operator has the bare forward product (VIE_OP_N) only");
    if (kind == VIE_OP_A && !eps_c) return fail(VIE_E_ARG, "vie_matvec_pwl: eps_c is required for VIE_OP_A");
    if (ws_bytes < vie_pwl_workspace_bytes(op, dtype, nrhs))
        return fail(VIE_E_ARG, "vie_matvec_pwl: workspace too small");
    const OpView& v = op->blk[0]->d.view;
    const size_t vbytes = (size_t)nrhs * 12 * v.n[0] * v.n[1] * v.n[2] * (dtype == VIE_C128 ? 16 : 8);
    const char* xb = (const char*)x;
    const char* yb = (const char*)y;
    if (!(xb + vbytes <= yb || yb + vbytes <= xb)) return fail(VIE_E_ARG, "vie_matvec_pwl: x and y overlap");
    const int mode = kind == VIE_OP_A ? (adjoint ? MODE_AH : MODE_A) : (adjoint ? MODE_NH : MODE_N);
    hipStream_t s = (hipStream_t)stream;
    std::string err;
    hipError_t e = dtype == VIE_C128
                       ? pwl_matvec<double, double>(*op, mode, (const c2<double>*)eps_c, (const c2<double>*)x,
                                                    (c2<double>*)y, (c2<double>*)ws, nrhs, s, err)
                       : pwl_matvec<float, float>(*op, mode, (const c2<float>*)eps_c, (const c2<float>*)x,
                                                  (c2<float>*)y, (c2<float>*)ws, nrhs, s, err);
    if (e != hipSuccess) {
        if (!err.empty()) return fail(VIE_E_UNSUPPORTED, "vie_matvec_pwl: " + err);
        return hip_fail(e, "vie_matvec_pwl launch");
    }
    return VIE_OK;
}

size_t vie_jm_pwl_workspace_bytes(const vie_pwl_op* op_n, const vie_pwl_op* op_k, int dtype)
{
    if (!op_n || !op_k || !op_n->blk[0] || !op_k->blk[0] || (dtype != VIE_C64 && dtype != VIE_C128)) return 0;
    const OpView& v = op_n->blk[0]->d.view;
    const size_t vec = (size_t)2 * 12 * v.n[0] * v.n[1] * v.n[2] * (dtype == VIE_C128 ? 16 : 8);
    const size_t mv = std::max(vie_pwl_workspace_bytes(op_n, dtype, 2), vie_pwl_workspace_bytes(op_k, dtype, 2));
    return 2 * al256(vec) + mv;
}

vie_status vie_matvec_jm_pwl(const vie_pwl_op* op_n, const vie_pwl_op* op_k, int dtype, double h, double omega,
                             const void* eps_c, const void* mu_c, const void* x, void* y, void* ws, size_t ws_bytes,
                             void* stream)
{
    if (!op_n || !op_k || !op_n->blk[0] || !op_k->blk[0] || !eps_c || !mu_c || !x || !y || !ws || !(h > 0) ||
        !(omega > 0))
        return fail(VIE_E_ARG, "vie_matvec_jm_pwl: bad argument");
    if (op_n->fam != 0 || op_k->fam != 1)
        return fail(VIE_E_ARG, "vie_matvec_jm_pwl: needs an N operator and a K operator");
    const OpView& v = op_n->blk[0]->d.view;
    for (int a = 0; a < 3; ++a)
        if (op_k->blk[0]->d.view.n[a] != v.n[a]) return fail(VIE_E_ARG, "vie_matvec_jm_pwl: N and K grids differ");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_matvec_jm_pwl: bad dtype");
    if (ws_bytes < vie_jm_pwl_workspace_bytes(op_n, op_k, dtype))
        return fail(VIE_E_ARG, "vie_matvec_jm_pwl: workspace too small");
    const long nv = (long)v.n[0] * v.n[1] * v.n[2];
    const size_t vec = (size_t)2 * 12 * nv * (dtype == VIE_C128 ? 16 : 8);
    const char* xb = (const char*)x;
    const char* yb = (const char*)y;
    if (!(xb + vec <= yb || yb + vec <= xb)) return fail(VIE_E_ARG, "vie_matvec_jm_pwl: x and y overlap");
    char* w = (char*)ws;
    void* NX = w;
    void* KX = w + al256(vec);
    void* mw = w + 2 * al256(vec);
    const size_t mb = ws_bytes - 2 * al256(vec);
    hipStream_t s = (hipStream_t)stream;
    // [J; M] as two right-hand sides of each operator
    if (jm_mixed_products && dtype == VIE_C128) {
        // FP64 vectors, products in FP32 (the inner operator of a refined solve)
        std::string err;
        hipError_t he = pwl_matvec<double, float>(*op_n, MODE_N, nullptr, (const c2<double>*)x, (c2<double>*)NX,
                                                  (c2<float>*)mw, 2, s, err);
        if (he == hipSuccess)
            he = pwl_matvec<double, float>(*op_k, MODE_N, nullptr, (const c2<double>*)x, (c2<double>*)KX,
                                           (c2<float>*)mw, 2, s, err);
        if (he != hipSuccess)
            return err.empty() ? hip_fail(he, "vie_matvec_jm_pwl") : fail(VIE_E_UNSUPPORTED, "vie_matvec_jm_pwl: " + err);
    } else {
        vie_status st = vie_matvec_pwl(op_n, VIE_OP_N, 0, dtype, nullptr, x, NX, 2, mw, mb, stream);
        if (st != VIE_OK) return st;
        st = vie_matvec_pwl(op_k, VIE_OP_N, 0, dtype, nullptr, x, KX, 2, mw, mb, stream);
        if (st != VIE_OK) return st;
    }
    const double EPS0 = 8.8541878128e-12, C0 = 299792458.0;
    const double MU0 = 1.0 / (EPS0 * C0 * C0);
    hipError_t e;
    if (dtype == VIE_C128)
        e = kr_jm_combine<double>((const c2<double>*)eps_c, (const c2<double>*)mu_c, (const c2<double>*)x,
                                  (const c2<double>*)NX, (const c2<double>*)KX, omega * EPS0 * h, omega * MU0 * h,
                                  (c2<double>*)y, nv, 12, s);
    else
        e = kr_jm_combine<float>((const c2<float>*)eps_c, (const c2<float>*)mu_c, (const c2<float>*)x,
                                 (const c2<float>*)NX, (const c2<float>*)KX, omega * EPS0 * h, omega * MU0 * h,
                                 (c2<float>*)y, nv, 12, s);
    if (e != hipSuccess) return hip_fail(e, "vie_matvec_jm_pwl");
    return VIE_OK;
}

}  // extern "C"
