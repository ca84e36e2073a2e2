// Five-pass FFT-VIE matvec for gfx950.
//
// The Toeplitz product N u (Sec. II-B) is a circular convolution after zero
// padding every current component to L_i = 2 n_i per axis.  The 3-D FFT is
// done as three sweeps of 1-D FFTs, forward then inverse, with the Fourier-
// domain 3x3 component product in the middle:
//
//   pass X+  pad x to L1, FFT along x          u  [q][k][j][i]   -> S1 [q][k][i'][j]
//   pass Y+  pad y to L2, FFT along y          S1                -> S2 [q][j'][i'][k]
//   pass Z*  pad z, FFT along z, reconstruct N^_c on the fly from the Tucker
//            form, Y^_p = sum_q N^_pq X^_q, inverse FFT along z, crop z  (S2 in place)
//   pass Y-  inverse FFT along y, crop y       S2                -> S3 [q][k][i'][j]
//   pass X-  inverse FFT along x, crop x, contrast epilogue     S3 -> y  [q][k][j][i]
//
// Each pass writes its output transposed so that the next FFT axis is the
// contiguous one for the Z pass and global accesses of every pass are runs of
// at least W (= 16 complex64 / 8 complex128) contiguous elements.  Within a
// block the W pencils of a tile sit in LDS as [element][pencil] (X and Y
// passes) or [pencil][element] (Z pass) and are transformed by the Stockham
// stages of fft_device.h.
//
// Z pass and the Tucker form (eq. 13-14, Sec. V-A/B): for a pencil (k1, k2)
//   N^_c(k1, k2, k3) = sum_g V_c[g] U3^_c(k3, g),
//   V_c[g] = sum_a U1^_c(k1, a) sum_b G_c[a, b, g] U2^_c(k2, b).
// The embedded factor columns are even or odd, so U^_a(L_a - k) =
// s_a(c) U^_a(k): one block handles the (up to) four mirror pencils
// (k1, k2), (L1-k1, k2), (k1, L2-k2), (L1-k1, L2-k2), reconstructs
// N^_c(k1, k2, k3) once for k3 in [0, n3] and applies the parity signs
// (this is the decompression of Sec. V-B done per pencil quad; nothing
// dense is stored).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <type_traits>

#include "fft_device.h"

#include "vie_internal.h"

namespace vie {

static constexpr int NT = 256;   // threads per block in every pass

int g_kernel_path = 0;
int g_batch_mode = 0;

// component parities: s_a(c) = -1 iff c is off-diagonal and a is one of its axes
__device__ __forceinline__ int comp_sign(int fam, int c, int f1, int f2, int f3)
{
    // c: 0 xx, 1 yy, 2 zz, 3 xy, 4 xz, 5 yz
    int neg = (comp_odd(fam, c, 0) & f1) ^ (comp_odd(fam, c, 1) & f2) ^ (comp_odd(fam, c, 2) & f3);
    return neg ? -1 : 1;
}

template <typename T>
__device__ __forceinline__ void load_tw(c2<T>* dst, const c2<T>* src, int L, int tid)
{
    for (int m = tid; m < L; m += NT) dst[m] = src[m];
}

// ------------------------------- pass X+ --------------------------------
template <typename TV, typename T, int W, int MAXE, int LC = 0>
__device__ __forceinline__ void xfwd_body(const c2<TV>* __restrict__ x, const c2<TV>* __restrict__ eps,
                                             c2<T>* __restrict__ S1, FftPlan pl, const c2<T>* __restrict__ tw,
                                             int n1, int n2, int n3, int mode, const int* __restrict__ rhs_map, int bx, int by, int bz)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T>* buf = reinterpret_cast<c2<T>*>(smem_raw);
    const int L1 = LC ? LC : pl.L;
    c2<T>* tws = buf + (size_t)L1 * (W + 1);
    const int tid = threadIdx.x;
    const int j0 = bx * W, k = by;
    const int zq = bz;               // launch rhs * 3 + q
    const int q = zq % 3, bl = zq / 3;
    const int b = rhs_map ? rhs_map[bl] : bl;
    const long bq = (long)b * 3 + q;
    const long bq_out = (long)bl * 3 + q;
    load_tw(tws, tw, L1, tid);
    for (int e = tid; e < W * n1; e += NT) {
        int w = e / n1, i = e - w * n1;
        int j = j0 + w;
        c2<T> v = mk<T>(0, 0);
        if (j < n2) {
            long idx = ((bq * n3 + k) * n2 + j) * n1 + i;
            c2<T> u = cvt<T>(x[idx]);
            if (mode == MODE_AH) {       // pre-scale by conj(chi) = conj(eps) - 1
                c2<T> ep = cvt<T>(eps[((long)k * n2 + j) * n1 + i]);
                c2<T> chi = mk<T>(ep.x - (T)1, -ep.y);
                v = chi * u;
            } else {
                v = u;
            }
        }
        buf[i * (W + 1) + w] = v;
    }
    for (int e = tid; e < W * (L1 - n1); e += NT) {
        int w = e % W, i = n1 + e / W;
        buf[i * (W + 1) + w] = mk<T>(0, 0);
    }
    __syncthreads();
    fft_lds_len<-1, true, MAXE, LC>(buf, W, 1, W + 1, pl, tws, tid, NT);
    for (int e = tid; e < W * L1; e += NT) {
        int w = e % W, i = e / W;
        int j = j0 + w;
        if (j < n2) S1[((bq_out * n3 + k) * L1 + i) * n2 + j] = buf[i * (W + 1) + w];
    }
}

// ------------------------------- pass Y+ --------------------------------
template <typename T, int W, int MAXE, int LC = 0>
__device__ __forceinline__ void yfwd_body(const c2<T>* __restrict__ S1, c2<T>* __restrict__ S2, FftPlan pl,
                                             const c2<T>* __restrict__ tw, int L1, int n2, int n3, int bx, int by, int bz)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T>* buf = reinterpret_cast<c2<T>*>(smem_raw);
    const int L2 = LC ? LC : pl.L;
    c2<T>* tws = buf + (size_t)L2 * (W + 1);
    const int tid = threadIdx.x;
    const int k0 = bx * W, i = by;
    const long bq = bz;
    load_tw(tws, tw, L2, tid);
    for (int e = tid; e < W * n2; e += NT) {
        int w = e / n2, j = e - w * n2;
        int k = k0 + w;
        c2<T> v = mk<T>(0, 0);
        if (k < n3) v = S1[((bq * n3 + k) * L1 + i) * n2 + j];
        buf[j * (W + 1) + w] = v;
    }
    for (int e = tid; e < W * (L2 - n2); e += NT) {
        int w = e % W, j = n2 + e / W;
        buf[j * (W + 1) + w] = mk<T>(0, 0);
    }
    __syncthreads();
    fft_lds_len<-1, true, MAXE, LC>(buf, W, 1, W + 1, pl, tws, tid, NT);
    for (int e = tid; e < W * L2; e += NT) {
        int w = e % W, j = e / W;
        int k = k0 + w;
        if (k < n3) S2[((bq * L2 + j) * L1 + i) * n3 + k] = buf[j * (W + 1) + w];
    }
}

// ------------------------------- pass Y- --------------------------------
template <typename T, int W, int MAXE, int LC = 0>
__device__ __forceinline__ void yinv_body(const c2<T>* __restrict__ S2, c2<T>* __restrict__ S3, FftPlan pl,
                                             const c2<T>* __restrict__ tw, int L1, int n2, int n3, int bx, int by, int bz)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T>* buf = reinterpret_cast<c2<T>*>(smem_raw);
    const int L2 = LC ? LC : pl.L;
    c2<T>* tws = buf + (size_t)L2 * (W + 1);
    const int tid = threadIdx.x;
    const int k0 = bx * W, i = by;
    const long bq = bz;
    load_tw(tws, tw, L2, tid);
    for (int e = tid; e < W * L2; e += NT) {
        int w = e % W, j = e / W;
        int k = k0 + w;
        c2<T> v = mk<T>(0, 0);
        if (k < n3) v = S2[((bq * L2 + j) * L1 + i) * n3 + k];
        buf[j * (W + 1) + w] = v;
    }
    __syncthreads();
    fft_lds_len<1, true, MAXE, LC>(buf, W, 1, W + 1, pl, tws, tid, NT);
    for (int e = tid; e < W * n2; e += NT) {
        int w = e / n2, j = e - w * n2;
        int k = k0 + w;
        if (k < n3) S3[((bq * n3 + k) * L1 + i) * n2 + j] = buf[j * (W + 1) + w];
    }
}

// ------------------------------- pass X- --------------------------------
template <typename TV, typename T, int W, int MAXE, int LC = 0>
__device__ __forceinline__ void xinv_body(const c2<T>* __restrict__ S3, const c2<TV>* __restrict__ x,
                                             const c2<TV>* __restrict__ eps, c2<TV>* __restrict__ y, FftPlan pl,
                                             const c2<T>* __restrict__ tw, int n1, int n2, int n3, int mode,
                                             const int* __restrict__ rhs_map, int bx, int by, int bz)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T>* buf = reinterpret_cast<c2<T>*>(smem_raw);
    const int L1 = LC ? LC : pl.L;
    c2<T>* tws = buf + (size_t)L1 * (W + 1);
    const int tid = threadIdx.x;
    const int j0 = bx * W, k = by;
    const int zq = bz;
    const int q = zq % 3, bl = zq / 3;
    const int b = rhs_map ? rhs_map[bl] : bl;
    const long bq_in = (long)bl * 3 + q;
    const long bq = (long)b * 3 + q;
    load_tw(tws, tw, L1, tid);
    for (int e = tid; e < W * L1; e += NT) {
        int w = e % W, i = e / W;
        int j = j0 + w;
        c2<T> v = mk<T>(0, 0);
        if (j < n2) v = S3[((bq_in * n3 + k) * L1 + i) * n2 + j];
        buf[i * (W + 1) + w] = v;
    }
    __syncthreads();
    fft_lds_len<1, true, MAXE, LC>(buf, W, 1, W + 1, pl, tws, tid, NT);
    for (int e = tid; e < W * n1; e += NT) {
        int w = e / n1, i = e - w * n1;
        int j = j0 + w;
        if (j >= n2) continue;
        long idx = ((bq * n3 + k) * n2 + j) * n1 + i;
        c2<T> r = buf[i * (W + 1) + w];
        c2<T> out;
        if (mode == MODE_A || mode == MODE_AH) {
            c2<T> u = cvt<T>(x[idx]);
            c2<T> ep = cvt<T>(eps[((long)k * n2 + j) * n1 + i]);
            if (mode == MODE_A) {        // eps u - chi r
                c2<T> chi = mk<T>(ep.x - (T)1, ep.y);
                out = ep * u - chi * r;
            } else {                     // conj(eps) u - r
                out = conj(ep) * u - r;
            }
        } else {
            out = r;
        }
        y[idx] = cvt<TV>(out);
    }
}

// ------------------------------- pass Z* --------------------------------
// Pencil groups: G = 4 (quads over (n1+1) x (n2+1) blocks), G = 2 (pairs
// along x over (n1+1) x L2 blocks) or G = 1 (single pencils over L1 x L2).
struct ZArgs {
    OpView v;
    int G;
    int conj;     // use conj(N^) (adjoint)
    int dense;    // read N^ from the dense half-spectrum store
};

template <typename T, typename TR>
struct ZFactors {
    const c2<TR>* core;
    const c2<TR>* fac;
    const c2<TR>* dense;
};

template <typename T, int MAXE>
__device__ __forceinline__ void zmid_body(c2<T>* __restrict__ S2, FftPlan pl, const c2<T>* __restrict__ tw,
                                             ZArgs a, const c2<T>* __restrict__ core,
                                             const c2<T>* __restrict__ fac, const c2<T>* __restrict__ dense, int bx, int by, int bz)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const OpView& v = a.v;
    const int n1 = v.n[0], n2 = v.n[1], n3 = v.n[2];
    const int L1 = v.L[0], L2 = v.L[1], L3 = v.L[2];
    const int tid = threadIdx.x;

    // ---- which pencils this block owns
    int k1, k2, f1base = 0, f2base = 0;
    int P = 0;
    int pk1[4], pk2[4], pf1[4], pf2[4];
    {
        int bidx = bx;
        if (a.G == 4) {
            k1 = bidx % (n1 + 1);
            k2 = bidx / (n1 + 1);
        } else if (a.G == 2) {
            k1 = bidx % (n1 + 1);
            int kk2 = bidx / (n1 + 1);
            k2 = kk2 <= n2 ? kk2 : L2 - kk2;
            f2base = kk2 > n2;
        } else {
            int kk1 = bidx % L1, kk2 = bidx / L1;
            k1 = kk1 <= n1 ? kk1 : L1 - kk1;
            f1base = kk1 > n1;
            k2 = kk2 <= n2 ? kk2 : L2 - kk2;
            f2base = kk2 > n2;
        }
        bool m1 = (a.G >= 2) && k1 > 0 && k1 < n1;
        bool m2 = (a.G == 4) && k2 > 0 && k2 < n2;
        for (int s2 = 0; s2 <= (m2 ? 1 : 0); ++s2)
            for (int s1 = 0; s1 <= (m1 ? 1 : 0); ++s1) {
                int f1 = f1base | s1, f2 = f2base | s2;
                pk1[P] = f1 ? L1 - k1 : k1;
                pk2[P] = f2 ? L2 - k2 : k2;
                pf1[P] = f1;
                pf2[P] = f2;
                ++P;
            }
    }
    const int b = by;

    // ---- LDS carve-up
    c2<T>* X = reinterpret_cast<c2<T>*>(smem_raw);           // [3*P][L3]
    c2<T>* NTt = X + (size_t)3 * a.G * L3;                   // [6][n3+1]
    c2<T>* Wc = NTt + (size_t)6 * (n3 + 1);                  // [rmax*rmax]
    c2<T>* Vc = Wc + (size_t)v.rmax * v.rmax;                // [6][rmax]
    c2<T>* tws = Vc + (size_t)6 * v.rmax;                    // [L3]
    load_tw(tws, tw, L3, tid);

    // ---- load the 3*P pencils (k < n3), zero padding
    for (int e = tid; e < 3 * P * L3; e += NT) {
        int s = e / L3, m = e - s * L3;
        int q = s / P, pe = s - q * P;
        c2<T> val = mk<T>(0, 0);
        if (m < n3) val = S2[((((long)b * 3 + q) * L2 + pk2[pe]) * L1 + pk1[pe]) * n3 + m];
        X[s * L3 + m] = val;
    }

    // ---- reconstruct N^_c(k1, k2, k3) for k3 in [0, n3]
    if (!a.dense) {
        for (int c = 0; c < 6; ++c) {
            const int r1 = v.r[c][0], r2 = v.r[c][1], r3 = v.r[c][2];
            const c2<T>* G = core + v.core_off[c];
            const c2<T>* U1 = fac + v.fac_off[c][0] + (long)k1 * r1;
            const c2<T>* U2 = fac + v.fac_off[c][1] + (long)k2 * r2;
            for (int e = tid; e < r1 * r3; e += NT) {
                int al = e / r3, ga = e - al * r3;
                c2<T> acc = mk<T>(0, 0);
                for (int be = 0; be < r2; ++be) fma_c(acc, G[((long)al * r2 + be) * r3 + ga], U2[be]);
                Wc[e] = acc;
            }
            __syncthreads();
            for (int ga = tid; ga < r3; ga += NT) {
                c2<T> acc = mk<T>(0, 0);
                for (int al = 0; al < r1; ++al) fma_c(acc, U1[al], Wc[al * r3 + ga]);
                Vc[c * v.rmax + ga] = acc;
            }
            __syncthreads();
        }
        for (int e = tid; e < 6 * (n3 + 1); e += NT) {
            int c = e / (n3 + 1), kk = e - c * (n3 + 1);
            const int r3 = v.r[c][2];
            const c2<T>* U3 = fac + v.fac_off[c][2] + (long)kk * r3;
            c2<T> acc = mk<T>(0, 0);
            for (int ga = 0; ga < r3; ++ga) fma_c(acc, Vc[c * v.rmax + ga], U3[ga]);
            NTt[e] = acc;
        }
    } else {
        // dense half spectrum [c][k2][k1][k3], (n1+1)(n2+1)(n3+1) per component
        const long per = (long)(n1 + 1) * (n2 + 1) * (n3 + 1);
        for (int e = tid; e < 6 * (n3 + 1); e += NT) {
            int c = e / (n3 + 1), kk = e - c * (n3 + 1);
            NTt[e] = dense[c * per + ((long)k2 * (n1 + 1) + k1) * (n3 + 1) + kk];
        }
    }
    __syncthreads();

    // ---- forward FFT along z of all 3*P pencils
    fft_lds<-1, false, MAXE>(X, 3 * P, L3, 1, pl, tws, tid, NT);

    // ---- 3x3 component product with parity signs
    for (int e = tid; e < P * L3; e += NT) {
        int pe = e / L3, m = e - pe * L3;
        int f3 = m > n3;
        int kk = f3 ? L3 - m : m;
        c2<T> N[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            c2<T> t = NTt[c * (n3 + 1) + kk];
            if (comp_sign(v.fam, c, pf1[pe], pf2[pe], f3) < 0) t = mk<T>(-t.x, -t.y);
            N[c] = a.conj ? conj(t) : t;
        }
        // the pair (q, p) below the diagonal is N_pq (symmetric family) or
        // -K_pq (antisymmetric family)
        const T lo = v.fam ? (T)-1 : (T)1;
        c2<T> x0 = X[(0 * P + pe) * L3 + m], x1 = X[(1 * P + pe) * L3 + m], x2 = X[(2 * P + pe) * L3 + m];
        c2<T> y0 = N[0] * x0 + N[3] * x1 + N[4] * x2;
        c2<T> y1 = lo * (N[3] * x0) + N[1] * x1 + N[5] * x2;
        c2<T> y2 = lo * (N[4] * x0 + N[5] * x1) + N[2] * x2;
        X[(0 * P + pe) * L3 + m] = y0;
        X[(1 * P + pe) * L3 + m] = y1;
        X[(2 * P + pe) * L3 + m] = y2;
    }
    __syncthreads();

    // ---- inverse FFT along z and cropped store
    fft_lds<1, false, MAXE>(X, 3 * P, L3, 1, pl, tws, tid, NT);
    for (int e = tid; e < 3 * P * n3; e += NT) {
        int s = e / n3, m = e - s * n3;
        int q = s / P, pe = s - q * P;
        S2[((((long)b * 3 + q) * L2 + pk2[pe]) * L1 + pk1[pe]) * n3 + m] = X[s * L3 + m];
    }
}

// ----------------------- single-instance kernels --------------------------
template <typename TV, typename T, int W, int MAXE, int LC = 0>
__global__ void __launch_bounds__(NT) k_xfwd(const c2<TV>* __restrict__ x, const c2<TV>* __restrict__ eps,
                                             c2<T>* __restrict__ S1, FftPlan pl, const c2<T>* __restrict__ tw,
                                             int n1, int n2, int n3, int mode, const int* __restrict__ rhs_map)
{
    xfwd_body<TV, T, W, MAXE, LC>(x, eps, S1, pl, tw, n1, n2, n3, mode, rhs_map, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <typename T, int W, int MAXE, int LC = 0>
__global__ void __launch_bounds__(NT) k_yfwd(const c2<T>* __restrict__ S1, c2<T>* __restrict__ S2, FftPlan pl,
                                             const c2<T>* __restrict__ tw, int L1, int n2, int n3)
{
    yfwd_body<T, W, MAXE, LC>(S1, S2, pl, tw, L1, n2, n3, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <typename T, int W, int MAXE, int LC = 0>
__global__ void __launch_bounds__(NT) k_yinv(const c2<T>* __restrict__ S2, c2<T>* __restrict__ S3, FftPlan pl,
                                             const c2<T>* __restrict__ tw, int L1, int n2, int n3)
{
    yinv_body<T, W, MAXE, LC>(S2, S3, pl, tw, L1, n2, n3, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <typename TV, typename T, int W, int MAXE, int LC = 0>
__global__ void __launch_bounds__(NT) k_xinv(const c2<T>* __restrict__ S3, const c2<TV>* __restrict__ x,
                                             const c2<TV>* __restrict__ eps, c2<TV>* __restrict__ y, FftPlan pl,
                                             const c2<T>* __restrict__ tw, int n1, int n2, int n3, int mode,
                                             const int* __restrict__ rhs_map)
{
    xinv_body<TV, T, W, MAXE, LC>(S3, x, eps, y, pl, tw, n1, n2, n3, mode, rhs_map, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <typename T, int MAXE>
__global__ void __launch_bounds__(NT) k_zmid(c2<T>* __restrict__ S2, FftPlan pl, const c2<T>* __restrict__ tw,
                                             ZArgs a, const c2<T>* __restrict__ core,
                                             const c2<T>* __restrict__ fac, const c2<T>* __restrict__ dense)
{
    zmid_body<T, MAXE>(S2, pl, tw, a, core, fac, dense, blockIdx.x, blockIdx.y, blockIdx.z);
}

// ------------------------ multi-instance kernels ---------------------------
// One launch per pass covers every instance of a batch (grids of different
// sizes): block b belongs to the instance whose [off, off + cnt) range holds
// it and is decoded into that instance's tile coordinates.
__device__ __forceinline__ int find_inst(const InstDev* __restrict__ tab, int count, int pass, int b)
{
    int i = 0;
    while (i + 1 < count && b >= tab[i + 1].off[pass]) ++i;
    return i;
}

template <typename TV, typename T, int W, int MAXE>
__global__ void __launch_bounds__(NT) k_xfwd_multi(const InstDev* __restrict__ tab, int count, int mode)
{
    const InstDev& I = tab[find_inst(tab, count, 0, blockIdx.x)];
    const int t = blockIdx.x - I.off[0];
    const int n1 = I.v.n[0], n2 = I.v.n[1], n3 = I.v.n[2];
    const int gx = (n2 + W - 1) / W;
    xfwd_body<TV, T, W, MAXE>((const c2<TV>*)I.x, (const c2<TV>*)I.eps, (c2<T>*)I.S1, I.plan[0],
                              (const c2<T>*)I.tw[0], n1, n2, n3, mode, I.map, t % gx, (t / gx) % n3,
                              t / (gx * n3));
}

template <typename T, int W, int MAXE>
__global__ void __launch_bounds__(NT) k_yfwd_multi(const InstDev* __restrict__ tab, int count)
{
    const InstDev& I = tab[find_inst(tab, count, 1, blockIdx.x)];
    const int t = blockIdx.x - I.off[1];
    const int n2 = I.v.n[1], n3 = I.v.n[2], L1 = I.v.L[0];
    const int gx = (n3 + W - 1) / W;
    yfwd_body<T, W, MAXE>((const c2<T>*)I.S1, (c2<T>*)I.S2, I.plan[1], (const c2<T>*)I.tw[1], L1, n2, n3, t % gx,
                          (t / gx) % L1, t / (gx * L1));
}

template <typename T, int MAXE>
__global__ void __launch_bounds__(NT) k_zmid_multi(const InstDev* __restrict__ tab, int count, int conj)
{
    const InstDev& I = tab[find_inst(tab, count, 2, blockIdx.x)];
    const int t = blockIdx.x - I.off[2];
    ZArgs za;
    za.v = I.v;
    za.G = I.G;
    za.conj = conj;
    za.dense = 0;
    const int nblk = I.cnt[2] / I.nact;
    zmid_body<T, MAXE>((c2<T>*)I.S2, I.plan[2], (const c2<T>*)I.tw[2], za, (const c2<T>*)I.core,
                       (const c2<T>*)I.fac, nullptr, t % nblk, t / nblk, 0);
}

template <typename T, int W, int MAXE>
__global__ void __launch_bounds__(NT) k_yinv_multi(const InstDev* __restrict__ tab, int count)
{
    const InstDev& I = tab[find_inst(tab, count, 3, blockIdx.x)];
    const int t = blockIdx.x - I.off[3];
    const int n2 = I.v.n[1], n3 = I.v.n[2], L1 = I.v.L[0];
    const int gx = (n3 + W - 1) / W;
    yinv_body<T, W, MAXE>((const c2<T>*)I.S2, (c2<T>*)I.S1, I.plan[1], (const c2<T>*)I.tw[1], L1, n2, n3, t % gx,
                          (t / gx) % L1, t / (gx * L1));
}

template <typename TV, typename T, int W, int MAXE>
__global__ void __launch_bounds__(NT) k_xinv_multi(const InstDev* __restrict__ tab, int count, int mode)
{
    const InstDev& I = tab[find_inst(tab, count, 4, blockIdx.x)];
    const int t = blockIdx.x - I.off[4];
    const int n1 = I.v.n[0], n2 = I.v.n[1], n3 = I.v.n[2];
    const int gx = (n2 + W - 1) / W;
    xinv_body<TV, T, W, MAXE>((const c2<T>*)I.S1, (const c2<TV>*)I.x, (const c2<TV>*)I.eps, (c2<TV>*)I.y,
                              I.plan[0], (const c2<T>*)I.tw[0], n1, n2, n3, mode, I.map, t % gx, (t / gx) % n3,
                              t / (gx * n3));
}

// ------------------------------- host side ------------------------------

// Optional per-pass timing: HIP events recorded on the launch stream around
// each pass while profiling is enabled; summed by prof_collect().
namespace {
struct ProfRec {
    int pass;
    hipEvent_t a, b;
};
bool g_prof = false;
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event()
{
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

struct PassTimer {
    int pass;
    hipStream_t s;
    hipEvent_t a = nullptr;
    PassTimer(int p, hipStream_t st) : pass(p), s(st)
    {
        if (g_prof) {
            a = prof_event();
            (void)hipEventRecord(a, s);
        }
    }
    ~PassTimer()
    {
        if (g_prof && a) {
            hipEvent_t b = prof_event();
            (void)hipEventRecord(b, s);
            g_prof_recs.push_back({pass, a, b});
        }
    }
};
}  // namespace

void prof_enable(int on)
{
    g_prof = on != 0;
}

bool prof_is_enabled() { return g_prof; }

int prof_collect(double* ms, int* counts, int npass)
{
    for (int p = 0; p < npass; ++p) {
        ms[p] = 0;
        counts[p] = 0;
    }
    int bad = 0;
    for (auto& r : g_prof_recs) {
        float t = 0;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
            ++bad;
        } else if (r.pass >= 0 && r.pass < npass) {
            ms[r.pass] += t;
            counts[r.pass] += 1;
        }
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    g_prof_recs.clear();
    return bad;
}

template <typename T>
static int tile_width(size_t max_lds, int L)
{
    int W = sizeof(T) == 4 ? 16 : 8;
    while (W > 1 && (size_t)(W + 1 + 1) * L * sizeof(c2<T>) > max_lds) W /= 2;
    return W;
}

size_t matvec_ws_elems(const DeviceOp& op, int nrhs)
{
    const OpView& v = op.view;
    size_t s2 = (size_t)3 * v.L[1] * v.L[0] * v.n[2];
    size_t s1 = (size_t)3 * v.n[2] * v.L[0] * v.n[1];
    return (s2 + s1) * (size_t)nrhs;
}

template <typename T>
static size_t z_lds_bytes(const OpView& v, int G)
{
    return sizeof(c2<T>) * ((size_t)3 * G * v.L[2] + 6 * (v.n[2] + 1) + (size_t)v.rmax * v.rmax +
                            6 * v.rmax + v.L[2]);
}

// Dispatch helpers on the tile width W (compile-time) for X/Y passes.
#define VIE_W_DISPATCH(W_, ...)                                          \
    switch (W_) {                                                        \
    case 16: { constexpr int Wc = 16; __VA_ARGS__; } break;              \
    case 8: { constexpr int Wc = 8; __VA_ARGS__; } break;                \
    case 4: { constexpr int Wc = 4; __VA_ARGS__; } break;                \
    case 2: { constexpr int Wc = 2; __VA_ARGS__; } break;                \
    default: { constexpr int Wc = 1; __VA_ARGS__; } break;               \
    }

// Default tile width of the mixed-radix X/Y kernels, and the lengths whose
// radix sequence those kernels take at compile time (the sphere series'
// 2n = 60 ... 300; the register-FFT lengths have kernels of their own)
template <typename T>
constexpr int kWDefault = sizeof(T) == 4 ? 16 : 8;

template <class F>
static void with_lc(int L, F&& f)
{
    switch (L) {
    case 60: f(std::integral_constant<int, 60>{}); break;
    case 120: f(std::integral_constant<int, 120>{}); break;
    case 180: f(std::integral_constant<int, 180>{}); break;
    case 240: f(std::integral_constant<int, 240>{}); break;
    case 300: f(std::integral_constant<int, 300>{}); break;
    default: f(std::integral_constant<int, 0>{}); break;
    }
}

// One pass of the matvec on explicit buffers (see launch_matvec for the
// layouts): pass 0 reads x and writes S1 (out), 1 reads S1 (in) and writes
// S2 (out), 2 transforms S2 in place (out), 3 reads S2 (in) and writes S3
// (out), 4 reads S3 (in) and writes y (out).  ident (passes 0 and 4 only):
// the transform is replaced by the identity, so only the pass's index maps
// (padding, transposes, cropping; pass 4 with the bare epilogue) remain.
template <typename TV, typename T>
hipError_t run_pass(const DeviceOp& op, int pass, int mode, int recon, const c2<TV>* eps, const c2<TV>* x,
                    const void* in, void* out, int nrhs, hipStream_t s, const int* rhs_map, std::string& err,
                    bool ident)
{
    const OpView& v = op.view;
    const int n1 = v.n[0], n2 = v.n[1], n3 = v.n[2];
    const int L1 = v.L[0], L2 = v.L[1], L3 = v.L[2];
    const c2<T>* tw[3];
    const c2<T>* core;
    const c2<T>* fac;
    const c2<T>* dense;
    if constexpr (sizeof(T) == 8) {
        for (int a = 0; a < 3; ++a) tw[a] = op.tw64[a];
        core = op.d64.core;
        fac = op.d64.fac;
        dense = op.dense64;
    } else {
        for (int a = 0; a < 3; ++a) tw[a] = op.tw32[a];
        core = op.d32.core;
        fac = op.d32.fac;
        dense = op.dense32;
    }
    constexpr int MAXE_XY = 32;   // W * L <= MAXE * NT for W*L <= 8192
    constexpr int MAXE_Z = 24;    // 3 * G * L3 <= 6144
    const bool allow_fast = g_kernel_path == 0;
    // the identity "transform": a plan without stages leaves the LDS tile as loaded
    FftPlan id0 = op.plan[0];
    id0.nst = 0;
    const FftPlan& px = ident ? id0 : op.plan[0];
    PassTimer timer(pass, s);
    if (pass == 0) {
        c2<T>* S1 = reinterpret_cast<c2<T>*>(out);
        if (ident) {
            if constexpr (std::is_same<TV, T>::value) {
                if (allow_fast && xy_ident_fast<T>(0, L1, nullptr, S1, x, tw[0], n1, n2, n3, L1, L2, nrhs, s))
                    return hipGetLastError();
            }
        } else if (allow_fast && xy_pass_fast<TV, T>(0, L1, nullptr, S1, x, eps, tw[0], n1, n2, n3, L1, L2, mode,
                                                     nrhs, rhs_map, s)) {
            return hipGetLastError();
        }
        int W = tile_width<T>(op.max_lds, L1);
        if ((size_t)W * L1 > (size_t)MAXE_XY * NT) { err = "x length too large"; return hipErrorInvalidValue; }
        size_t lds = (size_t)(W + 1) * L1 * sizeof(c2<T>) + (size_t)L1 * sizeof(c2<T>);
        dim3 grid((n2 + W - 1) / W, n3, nrhs * 3);
        VIE_W_DISPATCH(W, {
            auto launch = [&](auto lc) {
                auto kern = k_xfwd<TV, T, Wc, MAXE_XY, decltype(lc)::value>;
                (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                hipLaunchKernelGGL(kern, grid, dim3(NT), lds, s, x, eps, S1, px, tw[0], n1, n2, n3,
                                   ident ? (int)MODE_N : mode, rhs_map);
            };
            if constexpr (Wc == kWDefault<T>) with_lc(ident ? 0 : L1, launch);
            else launch(std::integral_constant<int, 0>{});
        });
    } else if (pass == 1) {
        const c2<T>* S1 = reinterpret_cast<const c2<T>*>(in);
        c2<T>* S2 = reinterpret_cast<c2<T>*>(out);
        if (allow_fast && xy_pass_fast<TV, T>(1, L2, S1, S2, x, eps, tw[1], n1, n2, n3, L1, L2, mode, nrhs,
                                              rhs_map, s))
            return hipGetLastError();
        int W = tile_width<T>(op.max_lds, L2);
        if ((size_t)W * L2 > (size_t)MAXE_XY * NT) { err = "y length too large"; return hipErrorInvalidValue; }
        size_t lds = (size_t)(W + 1) * L2 * sizeof(c2<T>) + (size_t)L2 * sizeof(c2<T>);
        dim3 grid((n3 + W - 1) / W, L1, nrhs * 3);
        VIE_W_DISPATCH(W, {
            auto launch = [&](auto lc) {
                auto kern = k_yfwd<T, Wc, MAXE_XY, decltype(lc)::value>;
                (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                hipLaunchKernelGGL(kern, grid, dim3(NT), lds, s, S1, S2, op.plan[1], tw[1], L1, n2, n3);
            };
            if constexpr (Wc == kWDefault<T>) with_lc(L2, launch);
            else launch(std::integral_constant<int, 0>{});
        });
    } else if (pass == 2) {
        c2<T>* S2 = reinterpret_cast<c2<T>*>(out);
        if (op.nhat_source == 1 && dense == nullptr) {
            err = "dense spectrum not materialised";
            return hipErrorInvalidValue;
        }
        if (allow_fast && z_pass_fast<T>(op, mode, recon, nrhs, S2, tw[2], core, fac, dense, s))
            return hipGetLastError();
        if (recon == 1) {
            err = "BF16 z pass could not be launched";
            return hipErrorInvalidValue;
        }
        int G = 4;
        while (G > 1 && z_lds_bytes<T>(v, G) > op.max_lds) G /= 2;
        size_t lds = z_lds_bytes<T>(v, G);
        if (lds > op.max_lds) { err = "z pass does not fit in LDS"; return hipErrorInvalidValue; }
        if ((size_t)3 * G * L3 > (size_t)MAXE_Z * NT) { err = "z length too large"; return hipErrorInvalidValue; }
        ZArgs za;
        za.v = v;
        za.G = G;
        za.conj = (mode == MODE_AH || mode == MODE_NH);
        za.dense = op.nhat_source == 1;
        int nblk = G == 4 ? (n1 + 1) * (n2 + 1) : (G == 2 ? (n1 + 1) * L2 : L1 * L2);
        dim3 grid(nblk, nrhs);
        auto kern = k_zmid<T, MAXE_Z>;
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, grid, dim3(NT), lds, s, S2, op.plan[2], tw[2], za, core, fac, dense);
    } else if (pass == 3) {
        const c2<T>* S2 = reinterpret_cast<const c2<T>*>(in);
        c2<T>* S3 = reinterpret_cast<c2<T>*>(out);
        if (allow_fast && xy_pass_fast<TV, T>(2, L2, S2, S3, x, eps, tw[1], n1, n2, n3, L1, L2, mode, nrhs,
                                              rhs_map, s))
            return hipGetLastError();
        int W = tile_width<T>(op.max_lds, L2);
        size_t lds = (size_t)(W + 1) * L2 * sizeof(c2<T>) + (size_t)L2 * sizeof(c2<T>);
        dim3 grid((n3 + W - 1) / W, L1, nrhs * 3);
        VIE_W_DISPATCH(W, {
            auto launch = [&](auto lc) {
                auto kern = k_yinv<T, Wc, MAXE_XY, decltype(lc)::value>;
                (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                hipLaunchKernelGGL(kern, grid, dim3(NT), lds, s, S2, S3, op.plan[1], tw[1], L1, n2, n3);
            };
            if constexpr (Wc == kWDefault<T>) with_lc(L2, launch);
            else launch(std::integral_constant<int, 0>{});
        });
    } else {
        const c2<T>* S3 = reinterpret_cast<const c2<T>*>(in);
        c2<TV>* y = reinterpret_cast<c2<TV>*>(out);
        if (ident) {
            if constexpr (std::is_same<TV, T>::value) {
                if (allow_fast && xy_ident_fast<T>(3, L1, S3, y, nullptr, tw[0], n1, n2, n3, L1, L2, nrhs, s))
                    return hipGetLastError();
            }
        } else if (allow_fast && xy_pass_fast<TV, T>(3, L1, S3, y, x, eps, tw[0], n1, n2, n3, L1, L2, mode, nrhs,
                                                     rhs_map, s)) {
            return hipGetLastError();
        }
        int W = tile_width<T>(op.max_lds, L1);
        size_t lds = (size_t)(W + 1) * L1 * sizeof(c2<T>) + (size_t)L1 * sizeof(c2<T>);
        dim3 grid((n2 + W - 1) / W, n3, nrhs * 3);
        VIE_W_DISPATCH(W, {
            auto launch = [&](auto lc) {
                auto kern = k_xinv<TV, T, Wc, MAXE_XY, decltype(lc)::value>;
                (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                hipLaunchKernelGGL(kern, grid, dim3(NT), lds, s, S3, x, eps, y, px, tw[0], n1, n2, n3,
                                   ident ? (int)MODE_N : mode, rhs_map);
            };
            if constexpr (Wc == kWDefault<T>) with_lc(ident ? 0 : L1, launch);
            else launch(std::integral_constant<int, 0>{});
        });
    }
    return hipGetLastError();
}

template <typename TV, typename T>
hipError_t launch_matvec(const DeviceOp& op, int mode, int recon, const c2<TV>* eps, const c2<TV>* x,
                         c2<TV>* y, int nrhs, c2<T>* ws, hipStream_t s, const int* rhs_map,
                         std::string& err)
{
    const OpView& v = op.view;
    c2<T>* S2 = ws;
    c2<T>* S1 = ws + (size_t)3 * v.L[1] * v.L[0] * v.n[2] * nrhs;
    if (recon == 1 && (sizeof(T) != 4 || g_kernel_path != 0 || !bf16_recon_available(op))) {
        err = "BF16 reconstruction needs complex64, the register-FFT z pass (2 n3 = 128, 256 or 512) "
              "and z ranks <= 32";
        return hipErrorInvalidValue;
    }
    // X+ : x -> S1, Y+ : S1 -> S2, Z* : S2 in place, Y- : S2 -> S1 (S3), X- : S1 -> y
    void* const ins[5] = {nullptr, S1, S2, S2, S1};
    void* const outs[5] = {S1, S2, S2, S1, y};
    for (int p = 0; p < 5; ++p) {
        hipError_t e = run_pass<TV, T>(op, p, mode, recon, eps, x, ins[p], outs[p], nrhs, s, rhs_map, err, false);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t run_pass<float, float>(const DeviceOp&, int, int, int, const c2<float>*, const c2<float>*,
                                           const void*, void*, int, hipStream_t, const int*, std::string&, bool);
template hipError_t run_pass<double, double>(const DeviceOp&, int, int, int, const c2<double>*, const c2<double>*,
                                             const void*, void*, int, hipStream_t, const int*, std::string&, bool);
template hipError_t run_pass<double, float>(const DeviceOp&, int, int, int, const c2<double>*, const c2<double>*,
                                            const void*, void*, int, hipStream_t, const int*, std::string&, bool);

template hipError_t launch_matvec<float, float>(const DeviceOp&, int, int, const c2<float>*, const c2<float>*,
                                                c2<float>*, int, c2<float>*, hipStream_t, const int*,
                                                std::string&);
template hipError_t launch_matvec<double, double>(const DeviceOp&, int, int, const c2<double>*,
                                                  const c2<double>*, c2<double>*, int, c2<double>*, hipStream_t,
                                                  const int*, std::string&);
template hipError_t launch_matvec<double, float>(const DeviceOp&, int, int, const c2<double>*,
                                                 const c2<double>*, c2<double>*, int, c2<float>*, hipStream_t,
                                                 const int*, std::string&);

// ----------------------- multi-instance launcher ------------------------
template <typename TV, typename T>
hipError_t launch_matvec_multi(const std::vector<InstHost>& inst, int mode, InstDev* tab_dev, hipStream_t s,
                               std::string& err)
{
    constexpr int MAXE_XY = 32;
    constexpr int MAXE_Z = 24;
    const int count = (int)inst.size();
    // common tile width and z group: the most restrictive instance decides
    size_t max_lds = SIZE_MAX;
    int maxL = 1, maxL3 = 1;
    for (auto& h : inst) {
        max_lds = std::min(max_lds, h.op->max_lds);
        maxL = std::max(maxL, std::max(h.op->view.L[0], h.op->view.L[1]));
        maxL3 = std::max(maxL3, h.op->view.L[2]);
    }
    int W = tile_width<T>(max_lds, maxL);
    if ((size_t)W * maxL > (size_t)MAXE_XY * NT) { err = "length too large"; return hipErrorInvalidValue; }
    std::vector<InstDev> tab(count);
    int G = 4;
    for (int i = 0; i < count; ++i)
        while (G > 1 && z_lds_bytes<T>(inst[i].op->view, G) > max_lds) G /= 2;
    size_t lds_z = 0;
    for (int i = 0; i < count; ++i) lds_z = std::max(lds_z, z_lds_bytes<T>(inst[i].op->view, G));
    if (lds_z > max_lds || (size_t)3 * G * maxL3 > (size_t)MAXE_Z * NT) { err = "z pass does not fit"; return hipErrorInvalidValue; }
    int off[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < count; ++i) {
        const DeviceOp& op = *inst[i].op;
        const OpView& v = op.view;
        InstDev& d = tab[i];
        d.v = v;
        for (int a = 0; a < 3; ++a) {
            d.plan[a] = op.plan[a];
            d.tw[a] = sizeof(T) == 8 ? (const void*)op.tw64[a] : (const void*)op.tw32[a];
        }
        d.core = sizeof(T) == 8 ? (const void*)op.d64.core : (const void*)op.d32.core;
        d.fac = sizeof(T) == 8 ? (const void*)op.d64.fac : (const void*)op.d32.fac;
        d.x = inst[i].x;
        d.y = inst[i].y;
        d.eps = inst[i].eps;
        d.map = inst[i].map;
        d.nact = inst[i].nact;
        d.S2 = inst[i].ws;
        d.S1 = (char*)inst[i].ws + sizeof(c2<T>) * (size_t)3 * v.L[1] * v.L[0] * v.n[2] * inst[i].nact;
        d.G = G;
        const int n1 = v.n[0], n2 = v.n[1], n3 = v.n[2], L1 = v.L[0], L2 = v.L[1];
        const int nz = inst[i].nact * 3;
        d.cnt[0] = ((n2 + W - 1) / W) * n3 * nz;
        d.cnt[1] = ((n3 + W - 1) / W) * L1 * nz;
        d.cnt[2] = (G == 4 ? (n1 + 1) * (n2 + 1) : (G == 2 ? (n1 + 1) * L2 : L1 * L2)) * inst[i].nact;
        d.cnt[3] = d.cnt[1];
        d.cnt[4] = d.cnt[0];
        for (int p = 0; p < 5; ++p) {
            d.off[p] = off[p];
            off[p] += d.cnt[p];
        }
    }
    hipError_t e = hipMemcpyAsync(tab_dev, tab.data(), sizeof(InstDev) * count, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    size_t lds_xy = (size_t)(W + 1) * maxL * sizeof(c2<T>) + (size_t)maxL * sizeof(c2<T>);
    const int conj = (mode == MODE_AH || mode == MODE_NH);
    {
        PassTimer timer(0, s);
        VIE_W_DISPATCH(W, {
            auto kern = k_xfwd_multi<TV, T, Wc, MAXE_XY>;
            (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_xy);
            hipLaunchKernelGGL(kern, dim3(off[0]), dim3(NT), lds_xy, s, tab_dev, count, mode);
        });
    }
    {
        PassTimer timer(1, s);
        VIE_W_DISPATCH(W, {
            auto kern = k_yfwd_multi<T, Wc, MAXE_XY>;
            (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_xy);
            hipLaunchKernelGGL(kern, dim3(off[1]), dim3(NT), lds_xy, s, tab_dev, count);
        });
    }
    {
        PassTimer timer(2, s);
        auto kern = k_zmid_multi<T, MAXE_Z>;
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_z);
        hipLaunchKernelGGL(kern, dim3(off[2]), dim3(NT), lds_z, s, tab_dev, count, conj);
    }
    {
        PassTimer timer(3, s);
        VIE_W_DISPATCH(W, {
            auto kern = k_yinv_multi<T, Wc, MAXE_XY>;
            (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_xy);
            hipLaunchKernelGGL(kern, dim3(off[3]), dim3(NT), lds_xy, s, tab_dev, count);
        });
    }
    {
        PassTimer timer(4, s);
        VIE_W_DISPATCH(W, {
            auto kern = k_xinv_multi<TV, T, Wc, MAXE_XY>;
            (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_xy);
            hipLaunchKernelGGL(kern, dim3(off[4]), dim3(NT), lds_xy, s, tab_dev, count, mode);
        });
    }
    return hipGetLastError();
}

template hipError_t launch_matvec_multi<float, float>(const std::vector<InstHost>&, int, InstDev*, hipStream_t,
                                                      std::string&);
template hipError_t launch_matvec_multi<double, double>(const std::vector<InstHost>&, int, InstDev*, hipStream_t,
                                                        std::string&);
template hipError_t launch_matvec_multi<double, float>(const std::vector<InstHost>&, int, InstDev*, hipStream_t,
                                                       std::string&);

// ----------------------- sampled N^ (tests) ------------------------------
template <typename T>
__global__ void k_nhat_samples(OpView v, const c2<T>* __restrict__ core, const c2<T>* __restrict__ fac,
                               const int* __restrict__ idx, int count, double* __restrict__ out)
{
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= count) return;
    int c = idx[4 * m], kk[3] = {idx[4 * m + 1], idx[4 * m + 2], idx[4 * m + 3]};
    int f[3];
    for (int a = 0; a < 3; ++a) {
        f[a] = kk[a] > v.n[a];
        if (f[a]) kk[a] = v.L[a] - kk[a];
    }
    const int r1 = v.r[c][0], r2 = v.r[c][1], r3 = v.r[c][2];
    const c2<T>* G = core + v.core_off[c];
    const c2<T>* U1 = fac + v.fac_off[c][0] + (long)kk[0] * r1;
    const c2<T>* U2 = fac + v.fac_off[c][1] + (long)kk[1] * r2;
    const c2<T>* U3 = fac + v.fac_off[c][2] + (long)kk[2] * r3;
    c2<T> acc = mk<T>(0, 0);
    for (int al = 0; al < r1; ++al)
        for (int be = 0; be < r2; ++be) {
            c2<T> t = mk<T>(0, 0);
            for (int ga = 0; ga < r3; ++ga) fma_c(t, G[((long)al * r2 + be) * r3 + ga], U3[ga]);
            acc = acc + U1[al] * (U2[be] * t);
        }
    if (comp_sign(v.fam, c, f[0], f[1], f[2]) < 0) acc = mk<T>(-acc.x, -acc.y);
    out[2 * m] = (double)acc.x;
    out[2 * m + 1] = (double)acc.y;
}

hipError_t launch_nhat_samples(const DeviceOp& op, int prec, const int* idx_dev, int count, double* out_dev,
                               hipStream_t s)
{
    int nb = (count + 255) / 256;
    if (prec == 1)
        hipLaunchKernelGGL(k_nhat_samples<double>, dim3(nb), dim3(256), 0, s, op.view, op.d64.core, op.d64.fac,
                           idx_dev, count, out_dev);
    else
        hipLaunchKernelGGL(k_nhat_samples<float>, dim3(nb), dim3(256), 0, s, op.view, op.d32.core, op.d32.fac,
                           idx_dev, count, out_dev);
    return hipGetLastError();
}

// ----------------------- dense half spectrum -----------------------------
template <typename T>
__global__ void k_densify(OpView v, const c2<T>* __restrict__ core, const c2<T>* __restrict__ fac,
                          c2<T>* __restrict__ dense)
{
    // one block per (c, k2, k1), threads over k3
    const int n1 = v.n[0], n2 = v.n[1], n3 = v.n[2];
    int bidx = blockIdx.x;
    int k1 = bidx % (n1 + 1);
    int k2 = (bidx / (n1 + 1)) % (n2 + 1);
    int c = bidx / ((n1 + 1) * (n2 + 1));
    const int r1 = v.r[c][0], r2 = v.r[c][1], r3 = v.r[c][2];
    const c2<T>* G = core + v.core_off[c];
    const c2<T>* U1 = fac + v.fac_off[c][0] + (long)k1 * r1;
    const c2<T>* U2 = fac + v.fac_off[c][1] + (long)k2 * r2;
    __shared__ c2<T> Vs[128];
    for (int ga = threadIdx.x; ga < r3; ga += blockDim.x) {
        c2<T> acc = mk<T>(0, 0);
        for (int al = 0; al < r1; ++al) {
            c2<T> t = mk<T>(0, 0);
            for (int be = 0; be < r2; ++be) fma_c(t, G[((long)al * r2 + be) * r3 + ga], U2[be]);
            fma_c(acc, U1[al], t);
        }
        Vs[ga] = acc;
    }
    __syncthreads();
    const long per = (long)(n1 + 1) * (n2 + 1) * (n3 + 1);
    for (int kk = threadIdx.x; kk <= n3; kk += blockDim.x) {
        const c2<T>* U3 = fac + v.fac_off[c][2] + (long)kk * r3;
        c2<T> acc = mk<T>(0, 0);
        for (int ga = 0; ga < r3; ++ga) fma_c(acc, Vs[ga], U3[ga]);
        dense[c * per + ((long)k2 * (n1 + 1) + k1) * (n3 + 1) + kk] = acc;
    }
}

hipError_t launch_densify(DeviceOp& op, int with_c128, hipStream_t s)
{
    const OpView& v = op.view;
    if (v.rmax > 128) return hipErrorInvalidValue;
    long per = (long)(v.n[0] + 1) * (v.n[1] + 1) * (v.n[2] + 1);
    int nb = 6 * (v.n[0] + 1) * (v.n[1] + 1);
    hipError_t e;
    if (!op.dense32) {
        e = hipMalloc((void**)&op.dense32, sizeof(c2<float>) * 6 * per);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_densify<float>, dim3(nb), dim3(256), 0, s, v, op.d32.core, op.d32.fac, op.dense32);
    if (with_c128) {
        if (!op.dense64) {
            e = hipMalloc((void**)&op.dense64, sizeof(c2<double>) * 6 * per);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_densify<double>, dim3(nb), dim3(256), 0, s, v, op.d64.core, op.d64.fac,
                           op.dense64);
    }
    return hipGetLastError();
}

// Whether every instance has register-FFT kernels for all five passes.
template <typename T>
static bool batch_grouped_ok(const std::vector<InstHost>& req, int recon)
{
    if (g_kernel_path != 0) return false;
    for (const InstHost& h : req) {
        const DeviceOp& op = *h.op;
        const OpView& v = op.view;
        if (v.fam != 0) return false;
        if (!xy_fast_length(v.L[0]) || !xy_fast_length(v.L[1]) || !z_fast_length(v.L[2])) return false;
        if (op.nhat_source == 1 && (sizeof(T) == 8 ? (const void*)op.dense64 : (const void*)op.dense32) == nullptr)
            return false;
        if (recon == 1 && (sizeof(T) != 4 || !bf16_recon_available(op))) return false;
    }
    return true;
}

// One launch per pass and FFT length over every instance of the batch
// (register-FFT kernels; the per-instance descriptors are kernel arguments,
// at most kXYGroupMax / kZGroupMax instances per launch).
template <typename TV, typename T>
static hipError_t launch_batch_grouped(const std::vector<InstHost>& req, int mode, int recon, hipStream_t s,
                                       std::string& err)
{
    const int count = (int)req.size();
    const int conj = (mode == MODE_AH || mode == MODE_NH);
    auto tw_of = [](const DeviceOp& op, int axis) -> const c2<T>* {
        if constexpr (sizeof(T) == 8) return op.tw64[axis];
        else return op.tw32[axis];
    };
    for (int p = 0; p < 5; ++p) {
        PassTimer timer(p, s);
        const int kind = p < 2 ? p : p - 1;   // X+, Y+, (Z), Y-, X-
        const int axis = p == 2 ? 2 : ((kind == 0 || kind == 3) ? 0 : 1);
        const int gmax = p == 2 ? kZGroupMax : kXYGroupMax;
        std::vector<char> done(count, 0);
        for (int i = 0; i < count; ++i) {
            if (done[i]) continue;
            const int L = req[i].op->view.L[axis];
            XYGroup xg;
            ZGroup zg;
            xg.n = zg.n = 0;
            int off = 0, rmax = 0;
            const c2<T>* tw = tw_of(*req[i].op, axis);
            for (int j = i; j < count; ++j) {
                if (done[j] || req[j].op->view.L[axis] != L) continue;
                if ((p == 2 ? zg.n : xg.n) == gmax) break;   // the next launch takes the rest
                done[j] = 1;
                const InstHost& h = req[j];
                const DeviceOp& op = *h.op;
                const OpView& v = op.view;
                c2<T>* S2 = (c2<T>*)h.ws;
                c2<T>* S1 = S2 + (size_t)3 * v.L[1] * v.L[0] * v.n[2] * h.nact;
                if (p == 2) {
                    ZInst& z = zg.e[zg.n++];
                    z = ZInst{};
                    z.S2 = S2;
                    if constexpr (sizeof(T) == 8) {
                        z.core = op.d64.core;
                        z.fac = op.d64.fac;
                        z.dense = op.dense64;
                    } else {
                        z.core = op.d32.core;
                        z.fac = op.d32.fac;
                        z.dense = op.dense32;
                    }
                    z.f3m = op.b16.fac3m;
                    z.za.v = v;
                    z.za.conj = conj;
                    z.za.dense = op.nhat_source == 1;
                    z.za.chunk = op.zchunk;
                    z.nbx = (v.n[1] + 1) * ((v.n[0] + 1 + op.zchunk - 1) / op.zchunk);
                    z.off = off;
                    off += z.nbx * h.nact;
                    rmax = std::max(rmax, v.rmax);
                } else {
                    const int W = xy_fast_tile<TV, T>(L);
                    XYInst& e = xg.e[xg.n++];
                    e = XYInst{};
                    e.x = h.x;
                    e.eps = h.eps;
                    e.map = h.map;
                    e.a = XYArgs{v.n[0], v.n[1], v.n[2], v.L[0], v.L[1], mode};
                    if (kind == 0) { e.in = nullptr; e.out = S1; e.ntx = (v.n[1] + W - 1) / W; e.rows = v.n[2]; }
                    else if (kind == 1) { e.in = S1; e.out = S2; e.ntx = (v.n[2] + W - 1) / W; e.rows = v.L[0]; }
                    else if (kind == 2) { e.in = S2; e.out = S1; e.ntx = (v.n[2] + W - 1) / W; e.rows = v.L[0]; }
                    else { e.in = S1; e.out = h.y; e.ntx = (v.n[1] + W - 1) / W; e.rows = v.n[2]; }
                    e.off = off;
                    off += e.ntx * e.rows * 3 * h.nact;
                }
            }
            if (off == 0) continue;
            const bool ok = p == 2 ? z_group_fast<T>(L, conj, recon, rmax, req[i].op->max_lds, zg, off, tw, s)
                                   : xy_group_fast<TV, T>(kind, L, xg, off, tw, s);
            if (!ok) {
                err = "grouped register-FFT launch not available for this batch";
                return hipErrorInvalidValue;
            }
        }
    }
    return hipGetLastError();
}

template <typename TV, typename T>
hipError_t launch_batch(const std::vector<InstHost>& req, int mode, int recon, InstDev* tab, hipStream_t st,
                        std::string& err)
{
    if (req.empty()) return hipSuccess;
    if (req.size() > 1 && g_batch_mode == 0 && batch_grouped_ok<T>(req, recon))
        return launch_batch_grouped<TV, T>(req, mode, recon, st, err);
    if (req.size() == 1 || g_batch_mode == 0) {
        for (const InstHost& h : req) {
            hipError_t e = launch_matvec<TV, T>(*h.op, mode, recon, (const c2<TV>*)h.eps, (const c2<TV>*)h.x,
                                                (c2<TV>*)h.y, h.nact, (c2<T>*)h.ws, st, h.map, err);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    if (recon != 0) {
        err = "BF16 reconstruction is not available in the single-launch batch mode";
        return hipErrorInvalidValue;
    }
    return launch_matvec_multi<TV, T>(req, mode, tab, st, err);
}

template hipError_t launch_batch<float, float>(const std::vector<InstHost>&, int, int, InstDev*, hipStream_t,
                                               std::string&);
template hipError_t launch_batch<double, double>(const std::vector<InstHost>&, int, int, InstDev*, hipStream_t,
                                                 std::string&);
template hipError_t launch_batch<double, float>(const std::vector<InstHost>&, int, int, InstDev*, hipStream_t,
                                                std::string&);


}  // namespace vie
