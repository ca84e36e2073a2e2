// Batched vector kernels of the GMRES driver (Arnoldi with classical
// Gram-Schmidt and one re-orthogonalisation, residuals, norms) and the
// voxel-wise gradient factor.  Systems are independent right-hand sides; a
// device map selects the systems that are still active, so converged ones
// cost nothing.  Vector v of system s sits at base + v*vstride + s*sstride
// (complex elements).  Reductions are two-stage (per-block partials, then a
// fixed-order sum), so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "krylov.h"

namespace vie {

static constexpr int KB = 256;       // threads per block
static constexpr int KEL = 8;        // elements per thread per block chunk

__device__ __forceinline__ c2<double> block_sum(c2<double> v, c2<double>* red)
{
    // wave64 tree reduction, then across the 4 waves of the block
    for (int off = 32; off > 0; off >>= 1) {
        v.x += __shfl_xor(v.x, off, 64);
        v.y += __shfl_xor(v.y, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    c2<double> t = mk<double>(0, 0);
    if (threadIdx.x == 0)
        for (int k = 0; k < KB / 64; ++k) t = t + red[k];
    return t;   // valid in thread 0
}

template <typename TK>
__global__ void __launch_bounds__(KB) k_mdot(const c2<TK>* __restrict__ V, long vstride, long sstride, int nvec,
                                             const c2<TK>* __restrict__ W, long wvoff, long n,
                                             const int* __restrict__ map, int nblk, c2<double>* __restrict__ partial)
{
    __shared__ c2<double> red[KB / 64];
    const int a = blockIdx.y, s = map[a];
    const long base = (long)blockIdx.x * KB * KEL;
    const c2<TK>* w = W + wvoff + s * sstride;
    c2<double> wl[KEL];
#pragma unroll
    for (int t = 0; t < KEL; ++t) {
        long i = base + t * KB + threadIdx.x;
        wl[t] = i < n ? cvt<double>(w[i]) : mk<double>(0, 0);
    }
    for (int v = 0; v < nvec; ++v) {
        const c2<TK>* vv = V + v * vstride + s * sstride;
        c2<double> acc = mk<double>(0, 0);
#pragma unroll
        for (int t = 0; t < KEL; ++t) {
            long i = base + t * KB + threadIdx.x;
            if (i < n) {
                c2<double> x = cvt<double>(vv[i]);
                acc = acc + mulc(wl[t], x);            // conj(v) * w
            }
        }
        c2<double> tot = block_sum(acc, red);
        if (threadIdx.x == 0) partial[((long)a * nvec + v) * nblk + blockIdx.x] = tot;
    }
}

__global__ void __launch_bounds__(KB) k_reduce(const c2<double>* __restrict__ partial, int nblk,
                                               c2<double>* __restrict__ out)
{
    __shared__ c2<double> red[KB / 64];
    const long row = blockIdx.x;
    c2<double> acc = mk<double>(0, 0);
    for (int b = threadIdx.x; b < nblk; b += KB) acc = acc + partial[row * nblk + b];
    c2<double> tot = block_sum(acc, red);
    if (threadIdx.x == 0) out[row] = tot;
}

// W[s] += sign * sum_v V_v[s] coef[a][v]
template <typename TK>
__global__ void __launch_bounds__(KB) k_maxpy(c2<TK>* __restrict__ W, long wvoff, long wsstride,
                                              const c2<TK>* __restrict__ V, long vstride, long sstride, int nvec,
                                              int cstride, const c2<double>* __restrict__ coef, double sign,
                                              long n, const int* __restrict__ map)
{
    const int a = blockIdx.y, s = map[a];
    const long base = (long)blockIdx.x * KB * KEL;
    c2<TK>* w = W + wvoff + s * wsstride;
    c2<double> acc[KEL];
#pragma unroll
    for (int t = 0; t < KEL; ++t) acc[t] = mk<double>(0, 0);
    for (int v = 0; v < nvec; ++v) {
        c2<double> cf = coef[(long)a * cstride + v];
        if (cf.x == 0.0 && cf.y == 0.0) continue;   // padding of shorter cycles: never touch those vectors
        const c2<TK>* vv = V + v * vstride + s * sstride;
#pragma unroll
        for (int t = 0; t < KEL; ++t) {
            long i = base + t * KB + threadIdx.x;
            if (i < n) acc[t] = acc[t] + cvt<double>(vv[i]) * cf;
        }
    }
#pragma unroll
    for (int t = 0; t < KEL; ++t) {
        long i = base + t * KB + threadIdx.x;
        if (i < n) {
            c2<double> o = cvt<double>(w[i]);
            o = o + sign * acc[t];
            w[i] = cvt<TK>(o);
        }
    }
}

template <typename TK>
__global__ void __launch_bounds__(KB) k_norm2(const c2<TK>* __restrict__ W, long wvoff, long sstride, long n,
                                              const int* __restrict__ map, int nblk,
                                              c2<double>* __restrict__ partial)
{
    __shared__ c2<double> red[KB / 64];
    const int a = blockIdx.y, s = map[a];
    const long base = (long)blockIdx.x * KB * KEL;
    const c2<TK>* w = W + wvoff + s * sstride;
    double acc = 0;
#pragma unroll
    for (int t = 0; t < KEL; ++t) {
        long i = base + t * KB + threadIdx.x;
        if (i < n) {
            c2<double> x = cvt<double>(w[i]);
            acc += x.x * x.x + x.y * x.y;
        }
    }
    c2<double> tot = block_sum(mk<double>(acc, 0.0), red);
    if (threadIdx.x == 0) partial[(long)a * nblk + blockIdx.x] = tot;
}

// dst[s] = src[s] / sqrt(norm2[a].x)  (zero if the norm is zero)
template <typename TK>
__global__ void __launch_bounds__(KB) k_scale_norm(c2<TK>* __restrict__ dst, long dvoff, const c2<TK>* __restrict__ src,
                                                   long svoff, long sstride, const c2<double>* __restrict__ norm2,
                                                   long n, const int* __restrict__ map)
{
    const int a = blockIdx.y, s = map[a];
    double nn = norm2[a].x;
    double sc = nn > 0 ? 1.0 / sqrt(nn) : 0.0;
    const long base = (long)blockIdx.x * KB * KEL;
#pragma unroll
    for (int t = 0; t < KEL; ++t) {
        long i = base + t * KB + threadIdx.x;
        if (i < n) {
            c2<double> x = cvt<double>(src[svoff + s * sstride + i]);
            dst[dvoff + s * sstride + i] = cvt<TK>(sc * x);
        }
    }
}

// R[s] = B[s] - R[s]
template <typename TK>
__global__ void __launch_bounds__(KB) k_residual(c2<TK>* __restrict__ R, const c2<TK>* __restrict__ B, long sstride,
                                                 long n, const int* __restrict__ map)
{
    const int a = blockIdx.y, s = map[a];
    const long base = (long)blockIdx.x * KB * KEL;
#pragma unroll
    for (int t = 0; t < KEL; ++t) {
        long i = base + t * KB + threadIdx.x;
        if (i < n) R[s * sstride + i] = B[s * sstride + i] - R[s * sstride + i];
    }
}

template <typename TO, typename TI>
__global__ void __launch_bounds__(KB) k_convert(c2<TO>* __restrict__ dst, const c2<TI>* __restrict__ src, long n)
{
    long i = (long)blockIdx.x * KB + threadIdx.x;
    if (i < n) dst[i] = cvt<TO>(src[i]);
}

// g_eps = Re X, g_sigma = Im X / (omega eps0), X = sum_q conj(z_q) E_q
template <typename T>
__global__ void __launch_bounds__(KB) k_field_gradient(const c2<T>* __restrict__ z, const c2<T>* __restrict__ E,
                                                       T* __restrict__ g_eps, T* __restrict__ g_sig, double oe0,
                                                       long V)
{
    long i = (long)blockIdx.x * KB + threadIdx.x;
    if (i >= V) return;
    c2<T> acc = mk<T>(0, 0);
    for (int q = 0; q < 3; ++q) acc = acc + mulc(E[q * V + i], z[q * V + i]);   // conj(z) E
    g_eps[i] = acc.x;
    g_sig[i] = (T)(acc.y / oe0);
}

// eps_c = eps_r - i sigma / (omega eps0);  b_q = i omega eps0 (eps_c - 1) e_q
template <typename T>
__global__ void __launch_bounds__(KB) k_problem(const T* __restrict__ eps_r, const T* __restrict__ sigma,
                                                const c2<T>* __restrict__ e_inc, c2<T>* __restrict__ eps_c,
                                                c2<T>* __restrict__ b, double oe0, long V)
{
    long i = (long)blockIdx.x * KB + threadIdx.x;
    if (i >= V) return;
    c2<T> ec = mk<T>(eps_r[i], (T)(-(double)sigma[i] / oe0));
    eps_c[i] = ec;
    c2<T> ce_chi = mk<T>((T)(-oe0 * (double)ec.y), (T)(oe0 * ((double)ec.x - 1.0)));   // i oe0 (eps_c - 1)
    for (int q = 0; q < 3; ++q) b[q * V + i] = ce_chi * e_inc[q * V + i];
}

// E = e_inc + (Nu - u) / (i omega eps0)
template <typename T>
__global__ void __launch_bounds__(KB) k_total_field(const c2<T>* __restrict__ e_inc, const c2<T>* __restrict__ u,
                                                    const c2<T>* __restrict__ Nu, c2<T>* __restrict__ E, double oe0,
                                                    long n)
{
    long i = (long)blockIdx.x * KB + threadIdx.x;
    if (i >= n) return;
    c2<T> d = Nu[i] - u[i];
    // d / (i oe0) = -i d / oe0
    E[i] = mk<T>(e_inc[i].x + (T)((double)d.y / oe0), e_inc[i].y - (T)((double)d.x / oe0));
}

// H = h_inc + h KJ (the physical K is h times the dimensionless tensor) and
// |b1+| = mu0 |H_x + i H_y| (eq. 18); nv voxels, components [3][nv]
template <typename T>
__global__ void __launch_bounds__(KB) k_magnetic_field(const c2<T>* __restrict__ h_inc, const c2<T>* __restrict__ KJ,
                                                       double h, double mu0, c2<T>* __restrict__ H, T* __restrict__ b1,
                                                       long nv)
{
    long i = (long)blockIdx.x * KB + threadIdx.x;
    if (i >= nv) return;
    c2<T> hq[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const long o = q * nv + i;
        hq[q] = mk<T>(h_inc[o].x + (T)h * KJ[o].x, h_inc[o].y + (T)h * KJ[o].y);
        H[o] = hq[q];
    }
    // H_x + i H_y
    const double re = (double)hq[0].x - (double)hq[1].y, im = (double)hq[0].y + (double)hq[1].x;
    b1[i] = (T)(mu0 * sqrt(re * re + im * im));
}

// Full JMVIE operator (eq. 4) from the N and K products of x = [J; M]:
//   y_J = eps J - chi_e N J + i ce_h chi_e K M
//   y_M = mu M  - chi_h N M - i cm_h chi_h K J
// (ce_h = omega eps0 h, cm_h = omega mu0 h; chi = contrast - 1); x, NX, KX,
// y are [2][nq][nv] (nq = 3 pulse components, or 12 piecewise-linear
// coefficients in the mass-normalised basis, whose mass term is the
// identity), eps and mu [nv]
template <typename T>
__global__ void __launch_bounds__(KB) k_jm_combine(const c2<T>* __restrict__ eps, const c2<T>* __restrict__ mu,
                                                   const c2<T>* __restrict__ x, const c2<T>* __restrict__ NX,
                                                   const c2<T>* __restrict__ KX, double ce_h, double cm_h,
                                                   c2<T>* __restrict__ y, long nv, int nq)
{
    long i = (long)blockIdx.x * KB + threadIdx.x;
    if (i >= nv) return;
    const c2<T> e = eps[i], m = mu[i];
    const c2<T> ce = mk<T>(e.x - (T)1, e.y), cmu = mk<T>(m.x - (T)1, m.y);
    const c2<T> ie = mk<T>(0, (T)ce_h) * ce, im = mk<T>(0, (T)cm_h) * cmu;
    for (int q = 0; q < nq; ++q) {
        const long oJ = q * nv + i, oM = (nq + q) * nv + i;
        y[oJ] = e * x[oJ] - ce * NX[oJ] + ie * KX[oM];
        y[oM] = m * x[oM] - cmu * NX[oM] - im * KX[oJ];
    }
}

// t = N^H g - g
template <typename T>
__global__ void __launch_bounds__(KB) k_adjoint_source(const c2<T>* __restrict__ g, const c2<T>* __restrict__ NHg,
                                                       c2<T>* __restrict__ t, long n)
{
    long i = (long)blockIdx.x * KB + threadIdx.x;
    if (i >= n) return;
    t[i] = NHg[i] - g[i];
}

// ---------------------------- launchers ---------------------------------
static inline int nblocks(long n) { return (int)((n + (long)KB * KEL - 1) / ((long)KB * KEL)); }

int krylov_nblk(long n) { return nblocks(n); }

template <typename TK>
hipError_t kr_mdot(const c2<TK>* V, long vstride, long sstride, int nvec, const c2<TK>* W, long wvoff, long n,
                   const int* map, int nact, c2<double>* partial, c2<double>* out, hipStream_t st)
{
    int nb = nblocks(n);
    hipLaunchKernelGGL(k_mdot<TK>, dim3(nb, nact), dim3(KB), 0, st, V, vstride, sstride, nvec, W, wvoff, n, map,
                       nb, partial);
    hipLaunchKernelGGL(k_reduce, dim3(nact * nvec), dim3(KB), 0, st, partial, nb, out);
    return hipGetLastError();
}

template <typename TK>
hipError_t kr_maxpy(c2<TK>* W, long wvoff, long wsstride, const c2<TK>* V, long vstride, long sstride, int nvec,
                    int cstride, const c2<double>* coef, double sign, long n, const int* map, int nact,
                    hipStream_t st)
{
    hipLaunchKernelGGL(k_maxpy<TK>, dim3(nblocks(n), nact), dim3(KB), 0, st, W, wvoff, wsstride, V, vstride,
                       sstride, nvec, cstride, coef, sign, n, map);
    return hipGetLastError();
}

template <typename TK>
hipError_t kr_norm2(const c2<TK>* W, long wvoff, long sstride, long n, const int* map, int nact,
                    c2<double>* partial, c2<double>* out, hipStream_t st)
{
    int nb = nblocks(n);
    hipLaunchKernelGGL(k_norm2<TK>, dim3(nb, nact), dim3(KB), 0, st, W, wvoff, sstride, n, map, nb, partial);
    hipLaunchKernelGGL(k_reduce, dim3(nact), dim3(KB), 0, st, partial, nb, out);
    return hipGetLastError();
}

template <typename TK>
hipError_t kr_scale_norm(c2<TK>* dst, long dvoff, const c2<TK>* src, long svoff, long sstride,
                         const c2<double>* norm2, long n, const int* map, int nact, hipStream_t st)
{
    hipLaunchKernelGGL(k_scale_norm<TK>, dim3(nblocks(n), nact), dim3(KB), 0, st, dst, dvoff, src, svoff, sstride,
                       norm2, n, map);
    return hipGetLastError();
}

template <typename TK>
hipError_t kr_residual(c2<TK>* R, const c2<TK>* B, long sstride, long n, const int* map, int nact, hipStream_t st)
{
    hipLaunchKernelGGL(k_residual<TK>, dim3(nblocks(n), nact), dim3(KB), 0, st, R, B, sstride, n, map);
    return hipGetLastError();
}

template <typename TO, typename TI>
hipError_t kr_convert(c2<TO>* dst, const c2<TI>* src, long n, hipStream_t st)
{
    hipLaunchKernelGGL((k_convert<TO, TI>), dim3((n + KB - 1) / KB), dim3(KB), 0, st, dst, src, n);
    return hipGetLastError();
}

template <typename T>
hipError_t kr_field_gradient(const c2<T>* z, const c2<T>* E, T* g_eps, T* g_sig, double oe0, long V,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_field_gradient<T>, dim3((V + KB - 1) / KB), dim3(KB), 0, st, z, E, g_eps, g_sig, oe0, V);
    return hipGetLastError();
}

template <typename T>
hipError_t kr_problem(const T* eps_r, const T* sigma, const c2<T>* e_inc, c2<T>* eps_c, c2<T>* b, double oe0, long V,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_problem<T>, dim3((V + KB - 1) / KB), dim3(KB), 0, st, eps_r, sigma, e_inc, eps_c, b, oe0, V);
    return hipGetLastError();
}

template <typename T>
hipError_t kr_total_field(const c2<T>* e_inc, const c2<T>* u, const c2<T>* Nu, c2<T>* E, double oe0, long n,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_total_field<T>, dim3((n + KB - 1) / KB), dim3(KB), 0, st, e_inc, u, Nu, E, oe0, n);
    return hipGetLastError();
}

template <typename T>
hipError_t kr_magnetic_field(const c2<T>* h_inc, const c2<T>* KJ, double h, double mu0, c2<T>* H, T* b1, long nv,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_magnetic_field<T>, dim3((nv + KB - 1) / KB), dim3(KB), 0, st, h_inc, KJ, h, mu0, H, b1, nv);
    return hipGetLastError();
}

template <typename T>
hipError_t kr_jm_combine(const c2<T>* eps, const c2<T>* mu, const c2<T>* x, const c2<T>* NX, const c2<T>* KX,
                         double ce_h, double cm_h, c2<T>* y, long nv, int nq, hipStream_t st)
{
    hipLaunchKernelGGL(k_jm_combine<T>, dim3((nv + KB - 1) / KB), dim3(KB), 0, st, eps, mu, x, NX, KX, ce_h, cm_h, y,
                       nv, nq);
    return hipGetLastError();
}

template <typename T>
hipError_t kr_adjoint_source(const c2<T>* g, const c2<T>* NHg, c2<T>* t, long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_adjoint_source<T>, dim3((n + KB - 1) / KB), dim3(KB), 0, st, g, NHg, t, n);
    return hipGetLastError();
}

#define VIE_KR_INST(TK)                                                                                          \
    template hipError_t kr_mdot<TK>(const c2<TK>*, long, long, int, const c2<TK>*, long, long, const int*, int,  \
                                    c2<double>*, c2<double>*, hipStream_t);                                      \
    template hipError_t kr_maxpy<TK>(c2<TK>*, long, long, const c2<TK>*, long, long, int, int,                   \
                                     const c2<double>*, double, long, const int*, int, hipStream_t);             \
    template hipError_t kr_norm2<TK>(const c2<TK>*, long, long, long, const int*, int, c2<double>*, c2<double>*, \
                                     hipStream_t);                                                               \
    template hipError_t kr_scale_norm<TK>(c2<TK>*, long, const c2<TK>*, long, long, const c2<double>*, long,     \
                                          const int*, int, hipStream_t);                                         \
    template hipError_t kr_residual<TK>(c2<TK>*, const c2<TK>*, long, long, const int*, int, hipStream_t);       \
    template hipError_t kr_field_gradient<TK>(const c2<TK>*, const c2<TK>*, TK*, TK*, double, long, hipStream_t); \
    template hipError_t kr_problem<TK>(const TK*, const TK*, const c2<TK>*, c2<TK>*, c2<TK>*, double, long,        \
                                       hipStream_t);                                                             \
    template hipError_t kr_total_field<TK>(const c2<TK>*, const c2<TK>*, const c2<TK>*, c2<TK>*, double, long,     \
                                           hipStream_t);                                                         \
    template hipError_t kr_adjoint_source<TK>(const c2<TK>*, const c2<TK>*, c2<TK>*, long, hipStream_t);          \
    template hipError_t kr_magnetic_field<TK>(const c2<TK>*, const c2<TK>*, double, double, c2<TK>*, TK*, long,   \
                                              hipStream_t);                                                      \
    template hipError_t kr_jm_combine<TK>(const c2<TK>*, const c2<TK>*, const c2<TK>*, const c2<TK>*,             \
                                          const c2<TK>*, double, double, c2<TK>*, long, int, hipStream_t);

VIE_KR_INST(float)
VIE_KR_INST(double)
template hipError_t kr_convert<float, double>(c2<float>*, const c2<double>*, long, hipStream_t);
template hipError_t kr_convert<double, float>(c2<double>*, const c2<float>*, long, hipStream_t);

}  // namespace vie
