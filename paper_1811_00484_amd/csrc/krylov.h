// Launchers of the batched Krylov vector kernels (krylov.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "dev_common.h"

namespace vie {

int krylov_nblk(long n);   // per-system partial count for a vector of n complex elements

// out[a*nvec + v] = <V_v[s], W[s]> = sum conj(V_v) W, s = map[a]
template <typename TK>
hipError_t kr_mdot(const c2<TK>* V, long vstride, long sstride, int nvec, const c2<TK>* W, long wvoff, long n,
                   const int* map, int nact, c2<double>* partial, c2<double>* out, hipStream_t st);
// W[s] += sign * sum_v V_v[s] coef[a*cstride + v]
template <typename TK>
hipError_t kr_maxpy(c2<TK>* W, long wvoff, long wsstride, const c2<TK>* V, long vstride, long sstride, int nvec,
                    int cstride, const c2<double>* coef, double sign, long n, const int* map, int nact,
                    hipStream_t st);
// out[a].x = ||W[s]||^2
template <typename TK>
hipError_t kr_norm2(const c2<TK>* W, long wvoff, long sstride, long n, const int* map, int nact,
                    c2<double>* partial, c2<double>* out, hipStream_t st);
// dst[s] = src[s] / sqrt(norm2[a].x)
template <typename TK>
hipError_t kr_scale_norm(c2<TK>* dst, long dvoff, const c2<TK>* src, long svoff, long sstride,
                         const c2<double>* norm2, long n, const int* map, int nact, hipStream_t st);
// R[s] = B[s] - R[s]
template <typename TK>
hipError_t kr_residual(c2<TK>* R, const c2<TK>* B, long sstride, long n, const int* map, int nact, hipStream_t st);
template <typename TO, typename TI>
hipError_t kr_convert(c2<TO>* dst, const c2<TI>* src, long n, hipStream_t st);
// g_eps = Re X, g_sigma = Im X / oe0 with X = sum_q conj(z_q) E_q per voxel
template <typename T>
hipError_t kr_field_gradient(const c2<T>* z, const c2<T>* E, T* g_eps, T* g_sig, double oe0, long V,
                             hipStream_t st);
// eps_c = eps_r - i sigma / oe0, b = i oe0 (eps_c - 1) e_inc   (oe0 = omega eps0)
template <typename T>
hipError_t kr_problem(const T* eps_r, const T* sigma, const c2<T>* e_inc, c2<T>* eps_c, c2<T>* b, double oe0, long V,
                      hipStream_t st);
// E = e_inc + (Nu - u) / (i oe0)
template <typename T>
hipError_t kr_total_field(const c2<T>* e_inc, const c2<T>* u, const c2<T>* Nu, c2<T>* E, double oe0, long n,
                          hipStream_t st);
// t = NHg - g
template <typename T>
hipError_t kr_magnetic_field(const c2<T>* h_inc, const c2<T>* KJ, double h, double mu0, c2<T>* H, T* b1, long nv,
                             hipStream_t st);
template <typename T>
hipError_t kr_jm_combine(const c2<T>* eps, const c2<T>* mu, const c2<T>* x, const c2<T>* NX, const c2<T>* KX,
                         double ce_h, double cm_h, c2<T>* y, long nv, int nq, hipStream_t st);
template <typename T>
hipError_t kr_adjoint_source(const c2<T>* g, const c2<T>* NHg, c2<T>* t, long n, hipStream_t st);

}  // namespace vie
