// One Tucker (eq. 14) or Tucker+CP (eq. 17) component applied element-wise
// to a vector on its own n1 x n2 x n3 grid, y = D .* x with
// D = G x1 U1 x2 U2 x3 U3: the "decompression and element-wise product" of
// Sec. V-B (Table II, timed in Table IV), done in one pass over x and y with
// no buffer for D.
//
//   Tucker: W(k)   = G x3 U3(k, :)           (r1 x r2 per k; first kernel)
//           V(j,k) = W(k) U2(j, :)^T          (r1 per (j, k); second kernel)
//   CP:     V_l(j,k) = lambda_l U2(j, l) U3(k, l) (the 4-D loop of Sec. V-B)
//   then    D(i,j,k) = U1(i, :) . V(j, k), y = D .* x   (third kernel)
// The third kernel walks the (i, j) plane flat (consecutive threads take
// consecutive i, wrapping into the next j), so no lane idles on ragged n1;
// each thread keeps its row U1(i, :) in registers (read coalesced from a
// transposed copy) and reads V(j, k) through the cache (the lanes of a
// wavefront share one or two j), for KT consecutive k.  HBM traffic: x in,
// y out, and V (r1 complex per (j, k)).
#include <hip/hip_runtime.h>

#include <string>

#include "vie.h"
#include "vie_internal.h"

namespace vie {
vie_status fail(vie_status st, const std::string& msg);
vie_status hip_fail(hipError_t e, const char* where);
}  // namespace vie

namespace {

using namespace vie;

constexpr int kRMax = 32;    // largest rank per mode
constexpr int kKT = 16;      // k rows per workgroup of the apply kernel
constexpr int kNT = 256;     // threads per workgroup of the apply kernel ((i, j) positions)

template <typename T>
__global__ void __launch_bounds__(256) k_core_z(const c2<T>* __restrict__ G, const c2<T>* __restrict__ U3, int r1,
                                                int r2, int r3, c2<T>* __restrict__ W)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (e >= r1 * r2) return;
    const c2<T>* g = G + (long)e * r3;
    const c2<T>* u = U3 + (long)k * r3;
    c2<T> acc = mk<T>(0, 0);
    for (int c = 0; c < r3; ++c) fma_c(acc, g[c], u[c]);
    W[(long)k * r1 * r2 + e] = acc;
}

template <typename T, bool CP>
__global__ void __launch_bounds__(256) k_vjk(const c2<T>* __restrict__ W, const c2<T>* __restrict__ lam,
                                             const c2<T>* __restrict__ U2, const c2<T>* __restrict__ U3,
                                             c2<T>* __restrict__ V, int n2, int n3, int r1, int r2, int r3)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n3 * n2 * r1) return;
    const int a = (int)(e % r1);
    const long jk = e / r1;
    const int j = (int)(jk % n2), k = (int)(jk / n2);
    c2<T> v = mk<T>(0, 0);
    if constexpr (CP) {
        v = lam[a] * (U2[(long)j * r2 + a] * U3[(long)k * r3 + a]);
    } else {
        const c2<T>* w = W + ((long)k * r1 + a) * r2;
        const c2<T>* u = U2 + (long)j * r2;
        for (int b = 0; b < r2; ++b) fma_c(v, w[b], u[b]);
    }
    V[e] = v;
}

// U1 (n1 x r1) into U1T (r1 x n1), so that the apply kernel's lanes read
// consecutive i of one column
template <typename T>
__global__ void __launch_bounds__(256) k_transpose(const c2<T>* __restrict__ U1, c2<T>* __restrict__ U1T, int n1,
                                                   int r1)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n1 * r1) return;
    const int a = (int)(e / n1), i = (int)(e - (long)a * n1);
    U1T[e] = U1[(long)i * r1 + a];
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_apply(const c2<T>* __restrict__ V, const c2<T>* __restrict__ U1T,
                                               const c2<T>* __restrict__ x, c2<T>* __restrict__ y, int n1,
                                               int n2, int n3, int r1)
{
    const long p = (long)blockIdx.x * kNT + threadIdx.x;
    const long plane = (long)n1 * n2;
    if (p >= plane) return;
    const int i = (int)(p % n1), j = (int)(p / n1);
    c2<T> u[kRMax];
#pragma unroll
    for (int a = 0; a < kRMax; ++a) u[a] = a < r1 ? U1T[(long)a * n1 + i] : mk<T>(0, 0);
    const int k0 = blockIdx.y * kKT;
    const int kend = min(kKT, n3 - k0);
    for (int kk = 0; kk < kend; ++kk) {
        const int k = k0 + kk;
        const c2<T>* v = V + ((long)k * n2 + j) * r1;
        c2<T> d = mk<T>(0, 0);
#pragma unroll
        for (int a = 0; a < kRMax; ++a)
            if (a < r1) fma_c(d, u[a], v[a]);
        const long o = (long)k * plane + p;
        y[o] = d * x[o];
    }
}

template <typename T>
hipError_t run(const int n[3], const int r[3], int cp, const void* core, const void* u1, const void* u2,
               const void* u3, const void* x, void* y, void* ws, hipStream_t s)
{
    const c2<T>* G = (const c2<T>*)core;
    c2<T>* U1T = (c2<T>*)ws;
    c2<T>* W = U1T + (size_t)n[0] * r[0];
    c2<T>* V = W + (cp ? 0 : (size_t)n[2] * r[0] * r[1]);
    hipLaunchKernelGGL((k_transpose<T>), dim3((unsigned)(((long)n[0] * r[0] + 255) / 256)), dim3(256), 0, s,
                       (const c2<T>*)u1, U1T, n[0], r[0]);
    const long nv = (long)n[2] * n[1] * r[0];
    const dim3 gv((unsigned)((nv + 255) / 256));
    if (cp) {
        hipLaunchKernelGGL((k_vjk<T, true>), gv, dim3(256), 0, s, nullptr, G, (const c2<T>*)u2, (const c2<T>*)u3, V,
                           n[1], n[2], r[0], r[1], r[2]);
    } else {
        dim3 gz((r[0] * r[1] + 255) / 256, n[2]);
        hipLaunchKernelGGL((k_core_z<T>), gz, dim3(256), 0, s, G, (const c2<T>*)u3, r[0], r[1], r[2], W);
        hipLaunchKernelGGL((k_vjk<T, false>), gv, dim3(256), 0, s, (const c2<T>*)W, nullptr, (const c2<T>*)u2,
                           (const c2<T>*)u3, V, n[1], n[2], r[0], r[1], r[2]);
    }
    const long plane = (long)n[0] * n[1];
    dim3 grid((unsigned)((plane + kNT - 1) / kNT), (n[2] + kKT - 1) / kKT);
    hipLaunchKernelGGL((k_apply<T>), grid, dim3(kNT), 0, s, (const c2<T>*)V, (const c2<T>*)U1T, (const c2<T>*)x,
                       (c2<T>*)y, n[0], n[1], n[2], r[0]);
    return hipGetLastError();
}

}  // namespace

extern "C" {

size_t vie_tucker_hadamard_ws_bytes(const int n[3], const int r[3], int cp, int dtype)
{
    if (!n || !r) return 0;
    const size_t el = dtype == VIE_C128 ? 16 : 8;
    return ((size_t)n[0] * r[0] + (cp ? 0 : (size_t)n[2] * r[0] * r[1]) + (size_t)n[2] * n[1] * r[0]) * el;
}

vie_status vie_tucker_hadamard(const int n[3], const int r[3], int cp, int dtype, const void* core, const void* u1,
                               const void* u2, const void* u3, const void* x, void* y, void* ws, size_t ws_bytes,
                               void* stream)
{
    using namespace vie;
    if (!n || !r || !core || !u1 || !u2 || !u3 || !x || !y)
        return fail(VIE_E_ARG, "vie_tucker_hadamard: null argument");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_tucker_hadamard: bad dtype");
    if (cp != 0 && cp != 1) return fail(VIE_E_ARG, "vie_tucker_hadamard: cp must be 0 or 1");
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 1 || n[a] > 65535) return fail(VIE_E_ARG, "vie_tucker_hadamard: n_i must be in [1, 65535]");
        if (r[a] < 1 || r[a] > kRMax) return fail(VIE_E_UNSUPPORTED, "vie_tucker_hadamard: ranks must be in [1, 32]");
    }
    if (cp && (r[1] != r[0] || r[2] != r[0]))
        return fail(VIE_E_ARG, "vie_tucker_hadamard: a CP form has r1 = r2 = r3");
    const size_t need = vie_tucker_hadamard_ws_bytes(n, r, cp, dtype);
    if (!ws || ws_bytes < need) return fail(VIE_E_ARG, "vie_tucker_hadamard: workspace too small");
    const size_t el = dtype == VIE_C128 ? 16 : 8;
    const size_t vb = (size_t)n[0] * n[1] * n[2] * el;
    const char* xb = (const char*)x;
    const char* yb = (const char*)y;
    if (xb != yb && !(xb + vb <= yb || yb + vb <= xb))
        return fail(VIE_E_ARG, "vie_tucker_hadamard: x and y overlap without being equal");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == VIE_C128 ? run<double>(n, r, cp, core, u1, u2, u3, x, y, ws, s)
                                     : run<float>(n, r, cp, core, u1, u2, u3, x, y, ws, s);
    if (e != hipSuccess) return hip_fail(e, "vie_tucker_hadamard launch");
    return VIE_OK;
}

}  // extern "C"
