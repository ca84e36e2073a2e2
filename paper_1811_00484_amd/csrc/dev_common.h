// Device-side complex arithmetic and small helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace vie {

// Radix plan of one FFT length: L = rad[0] * rad[1] * ... * rad[nst-1].
struct FftPlan {
    int L;
    int nst;
    int rad[12];
};

template <typename T>
struct alignas(2 * sizeof(T)) c2 {
    T x, y;
};

template <typename T>
__device__ __forceinline__ c2<T> mk(T a, T b)
{
    c2<T> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename T>
__device__ __forceinline__ c2<T> operator+(c2<T> a, c2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ c2<T> operator-(c2<T> a, c2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ c2<T> operator*(c2<T> a, c2<T> b)
{
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ c2<T> operator*(T s, c2<T> a) { return mk<T>(s * a.x, s * a.y); }
template <typename T>
__device__ __forceinline__ c2<T> conj(c2<T> a) { return mk<T>(a.x, -a.y); }
// a * conj(b)
template <typename T>
__device__ __forceinline__ c2<T> mulc(c2<T> a, c2<T> b)
{
    return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// acc += a * b
template <typename T>
__device__ __forceinline__ void fma_c(c2<T>& acc, c2<T> a, c2<T> b)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}
// multiply by dir * i  (dir = +1 or -1)
template <int DIR, typename T>
__device__ __forceinline__ c2<T> mul_i(c2<T> a)
{
    return DIR > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

template <typename TO, typename TI>
__device__ __forceinline__ c2<TO> cvt(c2<TI> a)
{
    return mk<TO>((TO)a.x, (TO)a.y);
}

}  // namespace vie
