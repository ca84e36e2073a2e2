// Mixed-radix Stockham FFT stages on LDS for batches of sequences.
//
// A sequence of length L lives in LDS with element m of sequence s at
// buf[s*ss + m*es].  Each stage of radix R computes L/R butterflies per
// sequence; butterfly j (sub-transform position k = j mod Ns, Ns = product
// of the previous radices) reads x[j + r L/R], applies the twiddles
// w^(r k / (Ns R)), does a length-R DFT and writes y[(j/Ns) Ns R + k + r Ns]
// (Stockham autosort: natural order in, natural order out, no bit
// reversal).  All butterflies of a stage are read into registers before a
// barrier and written back after it, so the transform is in place.
//
// Direction DIR = -1 is the forward transform exp(-2 pi i m k / L), DIR = +1
// the unnormalised inverse.  The twiddle table holds exp(-2 pi i m / L),
// m < L, computed on the host in FP64.
#pragma once
#include "dev_common.h"

namespace vie {

template <int DIR, typename T>
__device__ __forceinline__ void dft2(c2<T>* a)
{
    c2<T> t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4v(c2<T>& a0, c2<T>& a1, c2<T>& a2, c2<T>& a3)
{
    c2<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_i<DIR>(a1 - a3);
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + t3;
    a3 = t1 - t3;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(c2<T>* a)
{
    dft4v<DIR>(a[0], a[1], a[2], a[3]);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft8(c2<T>* a)
{
    c2<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    c2<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
    dft4v<DIR>(e0, e1, e2, e3);
    dft4v<DIR>(o0, o1, o2, o3);
    const T h = (T)0.70710678118654752440;
    // o1 *= (1 + DIR i)/sqrt2, o2 *= DIR i, o3 *= (-1 + DIR i)/sqrt2
    c2<T> w1 = mk<T>(h * (o1.x - (T)DIR * o1.y), h * (o1.y + (T)DIR * o1.x));
    c2<T> w2 = mul_i<DIR>(o2);
    c2<T> w3 = mk<T>(h * (-o3.x - (T)DIR * o3.y), h * (-o3.y + (T)DIR * o3.x));
    a[0] = e0 + o0;
    a[4] = e0 - o0;
    a[1] = e1 + w1;
    a[5] = e1 - w1;
    a[2] = e2 + w2;
    a[6] = e2 - w2;
    a[3] = e3 + w3;
    a[7] = e3 - w3;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft3(c2<T>* a)
{
    const T c = (T)0.86602540378443864676;   // sqrt(3)/2
    c2<T> s = a[1] + a[2], d = a[1] - a[2];
    c2<T> m = a[0] - (T)0.5 * s;
    c2<T> t = mul_i<DIR>((T)c * d);
    a[0] = a[0] + s;
    a[1] = m + t;
    a[2] = m - t;
}

// cos and sin of 2 pi j / R for odd R in {5, 7}
template <int R>
__device__ __forceinline__ double cosr(int j);
template <int R>
__device__ __forceinline__ double sinr(int j);
template <>
__device__ __forceinline__ double cosr<5>(int j)
{
    const double t[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410, -0.80901699437494742410,
                         0.30901699437494742410};
    return t[j];
}
template <>
__device__ __forceinline__ double sinr<5>(int j)
{
    const double t[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917, -0.58778525229247312917,
                         -0.95105651629515357212};
    return t[j];
}
template <>
__device__ __forceinline__ double cosr<7>(int j)
{
    const double t[7] = {1.0, 0.62348980185873353053, -0.22252093395631440429, -0.90096886790241912624,
                         -0.90096886790241912624, -0.22252093395631440429, 0.62348980185873353053};
    return t[j];
}
template <>
__device__ __forceinline__ double sinr<7>(int j)
{
    const double t[7] = {0.0, 0.78183148246802980871, 0.97492791218182360702, 0.43388373911755812048,
                         -0.43388373911755812048, -0.97492791218182360702, -0.78183148246802980871};
    return t[j];
}

// odd-length DFT by symmetric pairs: X_k = a0 + sum_m [(a_m + a_{R-m}) cos
// + DIR i (a_m - a_{R-m}) sin](2 pi m k / R)
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_odd(c2<T>* a)
{
    constexpr int H = (R - 1) / 2;
    c2<T> sm[H], df[H];
#pragma unroll
    for (int m = 1; m <= H; ++m) {
        sm[m - 1] = a[m] + a[R - m];
        df[m - 1] = a[m] - a[R - m];
    }
    c2<T> out[R];
    c2<T> x0 = a[0];
#pragma unroll
    for (int m = 0; m < H; ++m) x0 = x0 + sm[m];
    out[0] = x0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        c2<T> A = a[0], B = mk<T>(0, 0);
#pragma unroll
        for (int m = 1; m <= H; ++m) {
            int j = (m * k) % R;
            A = A + (T)cosr<R>(j) * sm[m - 1];
            B = B + (T)sinr<R>(j) * df[m - 1];
        }
        c2<T> iB = mul_i<DIR>(B);
        out[k] = A + iB;
        out[R - k] = A - iB;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) a[k] = out[k];
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dftR(c2<T>* a)
{
    if constexpr (R == 2) dft2<DIR>(a);
    else if constexpr (R == 3) dft3<DIR>(a);
    else if constexpr (R == 4) dft4<DIR>(a);
    else if constexpr (R == 8) dft8<DIR>(a);
    else dft_odd<R, DIR>(a);
}

template <int R, int DIR, bool SEQFAST, int MAXE, typename T>
__device__ __forceinline__ void stage_r(c2<T>* buf, int nseq, int ss, int es, int L, int Ns,
                                        const c2<T>* tw, int tid, int nthr)
{
    constexpr int MB = (MAXE + R - 1) / R;
    const int nb = L / R;
    const int total = nseq * nb;
    const int tstep = L / (Ns * R);
    c2<T> v[MB][R];
    int sv[MB], jv[MB];
#pragma unroll
    for (int u = 0; u < MB; ++u) {
        int e = tid + u * nthr;
        sv[u] = -1;
        jv[u] = 0;
        if (e < total) {
            int s, j;
            if (SEQFAST) {
                s = e % nseq;
                j = e / nseq;
            } else {
                s = e / nb;
                j = e - s * nb;
            }
            sv[u] = s;
            jv[u] = j;
            const c2<T>* p = buf + s * ss;
#pragma unroll
            for (int r = 0; r < R; ++r) v[u][r] = p[(j + r * nb) * es];
            if (Ns > 1) {
                int k = j % Ns;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    c2<T> w = tw[r * k * tstep];
                    v[u][r] = (DIR < 0) ? v[u][r] * w : mulc(v[u][r], w);
                }
            }
            dftR<R, DIR>(v[u]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MB; ++u) {
        if (sv[u] >= 0) {
            int j = jv[u];
            int k = j % Ns;
            int idx = (j / Ns) * Ns * R + k;
            c2<T>* p = buf + sv[u] * ss;
#pragma unroll
            for (int r = 0; r < R; ++r) p[(idx + r * Ns) * es] = v[u][r];
        }
    }
    __syncthreads();
}

// Full transform of `nseq` sequences; requires nseq * L <= MAXE * nthr.
template <int DIR, bool SEQFAST, int MAXE, typename T>
__device__ void fft_lds(c2<T>* buf, int nseq, int ss, int es, const FftPlan& pl, const c2<T>* tw,
                        int tid, int nthr)
{
    int Ns = 1;
    for (int st = 0; st < pl.nst; ++st) {
        int R = pl.rad[st];
        switch (R) {
        case 8: stage_r<8, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, pl.L, Ns, tw, tid, nthr); break;
        case 4: stage_r<4, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, pl.L, Ns, tw, tid, nthr); break;
        case 2: stage_r<2, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, pl.L, Ns, tw, tid, nthr); break;
        case 3: stage_r<3, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, pl.L, Ns, tw, tid, nthr); break;
        case 5: stage_r<5, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, pl.L, Ns, tw, tid, nthr); break;
        case 7: stage_r<7, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, pl.L, Ns, tw, tid, nthr); break;
        default: break;
        }
        Ns *= R;
    }
}


// fft_lds with the radix sequence fixed at compile time for the lengths
// below (the stage index arithmetic then divides by constants); any other
// LC (0) takes the plan at run time.
template <int DIR, bool SEQFAST, int MAXE, int LC, typename T>
__device__ __forceinline__ void fft_lds_len(c2<T>* buf, int nseq, int ss, int es, const FftPlan& pl, const c2<T>* tw,
                                            int tid, int nthr)
{
    if constexpr (LC == 512) {
        stage_r<8, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 1, tw, tid, nthr);
        stage_r<8, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 8, tw, tid, nthr);
        stage_r<8, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 64, tw, tid, nthr);
    } else if constexpr (LC == 256) {
        stage_r<8, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 1, tw, tid, nthr);
        stage_r<8, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 8, tw, tid, nthr);
        stage_r<4, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 64, tw, tid, nthr);
    } else if constexpr (LC == 128) {
        stage_r<8, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 1, tw, tid, nthr);
        stage_r<4, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 8, tw, tid, nthr);
        stage_r<4, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 32, tw, tid, nthr);
    } else if constexpr (LC == 64) {
        stage_r<8, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 1, tw, tid, nthr);
        stage_r<8, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 8, tw, tid, nthr);
    } else if constexpr (LC == 300) {
        stage_r<5, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 1, tw, tid, nthr);
        stage_r<5, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 5, tw, tid, nthr);
        stage_r<4, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 25, tw, tid, nthr);
        stage_r<3, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 100, tw, tid, nthr);
    } else if constexpr (LC == 240) {
        stage_r<8, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 1, tw, tid, nthr);
        stage_r<5, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 8, tw, tid, nthr);
        stage_r<3, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 40, tw, tid, nthr);
        stage_r<2, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 120, tw, tid, nthr);
    } else if constexpr (LC == 180) {
        stage_r<5, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 1, tw, tid, nthr);
        stage_r<4, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 5, tw, tid, nthr);
        stage_r<3, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 20, tw, tid, nthr);
        stage_r<3, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 60, tw, tid, nthr);
    } else if constexpr (LC == 120) {
        stage_r<8, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 1, tw, tid, nthr);
        stage_r<5, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 8, tw, tid, nthr);
        stage_r<3, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 40, tw, tid, nthr);
    } else if constexpr (LC == 60) {
        stage_r<5, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 1, tw, tid, nthr);
        stage_r<4, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 5, tw, tid, nthr);
        stage_r<3, DIR, SEQFAST, MAXE>(buf, nseq, ss, es, LC, 20, tw, tid, nthr);
    } else {
        fft_lds<DIR, SEQFAST, MAXE>(buf, nseq, ss, es, pl, tw, tid, nthr);
    }
}

}  // namespace vie
