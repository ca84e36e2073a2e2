// Register-resident Stockham FFT for power-of-two lengths, radix 8/4/2.
//
// A pencil of length L is spread over TPP = L / E threads, E elements per
// thread.  In a stage of radix R (plan RADS, applied left to right) thread t
// owns butterflies j = t + TPP u, u < E / R; butterfly j reads
// x[j + r L/R], r < R, twiddles input r by w^(r k L / (Ns R)) with
// k = j mod Ns, Ns = product of the earlier radices, does a length-R DFT and
// writes y[(j / Ns) Ns R + k + r Ns].  Between stages the values go through
// LDS (one pencil slice of L elements, padded by one element every eight to
// spread the strided writes over the banks); the first stage reads the
// caller's registers and the last stage leaves its outputs in registers:
//
//   input  layout  v[u R0 + r]  = x[t + TPP u + r L/R0]        (R0 = first radix)
//   output layout  v[u Rl + r]  = X[t + TPP u + r L/Rl]        (Rl = last radix)
//
// The inverse plan is the forward plan reversed, so a forward transform's
// output layout is exactly the input layout of the inverse transform and the
// Fourier-domain product in between needs no data movement.
//
// Twiddles come from a per-plan LDS table laid out stage by stage (TwTable):
// the stage with Ns > 1 owns (R - 1) Ns entries, entry (r - 1) Ns + k =
// w^(r k L / (Ns R)), so the lanes of a wavefront read consecutive entries
// (or broadcast one), never several entries of one bank.
#pragma once
#include "dev_common.h"
#include "fft_device.h"

namespace vie {

template <int... R>
struct RadixList {
    static constexpr int n = sizeof...(R);
    static constexpr int v[sizeof...(R)] = {R...};
};

__device__ __forceinline__ int lds_pad(int a) { return a + (a >> 3); }

// Make LDS writes of this wavefront visible to its other lanes (a pencil
// whose threads all sit in one wavefront needs no block-wide barrier).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool WAVE>
__device__ __forceinline__ void stage_sync()
{
    if constexpr (WAVE) wave_sync();
    else __syncthreads();
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_reg(c2<T>* a)
{
    dftR<R, DIR>(a);
}

// One stage applied to the thread's registers.
template <int L, int TPP, int R, int NS, int DIR, typename T>
__device__ __forceinline__ void reg_stage(c2<T>* v, int t, const c2<T>* __restrict__ tw)
{
    constexpr int E = L / TPP;
    constexpr int NB = E / R;
    static_assert(E % R == 0, "radix must divide the elements per thread");
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        if constexpr (NS > 1) {
            const int j = t + TPP * u;
            const int k = j % NS;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                c2<T> w = tw[(r - 1) * NS + k];
                v[u * R + r] = (DIR < 0) ? v[u * R + r] * w : mulc(v[u * R + r], w);
            }
        }
        dft_reg<R, DIR>(v + u * R);
    }
}

// Write the outputs of a stage (radix R, Ns = NS) to LDS.
template <int L, int TPP, int R, int NS, typename T>
__device__ __forceinline__ void reg_store(const c2<T>* v, c2<T>* lds, int t)
{
    constexpr int E = L / TPP;
    constexpr int NB = E / R;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j = t + TPP * u;
        const int k = j % NS;
        const int idx = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lds_pad(idx + r * NS)] = v[u * R + r];
    }
}

// Read the inputs of a stage of radix R from LDS.
template <int L, int TPP, int R, typename T>
__device__ __forceinline__ void reg_load(c2<T>* v, const c2<T>* lds, int t)
{
    constexpr int E = L / TPP;
    constexpr int NB = E / R;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j = t + TPP * u;
#pragma unroll
        for (int r = 0; r < R; ++r) v[u * R + r] = lds[lds_pad(j + r * (L / R))];
    }
}

template <int... R>
struct Prod;
template <>
struct Prod<> {
    static constexpr int value = 1;
};
template <int R0, int... Rs>
struct Prod<R0, Rs...> {
    static constexpr int value = R0 * Prod<Rs...>::value;
};

// Recursive stage driver.  NS = product of the radices already applied.
// NSEQ pencils are transformed together (thread registers v[s*E ...] and LDS
// slices lds + s * stride); the barriers are shared.
template <int L, int TPP, int NSEQ, int DIR, int NS, bool WAVE, typename T, int R0, int... Rs>
struct RegFFTImpl {
    __device__ __forceinline__ static void run(c2<T>* v, c2<T>* lds, int stride, int t, const c2<T>* tw)
    {
        constexpr int E = L / TPP;
#pragma unroll
        for (int s = 0; s < NSEQ; ++s) reg_stage<L, TPP, R0, NS, DIR>(v + s * E, t, tw);
        if constexpr (sizeof...(Rs) > 0) {
            constexpr int RN = RadixList<Rs...>::v[0];
#pragma unroll
            for (int s = 0; s < NSEQ; ++s) reg_store<L, TPP, R0, NS>(v + s * E, lds + s * stride, t);
            stage_sync<WAVE>();
#pragma unroll
            for (int s = 0; s < NSEQ; ++s) reg_load<L, TPP, RN>(v + s * E, lds + s * stride, t);
            stage_sync<WAVE>();
            constexpr int OWN = NS > 1 ? (R0 - 1) * NS : 0;   // this stage's twiddle entries
            RegFFTImpl<L, TPP, NSEQ, DIR, NS * R0, WAVE, T, Rs...>::run(v, lds, stride, t, tw + OWN);
        }
    }
};

// WAVE: every pencil's TPP threads lie in one wavefront (TPP divides 64 and
// pencils are aligned to it), so the inter-stage transposes only need
// wavefront-level ordering.
template <int L, int TPP, int NSEQ, int DIR, typename T, int... Rs>
__device__ __forceinline__ void reg_fft(c2<T>* v, c2<T>* lds, int stride, int t, const c2<T>* tw)
{
    static_assert(Prod<Rs...>::value == L, "plan does not multiply to L");
    constexpr bool WAVE = (TPP <= 64) && (64 % TPP == 0);
    RegFFTImpl<L, TPP, NSEQ, DIR, 1, WAVE, T, Rs...>::run(v, lds, stride, t, tw);
}

// Stage-ordered twiddle table of a plan (radices Rs applied left to right,
// NS = product of the radices before them).
template <int L, int NS, int... Rs>
struct TwTable {
    static constexpr int size = 0;
    template <typename T>
    __device__ static void fill(c2<T>*, const c2<T>*, int, int)
    {
    }
};
template <int L, int NS, int R0, int... Rs>
struct TwTable<L, NS, R0, Rs...> {
    static constexpr int own = NS > 1 ? (R0 - 1) * NS : 0;
    static constexpr int size = own + TwTable<L, NS * R0, Rs...>::size;
    // tw: w^m, m < L, w = exp(-2 pi i / L)
    template <typename T>
    __device__ static void fill(c2<T>* dst, const c2<T>* __restrict__ tw, int tid, int nt)
    {
        for (int e = tid; e < own; e += nt) {
            const int r = e / NS + 1, k = e - (r - 1) * NS;
            dst[e] = tw[r * k * (L / (NS * R0))];
        }
        TwTable<L, NS * R0, Rs...>::fill(dst + own, tw, tid, nt);
    }
};

// LDS slice length (elements) for one pencil including the padding
template <int L>
struct PadLen {
    static constexpr int value = L + L / 8;
};

}  // namespace vie
