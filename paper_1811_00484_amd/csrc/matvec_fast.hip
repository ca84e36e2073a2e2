// Register-FFT kernels of the five matvec passes for the FFT lengths of the
// workloads that matter for throughput: 128, 256, 512 (radix 8/4) on every
// axis, and 192, 224 (radix 8/4/3, 7/4/2) for the x and y passes.  Same data layouts and results as the generic LDS-staged
// kernels in matvec.hip (which remain the path for lengths with factors 3,
// 5, 7), but each thread keeps its pencil elements in registers across the
// radix-8/4 stages (reg_fft.h) and LDS only carries the transposes between
// stages.
//
// X/Y passes: a block owns W pencils of one tile; global rows are staged
// through per-pencil LDS slices (stride PL = L + L/8 + 1 complex, odd so
// that both row-wise and pencil-wise walks are free of bank conflicts).
//
// Z pass: a block owns one canonical k2 (and its mirror L2 - k2) and a
// chunk of k1 quads.  W_c(k2) = G_c x2 U2_c(k2, :) is built once per block;
// per quad V_c = U1_c(k1, :) W_c and N^_c(k1, k2, k3) = sum_g V_c[g]
// U3_c(k3, g) for k3 in [0, n3] go to LDS, and each thread transforms the
// three components of its pencil in registers, so the 3 x 3 component
// product is thread-local.
#include <hip/hip_runtime.h>

#include "reg_fft.h"
#include "vie_internal.h"

// Extra complex elements at the end of every per-pencil LDS slice: the
// slice stride sets the bank offset between the pencils of a transposed
// row access.
#ifndef VIE_SLICE_EXTRA
#define VIE_SLICE_EXTRA 1
#endif

namespace vie {

// ---------------------------------------------------------------------------
// plans: forward plan and its reverse for the inverse
template <int L>
struct RegPlan;
template <>
struct RegPlan<512> {
    using TwF = TwTable<512, 1, 8, 8, 8>;
    using TwI = TwTable<512, 1, 8, 8, 8>;
    static constexpr int TWI = 0;
    static constexpr int TW = TWI + TwI::size;   // twiddle-table entries in LDS
    template <typename T>
    __device__ static void fill_tw(c2<T>* dst, const c2<T>* tw, int tid, int nt)
    {
        TwF::fill(dst, tw, tid, nt);
        
    }
    template <typename T, int TPP, int NSEQ, int DIR>
    __device__ static void fwd(c2<T>* v, c2<T>* lds, int st, int t, const c2<T>* tws)
    {
        reg_fft<512, TPP, NSEQ, DIR, T, 8, 8, 8>(v, lds, st, t, tws);
    }
    template <typename T, int TPP, int NSEQ, int DIR>
    __device__ static void inv(c2<T>* v, c2<T>* lds, int st, int t, const c2<T>* tws)
    {
        reg_fft<512, TPP, NSEQ, DIR, T, 8, 8, 8>(v, lds, st, t, tws + TWI);
    }
    static constexpr int RF0 = 8, RFL = 8, RI0 = 8, RIL = 8;
};
template <>
struct RegPlan<256> {
    using TwF = TwTable<256, 1, 8, 8, 4>;
    using TwI = TwTable<256, 1, 4, 8, 8>;
    static constexpr int TWI = TwF::size;
    static constexpr int TW = TWI + TwI::size;   // twiddle-table entries in LDS
    template <typename T>
    __device__ static void fill_tw(c2<T>* dst, const c2<T>* tw, int tid, int nt)
    {
        TwF::fill(dst, tw, tid, nt);
        TwI::fill(dst + TWI, tw, tid, nt);
    }
    template <typename T, int TPP, int NSEQ, int DIR>
    __device__ static void fwd(c2<T>* v, c2<T>* lds, int st, int t, const c2<T>* tws)
    {
        reg_fft<256, TPP, NSEQ, DIR, T, 8, 8, 4>(v, lds, st, t, tws);
    }
    template <typename T, int TPP, int NSEQ, int DIR>
    __device__ static void inv(c2<T>* v, c2<T>* lds, int st, int t, const c2<T>* tws)
    {
        reg_fft<256, TPP, NSEQ, DIR, T, 4, 8, 8>(v, lds, st, t, tws + TWI);
    }
    static constexpr int RF0 = 8, RFL = 4, RI0 = 4, RIL = 8;
};
template <>
struct RegPlan<128> {
    using TwF = TwTable<128, 1, 8, 4, 4>;
    using TwI = TwTable<128, 1, 4, 4, 8>;
    static constexpr int TWI = TwF::size;
    static constexpr int TW = TWI + TwI::size;   // twiddle-table entries in LDS
    template <typename T>
    __device__ static void fill_tw(c2<T>* dst, const c2<T>* tw, int tid, int nt)
    {
        TwF::fill(dst, tw, tid, nt);
        TwI::fill(dst + TWI, tw, tid, nt);
    }
    template <typename T, int TPP, int NSEQ, int DIR>
    __device__ static void fwd(c2<T>* v, c2<T>* lds, int st, int t, const c2<T>* tws)
    {
        reg_fft<128, TPP, NSEQ, DIR, T, 8, 4, 4>(v, lds, st, t, tws);
    }
    template <typename T, int TPP, int NSEQ, int DIR>
    __device__ static void inv(c2<T>* v, c2<T>* lds, int st, int t, const c2<T>* tws)
    {
        reg_fft<128, TPP, NSEQ, DIR, T, 4, 4, 8>(v, lds, st, t, tws + TWI);
    }
    static constexpr int RF0 = 8, RFL = 4, RI0 = 4, RIL = 8;
};
template <>
struct RegPlan<64> {
    using TwF = TwTable<64, 1, 8, 8>;
    using TwI = TwTable<64, 1, 8, 8>;
    static constexpr int TWI = 0;
    static constexpr int TW = TWI + TwI::size;   // twiddle-table entries in LDS
    template <typename T>
    __device__ static void fill_tw(c2<T>* dst, const c2<T>* tw, int tid, int nt)
    {
        TwF::fill(dst, tw, tid, nt);
        
    }
    template <typename T, int TPP, int NSEQ, int DIR>
    __device__ static void fwd(c2<T>* v, c2<T>* lds, int st, int t, const c2<T>* tws)
    {
        reg_fft<64, TPP, NSEQ, DIR, T, 8, 8>(v, lds, st, t, tws);
    }
    template <typename T, int TPP, int NSEQ, int DIR>
    __device__ static void inv(c2<T>* v, c2<T>* lds, int st, int t, const c2<T>* tws)
    {
        reg_fft<64, TPP, NSEQ, DIR, T, 8, 8>(v, lds, st, t, tws + TWI);
    }
    static constexpr int RF0 = 8, RFL = 8, RI0 = 8, RIL = 8;
};

template <>
struct RegPlan<192> {
    using TwF = TwTable<192, 1, 8, 8, 3>;
    using TwI = TwTable<192, 1, 3, 8, 8>;
    static constexpr int TWI = TwF::size;
    static constexpr int TW = TWI + TwI::size;   // twiddle-table entries in LDS
    template <typename T>
    __device__ static void fill_tw(c2<T>* dst, const c2<T>* tw, int tid, int nt)
    {
        TwF::fill(dst, tw, tid, nt);
        TwI::fill(dst + TWI, tw, tid, nt);
    }
    template <typename T, int TPP, int NSEQ, int DIR>
    __device__ static void fwd(c2<T>* v, c2<T>* lds, int st, int t, const c2<T>* tws)
    {
        reg_fft<192, TPP, NSEQ, DIR, T, 8, 8, 3>(v, lds, st, t, tws);
    }
    template <typename T, int TPP, int NSEQ, int DIR>
    __device__ static void inv(c2<T>* v, c2<T>* lds, int st, int t, const c2<T>* tws)
    {
        reg_fft<192, TPP, NSEQ, DIR, T, 3, 8, 8>(v, lds, st, t, tws + TWI);
    }
    static constexpr int RF0 = 8, RFL = 3, RI0 = 3, RIL = 8;
};
template <>
struct RegPlan<224> {
    using TwF = TwTable<224, 1, 7, 4, 4, 2>;
    using TwI = TwTable<224, 1, 2, 4, 4, 7>;
    static constexpr int TWI = TwF::size;
    static constexpr int TW = TWI + TwI::size;   // twiddle-table entries in LDS
    template <typename T>
    __device__ static void fill_tw(c2<T>* dst, const c2<T>* tw, int tid, int nt)
    {
        TwF::fill(dst, tw, tid, nt);
        TwI::fill(dst + TWI, tw, tid, nt);
    }
    template <typename T, int TPP, int NSEQ, int DIR>
    __device__ static void fwd(c2<T>* v, c2<T>* lds, int st, int t, const c2<T>* tws)
    {
        reg_fft<224, TPP, NSEQ, DIR, T, 7, 4, 4, 2>(v, lds, st, t, tws);
    }
    template <typename T, int TPP, int NSEQ, int DIR>
    __device__ static void inv(c2<T>* v, c2<T>* lds, int st, int t, const c2<T>* tws)
    {
        reg_fft<224, TPP, NSEQ, DIR, T, 2, 4, 4, 7>(v, lds, st, t, tws + TWI);
    }
    static constexpr int RF0 = 7, RFL = 2, RI0 = 2, RIL = 7;
};

template <int L>
struct PL {
    static constexpr int value = L + L / 8 + VIE_SLICE_EXTRA;
};

// ---------------------------------------------------------------------------
// X/Y passes.  KIND: 0 = X+, 1 = Y+, 2 = Y-, 3 = X-.
// One workgroup of an X/Y pass: pencil tile tx, row, component q, compact
// right-hand side bl (mapped through rhs_map).  IDENT replaces the transform
// by the identity (every element stays at its position), leaving the pass's
// index maps (padding, transposes, cropping, epilogue): the debug entry
// points check those bit for bit.
template <typename TV, typename T, int L, int E, int W, int KIND, bool IDENT = false>
__device__ __forceinline__ void xy_body(const void* __restrict__ in_, void* __restrict__ out_,
                                        const c2<TV>* __restrict__ x, const c2<TV>* __restrict__ eps,
                                        const c2<T>* __restrict__ tw, const XYArgs& a,
                                        const int* __restrict__ rhs_map, int tx, int row, int q, int bl)
{
    constexpr int TPP = L / E;
    constexpr int NT = W * TPP;
    constexpr int P = PL<L>::value;
    using Plan = RegPlan<L>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T>* buf = reinterpret_cast<c2<T>*>(smem_raw);           // [W][P]
    c2<T>* tws = buf + (size_t)W * P;                           // [Plan::TW]
    const int tid = threadIdx.x;
    Plan::fill_tw(tws, tw, tid, NT);

    const int n1 = a.n1, n2 = a.n2, n3 = a.n3, L1 = a.L1, L2 = a.L2;
    const long bqc = (long)bl * 3 + q;                           // compact (workspace) index
    const int b = rhs_map ? rhs_map[bl] : bl;
    const long bqv = (long)b * 3 + q;                           // vector index
    const int p0 = tx * W;                                      // first pencil of the tile
    // number of valid pencils in the tile and the transform's input length
    int npen, nin;
    if (KIND == 0) { npen = n2; nin = n1; }
    else if (KIND == 1) { npen = n3; nin = n2; }
    else if (KIND == 2) { npen = n3; nin = L2; }
    else { npen = n2; nin = L1; }

    const int w = tid / TPP, t = tid % TPP;
    const int pw = p0 + w;                                      // my pencil
    c2<T>* slice = buf + w * P;
    c2<T> v[E];

    if (KIND == 0 || KIND == 1) {
        // ---- rows contiguous per pencil: straight into the registers of
        //      the first stage (zero padding beyond nin)
        constexpr int R0 = Plan::RF0;
#pragma unroll
        for (int u = 0; u < E / R0; ++u)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int pos = t + TPP * u + r * (L / R0);
                c2<T> val = mk<T>(0, 0);
                if (pw < npen && pos < nin) {
                    if (KIND == 0) {
                        long idx = ((bqv * n3 + row) * n2 + pw) * n1 + pos;
                        val = cvt<T>(x[idx]);
                        if (a.mode == MODE_AH) {
                            c2<T> ep = cvt<T>(eps[((long)row * n2 + pw) * n1 + pos]);
                            val = mk<T>(ep.x - (T)1, -ep.y) * val;
                        }
                    } else {
                        const c2<T>* S1 = reinterpret_cast<const c2<T>*>(in_);
                        val = S1[((bqc * n3 + pw) * L1 + row) * n2 + pos];
                    }
                }
                v[u * R0 + r] = val;
            }
        __syncthreads();   // twiddle table complete (the FFT stages sync per wavefront only)
        if constexpr (IDENT) {
            constexpr int R0I = Plan::RF0;
#pragma unroll
            for (int u = 0; u < E / R0I; ++u)
#pragma unroll
                for (int r = 0; r < R0I; ++r) slice[lds_pad(t + TPP * u + r * (L / R0I))] = v[u * R0I + r];
        } else {
            Plan::template fwd<T, TPP, 1, -1>(v, slice, 0, t, tws);
            reg_store<L, TPP, Plan::RFL, L / Plan::RFL>(v, slice, t);
        }
        __syncthreads();
        // ---- transposed output [m][p0 + w], all L frequencies
        c2<T>* S = reinterpret_cast<c2<T>*>(out_);
        for (int e = tid; e < W * L; e += NT) {
            int ww = e % W, m = e / W;
            int p = p0 + ww;
            if (p >= npen) continue;
            c2<T> val = buf[ww * P + lds_pad(m)];
            if (KIND == 0) S[((bqc * n3 + row) * L1 + m) * n2 + p] = val;
            else S[((bqc * L2 + m) * L1 + row) * n3 + p] = val;
        }
    } else {
        // ---- X- epilogue operands (u, eps_c at the kept rows) are loaded
        //      together with the transposed input, so their latency is hidden
        //      behind the FFT (complex64: the LDS already limits the kernel to
        //      two workgroups per CU, so the registers are free)
        constexpr int RL = Plan::RIL;
        constexpr int RH = (RL + 1) / 2;                        // rows m < L/2 sit in r < RH
        constexpr bool PRE = KIND == 3 && sizeof(TV) == 4 && sizeof(T) == 4;
        constexpr int NPRE = PRE ? (E / RL) * RH : 1;
        const int nout = KIND == 2 ? n2 : n1;
        const bool contrast = a.mode == MODE_A || a.mode == MODE_AH;
        c2<TV> xpre[NPRE], epre[NPRE];
        // ---- transposed input: element m of pencil ww at [m][p0 + ww];
        //      all E loads of a thread are issued before the LDS writes
        {
            c2<T> tmp[E];
            const c2<T>* S = reinterpret_cast<const c2<T>*>(in_);
#pragma unroll
            for (int u = 0; u < E; ++u) {
                const int e = tid + u * NT;
                const int ww = e % W, m = e / W;
                const int p = p0 + ww;
                c2<T> val = mk<T>(0, 0);
                if (p < npen) {
                    if (KIND == 2) val = S[((bqc * L2 + m) * L1 + row) * n3 + p];
                    else val = S[((bqc * n3 + row) * L1 + m) * n2 + p];
                }
                tmp[u] = val;
            }
            if constexpr (PRE) {
                if (contrast && pw < npen) {
#pragma unroll
                    for (int u = 0; u < E / RL; ++u)
#pragma unroll
                        for (int r = 0; r < RH; ++r) {
                            const int m = t + TPP * u + r * (L / RL);
                            if (m < nout) {
                                xpre[u * RH + r] = x[((bqv * n3 + row) * n2 + pw) * n1 + m];
                                epre[u * RH + r] = eps[((long)row * n2 + pw) * n1 + m];
                            }
                        }
                }
            }
#pragma unroll
            for (int u = 0; u < E; ++u) {
                const int e = tid + u * NT;
                buf[(e % W) * P + lds_pad(e / W)] = tmp[u];
            }
        }
        __syncthreads();
        if constexpr (IDENT) {
#pragma unroll
            for (int u = 0; u < E / RL; ++u)
#pragma unroll
                for (int r = 0; r < RL; ++r) v[u * RL + r] = slice[lds_pad(t + TPP * u + r * (L / RL))];
        } else {
            reg_load<L, TPP, Plan::RI0>(v, slice, t);
            wave_sync();   // the slice is only rewritten by the lanes of this pencil's wavefront
            Plan::template inv<T, TPP, 1, 1>(v, slice, 0, t, tws);
        }
        // ---- cropped rows straight from the registers of the last stage
        if (pw < npen) {
#pragma unroll
            for (int u = 0; u < E / RL; ++u)
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    const int m = t + TPP * u + r * (L / RL);
                    if (m >= nout) continue;
                    const c2<T> rr = v[u * RL + r];
                    if (KIND == 2) {
                        c2<T>* S3 = reinterpret_cast<c2<T>*>(out_);
                        S3[((bqc * n3 + pw) * L1 + row) * n2 + m] = rr;
                    } else {
                        c2<TV>* y = reinterpret_cast<c2<TV>*>(out_);
                        long idx = ((bqv * n3 + row) * n2 + pw) * n1 + m;
                        c2<T> o;
                        if (contrast) {
                            c2<T> u0, ep;
                            if constexpr (PRE) {
                                // r < RH holds for every kept row (m < n1 = L/2)
                                u0 = cvt<T>(xpre[u * RH + (r < RH ? r : 0)]);
                                ep = cvt<T>(epre[u * RH + (r < RH ? r : 0)]);
                            } else {
                                u0 = cvt<T>(x[idx]);
                                ep = cvt<T>(eps[((long)row * n2 + pw) * n1 + m]);
                            }
                            if (a.mode == MODE_A) o = ep * u0 - mk<T>(ep.x - (T)1, ep.y) * rr;
                            else o = conj(ep) * u0 - rr;
                        } else {
                            o = rr;
                        }
                        y[idx] = cvt<TV>(o);
                    }
                }
        }
    }
}

template <typename TV, typename T, int L, int E, int W, int KIND, bool IDENT = false>
__global__ void __launch_bounds__(W*(L / E)) k_xy_fast(const void* __restrict__ in_, void* __restrict__ out_,
                                                       const c2<TV>* __restrict__ x, const c2<TV>* __restrict__ eps,
                                                       const c2<T>* __restrict__ tw, XYArgs a,
                                                       const int* __restrict__ rhs_map)
{
    int q, bl, tx, row;
    if (KIND == 3) {
        // The three components of one tile read the same eps_c rows in the
        // epilogue: give them workgroup ids g, g + 8, g + 16, which the
        // dispatcher sends (round robin over the 8 XCDs) to the same XCD one
        // after another, so two of the three reads hit its L2.
        const int lid = blockIdx.x, xcd = lid & 7, slot = lid >> 3;
        const int tile = (slot / 3) * 8 + xcd;
        const int ntx = (a.n2 + W - 1) / W;
        if (tile >= ntx * a.n3) return;
        q = slot % 3;
        bl = blockIdx.z;
        tx = tile % ntx;
        row = tile / ntx;
    } else {
        q = blockIdx.z % 3;
        bl = blockIdx.z / 3;
        tx = blockIdx.x;
        row = blockIdx.y;
    }
    xy_body<TV, T, L, E, W, KIND, IDENT>(in_, out_, x, eps, tw, a, rhs_map, tx, row, q, bl);
}

// Grouped launch over several instances with the same FFT length: workgroup
// ids are split by the instances' first-workgroup offsets (ascending); the
// descriptors are kernel arguments.
template <typename TV, typename T, int L, int E, int W, int KIND>
__global__ void __launch_bounds__(W*(L / E)) k_xy_fast_multi(const XYGroup g, const c2<T>* __restrict__ tw)
{
    int i = 0;
    while (i + 1 < g.n && (int)blockIdx.x >= g.e[i + 1].off) ++i;
    const XYInst& in = g.e[i];
    const int local = blockIdx.x - in.off;
    const int tx = local % in.ntx, t2 = local / in.ntx;
    const int row = t2 % in.rows, zq = t2 / in.rows;
    xy_body<TV, T, L, E, W, KIND>(in.in, in.out, (const c2<TV>*)in.x, (const c2<TV>*)in.eps, tw, in.a, in.map, tx,
                                  row, zq % 3, zq / 3);
}

// ---------------------------------------------------------------------------
// Z pass
template <int FAM>
__device__ __forceinline__ int zsign(int c, int f1, int f2, int f3)
{
    return ((comp_odd(FAM, c, 0) & f1) ^ (comp_odd(FAM, c, 1) & f2) ^ (comp_odd(FAM, c, 2) & f3)) ? -1 : 1;
}

// Load the three components of a pencil into the input layout of the
// forward plan (positions >= n3 are the zero padding).
template <typename T, int L3, int TPP, int R0>
__device__ __forceinline__ void z_load(c2<T> (&d)[3][8], const c2<T>* __restrict__ S2, long base, long cstride, int t,
                                       bool exists)
{
    constexpr int E = 8;
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int u = 0; u < E / R0; ++u)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int pos = t + TPP * u + r * (L3 / R0);
                d[q][u * R0 + r] = (exists && r < R0 / 2) ? S2[base + q * cstride + pos] : mk<T>(0, 0);
            }
}

// 3x3 component product in the output layout of the forward plan; FAM 1
// (K operators): antisymmetric pair, K's parities, zero diagonal
template <typename T, int L3, int TPP, int RL, bool CONJ, int FAM>
__device__ __forceinline__ void z_product(c2<T> (&d)[3][8], const c2<T>* NTt, int t, int f1, int f2)
{
    constexpr int E = 8;
    constexpr int N3 = L3 / 2;
#pragma unroll
    for (int u = 0; u < E / RL; ++u)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int m = t + TPP * u + r * (L3 / RL);
            const int f3 = m > N3;
            const int kk = f3 ? L3 - m : m;
            c2<T> Nc[6];
#pragma unroll
            for (int c = FAM ? 3 : 0; c < 6; ++c) {
                c2<T> tv = NTt[c * (N3 + 1) + kk];
                if (zsign<FAM>(c, f1, f2, f3) < 0) tv = mk<T>(-tv.x, -tv.y);
                Nc[c] = CONJ ? vie::conj(tv) : tv;
            }
            const int i = u * RL + r;
            c2<T> x0 = d[0][i], x1 = d[1][i], x2 = d[2][i];
            if constexpr (FAM == 0) {
                d[0][i] = Nc[0] * x0 + Nc[3] * x1 + Nc[4] * x2;
                d[1][i] = Nc[3] * x0 + Nc[1] * x1 + Nc[5] * x2;
                d[2][i] = Nc[4] * x0 + Nc[5] * x1 + Nc[2] * x2;
            } else {
                d[0][i] = Nc[3] * x1 + Nc[4] * x2;
                d[1][i] = Nc[5] * x2 - Nc[3] * x0;
                d[2][i] = mk<T>(0, 0) - (Nc[4] * x0 + Nc[5] * x1);
            }
        }
}

template <typename T, int L3, int TPP, int RIL>
__device__ __forceinline__ void z_store(const c2<T> (&d)[3][8], c2<T>* __restrict__ S2, long base, long cstride, int t)
{
    constexpr int E = 8;
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int u = 0; u < E / RIL; ++u)
#pragma unroll
            for (int r = 0; r < RIL / 2; ++r) S2[base + q * cstride + t + TPP * u + r * (L3 / RIL)] = d[q][u * RIL + r];
}

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// N^ tables of a quad pair from the BF16 z factors on MFMA (FP32 accumulate).
// Per component the pair's tables are the real product
//   [Re T_A, Im T_A, Re T_B, Im T_B] (rows k3) = [Re U3 | Im U3] (rows k3, 2 rh)
//     x [[Re V_A, Im V_A, Re V_B, Im V_B], [-Im V_A, Re V_A, -Im V_B, Re V_B]],
// done as 16 x 16 x 32 tiles (only the first 4 of the 16 output columns are
// used).  Each wavefront takes every NWV-th row tile; lane l holds A row
// l mod 16 and B column l mod 16 with K positions 8 (l / 16) .. +7 of each
// 32-wide step, and receives output rows 4 (l / 16) .. +3 of column l mod 16.
template <int L3>
__device__ __forceinline__ void z_tables_mfma(const OpView& v, const unsigned short* __restrict__ f3m,
                                              const c2<float>* Vc, c2<float>* tabA, c2<float>* tabB, int tid,
                                              int nt)
{
    constexpr int N3 = L3 / 2;
    constexpr int NTILE = (N3 + 1 + 15) / 16;
    const int rmax = v.rmax;
    const int lane = tid & 63, wv = tid >> 6, nwv = nt >> 6;
    const int col = lane & 15, grp = lane >> 4;
    float* fa = reinterpret_cast<float*>(tabA);
    float* fb = reinterpret_cast<float*>(tabB);
    const c2<float>* vq = Vc + ((col >> 1) & 1) * 6 * rmax;
#pragma unroll 1
    for (int c = 0; c < 6; ++c) {
        const int r3 = v.r[c][2], rh = v.rh[c];
        bf16x8 bop[2];
#pragma unroll
        for (int st = 0; st < 2; ++st)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 32 * st + 8 * grp + e;
                const bool hi = k >= rh;
                const int g = hi ? k - rh : k;
                const bool ok = (col < 4) & (k < 2 * rh) & (g < r3);
                const c2<float> w = vq[c * rmax + (ok ? g : 0)];
                const float re = hi ? -w.y : w.x, im = hi ? w.x : w.y;
                bop[st][e] = (__bf16)(ok ? ((col & 1) ? im : re) : 0.f);
            }
        const unsigned short* base = f3m + v.fac3m_off[c] + 8 * grp;
#pragma unroll 1
        for (int tile = wv; tile < NTILE; tile += nwv) {
            const unsigned short* row = base + (size_t)(tile * 16 + col) * (2 * rh);
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(row), bop[0], acc, 0, 0,
                                                          0);
            if (rh > 16)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(row + 32), bop[1],
                                                              acc, 0, 0, 0);
            if (col < 4) {
                float* dst = (col >> 1) ? fb : fa;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int kk = tile * 16 + 4 * grp + q;
                    if (kk <= N3) dst[2 * (c * (N3 + 1) + kk) + (col & 1)] = acc[q];
                }
            }
        }
    }
}

typedef __attribute__((ext_vector_type(4))) float f32x4m;

// N^ tables of a quad pair in FP32 on MFMA (v_mfma_f32_4x4x1f32: 16 blocks
// of 4 x 4 per instruction, FP32 accumulate).  Per component the pair's
// tables are the real product
//   [Re T_A; Im T_A; Re T_B; Im T_B] (4 rows x k3) = A (4 x 2 r3) B (2 r3 x k3),
// B's rows the real and imaginary parts of U3(k3, g), A's columns
// (Re V_A, Im V_A, Re V_B, Im V_B) against Re U3 and
// (-Im V_A, Re V_A, -Im V_B, Re V_B) against Im U3.  The z length fixes
// N3 / 64 = the number of wavefronts: wavefront w takes the 64 rows
// k3 = 64 w + lane of every component (block b of an instruction = rows
// 64 w + 4 b + 0..3; lane l supplies A row l mod 4 and B column l mod 4 of
// block l / 4 and receives the four rows of that column); the last row
// k3 = N3 is done on the vector ALUs by 12 threads.  Eight z-factor rows are
// loaded before their products, and four accumulators (Re / Im U3 halves,
// even / odd g) keep consecutive MFMAs independent.
template <int L3>
__device__ __forceinline__ void z_tables_mfma32(const OpView& v, const c2<float>* __restrict__ fac,
                                                const c2<float>* Vc, c2<float>* tabA, c2<float>* tabB, int tid)
{
    constexpr int N3 = L3 / 2;
    const int rmax = v.rmax;
    const int lane = tid & 63, wv = tid >> 6;
    const int k3 = 64 * wv + lane;
    const int qrow = lane & 3;
    const int qd = qrow >> 1, im = qrow & 1;
#pragma unroll 1
    for (int c = 0; c < 6; ++c) {
        const int r3 = v.r[c][2];
        const c2<float>* U3 = fac + v.fac3t_off[c] + k3;
        const c2<float>* vq = Vc + qd * 6 * rmax + c * rmax;
        f32x4m acc[4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        for (int g0 = 0; g0 < r3; g0 += 8) {
            // eight z-factor rows in flight, then their 16 products
            c2<float> uv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) uv[q] = g0 + q < r3 ? U3[(long)(g0 + q) * (N3 + 1)] : mk<float>(0, 0);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (g0 + q < r3) {
                    const c2<float> w = vq[g0 + q];
                    const float a0 = im ? w.y : w.x;     // coefficient of Re U3
                    const float a1 = im ? w.x : -w.y;    // coefficient of Im U3
                    acc[2 * (q & 1)] = __builtin_amdgcn_mfma_f32_4x4x1f32(a0, uv[q].x, acc[2 * (q & 1)], 0, 0, 0);
                    acc[2 * (q & 1) + 1] =
                        __builtin_amdgcn_mfma_f32_4x4x1f32(a1, uv[q].y, acc[2 * (q & 1) + 1], 0, 0, 0);
                }
            }
        }
        const int o = c * (N3 + 1) + k3;
        tabA[o] = mk<float>((acc[0][0] + acc[1][0]) + (acc[2][0] + acc[3][0]),
                            (acc[0][1] + acc[1][1]) + (acc[2][1] + acc[3][1]));
        tabB[o] = mk<float>((acc[0][2] + acc[1][2]) + (acc[2][2] + acc[3][2]),
                            (acc[0][3] + acc[1][3]) + (acc[2][3] + acc[3][3]));
    }
    if (tid < 12) {
        const int c = tid >> 1, q = tid & 1;
        const int r3 = v.r[c][2];
        const c2<float>* U3 = fac + v.fac3t_off[c] + N3;
        const c2<float>* vq = Vc + q * 6 * rmax + c * rmax;
        c2<float> acc = mk<float>(0, 0);
        for (int g = 0; g < r3; ++g) fma_c(acc, vq[g], U3[(long)g * (N3 + 1)]);
        (q ? tabB : tabA)[c * (N3 + 1) + N3] = acc;
    }
}

// REC: 0 = N^ tables in T on the vector ALUs, 1 = BF16 z factors on MFMA
// (T = float), 2 = a K operator (antisymmetric product, K parities; tables
// on the vector ALUs).
// One workgroup of the z pass: bx = canonical k2 + (n2 + 1) * chunk index,
// b = compact right-hand side.
template <typename T, int L3, bool CONJ, int REC>
__device__ __forceinline__ void z_body(c2<T>* __restrict__ S2, const c2<T>* __restrict__ tw, const ZFastArgs& a,
                                       const c2<T>* __restrict__ core, const c2<T>* __restrict__ fac,
                                       const c2<T>* __restrict__ dense, const unsigned short* __restrict__ f3m,
                                       int bx, int b)
{
    constexpr int TPP = L3 / 8;
    constexpr int NT = 4 * TPP;
    constexpr int P = PL<L3>::value;
    constexpr int N3 = L3 / 2;
    constexpr int NTS = 6 * (N3 + 1);                            // N^ table entries per quad
    using Plan = RegPlan<L3>;
    const OpView& v = a.v;
    const int n1 = v.n[0], n2 = v.n[1];
    const int L1 = v.L[0], L2 = v.L[1];
    const int rmax = v.rmax;
    const int tid = threadIdx.x;
    const int pe = tid / TPP, t = tid % TPP;
    const int s1 = pe & 1, s2 = pe >> 1;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    // X: per-pencil FFT transpose slices [4][P]; after the forward FFT of the
    // first quad of a pair the same region holds its N^ table, the second
    // quad's table has a region of its own
    c2<T>* X = reinterpret_cast<c2<T>*>(smem_raw);
    c2<T>* NTB = X + 4 * P;                                     // [6][N3+1]
    c2<T>* Wc = NTB + NTS;                                      // [6][wst]
    const int wst = v.cp ? rmax : rmax * rmax;                  // W_c stride per component
    c2<T>* Vc = Wc + 6 * wst;                                   // [2][6][rmax]
    c2<T>* tws = Vc + 12 * rmax;                                // [Plan::TW]
    Plan::fill_tw(tws, tw, tid, NT);

    const int k2 = bx % (n2 + 1);
    const int k1b = (bx / (n2 + 1)) * a.chunk;
    const int k1e = min(n1 + 1, k1b + a.chunk);
    const bool m2 = k2 > 0 && k2 < n2;
    const int pk2 = s2 ? L2 - k2 : k2;
    const long cstride = (long)L2 * L1 * N3;

    // ---- W_c(k2) = G_c x2 U2_c(k2, :) for the six components; for a
    //      superdiagonal core (Tucker+CP, eq. 17) only its diagonal
    //      W_c[l] = G_c[l,l,l] U2_c(k2, l) is nonzero and is all that is kept
    if (!a.dense && v.cp) {
        for (int e = tid; e < 6 * rmax; e += NT) {
            const int c = e / rmax, l = e - c * rmax;
            const int R = v.r[c][0];
            if (l < R)
                Wc[c * wst + l] = core[v.core_off[c] + (long)l * (R * R + R + 1)] *
                                               fac[v.fac_off[c][1] + (long)k2 * R + l];
        }
    } else if (!a.dense) {
        for (int c = 0; c < 6; ++c) {
            const int r1 = v.r[c][0], r2 = v.r[c][1], r3 = v.r[c][2];
            const c2<T>* G = core + v.core_off[c];
            const c2<T>* U2 = fac + v.fac_off[c][1] + (long)k2 * r2;
            for (int e = tid; e < r1 * r3; e += NT) {
                const int al = e / r3, ga = e - al * r3;
                const c2<T>* g = G + (long)al * r2 * r3 + ga;
                c2<T> acc = mk<T>(0, 0);
                for (int b0 = 0; b0 < r2; b0 += 8) {
                    c2<T> gv[8], uv[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const bool ok = b0 + q < r2;
                        gv[q] = ok ? g[(long)(b0 + q) * r3] : mk<T>(0, 0);
                        uv[q] = ok ? U2[b0 + q] : mk<T>(0, 0);
                    }
#pragma unroll
                    for (int q = 0; q < 8; ++q) fma_c(acc, gv[q], uv[q]);
                }
                Wc[c * wst + e] = acc;
            }
        }
    }
    __syncthreads();

    for (int kA = k1b; kA < k1e; kA += 2) {
        const int kB = kA + 1;
        const bool hasB = kB < k1e;
        // ---- quad A's pencils: loads issued first, in flight during the V phase
        const bool m1A = kA > 0 && kA < n1;
        const bool exA = (s1 == 0 || m1A) && (s2 == 0 || m2);
        const long baseA = (((long)b * 3 * L2 + pk2) * L1 + (s1 ? L1 - kA : kA)) * N3;
        c2<T> d[3][8];
        z_load<T, L3, TPP, Plan::RF0>(d, S2, baseA, cstride, t, exA);
        // ---- V_c = U1_c(k1, :) W_c for both quads of the pair (for a
        //      superdiagonal core the element-wise product with its diagonal)
        if (!a.dense && v.cp) {
            for (int e = tid; e < 12 * rmax; e += NT) {
                const int qd = e / (6 * rmax), rem = e - qd * 6 * rmax;
                const int c = rem / rmax, l = rem - c * rmax;
                const int R = v.r[c][0];
                if (l < R && (qd == 0 || hasB))
                    Vc[e] = fac[v.fac_off[c][0] + (long)(qd ? kB : kA) * R + l] * Wc[c * wst + l];
            }
        } else if (!a.dense) {
            for (int e = tid; e < 12 * rmax; e += NT) {
                const int qd = e / (6 * rmax), rem = e - qd * 6 * rmax;
                const int c = rem / rmax, ga = rem - c * rmax;
                const int r1 = v.r[c][0], r3 = v.r[c][2];
                const int k1 = qd ? kB : kA;
                if (ga < r3 && (qd == 0 || hasB)) {
                    const c2<T>* U1 = fac + v.fac_off[c][0] + (long)k1 * r1;
                    const c2<T>* w = Wc + c * wst + ga;
                    c2<T> acc = mk<T>(0, 0);
                    for (int a0 = 0; a0 < r1; a0 += 8) {
                        c2<T> uv[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) uv[q] = a0 + q < r1 ? U1[a0 + q] : mk<T>(0, 0);
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            if (a0 + q < r1) fma_c(acc, uv[q], w[(a0 + q) * r3]);
                    }
                    Vc[e] = acc;
                }
            }
        }
        // ---- quad A: forward FFT
#pragma unroll
        for (int q = 0; q < 3; ++q) Plan::template fwd<T, TPP, 1, -1>(d[q], X + pe * P, 0, t, tws);
        __syncthreads();   // slices free, Vc complete

        // ---- N^ tables of both quads: each z-factor element is loaded once
        //      and used for the two quads
        if (!a.dense && REC == 1) {
            if constexpr (REC == 1) z_tables_mfma<L3>(v, f3m, Vc, X, NTB, tid, NT);
#ifndef VIE_Z_TABLES_VALU
        } else if (!a.dense && sizeof(T) == 4) {
            if constexpr (sizeof(T) == 4) z_tables_mfma32<L3>(v, fac, Vc, X, NTB, tid);
#endif
        } else if (!a.dense) {
            for (int e = tid; e < NTS; e += NT) {
                const int c = e / (N3 + 1), kk = e - c * (N3 + 1);
                const int r3 = v.r[c][2];
                const c2<T>* U3 = fac + v.fac3t_off[c] + kk;
                const c2<T>* va = Vc + c * rmax;
                const c2<T>* vb = Vc + 6 * rmax + c * rmax;
                c2<T> accA = mk<T>(0, 0), accB = mk<T>(0, 0);
                for (int g0 = 0; g0 < r3; g0 += 8) {
                    c2<T> uv[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        uv[q] = g0 + q < r3 ? U3[(long)(g0 + q) * (N3 + 1)] : mk<T>(0, 0);
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        if (g0 + q < r3) {
                            fma_c(accA, va[g0 + q], uv[q]);
                            fma_c(accB, vb[g0 + q], uv[q]);
                        }
                    }
                }
                X[e] = accA;
                NTB[e] = accB;
            }
        } else {
            const long per = (long)(n1 + 1) * (n2 + 1) * (N3 + 1);
            for (int e = tid; e < NTS; e += NT) {
                const int c = e / (N3 + 1), kk = e - c * (N3 + 1);
                const c2<T>* src = dense + c * per + (long)k2 * (n1 + 1) * (N3 + 1) + kk;
                X[e] = src[(long)kA * (N3 + 1)];
                if (hasB) NTB[e] = src[(long)kB * (N3 + 1)];
            }
        }
        __syncthreads();   // tables complete
        z_product<T, L3, TPP, Plan::RFL, CONJ, REC == 2 ? 1 : 0>(d, X, t, s1, s2);
        __syncthreads();   // table A consumed: the slices are reused by the inverse FFT
#pragma unroll
        for (int q = 0; q < 3; ++q) Plan::template inv<T, TPP, 1, 1>(d[q], X + pe * P, 0, t, tws);
        if (exA) z_store<T, L3, TPP, Plan::RIL>(d, S2, baseA, cstride, t);

        // ---- quad B
        if (hasB) {
            const bool m1B = kB > 0 && kB < n1;
            const bool exB = (s1 == 0 || m1B) && (s2 == 0 || m2);
            const long baseB = (((long)b * 3 * L2 + pk2) * L1 + (s1 ? L1 - kB : kB)) * N3;
            // each wavefront now only touches its own pencil slice until the end of the pair
            z_load<T, L3, TPP, Plan::RF0>(d, S2, baseB, cstride, t, exB);
#pragma unroll
            for (int q = 0; q < 3; ++q) Plan::template fwd<T, TPP, 1, -1>(d[q], X + pe * P, 0, t, tws);
            z_product<T, L3, TPP, Plan::RFL, CONJ, REC == 2 ? 1 : 0>(d, NTB, t, s1, s2);
#pragma unroll
            for (int q = 0; q < 3; ++q) Plan::template inv<T, TPP, 1, 1>(d[q], X + pe * P, 0, t, tws);
            if (exB) z_store<T, L3, TPP, Plan::RIL>(d, S2, baseB, cstride, t);
        }
        __syncthreads();   // Vc, NTB and the slices are reused by the next pair
    }
}

template <typename T, int L3, bool CONJ, int REC>
__global__ void __launch_bounds__(4 * (L3 / 8), sizeof(T) == 4 ? 3 : 2)
    k_z_fast(c2<T>* __restrict__ S2, const c2<T>* __restrict__ tw, ZFastArgs a, const c2<T>* __restrict__ core,
             const c2<T>* __restrict__ fac, const c2<T>* __restrict__ dense,
             const unsigned short* __restrict__ f3m)
{
    z_body<T, L3, CONJ, REC>(S2, tw, a, core, fac, dense, f3m, blockIdx.x, blockIdx.y);
}

// Grouped launch over instances with the same z length (offsets ascending).
template <typename T, int L3, bool CONJ, int REC>
__global__ void __launch_bounds__(4 * (L3 / 8), sizeof(T) == 4 ? 3 : 2)
    k_z_fast_multi(const ZGroup g, const c2<T>* __restrict__ tw)
{
    int i = 0;
    while (i + 1 < g.n && (int)blockIdx.x >= g.e[i + 1].off) ++i;
    const ZInst& in = g.e[i];
    const int local = blockIdx.x - in.off;
    z_body<T, L3, CONJ, REC>((c2<T>*)in.S2, tw, in.za, (const c2<T>*)in.core, (const c2<T>*)in.fac,
                             (const c2<T>*)in.dense, in.f3m, local % in.nbx, local / in.nbx);
}

// ---------------------------------------------------------------------------
// host dispatch

// elements per thread: every radix of the plan must divide it; 8 threads per
// pencil for the mixed-radix lengths 192 = 8 8 3 and 224 = 7 4 4 2
template <typename T, int L>
static constexpr int xy_E()
{
    if constexpr (L == 192) return 24;
    else if constexpr (L == 224) return 28;
    else return sizeof(T) == 4 ? 32 : 16;
}

// pencils per workgroup (256 threads unless overridden at build time)
#ifndef VIE_XY_W512
#define VIE_XY_W512 0
#endif
#ifndef VIE_XY_W256
#define VIE_XY_W256 0
#endif
#ifndef VIE_XY_W128
#define VIE_XY_W128 0
#endif
template <typename T, int L>
static constexpr int xy_W()
{
    if constexpr (L == 512 && VIE_XY_W512 > 0) return VIE_XY_W512;
    else if constexpr (L == 256 && VIE_XY_W256 > 0) return VIE_XY_W256;
    else if constexpr (L == 128 && VIE_XY_W128 > 0) return VIE_XY_W128;
    else return 256 / (L / xy_E<T, L>());
}

template <typename TV, typename T, int L, int KIND, bool IDENT = false>
static void launch_xy(const void* in, void* out, const c2<TV>* x, const c2<TV>* eps, const c2<T>* tw,
                      const XYArgs& a, int grid_x, int grid_y, int nz, const int* rhs_map, hipStream_t s)
{
    constexpr int E = xy_E<T, L>();
    constexpr int W = xy_W<T, L>();
    constexpr int NT = W * (L / E);
    size_t lds = sizeof(c2<T>) * ((size_t)W * PL<L>::value + RegPlan<L>::TW);
    auto kern = k_xy_fast<TV, T, L, E, W, KIND, IDENT>;
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    dim3 grid((grid_x + W - 1) / W, grid_y, nz);
    if (KIND == 3) {
        // one dimension over (tile, component) in XCD-grouped order, z = rhs
        const long tiles = (long)grid.x * grid.y;
        grid = dim3((unsigned)(3 * ((tiles + 7) / 8) * 8), 1, nz / 3);
    }
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, s, in, out, x, eps, tw, a, rhs_map);
}

template <typename TV, typename T, int KIND>
static bool dispatch_xy(int L, const void* in, void* out, const c2<TV>* x, const c2<TV>* eps, const c2<T>* tw,
                        const XYArgs& a, int gx, int gy, int nz, const int* rhs_map, hipStream_t s)
{
    switch (L) {
    case 512: launch_xy<TV, T, 512, KIND>(in, out, x, eps, tw, a, gx, gy, nz, rhs_map, s); return true;
    case 256: launch_xy<TV, T, 256, KIND>(in, out, x, eps, tw, a, gx, gy, nz, rhs_map, s); return true;
    case 128: launch_xy<TV, T, 128, KIND>(in, out, x, eps, tw, a, gx, gy, nz, rhs_map, s); return true;
    case 192: launch_xy<TV, T, 192, KIND>(in, out, x, eps, tw, a, gx, gy, nz, rhs_map, s); return true;
    case 224: launch_xy<TV, T, 224, KIND>(in, out, x, eps, tw, a, gx, gy, nz, rhs_map, s); return true;
    default: return false;
    }
}

template <typename T, int L3>
static size_t zfast_lds(const OpView& v)
{
    static_assert(6 * (L3 / 2 + 1) <= 4 * PL<L3>::value, "N^ table must fit in the FFT slices");
    // W_c holds r1 x r3 per component, or the R diagonal weights of a
    // superdiagonal (Tucker+CP) core
    const size_t wst = v.cp ? (size_t)v.rmax : (size_t)v.rmax * v.rmax;
    return sizeof(c2<T>) * ((size_t)4 * PL<L3>::value + 6 * (L3 / 2 + 1) + 6 * wst + 12 * v.rmax +
                            RegPlan<L3>::TW);
}

template <typename T, int L3>
static hipError_t launch_z(const DeviceOp& op, int mode, int recon, int nrhs, c2<T>* S2, const c2<T>* tw,
                           const c2<T>* core, const c2<T>* fac, const c2<T>* dense, hipStream_t s)
{
    const OpView& v = op.view;
    ZFastArgs za;
    za.v = v;
    za.conj = (mode == MODE_AH || mode == MODE_NH);
    za.dense = op.nhat_source == 1;
    za.chunk = op.zchunk;
    int nchunk = (v.n[0] + 1 + za.chunk - 1) / za.chunk;
    size_t lds = zfast_lds<T, L3>(v);
    if (lds > op.max_lds) return hipErrorInvalidValue;
    auto kern = za.conj ? k_z_fast<T, L3, true, 0> : k_z_fast<T, L3, false, 0>;
    if constexpr (sizeof(T) == 4) {
        if (recon == 1) kern = za.conj ? k_z_fast<T, L3, true, 1> : k_z_fast<T, L3, false, 1>;
    }
    if (v.fam == 1) kern = k_z_fast<T, L3, false, 2>;
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3((v.n[1] + 1) * nchunk, nrhs), dim3(4 * (L3 / 8)), lds, s, S2, tw, za, core, fac,
                       dense, (const unsigned short*)op.b16.fac3m);
    return hipGetLastError();
}

// Entry points used by launch_matvec (matvec.hip), one per pass; each
// returns false when its FFT length has no register-FFT kernel.
template <typename TV, typename T>
bool xy_pass_fast(int kind, int L, const void* in, void* out, const c2<TV>* x, const c2<TV>* eps, const c2<T>* tw,
                  int n1, int n2, int n3, int L1, int L2, int mode, int nrhs, const int* rhs_map, hipStream_t s)
{
    XYArgs a{n1, n2, n3, L1, L2, mode};
    const int nz = nrhs * 3;
    switch (kind) {
    case 0: return dispatch_xy<TV, T, 0>(L, in, out, x, eps, tw, a, n2, n3, nz, rhs_map, s);
    case 1: return dispatch_xy<TV, T, 1>(L, in, out, x, eps, tw, a, n3, L1, nz, rhs_map, s);
    case 2: return dispatch_xy<TV, T, 2>(L, in, out, x, eps, tw, a, n3, L1, nz, rhs_map, s);
    default: return dispatch_xy<TV, T, 3>(L, in, out, x, eps, tw, a, n2, n3, nz, rhs_map, s);
    }
}

// The X+ (kind 0) and X- (kind 3) index maps with the identity in place of
// the transform (debug entry points; vector and compute types equal).
template <typename T, int KIND>
static bool dispatch_xy_ident(int L, const void* in, void* out, const c2<T>* x, const c2<T>* tw, const XYArgs& a,
                              int gx, int gy, int nz, hipStream_t s)
{
    switch (L) {
    case 512: launch_xy<T, T, 512, KIND, true>(in, out, x, nullptr, tw, a, gx, gy, nz, nullptr, s); return true;
    case 256: launch_xy<T, T, 256, KIND, true>(in, out, x, nullptr, tw, a, gx, gy, nz, nullptr, s); return true;
    case 128: launch_xy<T, T, 128, KIND, true>(in, out, x, nullptr, tw, a, gx, gy, nz, nullptr, s); return true;
    case 192: launch_xy<T, T, 192, KIND, true>(in, out, x, nullptr, tw, a, gx, gy, nz, nullptr, s); return true;
    case 224: launch_xy<T, T, 224, KIND, true>(in, out, x, nullptr, tw, a, gx, gy, nz, nullptr, s); return true;
    default: return false;
    }
}

template <typename T>
bool xy_ident_fast(int kind, int L, const void* in, void* out, const c2<T>* x, const c2<T>* tw, int n1, int n2,
                   int n3, int L1, int L2, int nrhs, hipStream_t s)
{
    const int nz = nrhs * 3;
    if (kind == 0) {
        XYArgs a{n1, n2, n3, L1, L2, MODE_N};
        return dispatch_xy_ident<T, 0>(L, in, out, x, tw, a, n2, n3, nz, s);
    }
    XYArgs a{n1, n2, n3, L1, L2, MODE_N};
    return dispatch_xy_ident<T, 3>(L, in, out, x, tw, a, n2, n3, nz, s);
}
template bool xy_ident_fast<float>(int, int, const void*, void*, const c2<float>*, const c2<float>*, int, int, int,
                                   int, int, int, hipStream_t);
template bool xy_ident_fast<double>(int, int, const void*, void*, const c2<double>*, const c2<double>*, int, int,
                                    int, int, int, int, hipStream_t);

bool bf16_recon_available(const DeviceOp& op)
{
    const OpView& v = op.view;
    if (v.fam != 0 || !op.b16.fac3m) return false;
    if (v.L[2] != 512 && v.L[2] != 256 && v.L[2] != 128) return false;
    for (int c = 0; c < 6; ++c)
        if (v.rh[c] == 0) return false;
    return true;
}

template <typename T>
bool z_pass_fast(const DeviceOp& op, int mode, int recon, int nrhs, c2<T>* S2, const c2<T>* tw, const c2<T>* core,
                 const c2<T>* fac, const c2<T>* dense, hipStream_t s)
{
    const OpView& v = op.view;
    // K operators: forward product only (the API rejects the others)
    if (v.fam != 0 && (mode == MODE_AH || mode == MODE_NH || recon == 1)) return false;
    if (recon == 1 && (sizeof(T) != 4 || !bf16_recon_available(op))) return false;
    switch (v.L[2]) {
    case 512:
        if (zfast_lds<T, 512>(v) > op.max_lds) return false;
        return launch_z<T, 512>(op, mode, recon, nrhs, S2, tw, core, fac, dense, s) == hipSuccess;
    case 256:
        if (zfast_lds<T, 256>(v) > op.max_lds) return false;
        return launch_z<T, 256>(op, mode, recon, nrhs, S2, tw, core, fac, dense, s) == hipSuccess;
    case 128:
        if (zfast_lds<T, 128>(v) > op.max_lds) return false;
        return launch_z<T, 128>(op, mode, recon, nrhs, S2, tw, core, fac, dense, s) == hipSuccess;
    default: return false;
    }
}

// ---- grouped launches (one per pass and FFT length over a batch)
template <typename TV, typename T, int L, int KIND>
static void launch_xy_group(const XYGroup& g, int nblocks, const c2<T>* tw, hipStream_t s)
{
    constexpr int E = xy_E<T, L>();
    constexpr int W = xy_W<T, L>();
    constexpr int NT = W * (L / E);
    size_t lds = sizeof(c2<T>) * ((size_t)W * PL<L>::value + RegPlan<L>::TW);
    auto kern = k_xy_fast_multi<TV, T, L, E, W, KIND>;
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(NT), lds, s, g, tw);
}

template <typename TV, typename T, int KIND>
static bool dispatch_xy_group(int L, const XYGroup& g, int nblocks, const c2<T>* tw, hipStream_t s)
{
    switch (L) {
    case 512: launch_xy_group<TV, T, 512, KIND>(g, nblocks, tw, s); return true;
    case 256: launch_xy_group<TV, T, 256, KIND>(g, nblocks, tw, s); return true;
    case 128: launch_xy_group<TV, T, 128, KIND>(g, nblocks, tw, s); return true;
    case 192: launch_xy_group<TV, T, 192, KIND>(g, nblocks, tw, s); return true;
    case 224: launch_xy_group<TV, T, 224, KIND>(g, nblocks, tw, s); return true;
    default: return false;
    }
}

template <typename TV, typename T>
int xy_fast_tile(int L)
{
    switch (L) {
    case 512: return xy_W<T, 512>();
    case 256: return xy_W<T, 256>();
    case 128: return xy_W<T, 128>();
    case 192: return xy_W<T, 192>();
    case 224: return xy_W<T, 224>();
    default: return 0;
    }
}

template <typename TV, typename T>
bool xy_group_fast(int kind, int L, const XYGroup& g, int nblocks, const c2<T>* tw, hipStream_t s)
{
    switch (kind) {
    case 0: return dispatch_xy_group<TV, T, 0>(L, g, nblocks, tw, s);
    case 1: return dispatch_xy_group<TV, T, 1>(L, g, nblocks, tw, s);
    case 2: return dispatch_xy_group<TV, T, 2>(L, g, nblocks, tw, s);
    default: return dispatch_xy_group<TV, T, 3>(L, g, nblocks, tw, s);
    }
}

template <typename T, int L3>
static void launch_z_group(int conj, int recon, int rmax, const ZGroup& g, int nblocks, const c2<T>* tw,
                           hipStream_t s)
{
    OpView dummy{};
    dummy.rmax = rmax;
    size_t lds = zfast_lds<T, L3>(dummy);
    auto kern = conj ? k_z_fast_multi<T, L3, true, 0> : k_z_fast_multi<T, L3, false, 0>;
    if constexpr (sizeof(T) == 4) {
        if (recon == 1) kern = conj ? k_z_fast_multi<T, L3, true, 1> : k_z_fast_multi<T, L3, false, 1>;
    }
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(4 * (L3 / 8)), lds, s, g, tw);
}

template <typename T>
bool z_group_fast(int L3, int conj, int recon, int rmax, size_t max_lds, const ZGroup& g, int nblocks,
                  const c2<T>* tw, hipStream_t s)
{
    OpView dummy{};
    dummy.rmax = rmax;
    switch (L3) {
    case 512:
        if (zfast_lds<T, 512>(dummy) > max_lds) return false;
        launch_z_group<T, 512>(conj, recon, rmax, g, nblocks, tw, s);
        return true;
    case 256:
        if (zfast_lds<T, 256>(dummy) > max_lds) return false;
        launch_z_group<T, 256>(conj, recon, rmax, g, nblocks, tw, s);
        return true;
    case 128:
        if (zfast_lds<T, 128>(dummy) > max_lds) return false;
        launch_z_group<T, 128>(conj, recon, rmax, g, nblocks, tw, s);
        return true;
    default: return false;
    }
}

bool z_fast_length(int L3) { return L3 == 512 || L3 == 256 || L3 == 128; }
bool xy_fast_length(int L) { return L == 512 || L == 256 || L == 128 || L == 192 || L == 224; }

template bool xy_group_fast<float, float>(int, int, const XYGroup&, int, const c2<float>*, hipStream_t);
template bool xy_group_fast<double, double>(int, int, const XYGroup&, int, const c2<double>*, hipStream_t);
template bool xy_group_fast<double, float>(int, int, const XYGroup&, int, const c2<float>*, hipStream_t);
template int xy_fast_tile<float, float>(int);
template int xy_fast_tile<double, double>(int);
template int xy_fast_tile<double, float>(int);
template bool z_group_fast<float>(int, int, int, int, size_t, const ZGroup&, int, const c2<float>*, hipStream_t);
template bool z_group_fast<double>(int, int, int, int, size_t, const ZGroup&, int, const c2<double>*, hipStream_t);

#define VIE_XYF_INST(TV, T)                                                                                        \
    template bool xy_pass_fast<TV, T>(int, int, const void*, void*, const c2<TV>*, const c2<TV>*, const c2<T>*, int, \
                                      int, int, int, int, int, int, const int*, hipStream_t);
VIE_XYF_INST(float, float)
VIE_XYF_INST(double, double)
VIE_XYF_INST(double, float)
template bool z_pass_fast<float>(const DeviceOp&, int, int, int, c2<float>*, const c2<float>*, const c2<float>*,
                                 const c2<float>*, const c2<float>*, hipStream_t);
template bool z_pass_fast<double>(const DeviceOp&, int, int, int, c2<double>*, const c2<double>*,
                                  const c2<double>*, const c2<double>*, const c2<double>*, hipStream_t);

}  // namespace vie
