// Internal types shared by the C ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "dev_common.h"

namespace vie {

// Device view of the compressed operator (passed to kernels by value).
// Fourier factors of component c along axis a: rows 0..n_a of the DFT of the
// embedded factor columns, row-major (n_a + 1) x r_a, at fac + fac_off[c][a];
// the z factor again column-major ((n3 + 1) contiguous per column) at
// fac + fac3t_off[c].
// Cores: [r1][r2][r3] (r3 fastest) at core + core_off[c], scaled by
// 1 / (8 n1 n2 n3) so the inverse FFTs can stay unnormalised.
// Parity of component c (xx, yy, zz, xy, xz, yz) of an operator family
// along axis a: 1 if the defining tensor is odd along that axis.  N: an
// off-diagonal component is odd along both of its axes.  K (the curl
// kernel eps_psq d_s g): xy is odd along z, xz along y, yz along x.
__host__ __device__ inline int comp_odd(int fam, int c, int a)
{
    if (fam == 0) return (c == 3 && a != 2) || (c == 4 && a != 1) || (c == 5 && a != 0);
    return (c == 3 && a == 2) || (c == 4 && a == 1) || (c == 5 && a == 0);
}

// parity of component c of an operator view along axis a (family and
// piecewise-linear pair together)
__host__ __device__ inline int view_odd(int fam, int lmask, int c, int a)
{
    return comp_odd(fam, c, a) ^ ((lmask >> a) & 1);
}

struct OpView {
    int n[3];
    int L[3];
    int r[6][3];
    int core_off[6];
    int fac_off[6][3];
    int fac3t_off[6];   // z factor transposed: [r3][n3 + 1]
    int rmax;
    // BF16 z factor for the MFMA reconstruction: per component 16 * ceil((n3 + 1) / 16)
    // rows k3 of 2 rh bf16 values [Re U3(k3, 0..rh) | Im U3(k3, 0..rh)], zero beyond
    // r3 and beyond row n3; rh = 16 ceil(r3 / 16) (0 when r3 > 32: not available)
    int rh[6];
    int fac3m_off[6];
    // operator family: 0 = N (symmetric component pair, six components),
    // 1 = K (antisymmetric pair: components xy, xz, yz in slots 3..5, slots
    // 0..2 zero)
    int fam;
    // extra parities of a piecewise-linear block (bit a: odd along axis a):
    // the pair (l, l') of basis functions flips the parity along a when
    // exactly one of them is linear along a; 0 for the pulse basis
    int lmask;
    // 1: every core is superdiagonal (r1 = r2 = r3 = R, a Tucker+CP form,
    // eq. 17): the z pass forms V_c(k1, k2, l) = G_c[l,l,l] U1_c(k1, l)
    // U2_c(k2, l) directly instead of contracting the core
    int cp;
};

template <typename T>
struct OpBuffers {
    c2<T>* core = nullptr;
    c2<T>* fac = nullptr;
};

struct BF16Buffers {
    // interleaved (re, im) bf16 pairs, same offsets as OpView
    unsigned short* core = nullptr;
    unsigned short* fac = nullptr;
    unsigned short* fac3m = nullptr;   // MFMA layout of the z factors (OpView::fac3m_off)
};

struct DeviceOp {
    OpView view;
    FftPlan plan[3];
    OpBuffers<double> d64;
    OpBuffers<float> d32;
    BF16Buffers b16;
    // twiddle tables exp(-2 pi i m / L_a), m < L_a, per axis
    c2<double>* tw64[3] = {nullptr, nullptr, nullptr};
    c2<float>* tw32[3] = {nullptr, nullptr, nullptr};
    // dense half-spectrum stores [c][k2][k1][k3] over (n1+1)(n2+1)(n3+1)
    c2<float>* dense32 = nullptr;
    c2<double>* dense64 = nullptr;
    int nhat_source = 0;
    size_t tucker_bytes = 0;   // cores + factors, each once, complex64
    size_t device_bytes = 0;   // everything the operator holds on the device
    int device = 0;
    size_t max_lds = 65536;
    int zchunk = 16;   // k1 mirror quads per z-pass workgroup (vie_autotune)
};

// Arguments of the register-FFT passes.
struct XYArgs {
    int n1, n2, n3, L1, L2;
    int mode;
};
struct ZFastArgs {
    OpView v;
    int conj;
    int dense;
    int chunk;     // k1 quads per workgroup
};

// Per-instance descriptors of a grouped register-FFT launch (one launch per
// pass and FFT length over every instance of a batch with that length).
struct XYInst {
    const void* in;
    void* out;
    const void* x;
    const void* eps;
    const int* map;
    XYArgs a;
    int off;    // first workgroup of the instance
    int ntx;    // pencil tiles
    int rows;   // rows per component
};
struct ZInst {
    void* S2;
    const void* core;
    const void* fac;
    const void* dense;
    const unsigned short* f3m;
    ZFastArgs za;
    int off;    // first workgroup of the instance
    int nbx;    // workgroups per right-hand side
};

// One instance of a multi-instance matvec (several grids, one launch per pass).
struct InstDev {
    OpView v;
    FftPlan plan[3];
    const void* tw[3];
    const void* core;
    const void* fac;
    const void* x;
    void* y;
    const void* eps;
    const int* map;   // active right-hand sides of this instance (nullptr = 0..nact-1)
    void* S1;
    void* S2;
    int nact;
    int G;
    int off[5];       // first block of the instance in each pass
    int cnt[5];       // blocks of the instance in each pass
};

struct InstHost {
    const DeviceOp* op;
    const void* x;
    void* y;
    const void* eps;
    const int* map;
    int nact;
    void* ws;         // matvec workspace of this instance (matvec_ws_elems(op, nact) elements)
};

// matvec modes
enum { MODE_A = 0, MODE_AH = 1, MODE_N = 2, MODE_NH = 3 };

// Set by the refined JM solve around its inner operator applications: the
// N and K products of vie_matvec_jm then run in FP32 on FP64 vectors
// (per host thread).
extern thread_local bool jm_mixed_products;

// Launch the five-pass matvec.  TV: vector element type, T: compute type.
// recon: 0 = same as T, 1 = BF16 (T = float only).
template <typename TV, typename T>
hipError_t launch_matvec(const DeviceOp& op, int mode, int recon, const c2<TV>* eps, const c2<TV>* x,
                         c2<TV>* y, int nrhs, c2<T>* ws, hipStream_t s, const int* rhs_map,
                         std::string& err);

// One pass p of the matvec on explicit buffers: 0 x -> S1, 1 S1 -> S2, 2 S2 in
// place (out), 3 S2 -> S3, 4 S3 -> y; ident (passes 0 and 4) replaces the
// transform by the identity.
template <typename TV, typename T>
hipError_t run_pass(const DeviceOp& op, int pass, int mode, int recon, const c2<TV>* eps, const c2<TV>* x,
                    const void* in, void* out, int nrhs, hipStream_t s, const int* rhs_map, std::string& err,
                    bool ident);

// Multi-instance matvec: one launch per pass over all instances (mixed-radix
// LDS kernels).  tab_dev: device scratch for the instance table.
template <typename TV, typename T>
hipError_t launch_matvec_multi(const std::vector<InstHost>& inst, int mode, InstDev* tab_dev, hipStream_t s,
                               std::string& err);

// Sampled Fourier-domain tensor values for tests.
hipError_t launch_nhat_samples(const DeviceOp& op, int prec, const int* idx_dev, int count,
                               double* out_dev, hipStream_t s);

// Materialise dense half-spectrum stores.
hipError_t launch_densify(DeviceOp& op, int with_c128, hipStream_t s);

size_t matvec_ws_elems(const DeviceOp& op, int nrhs);   // complex elements per workspace

// Instances per grouped launch (descriptors travel in the kernel arguments).
constexpr int kXYGroupMax = 24;
constexpr int kZGroupMax = 8;
struct XYGroup {
    int n;
    XYInst e[kXYGroupMax];
};
struct ZGroup {
    int n;
    ZInst e[kZGroupMax];
};

// register-FFT variants of the passes (matvec_fast.hip); false = not available
template <typename TV, typename T>
bool xy_pass_fast(int kind, int L, const void* in, void* out, const c2<TV>* x, const c2<TV>* eps, const c2<T>* tw,
                  int n1, int n2, int n3, int L1, int L2, int mode, int nrhs, const int* rhs_map, hipStream_t s);
// the X+ (kind 0) or X- (kind 3, bare epilogue) register kernel with the
// identity in place of the transform; false = no register kernel for L
template <typename T>
bool xy_ident_fast(int kind, int L, const void* in, void* out, const c2<T>* x, const c2<T>* tw, int n1, int n2,
                   int n3, int L1, int L2, int nrhs, hipStream_t s);
// recon 1: N^ tables from the BF16 z factors on MFMA (T = float only)
template <typename T>
bool z_pass_fast(const DeviceOp& op, int mode, int recon, int nrhs, c2<T>* S2, const c2<T>* tw, const c2<T>* core,
                 const c2<T>* fac, const c2<T>* dense, hipStream_t s);
// whether the BF16 MFMA reconstruction can run for this operator
bool bf16_recon_available(const DeviceOp& op);
// grouped register-FFT launches over a batch (instance tables on the device)
bool xy_fast_length(int L);
bool z_fast_length(int L3);
template <typename TV, typename T>
int xy_fast_tile(int L);   // pencils per workgroup of the X/Y kernels at length L
template <typename TV, typename T>
bool xy_group_fast(int kind, int L, const XYGroup& g, int nblocks, const c2<T>* tw, hipStream_t s);
template <typename T>
bool z_group_fast(int L3, int conj, int recon, int rmax, size_t max_lds, const ZGroup& g, int nblocks,
                  const c2<T>* tw, hipStream_t s);
// 0 = choose per pass (register FFT where the length allows), 1 = generic kernels only
extern int g_kernel_path;
// multi-instance batches: 0 = each instance's passes on its own (register-FFT)
// launches, back to back on the stream; 1 = one launch per pass over every
// instance (mixed-radix LDS kernels)
extern int g_batch_mode;

// Matvec of a multi-instance batch under g_batch_mode (recon: single-launch
// mode supports FP32/FP64 reconstruction only).
template <typename TV, typename T>
hipError_t launch_batch(const std::vector<InstHost>& inst, int mode, int recon, InstDev* tab_dev, hipStream_t s,
                        std::string& err);

// per-pass event timing (passes 0..4 = X+, Y+, Z*, Y-, X-)
void prof_enable(int on);
bool prof_is_enabled();
int prof_collect(double* ms, int* counts, int npass);

// Krylov helpers (batched over systems); T = double or float.
template <typename T>
struct KrylovArgs;

}  // namespace vie

// opaque handle of the C ABI
struct vie_op {
    vie::DeviceOp d;
};

namespace vie {
// one (l, l') block of a piecewise-linear operator as the z pass reads it
template <typename T>
struct PwlBlock {
    OpView v;
    const c2<T>* core;
    const c2<T>* fac;
};
// the ten stored basis pairs (l <= l'; 0 = pulse, 1..3 = linear along x, y, z)
constexpr int kPwlPairs[10][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {1, 1}, {1, 2}, {1, 3}, {2, 2}, {2, 3}, {3, 3}};
}  // namespace vie

// opaque handle of a piecewise-linear operator: ten six-component blocks
// (fam 0, N) or ten antisymmetric blocks with slots 3..5 = xy, xz, yz (fam 1, K)
struct vie_pwl_op {
    vie_op* blk[10];
    vie::PwlBlock<float>* dev32 = nullptr;    // device copies of the ten block views
    vie::PwlBlock<double>* dev64 = nullptr;
    int rmax = 1;
    int fam = 0;
};

