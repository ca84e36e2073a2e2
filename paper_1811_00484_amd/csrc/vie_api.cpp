// C ABI of the Tucker-compressed FFT-VIE library: operator construction,
// matvecs and test entry points.  The GMRES driver is in solve.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/vie.h"
#include "host_compress.h"
#include "host_cross.h"
#include "krylov.h"
#include "vie_internal.h"

namespace vie {

thread_local std::string g_last_error;
thread_local bool jm_mixed_products = false;

vie_status fail(vie_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

vie_status hip_fail(hipError_t e, const char* where)
{
    return fail(VIE_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

static bool make_plan(int L, FftPlan& p)
{
    p.L = L;
    p.nst = 0;
    int rem = L;
    const int order[] = {8, 4, 2, 3, 5, 7};
    for (int R : order) {
        while (rem % R == 0) {
            if (p.nst >= 12) return false;
            // avoid a radix-4/8 that would leave a lone factor of 2 unusable: fine either way
            p.rad[p.nst++] = R;
            rem /= R;
        }
    }
    return rem == 1;
}

static void free_op(DeviceOp& d)
{
    (void)hipFree(d.d64.core);
    (void)hipFree(d.d64.fac);
    (void)hipFree(d.d32.core);
    (void)hipFree(d.d32.fac);
    (void)hipFree(d.b16.core);
    (void)hipFree(d.b16.fac);
    (void)hipFree(d.b16.fac3m);
    for (int a = 0; a < 3; ++a) {
        (void)hipFree(d.tw64[a]);
        (void)hipFree(d.tw32[a]);
    }
    (void)hipFree(d.dense32);
    (void)hipFree(d.dense64);
}

static unsigned short to_bf16(float f)
{
    unsigned int u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);   // inf / nan
    unsigned int lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;                                                        // round to nearest even
    return (unsigned short)(u >> 16);
}

static vie_status build_operator(const int n[3], const FftPlan plans[3], TuckerComponent tc[6], vie_op** out,
                                 vie_compress_info* info, std::chrono::steady_clock::time_point t0, int fam = 0,
                                 int lmask = 0, double scale = 1.0)
{
    using cd = std::complex<double>;
    const long V = (long)n[0] * n[1] * n[2];
    // pack cores (scaled by 1/M) and Fourier factors
    DeviceOp d;
    OpView& v = d.view;
    v.fam = fam;
    v.lmask = lmask;
    int rmax = 1;
    int core_tot = 0, fac_tot = 0;
    for (int a = 0; a < 3; ++a) {
        v.n[a] = n[a];
        v.L[a] = 2 * n[a];
        d.plan[a] = plans[a];
    }
    for (int c = 0; c < 6; ++c) {
        for (int a = 0; a < 3; ++a) {
            v.r[c][a] = tc[c].r[a];
            rmax = std::max(rmax, tc[c].r[a]);
        }
        v.core_off[c] = core_tot;
        core_tot += tc[c].r[0] * tc[c].r[1] * tc[c].r[2];
        for (int a = 0; a < 3; ++a) {
            v.fac_off[c][a] = fac_tot;
            fac_tot += (n[a] + 1) * tc[c].r[a];
        }
    }
    const int fac_unique = fac_tot;
    // z factors also stored transposed ([g][k3]) for coalesced pencil-wise reads
    for (int c = 0; c < 6; ++c) {
        v.fac3t_off[c] = fac_tot;
        fac_tot += (n[2] + 1) * tc[c].r[2];
    }
    v.rmax = rmax;
    if (rmax > 64) return fail(VIE_E_UNSUPPORTED, "vie_compress: Tucker rank above 64");
    // superdiagonal cores (Tucker+CP forms) take the z pass's CP branch
    v.cp = 1;
    for (int c = 0; c < 6 && v.cp; ++c) {
        const int R = tc[c].r[0];
        if (tc[c].r[1] != R || tc[c].r[2] != R) {
            v.cp = 0;
            break;
        }
        for (int a = 0; a < R && v.cp; ++a)
            for (int b = 0; b < R && v.cp; ++b)
                for (int g = 0; g < R; ++g)
                    if (!(a == b && b == g) && tc[c].G[((size_t)a * R + b) * R + g] != cd(0.0)) {
                        v.cp = 0;
                        break;
                    }
    }
    // 1/M of the inverse transform, and the block's scale (piecewise-linear
    // blocks in the mass-normalised basis)
    const double invM = scale / (8.0 * (double)V);
    std::vector<cd> hcore(core_tot), hfac(fac_tot);
    for (int c = 0; c < 6; ++c) {
        for (size_t t = 0; t < tc[c].G.size(); ++t) hcore[v.core_off[c] + t] = tc[c].G[t] * invM;
        for (int a = 0; a < 3; ++a) {
            std::vector<cd> Uh;
            fourier_factor(tc[c].U[a], n[a], tc[c].r[a], view_odd(fam, lmask, c, a) ? -1 : 1, Uh);
            std::copy(Uh.begin(), Uh.end(), hfac.begin() + v.fac_off[c][a]);
            if (a == 2) {
                const int r3 = tc[c].r[2];
                for (int k = 0; k <= n[2]; ++k)
                    for (int g = 0; g < r3; ++g) hfac[v.fac3t_off[c] + (size_t)g * (n[2] + 1) + k] = Uh[(size_t)k * r3 + g];
            }
        }
    }
    // BF16 z factors in the row layout of the MFMA reconstruction
    const int ntile3 = (n[2] + 1 + 15) / 16;
    int m3_tot = 0;
    for (int c = 0; c < 6; ++c) {
        const int r3 = tc[c].r[2];
        v.rh[c] = r3 <= 16 ? 16 : (r3 <= 32 ? 32 : 0);
        v.fac3m_off[c] = m3_tot;
        m3_tot += ntile3 * 16 * 2 * v.rh[c];
    }
    std::vector<unsigned short> h3m((size_t)std::max(m3_tot, 1), 0);
    for (int c = 0; c < 6; ++c) {
        const int r3 = tc[c].r[2], rh = v.rh[c];
        if (rh == 0) continue;
        for (int k = 0; k <= n[2]; ++k)
            for (int g = 0; g < r3; ++g) {
                const cd u = hfac[v.fac_off[c][2] + (size_t)k * r3 + g];
                unsigned short* row = h3m.data() + v.fac3m_off[c] + (size_t)k * 2 * rh;
                row[g] = to_bf16((float)u.real());
                row[rh + g] = to_bf16((float)u.imag());
            }
    }
    // device upload
    hipError_t e;
    e = hipGetDevice(&d.device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, d.device) == hipSuccess && lds > 0)
        d.max_lds = (size_t)lds;
    auto upload = [&](const std::vector<cd>& src, void** dst64, void** dst32, void** dst16) -> hipError_t {
        size_t m = src.size();
        std::vector<c2<double>> h64(m);
        std::vector<c2<float>> h32(m);
        std::vector<unsigned short> h16(2 * m);
        for (size_t t = 0; t < m; ++t) {
            h64[t].x = src[t].real();
            h64[t].y = src[t].imag();
            h32[t].x = (float)src[t].real();
            h32[t].y = (float)src[t].imag();
            h16[2 * t] = to_bf16((float)src[t].real());
            h16[2 * t + 1] = to_bf16((float)src[t].imag());
        }
        hipError_t er;
        if ((er = hipMalloc(dst64, m * sizeof(c2<double>))) != hipSuccess) return er;
        if ((er = hipMalloc(dst32, m * sizeof(c2<float>))) != hipSuccess) return er;
        if ((er = hipMalloc(dst16, m * 4)) != hipSuccess) return er;
        if ((er = hipMemcpy(*dst64, h64.data(), m * sizeof(c2<double>), hipMemcpyHostToDevice)) != hipSuccess)
            return er;
        if ((er = hipMemcpy(*dst32, h32.data(), m * sizeof(c2<float>), hipMemcpyHostToDevice)) != hipSuccess)
            return er;
        return hipMemcpy(*dst16, h16.data(), m * 4, hipMemcpyHostToDevice);
    };
    e = upload(hcore, (void**)&d.d64.core, (void**)&d.d32.core, (void**)&d.b16.core);
    if (e == hipSuccess) e = upload(hfac, (void**)&d.d64.fac, (void**)&d.d32.fac, (void**)&d.b16.fac);
    if (e == hipSuccess) e = hipMalloc((void**)&d.b16.fac3m, h3m.size() * sizeof(unsigned short));
    if (e == hipSuccess)
        e = hipMemcpy(d.b16.fac3m, h3m.data(), h3m.size() * sizeof(unsigned short), hipMemcpyHostToDevice);
    for (int a = 0; a < 3 && e == hipSuccess; ++a) {
        int L = v.L[a];
        std::vector<c2<double>> t64(L);
        std::vector<c2<float>> t32(L);
        for (int m = 0; m < L; ++m) {
            const cd w = twiddle(m, L);
            t64[m].x = w.real();
            t64[m].y = w.imag();
            t32[m].x = (float)t64[m].x;
            t32[m].y = (float)t64[m].y;
        }
        e = hipMalloc((void**)&d.tw64[a], L * sizeof(c2<double>));
        if (e == hipSuccess) e = hipMalloc((void**)&d.tw32[a], L * sizeof(c2<float>));
        if (e == hipSuccess) e = hipMemcpy(d.tw64[a], t64.data(), L * sizeof(c2<double>), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d.tw32[a], t32.data(), L * sizeof(c2<float>), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        free_op(d);
        return e == hipErrorOutOfMemory ? fail(VIE_E_NOMEM, "vie_compress: device allocation failed")
                                        : hip_fail(e, "vie_compress upload");
    }
    // a Tucker+CP operator's compressed form is its factors and the R weights
    // on the core's diagonal
    size_t core_unique = core_tot;
    if (v.cp) {
        core_unique = 0;
        for (int c = 0; c < 6; ++c) core_unique += tc[c].r[0];
    }
    d.tucker_bytes = (core_unique + fac_unique) * sizeof(c2<float>);
    size_t twb = 0;
    for (int a = 0; a < 3; ++a) twb += (size_t)v.L[a] * (sizeof(c2<double>) + sizeof(c2<float>));
    d.device_bytes = (size_t)(core_tot + fac_tot) * (sizeof(c2<double>) + sizeof(c2<float>) + 4) +
                     h3m.size() * sizeof(unsigned short) + twb;
    vie_op* op = new vie_op;
    op->d = d;
    *out = op;
    if (info) {
        for (int c = 0; c < 6; ++c) {
            for (int a = 0; a < 3; ++a) info->ranks[c][a] = tc[c].r[a];
            info->tail_bound[c] = tc[c].tail_rel;
            info->fro_norm[c] = tc[c].fro;
        }
        info->tucker_bytes_c64 = d.tucker_bytes;
        info->dense_bytes_c64 = (size_t)6 * 8 * (size_t)V * sizeof(c2<float>);
        info->device_bytes = d.device_bytes;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->cp = v.cp;
    }
    return VIE_OK;
}

}  // namespace vie

using namespace vie;

// HOSVD of `count` defining tensors, one(c, buffer) each: on grids of at most
// 2^18 voxels one tensor per host thread (its loops serial: on such short
// unfoldings the threads' start-up outweighs the work inside one tensor), on
// larger ones one after another with the threads inside each.  Results do not
// depend on the choice.
template <typename F>
static void for_components(int count, long V, F one)
{
    using cd = std::complex<double>;
    if (V <= (1L << 18)) {
        parallel_jobs(count, [&](int c) {
            std::vector<cd> A((size_t)V);
            one(c, A);
        });
    } else {
        std::vector<cd> A((size_t)V);
        for (int c = 0; c < count; ++c) one(c, A);
    }
}

extern "C" {

const char* vie_last_error(void) { return g_last_error.c_str(); }

const char* vie_version(void) { return "vie-gfx950 0.1"; }

static vie_status compress_common(const int n[3], const double* green, const vie_compress_opts* opts, int cp_rank,
                                  int cp_iters, vie_op** out, vie_compress_info* info, double* cp_err,
                                  int lmask = 0, double scale = 1.0);
static vie_status pwl_upload(vie_pwl_op* P, const char* who);

vie_status vie_compress(const int n[3], const double* green, const vie_compress_opts* opts, vie_op** out,
                        vie_compress_info* info)
{
    return compress_common(n, green, opts, -1, 0, out, info, nullptr);
}

vie_status vie_compress_cp(const int n[3], const double* green, const vie_compress_opts* opts, int cp_rank,
                           int cp_iters, vie_op** out, vie_compress_info* info, double cp_rel_err[6])
{
    if (cp_rank < 0 || cp_iters < 0) return fail(VIE_E_ARG, "vie_compress_cp: negative CP rank or iterations");
    return compress_common(n, green, opts, cp_rank, cp_iters == 0 ? 1000 : cp_iters, out, info, cp_rel_err);
}

static vie_status compress_k_common(const int n[3], const double* green_k, const vie_compress_opts* opts,
                                    vie_op** out, vie_compress_info* info, int lmask, double scale);

vie_status vie_compress_k(const int n[3], const double* green_k, const vie_compress_opts* opts, vie_op** out,
                          vie_compress_info* info)
{
    return compress_k_common(n, green_k, opts, out, info, 0, 1.0);
}

// lmask, scale: as compress_common (piecewise-linear blocks)
static vie_status compress_k_common(const int n[3], const double* green_k, const vie_compress_opts* opts,
                                    vie_op** out, vie_compress_info* info, int lmask, double scale)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!n || !green_k || !out) return fail(VIE_E_ARG, "vie_compress_k: null argument");
    *out = nullptr;
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || n[a] > 256) return fail(VIE_E_UNSUPPORTED, "vie_compress_k: n_i must be in [1, 256]");
    vie_compress_opts o = opts ? *opts : vie_compress_opts{1e-6, 0, 0};
    if (!(o.tol > 0 && o.tol < 1) || (o.trunc_rule != 0 && o.trunc_rule != 1) || o.max_rank < 0)
        return fail(VIE_E_ARG, "vie_compress_k: bad options");
    FftPlan plans[3];
    for (int a = 0; a < 3; ++a)
        if (!make_plan(2 * n[a], plans[a]))
            return fail(VIE_E_UNSUPPORTED, "vie_compress_k: 2 n_i must factor into 2, 3, 5, 7");
    const long V = (long)n[0] * n[1] * n[2];
    for (long t = 0; t < 6 * V; ++t)
        if (!std::isfinite(green_k[t])) return fail(VIE_E_NONFINITE, "vie_compress_k: non-finite tensor");
    using cd = std::complex<double>;
    TuckerComponent tc[6];
    // slots 0..2 (the zero diagonal of an antisymmetric pair): rank-1 zero forms
    for (int c = 0; c < 3; ++c) {
        for (int a = 0; a < 3; ++a) {
            tc[c].r[a] = 1;
            tc[c].U[a].assign((size_t)n[a], cd(0.0));
            tc[c].sv[a].assign((size_t)n[a], 0.0);
        }
        tc[c].G.assign(1, cd(0.0));
        tc[c].tail_rel = 0;
        tc[c].fro = 0;
    }
    int rc[6] = {0, 0, 0, 0, 0, 0};
    for_components(3, V, [&](int j3, std::vector<cd>& A) {
        const int c = 3 + j3;
        const double* g = green_k + 2 * (size_t)j3 * V;
        for (long t = 0; t < V; ++t) A[t] = cd(g[2 * t], g[2 * t + 1]);
        // zero at zero offset along the axes the component is odd along
        for (int k = 0; k < n[2]; ++k)
            for (int j = 0; j < n[1]; ++j)
                for (int i = 0; i < n[0]; ++i)
                    if ((view_odd(1, lmask, c, 0) && i == 0) || (view_odd(1, lmask, c, 1) && j == 0) ||
                        (view_odd(1, lmask, c, 2) && k == 0))
                        A[((long)k * n[1] + j) * n[0] + i] = 0.0;
        rc[c] = hosvd_component(A.data(), n, o.tol, o.trunc_rule, o.max_rank, tc[c]);
    });
    for (int c = 3; c < 6; ++c)
        if (rc[c] != 0) return fail(VIE_E_UNSUPPORTED, "vie_compress_k: max_rank too small for tol");
    return build_operator(n, plans, tc, out, info, t0, 1, lmask, scale);
}

static vie_status compress_common(const int n[3], const double* green, const vie_compress_opts* opts, int cp_rank,
                                  int cp_iters, vie_op** out, vie_compress_info* info, double* cp_err, int lmask,
                                  double scale)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!n || !green || !out) return fail(VIE_E_ARG, "vie_compress: null argument");
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || n[a] > 256) return fail(VIE_E_UNSUPPORTED, "vie_compress: n_i must be in [1, 256]");
    double tol = opts ? opts->tol : 1e-6;
    int rule = opts ? opts->trunc_rule : 0;
    int max_rank = opts ? opts->max_rank : 0;
    if (!(tol > 0.0) || !std::isfinite(tol) || (rule != 0 && rule != 1) || max_rank < 0)
        return fail(VIE_E_ARG, "vie_compress: bad options");
    const long V = (long)n[0] * n[1] * n[2];
    FftPlan plans[3];
    for (int a = 0; a < 3; ++a)
        if (!make_plan(2 * n[a], plans[a]))
            return fail(VIE_E_UNSUPPORTED, "vie_compress: 2 n_i must factor into 2, 3, 5, 7");
    for (long t = 0; t < 12 * V; ++t)
        if (!std::isfinite(green[t])) return fail(VIE_E_NONFINITE, "vie_compress: non-finite Green's tensor");

    using cd = std::complex<double>;
    TuckerComponent tc[6];
    int odd[6][3];
    for (int c = 0; c < 6; ++c)
        for (int a = 0; a < 3; ++a) odd[c][a] = view_odd(0, lmask, c, a);
    int rc[6] = {0, 0, 0, 0, 0, 0};
    for_components(6, V, [&](int c, std::vector<cd>& A) {
        const double* g = green + 2 * (size_t)c * V;
        for (long t = 0; t < V; ++t) A[t] = cd(g[2 * t], g[2 * t + 1]);
        // an odd component vanishes at zero offset along its odd axes
        for (int k = 0; k < n[2]; ++k)
            for (int j = 0; j < n[1]; ++j)
                for (int i = 0; i < n[0]; ++i)
                    if ((odd[c][0] && i == 0) || (odd[c][1] && j == 0) || (odd[c][2] && k == 0))
                        A[((long)k * n[1] + j) * n[0] + i] = 0.0;
        rc[c] = hosvd_component(A.data(), n, tol, rule, max_rank, tc[c]);
    });
    for (int c = 0; c < 6; ++c)
        if (rc[c] != 0) return fail(VIE_E_UNSUPPORTED, "vie_compress: max_rank too small for tol");
    if (cp_rank >= 0) {
        // Alg. 2: CP of each core, Tucker+CP factors W^a = U^a V^a, and a
        // superdiagonal core so that eq. 17 is the Tucker form with it
        for (int c = 0; c < 6; ++c) {
            TuckerComponent& t = tc[c];
            const int rmin = std::min(t.r[0], std::min(t.r[1], t.r[2]));
            const int R = cp_rank == 0 ? rmin : cp_rank;
            if (R > 64) return fail(VIE_E_UNSUPPORTED, "vie_compress_cp: CP rank above 64");
            std::vector<cd> Vf[3];
            const double e = cp_als(t.G, t.r, R, cp_iters, Vf);
            if (cp_err) cp_err[c] = e;
            for (int a = 0; a < 3; ++a) {
                // row 0 of an odd axis stays exactly zero, as the odd
                // embedding needs (U's row there is zero up to rounding, and
                // the large cancelling terms of a near-degenerate CP fit
                // would amplify that rounding)
                std::vector<cd> W((size_t)n[a] * R, 0);
                for (int i = odd[c][a] ? 1 : 0; i < n[a]; ++i)
                    for (int l = 0; l < R; ++l) {
                        cd acc = 0;
                        for (int k = 0; k < t.r[a]; ++k) acc += t.U[a][(size_t)i * t.r[a] + k] * Vf[a][(size_t)k * R + l];
                        W[(size_t)i * R + l] = acc;
                    }
                t.U[a] = W;
                t.r[a] = R;
            }
            t.G.assign((size_t)R * R * R, 0);
            for (int l = 0; l < R; ++l) t.G[((size_t)l * R + l) * R + l] = 1.0;
        }
    }
    return build_operator(n, plans, tc, out, info, t0, 0, lmask, scale);
}

static vie_status cross_params(const vie_cross_opts* opts, CrossParams& p, const char* who)
{
    if (opts) {
        p.tol = opts->tol;
        p.rule = opts->trunc_rule;
        p.max_rank = opts->max_rank;
        p.oversample = opts->oversample == 0 ? 8 : opts->oversample;
        p.max_sweeps = opts->max_sweeps == 0 ? 8 : opts->max_sweeps;
        p.n_sample = opts->n_sample;
        p.seed = opts->seed;
    }
    if (!(p.tol > 0.0 && p.tol < 1.0) || (p.rule != 0 && p.rule != 1) || p.max_rank < 0 || p.max_rank > 64 ||
        p.oversample < 0 || p.oversample > 16 || p.max_sweeps < 1 || p.max_sweeps > 100 || p.n_sample < 0 ||
        p.n_sample > (1 << 24))
        return fail(VIE_E_ARG, std::string(who) + ": bad options");
    return VIE_OK;
}

static vie_status cross_status(int rc, const std::string& err, const char* who)
{
    if (rc == 0) return VIE_OK;
    if (rc == -4) return fail(VIE_E_NONFINITE, std::string(who) + ": " + err);
    if (rc == -1) return fail(VIE_E_ARG, std::string(who) + ": " + err);
    return fail(VIE_E_UNSUPPORTED, std::string(who) + ": " + err);
}

vie_status vie_compress_cross(const int n[3], vie_entry_fn fn, void* ctx, const vie_cross_opts* opts,
                              vie_op** out, vie_compress_info* info, vie_cross_info* xinfo)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!n || !fn || !out) return fail(VIE_E_ARG, "vie_compress_cross: null argument");
    *out = nullptr;
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || n[a] > 256) return fail(VIE_E_UNSUPPORTED, "vie_compress_cross: n_i must be in [1, 256]");
    CrossParams p;
    vie_status st = cross_params(opts, p, "vie_compress_cross");
    if (st != VIE_OK) return st;
    FftPlan plans[3];
    for (int a = 0; a < 3; ++a)
        if (!make_plan(2 * n[a], plans[a]))
            return fail(VIE_E_UNSUPPORTED, "vie_compress_cross: 2 n_i must factor into 2, 3, 5, 7");
    TuckerComponent tc[6];
    vie_cross_info xi;
    std::memset(&xi, 0, sizeof(xi));
    for (int c = 0; c < 6; ++c) {
        int odd[3];
        for (int a = 0; a < 3; ++a) odd[a] = comp_odd(0, c, a);
        CrossStats cs;
        std::string err;
        const int rc = tucker_cross(fn, ctx, c, odd, n, p, tc[c], cs, err);
        if (rc != 0) return cross_status(rc, err, "vie_compress_cross");
        xi.evals[c] = cs.evals;
        xi.evals_sample[c] = cs.evals_sample;
        xi.sweeps[c] = cs.sweeps;
        xi.sample_rel_err[c] = cs.sample_rel_err;
    }
    xi.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    st = build_operator(n, plans, tc, out, info, t0);
    if (st == VIE_OK && xinfo) *xinfo = xi;
    return st;
}

// host-only cross of one component whose parity zeros are odd[3]; the
// counts go to slot `slot` of xinfo
static vie_status tucker_cross_host(const char* who, const int n[3], vie_entry_fn fn, void* ctx, int comp,
                                    const int odd[3], int slot, const vie_cross_opts* opts, int ranks[3], double* core,
                                    size_t core_cap, double* factors, size_t fac_cap, vie_cross_info* xinfo)
{
    auto t0 = std::chrono::steady_clock::now();
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || n[a] > 65536) return fail(VIE_E_ARG, std::string(who) + ": n_i must be in [1, 65536]");
    CrossParams p;
    vie_status st = cross_params(opts, p, who);
    if (st != VIE_OK) return st;
    TuckerComponent tc;
    CrossStats cs;
    std::string err;
    const int rc = tucker_cross(fn, ctx, comp, odd, n, p, tc, cs, err);
    if (rc != 0) return cross_status(rc, err, who);
    for (int a = 0; a < 3; ++a) ranks[a] = tc.r[a];
    if (xinfo) {
        xinfo->evals[slot] = cs.evals;
        xinfo->evals_sample[slot] = cs.evals_sample;
        xinfo->sweeps[slot] = cs.sweeps;
        xinfo->sample_rel_err[slot] = cs.sample_rel_err;
        xinfo->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    const size_t ng = (size_t)tc.r[0] * tc.r[1] * tc.r[2];
    const size_t nf = (size_t)n[0] * tc.r[0] + (size_t)n[1] * tc.r[1] + (size_t)n[2] * tc.r[2];
    if ((core && core_cap < ng) || (factors && fac_cap < nf))
        return fail(VIE_E_ARG, std::string(who) + ": output buffer too small for ranks (" + std::to_string(tc.r[0]) +
                                   ", " + std::to_string(tc.r[1]) + ", " + std::to_string(tc.r[2]) + ")");
    if (core)
        for (size_t t = 0; t < ng; ++t) {
            core[2 * t] = tc.G[t].real();
            core[2 * t + 1] = tc.G[t].imag();
        }
    if (factors) {
        size_t o = 0;
        for (int a = 0; a < 3; ++a)
            for (const auto& v : tc.U[a]) {
                factors[2 * o] = v.real();
                factors[2 * o + 1] = v.imag();
                ++o;
            }
    }
    return VIE_OK;
}

vie_status vie_tucker_cross(const int n[3], vie_entry_fn fn, void* ctx, int comp, const vie_cross_opts* opts,
                            int ranks[3], double* core, size_t core_cap, double* factors, size_t fac_cap,
                            vie_cross_info* xinfo)
{
    if (!n || !fn || !ranks) return fail(VIE_E_ARG, "vie_tucker_cross: null argument");
    if (comp < 0 || comp > 5) return fail(VIE_E_ARG, "vie_tucker_cross: comp must be in [0, 5]");
    int odd[3];
    for (int a = 0; a < 3; ++a) odd[a] = comp_odd(0, comp, a);
    return tucker_cross_host("vie_tucker_cross", n, fn, ctx, comp, odd, comp, opts, ranks, core, core_cap, factors,
                             fac_cap, xinfo);
}

vie_status vie_tucker_cross_pwl(const int n[3], vie_entry_fn fn, void* ctx, int comp, const vie_cross_opts* opts,
                                int ranks[3], double* core, size_t core_cap, double* factors, size_t fac_cap,
                                vie_cross_info* xinfo)
{
    if (!n || !fn || !ranks) return fail(VIE_E_ARG, "vie_tucker_cross_pwl: null argument");
    if (comp < 0 || comp > 89) return fail(VIE_E_ARG, "vie_tucker_cross_pwl: comp must be in [0, 89]");
    // 0..59: N, pair comp / 6, dyadic component comp % 6; 60..89: K, pair
    // (comp - 60) / 3, component xy, xz, yz = (comp - 60) % 3 (K's slots 3..5)
    const bool isk = comp >= 60;
    const int pair = isk ? (comp - 60) / 3 : comp / 6;
    const int c = isk ? 3 + (comp - 60) % 3 : comp % 6;
    const int la = kPwlPairs[pair][0], lb = kPwlPairs[pair][1];
    int lmask = 0;
    for (int a = 0; a < 3; ++a) lmask |= (((la == a + 1) + (lb == a + 1)) & 1) << a;
    int odd[3];
    for (int a = 0; a < 3; ++a) odd[a] = view_odd(isk ? 1 : 0, lmask, c, a);
    return tucker_cross_host("vie_tucker_cross_pwl", n, fn, ctx, comp, odd, c, opts, ranks, core, core_cap, factors,
                             fac_cap, xinfo);
}

vie_status vie_op_from_tucker(const int n[3], const int ranks[6][3], const double* cores, const double* factors,
                              vie_op** out, vie_compress_info* info)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!n || !ranks || !cores || !factors || !out) return fail(VIE_E_ARG, "vie_op_from_tucker: null argument");
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || n[a] > 256) return fail(VIE_E_UNSUPPORTED, "vie_op_from_tucker: n_i must be in [1, 256]");
    FftPlan plans[3];
    for (int a = 0; a < 3; ++a)
        if (!make_plan(2 * n[a], plans[a]))
            return fail(VIE_E_UNSUPPORTED, "vie_op_from_tucker: 2 n_i must factor into 2, 3, 5, 7");
    using cd = std::complex<double>;
    int odd[6][3];
    for (int c = 0; c < 6; ++c)
        for (int a = 0; a < 3; ++a) odd[c][a] = comp_odd(0, c, a);
    TuckerComponent tc[6];
    size_t co = 0, fo = 0;
    for (int c = 0; c < 6; ++c) {
        for (int a = 0; a < 3; ++a) {
            const int r = ranks[c][a];
            if (r < 1 || r > n[a] || r > 64) return fail(VIE_E_ARG, "vie_op_from_tucker: ranks must be in [1, min(n_a, 64)]");
            tc[c].r[a] = r;
        }
        const size_t ng = (size_t)tc[c].r[0] * tc[c].r[1] * tc[c].r[2];
        tc[c].G.resize(ng);
        for (size_t t = 0; t < ng; ++t) tc[c].G[t] = cd(cores[2 * (co + t)], cores[2 * (co + t) + 1]);
        co += ng;
        for (int a = 0; a < 3; ++a) {
            const size_t nu = (size_t)n[a] * tc[c].r[a];
            tc[c].U[a].resize(nu);
            for (size_t t = 0; t < nu; ++t) tc[c].U[a][t] = cd(factors[2 * (fo + t)], factors[2 * (fo + t) + 1]);
            fo += nu;
            if (odd[c][a])
                for (int g = 0; g < tc[c].r[a]; ++g)
                    if (tc[c].U[a][g] != cd(0.0))
                        return fail(VIE_E_ARG, "vie_op_from_tucker: an off-diagonal component's factor along one of "
                                               "its odd axes must have a zero row 0");
        }
    }
    for (size_t t = 0; t < 2 * co; ++t)
        if (!std::isfinite(cores[t])) return fail(VIE_E_NONFINITE, "vie_op_from_tucker: non-finite core");
    for (size_t t = 0; t < 2 * fo; ++t)
        if (!std::isfinite(factors[t])) return fail(VIE_E_NONFINITE, "vie_op_from_tucker: non-finite factor");
    return build_operator(n, plans, tc, out, info, t0);
}

vie_status vie_op_destroy(vie_op* op)
{
    if (!op) return VIE_OK;
    free_op(op->d);
    delete op;
    return VIE_OK;
}

vie_status vie_pwl_op_destroy(vie_pwl_op* op)
{
    if (!op) return VIE_OK;
    for (int b = 0; b < 10; ++b) vie_op_destroy(op->blk[b]);
    if (op->dev32) (void)hipFree(op->dev32);
    if (op->dev64) (void)hipFree(op->dev64);
    delete op;
    return VIE_OK;
}

vie_status vie_compress_pwl(const int n[3], const double* green_pwl, const vie_compress_opts* opts, int cp_rank,
                            int cp_iters, vie_pwl_op** out, vie_compress_info* info)
{
    if (!n || !green_pwl || !out) return fail(VIE_E_ARG, "vie_compress_pwl: null argument");
    *out = nullptr;
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || n[a] > 256) return fail(VIE_E_UNSUPPORTED, "vie_compress_pwl: n_i must be in [1, 256]");
    if (cp_rank < -1 || cp_iters < 0) return fail(VIE_E_ARG, "vie_compress_pwl: bad CP rank or iterations");
    const size_t V = (size_t)n[0] * n[1] * n[2];
    const double s12 = std::sqrt(12.0);
    vie_pwl_op* P = new vie_pwl_op();
    for (int b = 0; b < 10; ++b) P->blk[b] = nullptr;
    for (int b = 0; b < 10; ++b) {
        const int la = kPwlPairs[b][0], lb = kPwlPairs[b][1];
        int lmask = 0;
        for (int a = 0; a < 3; ++a) lmask |= (((la == a + 1) + (lb == a + 1)) & 1) << a;
        // the mass-normalised basis scales the linear functions by sqrt 12
        const double scale = (la ? s12 : 1.0) * (lb ? s12 : 1.0);
        vie_status st = compress_common(n, green_pwl + (size_t)b * 12 * V, opts, cp_rank,
                                        cp_rank >= 0 && cp_iters == 0 ? 1000 : cp_iters, &P->blk[b],
                                        info ? &info[b] : nullptr, nullptr, lmask, scale);
        if (st != VIE_OK) {
            std::string msg = vie_last_error();
            vie_pwl_op_destroy(P);
            return fail(st, "vie_compress_pwl: block " + std::to_string(b) + ": " + msg);
        }
        P->rmax = std::max(P->rmax, P->blk[b]->d.view.rmax);
    }
    vie_status st = pwl_upload(P, "vie_compress_pwl");
    if (st == VIE_OK) *out = P;
    return st;
}

vie_status vie_compress_pwl_k(const int n[3], const double* green_pwl_k, const vie_compress_opts* opts,
                              vie_pwl_op** out, vie_compress_info* info)
{
    if (!n || !green_pwl_k || !out) return fail(VIE_E_ARG, "vie_compress_pwl_k: null argument");
    *out = nullptr;
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || n[a] > 256) return fail(VIE_E_UNSUPPORTED, "vie_compress_pwl_k: n_i must be in [1, 256]");
    const size_t V = (size_t)n[0] * n[1] * n[2];
    const double s12 = std::sqrt(12.0);
    vie_pwl_op* P = new vie_pwl_op();
    P->fam = 1;
    for (int b = 0; b < 10; ++b) P->blk[b] = nullptr;
    for (int b = 0; b < 10; ++b) {
        const int la = kPwlPairs[b][0], lb = kPwlPairs[b][1];
        int lmask = 0;
        for (int a = 0; a < 3; ++a) lmask |= (((la == a + 1) + (lb == a + 1)) & 1) << a;
        const double scale = (la ? s12 : 1.0) * (lb ? s12 : 1.0);
        vie_status st = compress_k_common(n, green_pwl_k + (size_t)b * 6 * V, opts, &P->blk[b],
                                          info ? &info[b] : nullptr, lmask, scale);
        if (st != VIE_OK) {
            std::string msg = vie_last_error();
            vie_pwl_op_destroy(P);
            return fail(st, "vie_compress_pwl_k: block " + std::to_string(b) + ": " + msg);
        }
        P->rmax = std::max(P->rmax, P->blk[b]->d.view.rmax);
    }
    vie_status st = pwl_upload(P, "vie_compress_pwl_k");
    if (st == VIE_OK) *out = P;
    return st;
}

}  // extern "C"

// device copies of the ten block views (the z pass reads them by pair)
static vie_status pwl_upload(vie_pwl_op* P, const char* who)
{
    PwlBlock<float> h32[10];
    PwlBlock<double> h64[10];
    for (int b = 0; b < 10; ++b) {
        const DeviceOp& d = P->blk[b]->d;
        h32[b].v = d.view;
        h32[b].core = d.d32.core;
        h32[b].fac = d.d32.fac;
        h64[b].v = d.view;
        h64[b].core = d.d64.core;
        h64[b].fac = d.d64.fac;
    }
    hipError_t e = hipMalloc((void**)&P->dev32, sizeof(h32));
    if (e == hipSuccess) e = hipMalloc((void**)&P->dev64, sizeof(h64));
    if (e == hipSuccess) e = hipMemcpy(P->dev32, h32, sizeof(h32), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(P->dev64, h64, sizeof(h64), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        vie_pwl_op_destroy(P);
        return hip_fail(e, (std::string(who) + " upload").c_str());
    }
    return VIE_OK;
}

extern "C" {

vie_status vie_op_query(const vie_op* op, int n[3], int ranks[6][3])
{
    if (!op) return fail(VIE_E_ARG, "vie_op_query: null op");
    if (n)
        for (int a = 0; a < 3; ++a) n[a] = op->d.view.n[a];
    if (ranks)
        for (int c = 0; c < 6; ++c)
            for (int a = 0; a < 3; ++a) ranks[c][a] = op->d.view.r[c][a];
    return VIE_OK;
}

vie_status vie_op_densify(vie_op* op, int with_c128)
{
    if (!op) return fail(VIE_E_ARG, "vie_op_densify: null op");
    hipError_t e = launch_densify(op->d, with_c128, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "vie_op_densify");
    return VIE_OK;
}

vie_status vie_op_set_nhat(vie_op* op, int source)
{
    if (!op || (source != VIE_NHAT_TUCKER && source != VIE_NHAT_DENSE))
        return fail(VIE_E_ARG, "vie_op_set_nhat: bad argument");
    if (source == VIE_NHAT_DENSE && !op->d.dense32)
        return fail(VIE_E_ARG, "vie_op_set_nhat: call vie_op_densify first");
    op->d.nhat_source = source;
    return VIE_OK;
}

size_t vie_workspace_bytes(const vie_op* op, int dtype, int nrhs)
{
    if (!op || nrhs < 1) return 0;
    size_t el = dtype == VIE_C128 ? sizeof(c2<double>) : sizeof(c2<float>);
    return matvec_ws_elems(op->d, nrhs) * el;
}

}  // extern "C"

namespace vie {

vie_status matvec_common(const vie_op* op, int mode, int dtype, int recon, const void* eps, const void* x,
                         void* y, int nrhs, void* ws, size_t ws_bytes, void* stream, const int* rhs_map)
{
    if (!op || !x || !y || !ws || nrhs < 1) return fail(VIE_E_ARG, "vie_matvec: null argument or nrhs < 1");
    if (op->d.view.fam != 0 && mode != MODE_N)
        return fail(VIE_E_UNSUPPORTED, "vie_matvec: a K operator has the bare forward product (VIE_OP_N) only");
    bool needs_eps = (mode == MODE_A || mode == MODE_AH);
    if (needs_eps && !eps) return fail(VIE_E_ARG, "vie_matvec: eps_c is required for VIE_OP_A");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_matvec: bad dtype");
    if (recon < VIE_RECON_AUTO || recon > VIE_RECON_FP64) return fail(VIE_E_ARG, "vie_matvec: bad recon");
    if (dtype == VIE_C64 && recon == VIE_RECON_FP64)
        return fail(VIE_E_UNSUPPORTED, "vie_matvec: FP64 reconstruction needs VIE_C128");
    if (dtype == VIE_C128 && (recon == VIE_RECON_FP32 || recon == VIE_RECON_BF16))
        return fail(VIE_E_UNSUPPORTED, "vie_matvec: reduced reconstruction needs VIE_C64");
    size_t need = vie_workspace_bytes(op, dtype, nrhs);
    if (ws_bytes < need) return fail(VIE_E_ARG, "vie_matvec: workspace too small");
    const OpView& v = op->d.view;
    size_t vbytes = (size_t)nrhs * 3 * v.n[0] * v.n[1] * v.n[2] * (dtype == VIE_C128 ? 16 : 8);
    const char* xb = (const char*)x;
    const char* yb = (const char*)y;
    if (!(xb + vbytes <= yb || yb + vbytes <= xb)) return fail(VIE_E_ARG, "vie_matvec: x and y overlap");
    hipStream_t s = (hipStream_t)stream;
    std::string err;
    hipError_t e;
    if (dtype == VIE_C128)
        e = launch_matvec<double, double>(op->d, mode, 0, (const c2<double>*)eps, (const c2<double>*)x,
                                          (c2<double>*)y, nrhs, (c2<double>*)ws, s, rhs_map, err);
    else
        e = launch_matvec<float, float>(op->d, mode, recon == VIE_RECON_BF16 ? 1 : 0, (const c2<float>*)eps,
                                        (const c2<float>*)x,
                                        (c2<float>*)y, nrhs, (c2<float>*)ws, s, rhs_map, err);
    if (e != hipSuccess) {
        if (!err.empty()) return fail(VIE_E_UNSUPPORTED, "vie_matvec: " + err);
        return hip_fail(e, "vie_matvec launch");
    }
    return VIE_OK;
}

}  // namespace vie

extern "C" {

vie_status vie_matvec(const vie_op* op, int kind, int dtype, int recon, const void* eps_c, const void* x, void* y,
                      int nrhs, void* ws, size_t ws_bytes, void* stream)
{
    if (kind != VIE_OP_A && kind != VIE_OP_N) return fail(VIE_E_ARG, "vie_matvec: bad kind");
    return matvec_common(op, kind == VIE_OP_A ? MODE_A : MODE_N, dtype, recon, eps_c, x, y, nrhs, ws, ws_bytes,
                         stream, nullptr);
}

vie_status vie_matvec_adjoint(const vie_op* op, int kind, int dtype, int recon, const void* eps_c, const void* x,
                              void* y, int nrhs, void* ws, size_t ws_bytes, void* stream)
{
    if (kind != VIE_OP_A && kind != VIE_OP_N) return fail(VIE_E_ARG, "vie_matvec_adjoint: bad kind");
    return matvec_common(op, kind == VIE_OP_A ? MODE_AH : MODE_NH, dtype, recon, eps_c, x, y, nrhs, ws, ws_bytes,
                         stream, nullptr);
}

static size_t align_up256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t vie_jm_workspace_bytes(const vie_op* op_n, const vie_op* op_k, int dtype)
{
    if (!op_n || !op_k || (dtype != VIE_C64 && dtype != VIE_C128)) return 0;
    const OpView& v = op_n->d.view;
    const size_t vec = (size_t)2 * 3 * v.n[0] * v.n[1] * v.n[2] * (dtype == VIE_C128 ? 16 : 8);
    const size_t mv = std::max(vie_workspace_bytes(op_n, dtype, 2), vie_workspace_bytes(op_k, dtype, 2));
    return 2 * align_up256(vec) + mv;
}

vie_status vie_matvec_jm(const vie_op* op_n, const vie_op* op_k, int dtype, double h, double omega, const void* eps_c,
                         const void* mu_c, const void* x, void* y, void* ws, size_t ws_bytes, void* stream)
{
    if (!op_n || !op_k || !eps_c || !mu_c || !x || !y || !ws || !(h > 0) || !(omega > 0))
        return fail(VIE_E_ARG, "vie_matvec_jm: bad argument");
    if (op_n->d.view.fam != 0 || op_k->d.view.fam != 1)
        return fail(VIE_E_ARG, "vie_matvec_jm: needs an N operator and a K operator");
    const OpView& v = op_n->d.view;
    for (int a = 0; a < 3; ++a)
        if (op_k->d.view.n[a] != v.n[a]) return fail(VIE_E_ARG, "vie_matvec_jm: N and K grids differ");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_matvec_jm: bad dtype");
    const size_t need = vie_jm_workspace_bytes(op_n, op_k, dtype);
    if (ws_bytes < need) return fail(VIE_E_ARG, "vie_matvec_jm: workspace too small");
    const long nv = (long)v.n[0] * v.n[1] * v.n[2];
    const size_t vec = (size_t)2 * 3 * nv * (dtype == VIE_C128 ? 16 : 8);
    const char* xb = (const char*)x;
    const char* yb = (const char*)y;
    if (!(xb + vec <= yb || yb + vec <= xb)) return fail(VIE_E_ARG, "vie_matvec_jm: x and y overlap");
    char* w = (char*)ws;
    void* NX = w;
    void* KX = w + align_up256(vec);
    void* mw = w + 2 * align_up256(vec);
    const size_t mb = ws_bytes - 2 * align_up256(vec);
    // [J; M] as two right-hand sides of each operator
    vie_status st;
    if (jm_mixed_products && dtype == VIE_C128) {
        // FP64 vectors, products computed in FP32 (the inner operator of a
        // refined solve)
        std::string err;
        hipError_t he = launch_matvec<double, float>(op_n->d, MODE_N, 0, nullptr, (const c2<double>*)x,
                                                     (c2<double>*)NX, 2, (c2<float>*)mw, (hipStream_t)stream,
                                                     nullptr, err);
        if (he == hipSuccess)
            he = launch_matvec<double, float>(op_k->d, MODE_N, 0, nullptr, (const c2<double>*)x, (c2<double>*)KX, 2,
                                              (c2<float>*)mw, (hipStream_t)stream, nullptr, err);
        if (he != hipSuccess) return err.empty() ? hip_fail(he, "vie_matvec_jm") : fail(VIE_E_UNSUPPORTED, err);
    } else {
        st = matvec_common(op_n, MODE_N, dtype, VIE_RECON_AUTO, nullptr, x, NX, 2, mw, mb, stream, nullptr);
        if (st != VIE_OK) return st;
        st = matvec_common(op_k, MODE_N, dtype, VIE_RECON_AUTO, nullptr, x, KX, 2, mw, mb, stream, nullptr);
        if (st != VIE_OK) return st;
    }
    const double EPS0 = 8.8541878128e-12, C0 = 299792458.0;
    const double MU0 = 1.0 / (EPS0 * C0 * C0);
    hipError_t e;
    if (dtype == VIE_C128)
        e = kr_jm_combine<double>((const c2<double>*)eps_c, (const c2<double>*)mu_c, (const c2<double>*)x,
                                  (const c2<double>*)NX, (const c2<double>*)KX, omega * EPS0 * h, omega * MU0 * h,
                                  (c2<double>*)y, nv, 3, (hipStream_t)stream);
    else
        e = kr_jm_combine<float>((const c2<float>*)eps_c, (const c2<float>*)mu_c, (const c2<float>*)x,
                                 (const c2<float>*)NX, (const c2<float>*)KX, omega * EPS0 * h, omega * MU0 * h,
                                 (c2<float>*)y, nv, 3, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "vie_matvec_jm");
    return VIE_OK;
}

// Buffer sizes (complex elements per right-hand side) of the pass layouts.
static size_t pass_elems(const OpView& v, int which)
{
    const size_t n1 = v.n[0], n2 = v.n[1], n3 = v.n[2], L1 = v.L[0], L2 = v.L[1];
    switch (which) {
    case 0: return 3 * n3 * n2 * n1;   // vector [3][n3][n2][n1]
    case 1: return 3 * n3 * L1 * n2;   // S1 / S3 [3][n3][L1][n2]
    default: return 3 * L2 * L1 * n3;  // S2 [3][L2][L1][n3]
    }
}

static bool disjoint(const void* a, size_t na, const void* b, size_t nb)
{
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa + na <= pb || pb + nb <= pa;
}

static vie_status debug_pass_common(const char* who, const vie_op* op, int pass, int mode, int dtype, int recon,
                                    const void* eps_c, const void* x, const void* in, void* out, int nrhs,
                                    void* stream, bool ident)
{
    std::string w(who);
    if (!op || !out || nrhs < 1) return fail(VIE_E_ARG, w + ": null argument or nrhs < 1");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, w + ": bad dtype");
    if (pass < 0 || pass > 4) return fail(VIE_E_ARG, w + ": pass must be 0..4");
    const OpView& v = op->d.view;
    if (v.fam != 0 && (mode != MODE_N || recon == VIE_RECON_BF16))
        return fail(VIE_E_UNSUPPORTED, w + ": a K operator has the bare forward product only");
    const bool needs_eps = mode == MODE_A || mode == MODE_AH;
    const bool needs_x = pass == 0 || (pass == 4 && needs_eps);
    if (needs_x && !x) return fail(VIE_E_ARG, w + ": x is required by this pass and mode");
    if (((pass == 0 && mode == MODE_AH) || (pass == 4 && needs_eps)) && !eps_c)
        return fail(VIE_E_ARG, w + ": eps_c is required by this pass and mode");
    if (pass != 0 && !in) return fail(VIE_E_ARG, w + ": in is required by passes 1..4");
    if (recon < VIE_RECON_AUTO || recon > VIE_RECON_FP64) return fail(VIE_E_ARG, w + ": bad recon");
    if ((dtype == VIE_C64 && recon == VIE_RECON_FP64) ||
        (dtype == VIE_C128 && (recon == VIE_RECON_FP32 || recon == VIE_RECON_BF16)))
        return fail(VIE_E_UNSUPPORTED, w + ": recon does not match dtype");
    if (recon == VIE_RECON_BF16 && (g_kernel_path != 0 || !bf16_recon_available(op->d)))
        return fail(VIE_E_UNSUPPORTED, w + ": BF16 reconstruction is not available for this operator");
    const size_t el = dtype == VIE_C128 ? 16 : 8;
    static const int in_layout[5] = {0, 1, 2, 2, 1};
    static const int out_layout[5] = {1, 2, 2, 1, 0};
    const size_t nin = pass_elems(v, in_layout[pass]) * nrhs * el;
    const size_t nout = pass_elems(v, out_layout[pass]) * nrhs * el;
    if (pass != 2) {
        if (pass != 0 && !disjoint(in, nin, out, nout)) return fail(VIE_E_ARG, w + ": in and out overlap");
        if (x && pass == 0 && !disjoint(x, nin, out, nout)) return fail(VIE_E_ARG, w + ": x and out overlap");
        if (x && pass == 4 && !disjoint(x, nout, out, nout)) return fail(VIE_E_ARG, w + ": x and out overlap");
    } else if (in != out && !disjoint(in, nin, out, nout)) {
        return fail(VIE_E_ARG, w + ": in and out partly overlap");
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (pass == 2 && in != out) e = hipMemcpyAsync(out, in, nin, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, w.c_str());
    std::string err;
    if (dtype == VIE_C128)
        e = run_pass<double, double>(op->d, pass, mode, 0, (const c2<double>*)eps_c, (const c2<double>*)x, in, out,
                                     nrhs, s, nullptr, err, ident);
    else
        e = run_pass<float, float>(op->d, pass, mode, recon == VIE_RECON_BF16 ? 1 : 0, (const c2<float>*)eps_c,
                                   (const c2<float>*)x, in, out, nrhs, s, nullptr, err, ident);
    if (e != hipSuccess) {
        if (!err.empty()) return fail(VIE_E_UNSUPPORTED, w + ": " + err);
        return hip_fail(e, w.c_str());
    }
    return VIE_OK;
}

vie_status vie_debug_pad(const vie_op* op, int dtype, const void* x, void* s1, int nrhs, void* stream)
{
    if (!x) return fail(VIE_E_ARG, "vie_debug_pad: null argument");
    return debug_pass_common("vie_debug_pad", op, 0, MODE_N, dtype, VIE_RECON_AUTO, nullptr, x, nullptr, s1, nrhs,
                             stream, true);
}

vie_status vie_debug_crop(const vie_op* op, int dtype, const void* s3, void* y, int nrhs, void* stream)
{
    if (!s3) return fail(VIE_E_ARG, "vie_debug_crop: null argument");
    return debug_pass_common("vie_debug_crop", op, 4, MODE_N, dtype, VIE_RECON_AUTO, nullptr, nullptr, s3, y, nrhs,
                             stream, true);
}

vie_status vie_debug_pass(const vie_op* op, int pass, int kind, int adjoint, int dtype, int recon,
                          const void* eps_c, const void* x, const void* in, void* out, int nrhs, void* stream)
{
    if (kind != VIE_OP_A && kind != VIE_OP_N) return fail(VIE_E_ARG, "vie_debug_pass: bad kind");
    const int mode = kind == VIE_OP_A ? (adjoint ? MODE_AH : MODE_A) : (adjoint ? MODE_NH : MODE_N);
    return debug_pass_common("vie_debug_pass", op, pass, mode, dtype, recon, eps_c, x, in, out, nrhs, stream, false);
}

vie_status vie_debug_nhat(const vie_op* op, int dtype, int recon, const int* idx, int count, double* out)
{
    if (!op || !idx || !out || count < 0) return fail(VIE_E_ARG, "vie_debug_nhat: bad argument");
    (void)recon;
    if (count == 0) return VIE_OK;
    const OpView& v = op->d.view;
    for (int m = 0; m < count; ++m) {
        if (idx[4 * m] < 0 || idx[4 * m] > 5) return fail(VIE_E_ARG, "vie_debug_nhat: bad component");
        for (int a = 0; a < 3; ++a)
            if (idx[4 * m + 1 + a] < 0 || idx[4 * m + 1 + a] >= v.L[a])
                return fail(VIE_E_ARG, "vie_debug_nhat: index out of range");
    }
    int* didx = nullptr;
    double* dout = nullptr;
    hipError_t e = hipMalloc((void**)&didx, sizeof(int) * 4 * count);
    if (e == hipSuccess) e = hipMalloc((void**)&dout, sizeof(double) * 2 * count);
    if (e == hipSuccess) e = hipMemcpy(didx, idx, sizeof(int) * 4 * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_nhat_samples(op->d, dtype == VIE_C128 ? 1 : 0, didx, count, dout, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, dout, sizeof(double) * 2 * count, hipMemcpyDeviceToHost);
    (void)hipFree(didx);
    (void)hipFree(dout);
    if (e != hipSuccess) return hip_fail(e, "vie_debug_nhat");
    return VIE_OK;
}

vie_status vie_debug_hosvd(const int n[3], const double* tensor, double tol, int rule, int ranks[3], double* svals,
                           double* recon, double* tail)
{
    if (!n || !tensor || !ranks) return fail(VIE_E_ARG, "vie_debug_hosvd: null argument");
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || n[a] > 512) return fail(VIE_E_ARG, "vie_debug_hosvd: bad size");
    if (!(tol > 0) || (rule != 0 && rule != 1)) return fail(VIE_E_ARG, "vie_debug_hosvd: bad tol/rule");
    using cd = std::complex<double>;
    long V = (long)n[0] * n[1] * n[2];
    std::vector<cd> A(V);
    for (long t = 0; t < V; ++t) A[t] = cd(tensor[2 * t], tensor[2 * t + 1]);
    TuckerComponent tc;
    hosvd_component(A.data(), n, tol, rule, 0, tc);
    for (int a = 0; a < 3; ++a) ranks[a] = tc.r[a];
    if (svals) {
        int off = 0;
        for (int a = 0; a < 3; ++a)
            for (int k = 0; k < n[a]; ++k) svals[off++] = tc.sv[a][k];
    }
    if (tail) *tail = tc.tail_rel;
    if (recon) {
        int r1 = tc.r[0], r2 = tc.r[1], r3 = tc.r[2];
        for (int k = 0; k < n[2]; ++k)
            for (int j = 0; j < n[1]; ++j)
                for (int i = 0; i < n[0]; ++i) {
                    cd acc = 0;
                    for (int al = 0; al < r1; ++al)
                        for (int be = 0; be < r2; ++be)
                            for (int ga = 0; ga < r3; ++ga)
                                acc += tc.G[((size_t)al * r2 + be) * r3 + ga] * tc.U[0][(size_t)i * r1 + al] *
                                       tc.U[1][(size_t)j * r2 + be] * tc.U[2][(size_t)k * r3 + ga];
                    long t = ((long)k * n[1] + j) * n[0] + i;
                    recon[2 * t] = acc.real();
                    recon[2 * t + 1] = acc.imag();
                }
    }
    return VIE_OK;
}

vie_status vie_debug_cp(const int r[3], const double* core, int R, int iters, double* V, double* rel_err)
{
    if (!r || !core || !V) return fail(VIE_E_ARG, "vie_debug_cp: null argument");
    for (int a = 0; a < 3; ++a)
        if (r[a] < 1 || r[a] > 64) return fail(VIE_E_ARG, "vie_debug_cp: bad core size");
    if (R < 1 || R > 64 || iters < 0) return fail(VIE_E_ARG, "vie_debug_cp: bad CP rank or iteration count");
    using cd = std::complex<double>;
    const size_t nG = (size_t)r[0] * r[1] * r[2];
    std::vector<cd> G(nG);
    for (size_t t = 0; t < nG; ++t) G[t] = cd(core[2 * t], core[2 * t + 1]);
    std::vector<cd> Vf[3];
    const double e = cp_als(G, r, R, iters, Vf);
    size_t off = 0;
    for (int a = 0; a < 3; ++a)
        for (const cd& x : Vf[a]) {
            V[2 * off] = x.real();
            V[2 * off + 1] = x.imag();
            ++off;
        }
    if (rel_err) *rel_err = e;
    return VIE_OK;
}

vie_status vie_profile_enable(int on)
{
    prof_enable(on);
    return VIE_OK;
}

vie_status vie_profile_collect(double ms[5], int counts[5])
{
    if (!ms || !counts) return fail(VIE_E_ARG, "vie_profile_collect: null argument");
    int bad = prof_collect(ms, counts, 5);
    if (bad) return fail(VIE_E_HIP, "vie_profile_collect: event query failed");
    return VIE_OK;
}

vie_status vie_set_kernel_path(int path)
{
    if (path != 0 && path != 1) return fail(VIE_E_ARG, "vie_set_kernel_path: 0 or 1");
    g_kernel_path = path;
    return VIE_OK;
}

vie_status vie_set_batch_mode(int mode)
{
    if (mode != 0 && mode != 1) return fail(VIE_E_ARG, "vie_set_batch_mode: 0 or 1");
    g_batch_mode = mode;
    return VIE_OK;
}

vie_status vie_autotune(vie_op* op, int dtype, int nrhs, void* ws, size_t ws_bytes, void* stream, double ms[4],
                        int* chosen)
{
    if (!op || !ws || nrhs < 1) return fail(VIE_E_ARG, "vie_autotune: null argument or nrhs < 1");
    if (op->d.view.fam != 0) return fail(VIE_E_UNSUPPORTED, "vie_autotune: N operators only");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_autotune: bad dtype");
    if (ws_bytes < vie_workspace_bytes(op, dtype, nrhs)) return fail(VIE_E_ARG, "vie_autotune: workspace too small");
    if (ms)
        for (int k = 0; k < 4; ++k) ms[k] = 0.0;
    DeviceOp& d = op->d;
    const OpView& v = d.view;
    if (chosen) *chosen = d.zchunk;
    if (g_kernel_path != 0 || (v.L[2] != 128 && v.L[2] != 256 && v.L[2] != 512)) return VIE_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t el = dtype == VIE_C128 ? sizeof(c2<double>) : sizeof(c2<float>);
    const size_t s2 = (size_t)3 * v.L[1] * v.L[0] * v.n[2] * nrhs;
    hipError_t e = hipMemsetAsync(ws, 0, s2 * el, s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int cand[4] = {4, 8, 16, 32};
    const int keep = d.zchunk;
    int best_c = keep;
    double best = 1e300;
    auto run = [&]() -> bool {
        if (dtype == VIE_C128)
            return z_pass_fast<double>(d, MODE_A, 0, nrhs, (c2<double>*)ws, d.tw64[2], d.d64.core, d.d64.fac,
                                       d.dense64, s);
        return z_pass_fast<float>(d, MODE_A, 0, nrhs, (c2<float>*)ws, d.tw32[2], d.d32.core, d.d32.fac, d.dense32,
                                  s);
    };
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
        d.zchunk = cand[k];
        if (!run()) continue;   // shape not launchable (LDS): leave 0
        e = hipEventRecord(e0, s);
        const int reps = 3;
        bool ok = true;
        for (int r = 0; r < reps && ok; ++r) ok = run();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess || !ok) break;
        const double per = (double)t / reps;
        if (ms) ms[k] = per;
        if (per < best) {
            best = per;
            best_c = cand[k];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    d.zchunk = e == hipSuccess ? best_c : keep;
    if (e != hipSuccess) return hip_fail(e, "vie_autotune");
    if (chosen) *chosen = d.zchunk;
    return VIE_OK;
}

}  // extern "C"

struct vie_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

vie_status vie_matvec_graph(const vie_op* op, int kind, int adjoint, int dtype, int recon, const void* eps_c,
                            const void* x, void* y, int nrhs, void* ws, size_t ws_bytes, vie_graph** out)
{
    if (!out) return fail(VIE_E_ARG, "vie_matvec_graph: null output");
    *out = nullptr;
    if (kind != VIE_OP_A && kind != VIE_OP_N) return fail(VIE_E_ARG, "vie_matvec_graph: bad kind");
    if (prof_is_enabled()) return fail(VIE_E_ARG, "vie_matvec_graph: disable per-pass profiling before capturing");
    const int mode = kind == VIE_OP_A ? (adjoint ? MODE_AH : MODE_A) : (adjoint ? MODE_NH : MODE_N);
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "vie_matvec_graph stream");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "vie_matvec_graph capture");
    }
    vie_status st = matvec_common(op, mode, dtype, recon, eps_c, x, y, nrhs, ws, ws_bytes, cs, nullptr);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (st < 0) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess || !g) return hip_fail(e == hipSuccess ? hipErrorUnknown : e, "vie_matvec_graph end");
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "vie_matvec_graph instantiate");
    }
    vie_graph* h = new vie_graph;
    h->graph = g;
    h->exec = ge;
    *out = h;
    return VIE_OK;
}

vie_status vie_graph_launch(vie_graph* g, void* stream)
{
    if (!g || !g->exec) return fail(VIE_E_ARG, "vie_graph_launch: null graph");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "vie_graph_launch");
    return VIE_OK;
}

vie_status vie_graph_destroy(vie_graph* g)
{
    if (!g) return VIE_OK;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return VIE_OK;
}

}  // extern "C"
