// GMRES(m) for one system of a single operator: the full JMVIE system of
// eq. 4, unknown x = [J; M] (2 x 3 x n3 x n2 x n1 complex), operator
// vie_matvec_jm (the N and K products of J and M combined with the electric
// and magnetic contrasts); and the electric block in the piecewise-linear
// basis (12 x n3 x n2 x n1, operator vie_matvec_pwl).
// The Krylov basis stays on the device; classical Gram-Schmidt with a second
// pass on every step, dots accumulated in FP64 (krylov.hip); the Hessenberg
// column and Givens rotations on the host; restart on the true residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "../../include/vie.h"
#include "krylov.h"
#include "vie_internal.h"

namespace vie {
vie_status fail(vie_status st, const std::string& msg);
vie_status hip_fail(hipError_t e, const char* where);
vie_status pwl_apply_mixed(const vie_pwl_op* op, int mode, const void* eps, const void* x, void* y, void* ws,
                           hipStream_t s);

namespace {

using cd = std::complex<double>;

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device buffers of one GMRES(m) solve of n unknowns whose operator needs
// `opws` bytes of workspace.
struct KLayout {
    size_t V, R, op, partial, h1, h2, coef, nrm, map, total;
};

KLayout k_layout(long n, size_t opws, int dtype, int m)
{
    const size_t ek = dtype == VIE_C128 ? 16 : 8;
    KLayout L;
    size_t off = 0;
    L.V = off;
    off += al256((size_t)(m + 1) * n * ek);
    L.R = off;
    off += al256((size_t)n * ek);
    L.op = off;
    off += al256(opws);
    L.partial = off;
    off += al256((size_t)(m + 2) * krylov_nblk(n) * 16);
    L.h1 = off;
    off += al256((size_t)(m + 2) * 16);
    L.h2 = off;
    off += al256((size_t)(m + 2) * 16);
    L.coef = off;
    off += al256((size_t)(m + 1) * 16);
    L.nrm = off;
    off += al256(16);
    L.map = off;
    off += al256(sizeof(int));
    L.total = off;
    return L;
}

KLayout jm_layout(const vie_op* op_n, const vie_op* op_k, int dtype, int m)
{
    const OpView& v = op_n->d.view;
    return k_layout(6L * v.n[0] * v.n[1] * v.n[2], vie_jm_workspace_bytes(op_n, op_k, dtype), dtype, m);
}

// GMRES(m) on n unknowns: apply(in, out) is the operator (the restart
// residual), apply_inner(in, out) the one of the Arnoldi steps (the same, or
// FP32 products on FP64 vectors when refining); `who` names the entry point
// in errors.
template <typename TK, typename FA, typename FI>
vie_status gmres_run(long n, const KLayout& L, FA apply, FI apply_inner, bool refine, const c2<TK>* b, c2<TK>* x,
                     const vie_solve_opts& o, vie_solve_info* info, char* ws, hipStream_t st, const char* who)
{
    const int m = o.restart;
    c2<TK>* V = (c2<TK>*)(ws + L.V);
    c2<TK>* R = (c2<TK>*)(ws + L.R);
    c2<double>* partial = (c2<double>*)(ws + L.partial);
    c2<double>* dh1 = (c2<double>*)(ws + L.h1);
    c2<double>* dh2 = (c2<double>*)(ws + L.h2);
    c2<double>* dcoef = (c2<double>*)(ws + L.coef);
    c2<double>* dnrm = (c2<double>*)(ws + L.nrm);
    int* dmap = (int*)(ws + L.map);
    hipError_t e;
    auto sync_copy = [&](void* dst, const void* src, size_t bytes) {
        hipError_t er = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st);
        return er == hipSuccess ? hipStreamSynchronize(st) : er;
    };
    const int zero = 0;
    if ((e = hipMemcpyAsync(dmap, &zero, sizeof(int), hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_fail(e, who);
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, who);
    vie_solve_info inf{};
    if (info) {
        inf.history = info->history;
        inf.hist_cap = info->hist_cap;
    }
    c2<double> hn;
    if ((e = kr_norm2<TK>(b, 0, n, n, dmap, 1, partial, dnrm, st)) != hipSuccess) return hip_fail(e, "norm");
    if ((e = sync_copy(&hn, dnrm, sizeof(hn))) != hipSuccess) return hip_fail(e, "norm copy");
    const double bnorm = std::sqrt(hn.x);
    if (!std::isfinite(bnorm)) return fail(VIE_E_NONFINITE, std::string(who) + ": non-finite right-hand side");
    if ((e = hipMemsetAsync(x, 0, sizeof(c2<TK>) * n, st)) != hipSuccess) return hip_fail(e, who);
    vie_status status = VIE_NOT_CONVERGED;
    if (bnorm == 0.0) {
        inf.converged = 1;
        status = VIE_OK;
    }
    std::vector<cd> H((size_t)(m + 1) * m), g(m + 1), sn(m);
    std::vector<double> cs(m);
    std::vector<c2<double>> h1(m + 2), h2(m + 2);
    for (int outer = 0; bnorm > 0.0; ++outer) {
        // true residual R = b - A x
        vie_status s = apply(x, R);
        if (s != VIE_OK) return s;
        if (refine) inf.matvecs_fp64++;
        else inf.matvecs++;
        if ((e = kr_residual<TK>(R, b, n, n, dmap, 1, st)) != hipSuccess) return hip_fail(e, "residual");
        if ((e = kr_norm2<TK>(R, 0, n, n, dmap, 1, partial, dnrm, st)) != hipSuccess) return hip_fail(e, "norm");
        if ((e = sync_copy(&hn, dnrm, sizeof(hn))) != hipSuccess) return hip_fail(e, "norm copy");
        const double beta = std::sqrt(hn.x);
        if (!std::isfinite(beta)) return fail(VIE_E_NONFINITE, std::string(who) + ": non-finite residual");
        inf.rel_residual = beta / bnorm;
        if (inf.history && inf.hist_len < inf.hist_cap) inf.history[inf.hist_len++] = inf.rel_residual;
        if (inf.rel_residual <= o.tol) {
            inf.converged = 1;
            status = VIE_OK;
            break;
        }
        if (outer >= o.max_outer) break;
        if ((e = kr_scale_norm<TK>(V, 0, R, 0, n, dnrm, n, dmap, 1, st)) != hipSuccess) return hip_fail(e, "scale");
        std::fill(H.begin(), H.end(), cd(0.0));
        std::fill(g.begin(), g.end(), cd(0.0));
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            const long wo = (long)(j + 1) * n;
            if ((s = apply_inner(V + (long)j * n, V + wo)) != VIE_OK) return s;
            inf.matvecs++;
            // two classical Gram-Schmidt passes; the first also returns ||w||^2
            e = kr_mdot<TK>(V, n, n, j + 2, V, wo, n, dmap, 1, partial, dh1, st);
            if (e == hipSuccess) e = kr_maxpy<TK>(V, wo, n, V, n, n, j + 1, j + 2, dh1, -1.0, n, dmap, 1, st);
            if (e == hipSuccess) e = kr_mdot<TK>(V, n, n, j + 1, V, wo, n, dmap, 1, partial, dh2, st);
            if (e == hipSuccess) e = kr_maxpy<TK>(V, wo, n, V, n, n, j + 1, j + 1, dh2, -1.0, n, dmap, 1, st);
            if (e == hipSuccess) e = kr_norm2<TK>(V, wo, n, n, dmap, 1, partial, dnrm, st);
            if (e == hipSuccess) e = hipMemcpyAsync(h1.data(), dh1, sizeof(c2<double>) * (j + 2), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipMemcpyAsync(h2.data(), dh2, sizeof(c2<double>) * (j + 1), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = sync_copy(&hn, dnrm, sizeof(hn));
            if (e != hipSuccess) return hip_fail(e, who);
            cd* Hc = &H[(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) Hc[i] = cd(h1[i].x + h2[i].x, h1[i].y + h2[i].y);
            const double hj1 = std::sqrt(std::max(hn.x, 0.0));
            Hc[j + 1] = hj1;
            if (hj1 > 0.0) {
                if ((e = kr_scale_norm<TK>(V, wo, V, wo, n, dnrm, n, dmap, 1, st)) != hipSuccess)
                    return hip_fail(e, "scale");
            }
            // earlier rotations, then a new one that zeroes H[j+1][j]
            for (int i = 0; i < j; ++i) {
                const cd a = Hc[i], bb = Hc[i + 1];
                Hc[i] = cs[i] * a + sn[i] * bb;
                Hc[i + 1] = -std::conj(sn[i]) * a + cs[i] * bb;
            }
            {
                const cd a = Hc[j], bb = Hc[j + 1];
                double c;
                cd sv;
                if (std::abs(bb) == 0.0) {
                    c = 1.0;
                    sv = 0.0;
                } else if (std::abs(a) == 0.0) {
                    c = 0.0;
                    sv = 1.0;
                } else {
                    const double t = std::hypot(std::abs(a), std::abs(bb));
                    c = std::abs(a) / t;
                    sv = (a / std::abs(a)) * std::conj(bb) / t;
                }
                cs[j] = c;
                sn[j] = sv;
                Hc[j] = c * a + sv * bb;
                Hc[j + 1] = 0.0;
                g[j + 1] = -std::conj(sv) * g[j];
                g[j] = c * g[j];
            }
            k = j + 1;
            // refinement: each cycle asks for a relative reduction inner_tol
            const double stop = refine ? std::max(o.inner_tol * beta, 0.5 * o.tol * bnorm) : 0.5 * o.tol * bnorm;
            if (std::abs(g[j + 1]) <= stop || hj1 == 0.0) break;
        }
        // y = H(0:k, 0:k)^-1 g(0:k), x += V y
        std::vector<c2<double>> y(k);
        for (int i = k - 1; i >= 0; --i) {
            cd acc = g[i];
            for (int c = i + 1; c < k; ++c) acc -= H[(size_t)c * (m + 1) + i] * cd(y[c].x, y[c].y);
            const cd yi = acc / H[(size_t)i * (m + 1) + i];
            y[i] = mk<double>(yi.real(), yi.imag());
        }
        if ((e = hipMemcpyAsync(dcoef, y.data(), sizeof(c2<double>) * k, hipMemcpyHostToDevice, st)) != hipSuccess)
            return hip_fail(e, "coef");
        if ((e = kr_maxpy<TK>(x, 0, n, V, n, n, k, k, dcoef, 1.0, n, dmap, 1, st)) != hipSuccess)
            return hip_fail(e, "update");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "update");
        inf.restarts++;
        if (refine) inf.refine_steps++;
    }
    if (info) *info = inf;
    return status;
}

template <typename TK>
vie_status run_jm(const vie_op* op_n, const vie_op* op_k, int dtype, double h, double omega, const void* eps_c,
                  const void* mu_c, const c2<TK>* b, c2<TK>* x, const vie_solve_opts& o, vie_solve_info* info,
                  char* ws, hipStream_t st)
{
    const OpView& v = op_n->d.view;
    const long n = 6L * v.n[0] * v.n[1] * v.n[2];
    const KLayout L = jm_layout(op_n, op_k, dtype, o.restart);
    void* jw = ws + L.op;
    const size_t jwb = vie_jm_workspace_bytes(op_n, op_k, dtype);
    // refinement (o.refine, complex128 vectors): the Arnoldi steps use the
    // operator with FP32 products, the restart residual the FP64 one
    const bool refine = o.refine && sizeof(TK) == 8;
    auto apply_prec = [&](const c2<TK>* in, c2<TK>* out, bool mixed) {
        jm_mixed_products = mixed;
        vie_status r = vie_matvec_jm(op_n, op_k, dtype, h, omega, eps_c, mu_c, in, out, jw, jwb, st);
        jm_mixed_products = false;
        return r;
    };
    auto apply = [&](const c2<TK>* in, c2<TK>* out) { return apply_prec(in, out, false); };
    auto apply_inner = [&](const c2<TK>* in, c2<TK>* out) { return apply_prec(in, out, refine); };
    return gmres_run<TK>(n, L, apply, apply_inner, refine, b, x, o, info, ws, st, "vie_solve_jm");
}

KLayout pwl_layout(const vie_pwl_op* op, int dtype, int m)
{
    const OpView& v = op->blk[0]->d.view;
    return k_layout(12L * v.n[0] * v.n[1] * v.n[2], vie_pwl_workspace_bytes(op, dtype, 1), dtype, m);
}

template <typename TK>
vie_status run_pwl(const vie_pwl_op* op, int dtype, const void* eps_c, const c2<TK>* b, c2<TK>* x,
                   const vie_solve_opts& o, vie_solve_info* info, char* ws, hipStream_t st)
{
    const OpView& v = op->blk[0]->d.view;
    const long n = 12L * v.n[0] * v.n[1] * v.n[2];
    const KLayout L = pwl_layout(op, dtype, o.restart);
    void* pw = ws + L.op;
    const size_t pwb = vie_pwl_workspace_bytes(op, dtype, 1);
    const int mode = o.adjoint ? MODE_AH : MODE_A;
    const bool refine = o.refine && sizeof(TK) == 8;
    auto apply = [&](const c2<TK>* in, c2<TK>* out) {
        return vie_matvec_pwl(op, VIE_OP_A, o.adjoint, dtype, eps_c, in, out, 1, pw, pwb, (void*)st);
    };
    auto apply_inner = [&](const c2<TK>* in, c2<TK>* out) {
        if (refine) return pwl_apply_mixed(op, mode, eps_c, in, out, pw, st);
        return vie_matvec_pwl(op, VIE_OP_A, o.adjoint, dtype, eps_c, in, out, 1, pw, pwb, (void*)st);
    };
    return gmres_run<TK>(n, L, apply, apply_inner, refine, b, x, o, info, ws, st, "vie_solve_pwl");
}

KLayout jm_pwl_layout(const vie_pwl_op* op_n, const vie_pwl_op* op_k, int dtype, int m)
{
    const OpView& v = op_n->blk[0]->d.view;
    return k_layout(24L * v.n[0] * v.n[1] * v.n[2], vie_jm_pwl_workspace_bytes(op_n, op_k, dtype), dtype, m);
}

template <typename TK>
vie_status run_jm_pwl(const vie_pwl_op* op_n, const vie_pwl_op* op_k, int dtype, double h, double omega,
                      const void* eps_c, const void* mu_c, const c2<TK>* b, c2<TK>* x, const vie_solve_opts& o,
                      vie_solve_info* info, char* ws, hipStream_t st)
{
    const OpView& v = op_n->blk[0]->d.view;
    const long n = 24L * v.n[0] * v.n[1] * v.n[2];
    const KLayout L = jm_pwl_layout(op_n, op_k, dtype, o.restart);
    void* jw = ws + L.op;
    const size_t jwb = vie_jm_pwl_workspace_bytes(op_n, op_k, dtype);
    const bool refine = o.refine && sizeof(TK) == 8;
    auto apply_prec = [&](const c2<TK>* in, c2<TK>* out, bool mixed) {
        jm_mixed_products = mixed;
        vie_status r = vie_matvec_jm_pwl(op_n, op_k, dtype, h, omega, eps_c, mu_c, in, out, jw, jwb, st);
        jm_mixed_products = false;
        return r;
    };
    auto apply = [&](const c2<TK>* in, c2<TK>* out) { return apply_prec(in, out, false); };
    auto apply_inner = [&](const c2<TK>* in, c2<TK>* out) { return apply_prec(in, out, refine); };
    return gmres_run<TK>(n, L, apply, apply_inner, refine, b, x, o, info, ws, st, "vie_solve_jm_pwl");
}

}  // namespace
}  // namespace vie

using namespace vie;

extern "C" {

size_t vie_solve_jm_workspace_bytes(const vie_op* op_n, const vie_op* op_k, int dtype, const vie_solve_opts* opts)
{
    if (!op_n || !op_k || (dtype != VIE_C64 && dtype != VIE_C128)) return 0;
    const int m = opts ? opts->restart : 50;
    if (m < 1 || m > 200) return 0;
    return jm_layout(op_n, op_k, dtype, m).total;
}

vie_status vie_solve_jm(const vie_op* op_n, const vie_op* op_k, int dtype, double h, double omega, const void* eps_c,
                        const void* mu_c, const void* b, void* x, const vie_solve_opts* opts, vie_solve_info* info,
                        void* ws, size_t ws_bytes, void* stream)
{
    if (!op_n || !op_k || !eps_c || !mu_c || !b || !x || !ws || !(h > 0) || !(omega > 0))
        return fail(VIE_E_ARG, "vie_solve_jm: bad argument");
    if (op_n->d.view.fam != 0 || op_k->d.view.fam != 1)
        return fail(VIE_E_ARG, "vie_solve_jm: needs an N operator and a K operator");
    vie_solve_opts o;
    o.tol = 1e-6;
    o.restart = 50;
    o.max_outer = 200;
    o.adjoint = 0;
    o.refine = 0;
    o.inner_recon = VIE_RECON_FP32;
    o.inner_tol = 1e-4;
    if (opts) o = *opts;
    if (!(o.tol > 0) || o.restart < 1 || o.restart > 200 || o.max_outer < 0)
        return fail(VIE_E_ARG, "vie_solve_jm: bad options");
    if (o.adjoint) return fail(VIE_E_UNSUPPORTED, "vie_solve_jm: forward solves only");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_solve_jm: bad dtype");
    if (o.refine && (dtype != VIE_C128 || !(o.inner_tol > 0 && o.inner_tol < 1)))
        return fail(VIE_E_ARG, "vie_solve_jm: refinement needs VIE_C128 vectors and inner_tol in (0, 1)");
    if (ws_bytes < vie_solve_jm_workspace_bytes(op_n, op_k, dtype, &o))
        return fail(VIE_E_ARG, "vie_solve_jm: workspace too small");
    if (info && info->history && info->hist_cap < 0) return fail(VIE_E_ARG, "vie_solve_jm: bad history capacity");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == VIE_C128)
        return run_jm<double>(op_n, op_k, dtype, h, omega, eps_c, mu_c, (const c2<double>*)b, (c2<double>*)x, o, info,
                              (char*)ws, st);
    return run_jm<float>(op_n, op_k, dtype, h, omega, eps_c, mu_c, (const c2<float>*)b, (c2<float>*)x, o, info,
                         (char*)ws, st);
}

size_t vie_solve_pwl_workspace_bytes(const vie_pwl_op* op, int dtype, const vie_solve_opts* opts)
{
    if (!op || !op->blk[0] || (dtype != VIE_C64 && dtype != VIE_C128)) return 0;
    const int m = opts ? opts->restart : 50;
    if (m < 1 || m > 200) return 0;
    return pwl_layout(op, dtype, m).total;
}

vie_status vie_solve_pwl(const vie_pwl_op* op, int dtype, const void* eps_c, const void* b, void* x,
                         const vie_solve_opts* opts, vie_solve_info* info, void* ws, size_t ws_bytes, void* stream)
{
    if (!op || !op->blk[0] || !eps_c || !b || !x || !ws) return fail(VIE_E_ARG, "vie_solve_pwl: null argument");
    if (op->fam != 0) return fail(VIE_E_UNSUPPORTED, "vie_solve_pwl: the operator is a K operator");
    vie_solve_opts o;
    o.tol = 1e-6;
    o.restart = 50;
    o.max_outer = 200;
    o.adjoint = 0;
    o.refine = 0;
    o.inner_recon = VIE_RECON_FP32;
    o.inner_tol = 1e-4;
    if (opts) o = *opts;
    if (!(o.tol > 0) || o.restart < 1 || o.restart > 200 || o.max_outer < 0 || (o.adjoint != 0 && o.adjoint != 1) ||
        (o.refine != 0 && o.refine != 1))
        return fail(VIE_E_ARG, "vie_solve_pwl: bad options");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_solve_pwl: bad dtype");
    if (o.refine && (dtype != VIE_C128 || !(o.inner_tol > 0 && o.inner_tol < 1)))
        return fail(VIE_E_ARG, "vie_solve_pwl: refinement needs VIE_C128 vectors and inner_tol in (0, 1)");
    if (o.refine && o.inner_recon != VIE_RECON_FP32)
        return fail(VIE_E_UNSUPPORTED, "vie_solve_pwl: refinement takes FP32 inner products only");
    if (ws_bytes < vie_solve_pwl_workspace_bytes(op, dtype, &o))
        return fail(VIE_E_ARG, "vie_solve_pwl: workspace too small");
    if (info && info->history && info->hist_cap < 0) return fail(VIE_E_ARG, "vie_solve_pwl: bad history capacity");
    const OpView& v = op->blk[0]->d.view;
    const size_t vbytes = (size_t)12 * v.n[0] * v.n[1] * v.n[2] * (dtype == VIE_C128 ? 16 : 8);
    const char* xb = (const char*)x;
    const char* bb = (const char*)b;
    if (!(xb + vbytes <= bb || bb + vbytes <= xb)) return fail(VIE_E_ARG, "vie_solve_pwl: x and b overlap");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == VIE_C128)
        return run_pwl<double>(op, dtype, eps_c, (const c2<double>*)b, (c2<double>*)x, o, info, (char*)ws, st);
    return run_pwl<float>(op, dtype, eps_c, (const c2<float>*)b, (c2<float>*)x, o, info, (char*)ws, st);
}

size_t vie_solve_jm_pwl_workspace_bytes(const vie_pwl_op* op_n, const vie_pwl_op* op_k, int dtype,
                                        const vie_solve_opts* opts)
{
    if (!op_n || !op_k || !op_n->blk[0] || !op_k->blk[0] || (dtype != VIE_C64 && dtype != VIE_C128)) return 0;
    const int m = opts ? opts->restart : 50;
    if (m < 1 || m > 200) return 0;
    return jm_pwl_layout(op_n, op_k, dtype, m).total;
}

vie_status vie_solve_jm_pwl(const vie_pwl_op* op_n, const vie_pwl_op* op_k, int dtype, double h, double omega,
                            const void* eps_c, const void* mu_c, const void* b, void* x, const vie_solve_opts* opts,
                            vie_solve_info* info, void* ws, size_t ws_bytes, void* stream)
{
    if (!op_n || !op_k || !op_n->blk[0] || !op_k->blk[0] || !eps_c || !mu_c || !b || !x || !ws || !(h > 0) ||
        !(omega > 0))
        return fail(VIE_E_ARG, "vie_solve_jm_pwl: bad argument");
    if (op_n->fam != 0 || op_k->fam != 1)
        return fail(VIE_E_ARG, "vie_solve_jm_pwl: needs an N operator and a K operator");
    vie_solve_opts o;
    o.tol = 1e-6;
    o.restart = 50;
    o.max_outer = 200;
    o.adjoint = 0;
    o.refine = 0;
    o.inner_recon = VIE_RECON_FP32;
    o.inner_tol = 1e-4;
    if (opts) o = *opts;
    if (!(o.tol > 0) || o.restart < 1 || o.restart > 200 || o.max_outer < 0)
        return fail(VIE_E_ARG, "vie_solve_jm_pwl: bad options");
    if (o.adjoint) return fail(VIE_E_UNSUPPORTED, "vie_solve_jm_pwl: forward solves only");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_solve_jm_pwl: bad dtype");
    if (o.refine && (dtype != VIE_C128 || !(o.inner_tol > 0 && o.inner_tol < 1)))
        return fail(VIE_E_ARG, "vie_solve_jm_pwl: refinement needs VIE_C128 vectors and inner_tol in (0, 1)");
    if (o.refine && o.inner_recon != VIE_RECON_FP32)
        return fail(VIE_E_UNSUPPORTED, "vie_solve_jm_pwl: refinement takes FP32 inner products only");
    if (ws_bytes < vie_solve_jm_pwl_workspace_bytes(op_n, op_k, dtype, &o))
        return fail(VIE_E_ARG, "vie_solve_jm_pwl: workspace too small");
    if (info && info->history && info->hist_cap < 0) return fail(VIE_E_ARG, "vie_solve_jm_pwl: bad history capacity");
    const OpView& v = op_n->blk[0]->d.view;
    const size_t vbytes = (size_t)24 * v.n[0] * v.n[1] * v.n[2] * (dtype == VIE_C128 ? 16 : 8);
    const char* xb = (const char*)x;
    const char* bb = (const char*)b;
    if (!(xb + vbytes <= bb || bb + vbytes <= xb)) return fail(VIE_E_ARG, "vie_solve_jm_pwl: x and b overlap");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == VIE_C128)
        return run_jm_pwl<double>(op_n, op_k, dtype, h, omega, eps_c, mu_c, (const c2<double>*)b, (c2<double>*)x, o,
                                  info, (char*)ws, st);
    return run_jm_pwl<float>(op_n, op_k, dtype, h, omega, eps_c, mu_c, (const c2<float>*)b, (c2<float>*)x, o, info,
                             (char*)ws, st);
}

}  // extern "C"
