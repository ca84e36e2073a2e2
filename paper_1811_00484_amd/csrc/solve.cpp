// Restarted GMRES on the device for batches of independent right-hand sides
// (the paper's solver, Sec. VI-C: relative tolerance, restart length, outer
// limit), with an optional iterative-refinement mode:
//
//   plain   : every cycle restarts from the true residual r = b - A x in the
//             working precision; Arnoldi with classical Gram-Schmidt plus one
//             re-orthogonalisation pass (CGS2) in the working precision.
//   refine  : the true residual is formed with the FP64 operator; each cycle
//             solves A d = r approximately with FP64 Arnoldi on the FP32-
//             computed operator, and x += d.  Stops on the FP64 true residual.
//
// Vector work runs in the batched kernels of krylov.hip; the (m+1) x m
// Hessenberg matrices, their Givens rotations and the triangular solves are
// tiny and stay on the host (one device-to-host copy of j+2 coefficients per
// Arnoldi step and system).
#include <hip/hip_runtime.h>

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

namespace {

using cd = std::complex<double>;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Layout {
    size_t V, R, mws, partial, h1, h2, coef, nrm, map, total;
};

Layout layout(const DeviceOp& op, int dtype, int nrhs, int m, int refine)
{
    const OpView& v = op.view;
    long n = 3L * v.n[0] * v.n[1] * v.n[2];
    size_t ek = dtype == VIE_C128 ? 16 : 8;
    size_t mv_el = matvec_ws_elems(op, nrhs);
    size_t mv_bytes = mv_el * (dtype == VIE_C128 && !refine ? 16 : 8);
    if (refine) mv_bytes = mv_el * 16;   // FP64 residual matvec; the FP32 inner matvec uses half of it
    Layout L;
    size_t off = 0;
    L.V = off;
    off += align256((size_t)(m + 1) * nrhs * n * ek);
    L.R = off;
    off += align256((size_t)nrhs * n * ek);
    L.mws = off;
    off += align256(mv_bytes);
    L.partial = off;
    off += align256((size_t)nrhs * (m + 1) * krylov_nblk(n) * 16);
    L.h1 = off;
    off += align256((size_t)nrhs * (m + 1) * 16);
    L.h2 = off;
    off += align256((size_t)nrhs * (m + 1) * 16);
    L.coef = off;
    off += align256((size_t)nrhs * (m + 1) * 16);
    L.nrm = off;
    off += align256((size_t)nrhs * 16);
    L.map = off;
    off += align256((size_t)nrhs * 4);
    L.total = off;
    return L;
}

void givens(cd a, cd b, double& c, cd& s)
{
    if (b == 0.0) {
        c = 1.0;
        s = 0.0;
        return;
    }
    if (a == 0.0) {
        c = 0.0;
        s = 1.0;
        return;
    }
    double t = std::hypot(std::abs(a), std::abs(b));
    c = std::abs(a) / t;
    s = (a / std::abs(a)) * std::conj(b) / t;
}

struct SysState {
    std::vector<cd> H;   // (m+1) x m, column-major H[i + j*(m+1)]
    std::vector<cd> g;
    std::vector<double> cs;
    std::vector<cd> sn;
    int k = 0;           // Arnoldi steps completed in this cycle
    bool in_cycle = false;
    double beta0 = 0;
};

template <typename TK, typename TC>
vie_status run(const vie_op* opw, int mode, const c2<TK>* eps, const c2<TK>* b, c2<TK>* x, int nrhs,
               const vie_solve_opts& o, vie_solve_info* info, char* ws, const Layout& Lt, hipStream_t st)
{
    const DeviceOp& op = opw->d;
    const OpView& v = op.view;
    const long n = 3L * v.n[0] * v.n[1] * v.n[2];
    const int m = o.restart;
    const long sstride = n, vstride = (long)nrhs * n;
    c2<TK>* Vb = (c2<TK>*)(ws + Lt.V);
    c2<TK>* R = (c2<TK>*)(ws + Lt.R);
    void* mws = ws + Lt.mws;
    c2<double>* partial = (c2<double>*)(ws + Lt.partial);
    c2<double>* dh1 = (c2<double>*)(ws + Lt.h1);
    c2<double>* dh2 = (c2<double>*)(ws + Lt.h2);
    c2<double>* dcoef = (c2<double>*)(ws + Lt.coef);
    c2<double>* dnrm = (c2<double>*)(ws + Lt.nrm);
    int* dmap = (int*)(ws + Lt.map);
    hipError_t e;
    std::string err;

    auto upload_map = [&](const std::vector<int>& mp) -> hipError_t {
        hipError_t er = hipMemcpyAsync(dmap, mp.data(), sizeof(int) * mp.size(), hipMemcpyHostToDevice, st);
        if (er != hipSuccess) return er;
        return hipStreamSynchronize(st);
    };
    // matvec of the working (inner) operator, or of the FP64 residual operator
    auto mv_inner = [&](const c2<TK>* xin, c2<TK>* yout, int nact) -> hipError_t {
        return launch_matvec<TK, TC>(op, mode, 0, eps, xin, yout, nact, (c2<TC>*)mws, st, dmap, err);
    };
    auto mv_resid = [&](const c2<TK>* xin, c2<TK>* yout, int nact) -> hipError_t {
        if (o.refine) {
            if constexpr (sizeof(TK) == 8)
                return launch_matvec<double, double>(op, mode, 0, (const c2<double>*)eps, (const c2<double>*)xin,
                                                     (c2<double>*)yout, nact, (c2<double>*)mws, st, dmap, err);
        }
        return mv_inner(xin, yout, nact);
    };

    std::vector<double> bnorm(nrhs, 0.0);
    std::vector<int> all(nrhs);
    for (int s = 0; s < nrhs; ++s) all[s] = s;
    if ((e = upload_map(all)) != hipSuccess) return hip_fail(e, "vie_solve map");
    if ((e = kr_norm2<TK>(b, 0, sstride, n, dmap, nrhs, partial, dnrm, st)) != hipSuccess)
        return hip_fail(e, "vie_solve norm");
    {
        std::vector<c2<double>> h(nrhs);
        e = hipMemcpyAsync(h.data(), dnrm, sizeof(c2<double>) * nrhs, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "vie_solve norm copy");
        for (int s = 0; s < nrhs; ++s) {
            bnorm[s] = std::sqrt(h[s].x);
            if (!std::isfinite(bnorm[s])) return fail(VIE_E_NONFINITE, "vie_solve: non-finite right-hand side");
        }
    }
    std::vector<bool> conv(nrhs, false);
    std::vector<double> relres(nrhs, INFINITY);
    std::vector<int> mvs(nrhs, 0), mv64(nrhs, 0), cycles(nrhs, 0), steps(nrhs, 0);
    if (info)
        for (int s = 0; s < nrhs; ++s) info[s].hist_len = 0;
    // b == 0 -> x = 0 solves it
    for (int s = 0; s < nrhs; ++s)
        if (bnorm[s] == 0.0) {
            conv[s] = true;
            relres[s] = 0.0;
            (void)hipMemsetAsync(x + s * sstride, 0, sizeof(c2<TK>) * n, st);
        }
    std::vector<SysState> S(nrhs);
    for (auto& ss : S) {
        ss.H.assign((size_t)(m + 1) * m, 0.0);
        ss.g.assign(m + 1, 0.0);
        ss.cs.assign(m, 0.0);
        ss.sn.assign(m, 0.0);
    }
    bool nonfinite = false;

    for (int outer = 0;; ++outer) {
        std::vector<int> act;
        for (int s = 0; s < nrhs; ++s)
            if (!conv[s]) act.push_back(s);
        if (act.empty()) break;
        int na = (int)act.size();
        if ((e = upload_map(act)) != hipSuccess) return hip_fail(e, "vie_solve map");
        // ---- true residual R = b - A x
        if ((e = mv_resid(x, R, na)) != hipSuccess)
            return err.empty() ? hip_fail(e, "vie_solve matvec") : fail(VIE_E_UNSUPPORTED, err);
        for (int s : act) (o.refine ? mv64[s] : mvs[s])++;
        if ((e = kr_residual<TK>(R, b, sstride, n, dmap, na, st)) != hipSuccess) return hip_fail(e, "residual");
        if ((e = kr_norm2<TK>(R, 0, sstride, n, dmap, na, partial, dnrm, st)) != hipSuccess)
            return hip_fail(e, "norm");
        std::vector<c2<double>> hn(na);
        e = hipMemcpyAsync(hn.data(), dnrm, sizeof(c2<double>) * na, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "vie_solve copy");
        std::vector<int> cyc;
        for (int a = 0; a < na; ++a) {
            int s = act[a];
            double beta = std::sqrt(hn[a].x);
            if (!std::isfinite(beta)) {
                nonfinite = true;
                continue;
            }
            relres[s] = beta / bnorm[s];
            if (info && info[s].history && info[s].hist_len < info[s].hist_cap)
                info[s].history[info[s].hist_len++] = relres[s];
            if (relres[s] <= o.tol) {
                conv[s] = true;
                continue;
            }
            if (outer >= o.max_outer) continue;
            S[s].beta0 = beta;
            cyc.push_back(s);
        }
        if (nonfinite) return fail(VIE_E_NONFINITE, "vie_solve: non-finite residual");
        if (cyc.empty()) break;
        // ---- one GMRES(m) cycle on the systems in `cyc`
        int nc = (int)cyc.size();
        if ((e = upload_map(cyc)) != hipSuccess) return hip_fail(e, "vie_solve map");
        // V0 = R / beta: norms of R for the cyc systems are recomputed in cyc order
        if ((e = kr_norm2<TK>(R, 0, sstride, n, dmap, nc, partial, dnrm, st)) != hipSuccess)
            return hip_fail(e, "norm");
        if ((e = kr_scale_norm<TK>(Vb, 0, R, 0, sstride, dnrm, n, dmap, nc, st)) != hipSuccess)
            return hip_fail(e, "scale");
        for (int s : cyc) {
            SysState& ss = S[s];
            std::fill(ss.H.begin(), ss.H.end(), cd(0.0));
            std::fill(ss.g.begin(), ss.g.end(), cd(0.0));
            ss.g[0] = ss.beta0;
            ss.k = 0;
            ss.in_cycle = true;
        }
        std::vector<int> run_list = cyc;
        for (int j = 0; j < m && !run_list.empty(); ++j) {
            int nr = (int)run_list.size();
            if ((e = upload_map(run_list)) != hipSuccess) return hip_fail(e, "vie_solve map");
            c2<TK>* Vj = Vb + (long)j * vstride;
            c2<TK>* Vj1 = Vb + (long)(j + 1) * vstride;
            if ((e = mv_inner(Vj, Vj1, nr)) != hipSuccess)
                return err.empty() ? hip_fail(e, "vie_solve matvec") : fail(VIE_E_UNSUPPORTED, err);
            for (int s : run_list) mvs[s]++;
            // CGS2
            const long wvoff = (long)(j + 1) * vstride;
            e = kr_mdot<TK>(Vb, vstride, sstride, j + 1, Vb, wvoff, n, dmap, nr, partial, dh1, st);
            if (e == hipSuccess)
                e = kr_maxpy<TK>(Vb, wvoff, sstride, Vb, vstride, sstride, j + 1, j + 1, dh1, -1.0, n, dmap, nr, st);
            if (e == hipSuccess)
                e = kr_mdot<TK>(Vb, vstride, sstride, j + 1, Vb, wvoff, n, dmap, nr, partial, dh2, st);
            if (e == hipSuccess)
                e = kr_maxpy<TK>(Vb, wvoff, sstride, Vb, vstride, sstride, j + 1, j + 1, dh2, -1.0, n, dmap, nr, st);
            if (e == hipSuccess) e = kr_norm2<TK>(Vb, wvoff, sstride, n, dmap, nr, partial, dnrm, st);
            if (e == hipSuccess) e = kr_scale_norm<TK>(Vb, wvoff, Vb, wvoff, sstride, dnrm, n, dmap, nr, st);
            if (e != hipSuccess) return hip_fail(e, "vie_solve arnoldi");
            std::vector<c2<double>> h1((size_t)nr * (j + 1)), h2((size_t)nr * (j + 1)), hb(nr);
            e = hipMemcpyAsync(h1.data(), dh1, sizeof(c2<double>) * h1.size(), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(h2.data(), dh2, sizeof(c2<double>) * h2.size(), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipMemcpyAsync(hb.data(), dnrm, sizeof(c2<double>) * nr, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_fail(e, "vie_solve copy");
            std::vector<int> next;
            for (int a = 0; a < nr; ++a) {
                int s = run_list[a];
                SysState& ss = S[s];
                cd* Hc = &ss.H[(size_t)j * (m + 1)];
                for (int i = 0; i <= j; ++i) {
                    c2<double> t1 = h1[(size_t)a * (j + 1) + i], t2 = h2[(size_t)a * (j + 1) + i];
                    Hc[i] = cd(t1.x + t2.x, t1.y + t2.y);
                }
                double beta = std::sqrt(hb[a].x);
                Hc[j + 1] = beta;
                bool finite = std::isfinite(beta);
                for (int i = 0; i <= j; ++i) finite = finite && std::isfinite(Hc[i].real()) && std::isfinite(Hc[i].imag());
                if (!finite) {
                    nonfinite = true;
                    break;
                }
                for (int i = 0; i < j; ++i) {
                    cd aa = Hc[i], bb = Hc[i + 1];
                    Hc[i] = ss.cs[i] * aa + ss.sn[i] * bb;
                    Hc[i + 1] = -std::conj(ss.sn[i]) * aa + ss.cs[i] * bb;
                }
                givens(Hc[j], Hc[j + 1], ss.cs[j], ss.sn[j]);
                cd aa = Hc[j], bb = Hc[j + 1];
                Hc[j] = ss.cs[j] * aa + ss.sn[j] * bb;
                Hc[j + 1] = 0.0;
                ss.g[j + 1] = -std::conj(ss.sn[j]) * ss.g[j];
                ss.g[j] = ss.cs[j] * ss.g[j];
                ss.k = j + 1;
                steps[s]++;
                double est = std::abs(ss.g[j + 1]);
                double target = o.tol * bnorm[s];
                if (o.refine) target = std::max(o.inner_tol * ss.beta0, 0.5 * o.tol * bnorm[s]);
                bool stop = est <= target || beta == 0.0 || std::abs(Hc[j]) == 0.0;
                if (!stop) next.push_back(s);
            }
            if (nonfinite) return fail(VIE_E_NONFINITE, "vie_solve: non-finite Arnoldi quantity");
            run_list = next;
        }
        // ---- x += V y for every system of the cycle
        int kmax = 0;
        std::vector<c2<double>> coef((size_t)nc * m);
        for (int a = 0; a < nc; ++a) {
            SysState& ss = S[cyc[a]];
            int k = ss.k;
            kmax = std::max(kmax, k);
            std::vector<cd> y(k);
            for (int i = k - 1; i >= 0; --i) {
                cd acc = ss.g[i];
                for (int t = i + 1; t < k; ++t) acc -= ss.H[(size_t)t * (m + 1) + i] * y[t];
                cd d = ss.H[(size_t)i * (m + 1) + i];
                y[i] = std::abs(d) > 0.0 ? acc / d : cd(0.0);
            }
            for (int i = 0; i < m; ++i) {
                cd yy = i < k ? y[i] : cd(0.0);
                coef[(size_t)a * m + i].x = yy.real();
                coef[(size_t)a * m + i].y = yy.imag();
            }
            cycles[cyc[a]]++;
        }
        if ((e = upload_map(cyc)) != hipSuccess) return hip_fail(e, "vie_solve map");
        e = hipMemcpyAsync(dcoef, coef.data(), sizeof(c2<double>) * coef.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess && kmax > 0)
            e = kr_maxpy<TK>(x, 0, sstride, Vb, vstride, sstride, kmax, m, dcoef, 1.0, n, dmap, nc, st);
        if (e != hipSuccess) return hip_fail(e, "vie_solve update");
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "vie_solve sync");
    bool all_conv = true;
    for (int s = 0; s < nrhs; ++s) {
        all_conv = all_conv && conv[s];
        if (info) {
            info[s].matvecs = mvs[s];
            info[s].matvecs_fp64 = mv64[s];
            info[s].restarts = cycles[s];
            info[s].refine_steps = o.refine ? cycles[s] : 0;
            info[s].converged = conv[s] ? 1 : 0;
            info[s].rel_residual = relres[s];
        }
    }
    return all_conv ? VIE_OK : VIE_NOT_CONVERGED;
}

vie_solve_opts defaults(const vie_solve_opts* o)
{
    vie_solve_opts d;
    d.tol = 1e-6;
    d.restart = 50;
    d.max_outer = 200;
    d.adjoint = 0;
    d.refine = 0;
    d.inner_recon = VIE_RECON_FP32;
    d.inner_tol = 1e-4;
    return o ? *o : d;
}

}  // namespace
}  // namespace vie

using namespace vie;

extern "C" {

size_t vie_solve_workspace_bytes(const vie_op* op, int dtype, int nrhs, const vie_solve_opts* opts)
{
    if (!op || nrhs < 1) return 0;
    vie_solve_opts o = defaults(opts);
    if (o.restart < 1 || o.restart > 200) return 0;
    return layout(op->d, dtype, nrhs, o.restart, o.refine).total;
}

vie_status vie_solve(const vie_op* op, int dtype, const void* eps_c, const void* b, void* x, int nrhs,
                     const vie_solve_opts* opts, vie_solve_info* info, void* ws, size_t ws_bytes, void* stream)
{
    if (!op || !eps_c || !b || !x || !ws || nrhs < 1) return fail(VIE_E_ARG, "vie_solve: null argument or nrhs < 1");
    vie_solve_opts o = defaults(opts);
    if (!(o.tol > 0) || o.restart < 1 || o.restart > 200 || o.max_outer < 0 || (o.refine != 0 && o.refine != 1))
        return fail(VIE_E_ARG, "vie_solve: bad options");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_solve: bad dtype");
    if (o.refine && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_solve: refinement needs VIE_C128 vectors");
    if (o.refine && !(o.inner_tol > 0 && o.inner_tol < 1)) return fail(VIE_E_ARG, "vie_solve: inner_tol in (0, 1)");
    if (o.refine && o.inner_recon != VIE_RECON_FP32)
        return fail(VIE_E_UNSUPPORTED, "vie_solve: inner reconstruction must be FP32 in this build");
    Layout Lt = layout(op->d, dtype, nrhs, o.restart, o.refine);
    if (ws_bytes < Lt.total) return fail(VIE_E_ARG, "vie_solve: workspace too small");
    const OpView& v = op->d.view;
    size_t vbytes = (size_t)nrhs * 3 * v.n[0] * v.n[1] * v.n[2] * (dtype == VIE_C128 ? 16 : 8);
    const char* xb = (const char*)x;
    const char* bb = (const char*)b;
    if (!(xb + vbytes <= bb || bb + vbytes <= xb)) return fail(VIE_E_ARG, "vie_solve: x and b overlap");
    int mode = o.adjoint ? MODE_AH : MODE_A;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == VIE_C64)
        return run<float, float>(op, mode, (const c2<float>*)eps_c, (const c2<float>*)b, (c2<float>*)x, nrhs, o,
                                 info, (char*)ws, Lt, st);
    if (o.refine)
        return run<double, float>(op, mode, (const c2<double>*)eps_c, (const c2<double>*)b, (c2<double>*)x, nrhs,
                                  o, info, (char*)ws, Lt, st);
    return run<double, double>(op, mode, (const c2<double>*)eps_c, (const c2<double>*)b, (c2<double>*)x, nrhs, o,
                               info, (char*)ws, Lt, st);
}

vie_status vie_field_gradient(const vie_op* op, int dtype, const void* z, const void* E, double omega_eps0,
                              void* g_eps, void* g_sigma, void* stream)
{
    if (!op || !z || !E || !g_eps || !g_sigma || !(omega_eps0 > 0))
        return fail(VIE_E_ARG, "vie_field_gradient: bad argument");
    const OpView& v = op->d.view;
    long V = (long)v.n[0] * v.n[1] * v.n[2];
    hipError_t e;
    if (dtype == VIE_C128)
        e = kr_field_gradient<double>((const c2<double>*)z, (const c2<double>*)E, (double*)g_eps, (double*)g_sigma,
                                      omega_eps0, V, (hipStream_t)stream);
    else if (dtype == VIE_C64)
        e = kr_field_gradient<float>((const c2<float>*)z, (const c2<float>*)E, (float*)g_eps, (float*)g_sigma,
                                     omega_eps0, V, (hipStream_t)stream);
    else
        return fail(VIE_E_ARG, "vie_field_gradient: bad dtype");
    if (e != hipSuccess) return hip_fail(e, "vie_field_gradient");
    return VIE_OK;
}

vie_status vie_problem_setup(const vie_op* op, int dtype, const void* eps_r, const void* sigma, const void* e_inc,
                             double omega_eps0, void* eps_c, void* b, void* stream)
{
    if (!op || !eps_r || !sigma || !e_inc || !eps_c || !b || !(omega_eps0 > 0))
        return fail(VIE_E_ARG, "vie_problem_setup: bad argument");
    const OpView& v = op->d.view;
    long V = (long)v.n[0] * v.n[1] * v.n[2];
    hipError_t e;
    if (dtype == VIE_C128)
        e = kr_problem<double>((const double*)eps_r, (const double*)sigma, (const c2<double>*)e_inc,
                               (c2<double>*)eps_c, (c2<double>*)b, omega_eps0, V, (hipStream_t)stream);
    else if (dtype == VIE_C64)
        e = kr_problem<float>((const float*)eps_r, (const float*)sigma, (const c2<float>*)e_inc, (c2<float>*)eps_c,
                              (c2<float>*)b, omega_eps0, V, (hipStream_t)stream);
    else
        return fail(VIE_E_ARG, "vie_problem_setup: bad dtype");
    if (e != hipSuccess) return hip_fail(e, "vie_problem_setup");
    return VIE_OK;
}

vie_status vie_total_field(const vie_op* op, int dtype, const void* e_inc, const void* u, const void* Nu,
                           double omega_eps0, void* E, void* stream)
{
    if (!op || !e_inc || !u || !Nu || !E || !(omega_eps0 > 0)) return fail(VIE_E_ARG, "vie_total_field: bad argument");
    const OpView& v = op->d.view;
    long n = 3L * v.n[0] * v.n[1] * v.n[2];
    hipError_t e;
    if (dtype == VIE_C128)
        e = kr_total_field<double>((const c2<double>*)e_inc, (const c2<double>*)u, (const c2<double>*)Nu,
                                   (c2<double>*)E, omega_eps0, n, (hipStream_t)stream);
    else if (dtype == VIE_C64)
        e = kr_total_field<float>((const c2<float>*)e_inc, (const c2<float>*)u, (const c2<float>*)Nu, (c2<float>*)E,
                                  omega_eps0, n, (hipStream_t)stream);
    else
        return fail(VIE_E_ARG, "vie_total_field: bad dtype");
    if (e != hipSuccess) return hip_fail(e, "vie_total_field");
    return VIE_OK;
}

vie_status vie_adjoint_source(const vie_op* op, int dtype, const void* g, const void* NHg, void* t, void* stream)
{
    if (!op || !g || !NHg || !t) return fail(VIE_E_ARG, "vie_adjoint_source: bad argument");
    const OpView& v = op->d.view;
    long n = 3L * v.n[0] * v.n[1] * v.n[2];
    hipError_t e;
    if (dtype == VIE_C128)
        e = kr_adjoint_source<double>((const c2<double>*)g, (const c2<double>*)NHg, (c2<double>*)t, n,
                                      (hipStream_t)stream);
    else if (dtype == VIE_C64)
        e = kr_adjoint_source<float>((const c2<float>*)g, (const c2<float>*)NHg, (c2<float>*)t, n, (hipStream_t)stream);
    else
        return fail(VIE_E_ARG, "vie_adjoint_source: bad dtype");
    if (e != hipSuccess) return hip_fail(e, "vie_adjoint_source");
    return VIE_OK;
}

}  // extern "C"
