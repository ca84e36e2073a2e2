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

// Per-instance state of a (possibly multi-instance) batched GMRES solve.
// Selective re-orthogonalisation threshold: the second Gram-Schmidt pass is
// skipped when ||w'|| >= kReorthEta ||w||.  Used for FP64 bases when the
// cycle's target is loose enough (refinement inner cycles, or tol >= 1e-10)
// that an orthogonality loss of ~1e-13 per vector cannot matter.
constexpr double kReorthEta = 1e-3;

template <typename TK>
struct Inst {
    const DeviceOp* op = nullptr;
    const c2<TK>* eps = nullptr;
    const c2<TK>* b = nullptr;
    c2<TK>* x = nullptr;
    int nrhs = 0;
    vie_solve_info* info = nullptr;
    long n = 0;
    Layout Lt;
    char* ws = nullptr;
    c2<TK>* V = nullptr;
    c2<TK>* R = nullptr;
    void* mws = nullptr;
    c2<double>* partial = nullptr;
    c2<double>* dh1 = nullptr;
    c2<double>* dh2 = nullptr;
    c2<double>* dcoef = nullptr;
    c2<double>* dnrm = nullptr;
    int* dmap = nullptr;
    std::vector<double> bnorm, relres;
    std::vector<char> conv;
    std::vector<int> mvs, mv64, cycles;
    std::vector<SysState> S;
    std::vector<int> cyc, run;
    int reorth_steps = 0;   // Arnoldi steps that took the second Gram-Schmidt pass
};

// recon 1: BF16 MFMA reconstruction
template <typename TV, typename T>
hipError_t mv_dispatch(const std::vector<InstHost>& req, int mode, InstDev* tab, hipStream_t st, std::string& err,
                       int recon = 0)
{
    return launch_batch<TV, T>(req, mode, recon, tab, st, err);
}

template <typename TK, typename TC>
vie_status run_multi(std::vector<Inst<TK>>& I, int mode, const vie_solve_opts& o, InstDev* tab, hipStream_t st)
{
    const int m = o.restart;
    const int inner_recon = (o.refine && o.inner_recon == VIE_RECON_BF16) ? 1 : 0;
    const bool selective = sizeof(TK) == 8 && (o.refine || o.tol >= 1e-10);
    hipError_t e;
    std::string err;
    auto upload_map = [&](Inst<TK>& in, const std::vector<int>& mp) -> hipError_t {
        if (mp.empty()) return hipSuccess;
        hipError_t er = hipMemcpyAsync(in.dmap, mp.data(), sizeof(int) * mp.size(), hipMemcpyHostToDevice, st);
        if (er != hipSuccess) return er;
        return hipStreamSynchronize(st);
    };
    auto fetch = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        hipError_t er = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st);
        if (er != hipSuccess) return er;
        return hipStreamSynchronize(st);
    };
    // ---- right-hand side norms, zero right-hand sides
    for (auto& in : I) {
        const long n = in.n;
        std::vector<int> all(in.nrhs);
        for (int s = 0; s < in.nrhs; ++s) all[s] = s;
        if ((e = upload_map(in, all)) != hipSuccess) return hip_fail(e, "vie_solve map");
        if ((e = kr_norm2<TK>(in.b, 0, n, n, in.dmap, in.nrhs, in.partial, in.dnrm, st)) != hipSuccess)
            return hip_fail(e, "vie_solve norm");
        std::vector<c2<double>> h(in.nrhs);
        if ((e = fetch(h.data(), in.dnrm, sizeof(c2<double>) * in.nrhs)) != hipSuccess)
            return hip_fail(e, "vie_solve norm copy");
        in.bnorm.assign(in.nrhs, 0.0);
        in.relres.assign(in.nrhs, INFINITY);
        in.conv.assign(in.nrhs, 0);
        in.mvs.assign(in.nrhs, 0);
        in.mv64.assign(in.nrhs, 0);
        in.cycles.assign(in.nrhs, 0);
        in.S.assign(in.nrhs, SysState());
        for (auto& ss : in.S) {
            ss.H.assign((size_t)(m + 1) * m, 0.0);
            ss.g.assign(m + 1, 0.0);
            ss.cs.assign(m, 0.0);
            ss.sn.assign(m, 0.0);
        }
        if (in.info)
            for (int s = 0; s < in.nrhs; ++s) in.info[s].hist_len = 0;
        for (int s = 0; s < in.nrhs; ++s) {
            in.bnorm[s] = std::sqrt(h[s].x);
            if (!std::isfinite(in.bnorm[s])) return fail(VIE_E_NONFINITE, "vie_solve: non-finite right-hand side");
            if (in.bnorm[s] == 0.0) {
                in.conv[s] = 1;
                in.relres[s] = 0.0;
                (void)hipMemsetAsync(in.x + s * n, 0, sizeof(c2<TK>) * n, st);
            }
        }
    }
    std::vector<InstHost> req;
    for (int outer = 0;; ++outer) {
        // ---- true residual R = b - A x for every unconverged system
        req.clear();
        std::vector<std::vector<int>> act(I.size());
        for (size_t i = 0; i < I.size(); ++i) {
            Inst<TK>& in = I[i];
            for (int s = 0; s < in.nrhs; ++s)
                if (!in.conv[s]) act[i].push_back(s);
            if (act[i].empty()) continue;
            if ((e = upload_map(in, act[i])) != hipSuccess) return hip_fail(e, "vie_solve map");
            req.push_back({in.op, in.x, in.R, in.eps, in.dmap, (int)act[i].size(), in.mws});
        }
        if (req.empty()) break;
        if (o.refine) {
            if constexpr (sizeof(TK) == 8) e = mv_dispatch<double, double>(req, mode, tab, st, err);
        } else {
            e = mv_dispatch<TK, TC>(req, mode, tab, st, err);
        }
        if (e != hipSuccess) return err.empty() ? hip_fail(e, "vie_solve matvec") : fail(VIE_E_UNSUPPORTED, err);
        bool any_cycle = false;
        for (size_t i = 0; i < I.size(); ++i) {
            Inst<TK>& in = I[i];
            in.cyc.clear();
            if (act[i].empty()) continue;
            const int na = (int)act[i].size();
            const long n = in.n;
            for (int s : act[i]) (o.refine ? in.mv64[s] : in.mvs[s])++;
            if ((e = kr_residual<TK>(in.R, in.b, n, n, in.dmap, na, st)) != hipSuccess) return hip_fail(e, "residual");
            if ((e = kr_norm2<TK>(in.R, 0, n, n, in.dmap, na, in.partial, in.dnrm, st)) != hipSuccess)
                return hip_fail(e, "norm");
            std::vector<c2<double>> hn(na);
            if ((e = fetch(hn.data(), in.dnrm, sizeof(c2<double>) * na)) != hipSuccess) return hip_fail(e, "copy");
            for (int a = 0; a < na; ++a) {
                int s = act[i][a];
                double beta = std::sqrt(hn[a].x);
                if (!std::isfinite(beta)) return fail(VIE_E_NONFINITE, "vie_solve: non-finite residual");
                in.relres[s] = beta / in.bnorm[s];
                if (in.info && in.info[s].history && in.info[s].hist_len < in.info[s].hist_cap)
                    in.info[s].history[in.info[s].hist_len++] = in.relres[s];
                if (in.relres[s] <= o.tol) {
                    in.conv[s] = 1;
                    continue;
                }
                if (outer >= o.max_outer) continue;
                in.S[s].beta0 = beta;
                in.cyc.push_back(s);
            }
            if (in.cyc.empty()) continue;
            any_cycle = true;
            const int nc = (int)in.cyc.size();
            if ((e = upload_map(in, in.cyc)) != hipSuccess) return hip_fail(e, "vie_solve map");
            if ((e = kr_norm2<TK>(in.R, 0, n, n, in.dmap, nc, in.partial, in.dnrm, st)) != hipSuccess)
                return hip_fail(e, "norm");
            if ((e = kr_scale_norm<TK>(in.V, 0, in.R, 0, n, in.dnrm, n, in.dmap, nc, st)) != hipSuccess)
                return hip_fail(e, "scale");
            for (int s : in.cyc) {
                SysState& ss = in.S[s];
                std::fill(ss.H.begin(), ss.H.end(), cd(0.0));
                std::fill(ss.g.begin(), ss.g.end(), cd(0.0));
                ss.g[0] = ss.beta0;
                ss.k = 0;
            }
            in.run = in.cyc;
        }
        if (!any_cycle) break;
        // ---- one GMRES(m) cycle, all instances in lockstep
        for (int j = 0; j < m; ++j) {
            req.clear();
            for (auto& in : I) {
                if (in.run.empty()) continue;
                const long vstride = (long)in.nrhs * in.n;
                if ((e = upload_map(in, in.run)) != hipSuccess) return hip_fail(e, "vie_solve map");
                req.push_back({in.op, in.V + (long)j * vstride, in.V + (long)(j + 1) * vstride, in.eps, in.dmap,
                               (int)in.run.size(), in.mws});
            }
            if (req.empty()) break;
            if ((e = mv_dispatch<TK, TC>(req, mode, tab, st, err, inner_recon)) != hipSuccess)
                return err.empty() ? hip_fail(e, "vie_solve matvec") : fail(VIE_E_UNSUPPORTED, err);
            for (auto& in : I) {
                if (in.run.empty()) continue;
                const long n = in.n, vstride = (long)in.nrhs * n;
                const int nr = (int)in.run.size();
                for (int s : in.run) in.mvs[s]++;
                const long wvoff = (long)(j + 1) * vstride;
                // classical Gram-Schmidt; the first pass also returns ||w||^2
                // (w is basis slot j + 1, so it is the last of the j + 2 dots)
                e = kr_mdot<TK>(in.V, vstride, n, j + 2, in.V, wvoff, n, in.dmap, nr, in.partial, in.dh1, st);
                if (e == hipSuccess)
                    e = kr_maxpy<TK>(in.V, wvoff, n, in.V, vstride, n, j + 1, j + 2, in.dh1, -1.0, n, in.dmap, nr, st);
                if (e == hipSuccess) e = kr_norm2<TK>(in.V, wvoff, n, n, in.dmap, nr, in.partial, in.dnrm, st);
                std::vector<c2<double>> h1((size_t)nr * (j + 2)), h2((size_t)nr * (j + 1)), hb(nr);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(h1.data(), in.dh1, sizeof(c2<double>) * h1.size(), hipMemcpyDeviceToHost, st);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(hb.data(), in.dnrm, sizeof(c2<double>) * nr, hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e != hipSuccess) return hip_fail(e, "vie_solve arnoldi");
                // second pass (re-orthogonalisation) unless the first one lost
                // little of w to cancellation: ||w'|| >= eta ||w|| bounds the
                // loss of orthogonality of the new vector by ~ unit roundoff / eta
                // (the Daniel-Gragg-Kaufman-Stewart criterion).  FP32 bases
                // always take both passes.
                bool reorth = !selective;
                for (int a = 0; a < nr && !reorth; ++a) {
                    const double w0 = std::sqrt(std::max(h1[(size_t)a * (j + 2) + j + 1].x, 0.0));
                    const double w1 = std::sqrt(std::max(hb[a].x, 0.0));
                    reorth = !(w1 >= kReorthEta * w0);
                }
                if (reorth) {
                    ++in.reorth_steps;
                    e = kr_mdot<TK>(in.V, vstride, n, j + 1, in.V, wvoff, n, in.dmap, nr, in.partial, in.dh2, st);
                    if (e == hipSuccess)
                        e = kr_maxpy<TK>(in.V, wvoff, n, in.V, vstride, n, j + 1, j + 1, in.dh2, -1.0, n, in.dmap, nr,
                                         st);
                    if (e == hipSuccess) e = kr_norm2<TK>(in.V, wvoff, n, n, in.dmap, nr, in.partial, in.dnrm, st);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(h2.data(), in.dh2, sizeof(c2<double>) * h2.size(), hipMemcpyDeviceToHost,
                                           st);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(hb.data(), in.dnrm, sizeof(c2<double>) * nr, hipMemcpyDeviceToHost, st);
                } else {
                    std::fill(h2.begin(), h2.end(), mk<double>(0, 0));
                }
                if (e == hipSuccess) e = kr_scale_norm<TK>(in.V, wvoff, in.V, wvoff, n, in.dnrm, n, in.dmap, nr, st);
                if (e == hipSuccess && reorth) e = hipStreamSynchronize(st);
                if (e != hipSuccess) return hip_fail(e, "vie_solve arnoldi");
                std::vector<int> next;
                for (int a = 0; a < nr; ++a) {
                    int s = in.run[a];
                    SysState& ss = in.S[s];
                    cd* Hc = &ss.H[(size_t)j * (m + 1)];
                    for (int i2 = 0; i2 <= j; ++i2) {
                        c2<double> t1 = h1[(size_t)a * (j + 2) + i2], t2 = h2[(size_t)a * (j + 1) + i2];
                        Hc[i2] = cd(t1.x + t2.x, t1.y + t2.y);
                    }
                    double beta = std::sqrt(hb[a].x);
                    Hc[j + 1] = beta;
                    bool finite = std::isfinite(beta);
                    for (int i2 = 0; i2 <= j; ++i2)
                        finite = finite && std::isfinite(Hc[i2].real()) && std::isfinite(Hc[i2].imag());
                    if (!finite) return fail(VIE_E_NONFINITE, "vie_solve: non-finite Arnoldi quantity");
                    for (int i2 = 0; i2 < j; ++i2) {
                        cd aa = Hc[i2], bb = Hc[i2 + 1];
                        Hc[i2] = ss.cs[i2] * aa + ss.sn[i2] * bb;
                        Hc[i2 + 1] = -std::conj(ss.sn[i2]) * aa + ss.cs[i2] * bb;
                    }
                    givens(Hc[j], Hc[j + 1], ss.cs[j], ss.sn[j]);
                    cd aa = Hc[j], bb = Hc[j + 1];
                    Hc[j] = ss.cs[j] * aa + ss.sn[j] * bb;
                    Hc[j + 1] = 0.0;
                    ss.g[j + 1] = -std::conj(ss.sn[j]) * ss.g[j];
                    ss.g[j] = ss.cs[j] * ss.g[j];
                    ss.k = j + 1;
                    double est = std::abs(ss.g[j + 1]);
                    double target = o.tol * in.bnorm[s];
                    if (o.refine) target = std::max(o.inner_tol * ss.beta0, 0.5 * o.tol * in.bnorm[s]);
                    bool stop = est <= target || beta == 0.0 || std::abs(Hc[j]) == 0.0;
                    if (!stop) next.push_back(s);
                }
                in.run = next;
            }
        }
        // ---- x += V y for every system of the cycle
        for (auto& in : I) {
            if (in.cyc.empty()) continue;
            const long n = in.n, vstride = (long)in.nrhs * n;
            const int nc = (int)in.cyc.size();
            int kmax = 0;
            std::vector<c2<double>> coef((size_t)nc * m);
            for (int a = 0; a < nc; ++a) {
                SysState& ss = in.S[in.cyc[a]];
                int k = ss.k;
                kmax = std::max(kmax, k);
                std::vector<cd> y(k);
                for (int i2 = k - 1; i2 >= 0; --i2) {
                    cd acc = ss.g[i2];
                    for (int t = i2 + 1; t < k; ++t) acc -= ss.H[(size_t)t * (m + 1) + i2] * y[t];
                    cd d = ss.H[(size_t)i2 * (m + 1) + i2];
                    y[i2] = std::abs(d) > 0.0 ? acc / d : cd(0.0);
                }
                for (int i2 = 0; i2 < m; ++i2) {
                    cd yy = i2 < k ? y[i2] : cd(0.0);
                    coef[(size_t)a * m + i2].x = yy.real();
                    coef[(size_t)a * m + i2].y = yy.imag();
                }
                in.cycles[in.cyc[a]]++;
            }
            if ((e = upload_map(in, in.cyc)) != hipSuccess) return hip_fail(e, "vie_solve map");
            e = hipMemcpyAsync(in.dcoef, coef.data(), sizeof(c2<double>) * coef.size(), hipMemcpyHostToDevice, st);
            if (e == hipSuccess && kmax > 0)
                e = kr_maxpy<TK>(in.x, 0, n, in.V, vstride, n, kmax, m, in.dcoef, 1.0, n, in.dmap, nc, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_fail(e, "vie_solve update");
        }
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "vie_solve sync");
    bool all_conv = true;
    for (auto& in : I)
        for (int s = 0; s < in.nrhs; ++s) {
            all_conv = all_conv && in.conv[s];
            if (in.info) {
                in.info[s].matvecs = in.mvs[s];
                in.info[s].matvecs_fp64 = in.mv64[s];
                in.info[s].restarts = in.cycles[s];
                in.info[s].refine_steps = o.refine ? in.cycles[s] : 0;
                in.info[s].converged = in.conv[s] ? 1 : 0;
                in.info[s].rel_residual = in.relres[s];
            }
        }
    return all_conv ? VIE_OK : VIE_NOT_CONVERGED;
}

template <typename TK>
void bind_ws(Inst<TK>& in, char* ws)
{
    in.ws = ws;
    in.V = (c2<TK>*)(ws + in.Lt.V);
    in.R = (c2<TK>*)(ws + in.Lt.R);
    in.mws = ws + in.Lt.mws;
    in.partial = (c2<double>*)(ws + in.Lt.partial);
    in.dh1 = (c2<double>*)(ws + in.Lt.h1);
    in.dh2 = (c2<double>*)(ws + in.Lt.h2);
    in.dcoef = (c2<double>*)(ws + in.Lt.coef);
    in.dnrm = (c2<double>*)(ws + in.Lt.nrm);
    in.dmap = (int*)(ws + in.Lt.map);
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

// total workspace of a multi-instance solve: one instance table, then each
// instance's own layout, 256-byte aligned
size_t multi_ws_bytes(const vie_solve_instance* in, int count, int dtype, const vie_solve_opts& o)
{
    size_t tot = align256(sizeof(InstDev) * (size_t)count);
    for (int i = 0; i < count; ++i) tot += align256(layout(in[i].op->d, dtype, in[i].nrhs, o.restart, o.refine).total);
    return tot;
}

template <typename TK, typename TC>
vie_status solve_typed(const vie_solve_instance* in, int count, int dtype, const vie_solve_opts& o, int mode, char* ws,
                       hipStream_t st)
{
    std::vector<Inst<TK>> I(count);
    InstDev* tab = (InstDev*)ws;
    size_t off = align256(sizeof(InstDev) * (size_t)count);
    for (int i = 0; i < count; ++i) {
        Inst<TK>& d = I[i];
        d.op = &in[i].op->d;
        d.eps = (const c2<TK>*)in[i].eps_c;
        d.b = (const c2<TK>*)in[i].b;
        d.x = (c2<TK>*)in[i].x;
        d.nrhs = in[i].nrhs;
        d.info = in[i].info;
        d.n = 3L * d.op->view.n[0] * d.op->view.n[1] * d.op->view.n[2];
        d.Lt = layout(*d.op, dtype, d.nrhs, o.restart, o.refine);
        bind_ws(d, ws + off);
        off += align256(d.Lt.total);
    }
    return run_multi<TK, TC>(I, mode, o, tab, st);
}

vie_status solve_instances(const vie_solve_instance* in, int count, int dtype, const vie_solve_opts& o, int mode,
                           char* ws, hipStream_t st)
{
    if (dtype == VIE_C64) return solve_typed<float, float>(in, count, dtype, o, mode, ws, st);
    if (o.refine) return solve_typed<double, float>(in, count, dtype, o, mode, ws, st);
    return solve_typed<double, double>(in, count, dtype, o, mode, ws, st);
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
    vie_solve_instance one{op, nullptr, nullptr, nullptr, nrhs, nullptr};
    return multi_ws_bytes(&one, 1, dtype, o);
}

vie_status vie_solve(const vie_op* op, int dtype, const void* eps_c, const void* b, void* x, int nrhs,
                     const vie_solve_opts* opts, vie_solve_info* info, void* ws, size_t ws_bytes, void* stream)
{
    if (!op || !eps_c || !b || !x || !ws || nrhs < 1) return fail(VIE_E_ARG, "vie_solve: null argument or nrhs < 1");
    if (op->d.view.fam != 0) return fail(VIE_E_UNSUPPORTED, "vie_solve: N operators only");
    vie_solve_opts o = defaults(opts);
    if (!(o.tol > 0) || o.restart < 1 || o.restart > 200 || o.max_outer < 0 || (o.refine != 0 && o.refine != 1))
        return fail(VIE_E_ARG, "vie_solve: bad options");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_solve: bad dtype");
    if (o.refine && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_solve: refinement needs VIE_C128 vectors");
    if (o.refine && !(o.inner_tol > 0 && o.inner_tol < 1)) return fail(VIE_E_ARG, "vie_solve: inner_tol in (0, 1)");
    if (o.refine && o.inner_recon != VIE_RECON_FP32 && o.inner_recon != VIE_RECON_BF16)
        return fail(VIE_E_ARG, "vie_solve: inner_recon must be VIE_RECON_FP32 or VIE_RECON_BF16");
    {
        vie_solve_instance one{op, nullptr, nullptr, nullptr, nrhs, nullptr};
        if (ws_bytes < multi_ws_bytes(&one, 1, dtype, o)) return fail(VIE_E_ARG, "vie_solve: workspace too small");
    }
    const OpView& v = op->d.view;
    size_t vbytes = (size_t)nrhs * 3 * v.n[0] * v.n[1] * v.n[2] * (dtype == VIE_C128 ? 16 : 8);
    const char* xb = (const char*)x;
    const char* bb = (const char*)b;
    if (!(xb + vbytes <= bb || bb + vbytes <= xb)) return fail(VIE_E_ARG, "vie_solve: x and b overlap");
    int mode = o.adjoint ? MODE_AH : MODE_A;
    hipStream_t st = (hipStream_t)stream;
    vie_solve_instance one{op, eps_c, b, x, nrhs, info};
    return solve_instances(&one, 1, dtype, o, mode, (char*)ws, st);
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

vie_status vie_magnetic_field(const vie_op* op_k, int dtype, const void* h_inc, const void* KJ, double h, double mu0,
                              void* H, void* b1, void* stream)
{
    if (!op_k || !h_inc || !KJ || !H || !b1 || !(h > 0) || !(mu0 > 0))
        return fail(VIE_E_ARG, "vie_magnetic_field: bad argument");
    if (op_k->d.view.fam != 1) return fail(VIE_E_ARG, "vie_magnetic_field: needs a K operator (vie_compress_k)");
    const OpView& v = op_k->d.view;
    long nv = (long)v.n[0] * v.n[1] * v.n[2];
    hipError_t e;
    if (dtype == VIE_C128)
        e = kr_magnetic_field<double>((const c2<double>*)h_inc, (const c2<double>*)KJ, h, mu0, (c2<double>*)H,
                                      (double*)b1, nv, (hipStream_t)stream);
    else if (dtype == VIE_C64)
        e = kr_magnetic_field<float>((const c2<float>*)h_inc, (const c2<float>*)KJ, h, mu0, (c2<float>*)H, (float*)b1,
                                     nv, (hipStream_t)stream);
    else
        return fail(VIE_E_ARG, "vie_magnetic_field: bad dtype");
    if (e != hipSuccess) return hip_fail(e, "vie_magnetic_field");
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

static vie_status check_solve_opts(const vie_solve_opts& o, int dtype)
{
    if (!(o.tol > 0) || o.restart < 1 || o.restart > 200 || o.max_outer < 0 || (o.refine != 0 && o.refine != 1))
        return fail(VIE_E_ARG, "vie_solve: bad options");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_solve: bad dtype");
    if (o.refine && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_solve: refinement needs VIE_C128 vectors");
    if (o.refine && !(o.inner_tol > 0 && o.inner_tol < 1)) return fail(VIE_E_ARG, "vie_solve: inner_tol in (0, 1)");
    if (o.refine && o.inner_recon != VIE_RECON_FP32 && o.inner_recon != VIE_RECON_BF16)
        return fail(VIE_E_ARG, "vie_solve: inner_recon must be VIE_RECON_FP32 or VIE_RECON_BF16");
    return VIE_OK;
}

size_t vie_solve_multi_workspace_bytes(const vie_solve_instance* inst, int count, int dtype, const vie_solve_opts* opts)
{
    if (!inst || count < 1) return 0;
    vie_solve_opts o = defaults(opts);
    if (o.restart < 1 || o.restart > 200) return 0;
    for (int i = 0; i < count; ++i)
        if (!inst[i].op || inst[i].nrhs < 1) return 0;
    return multi_ws_bytes(inst, count, dtype, o);
}

vie_status vie_solve_multi(const vie_solve_instance* inst, int count, int dtype, const vie_solve_opts* opts, void* ws,
                           size_t ws_bytes, void* stream)
{
    if (!inst || count < 1 || !ws) return fail(VIE_E_ARG, "vie_solve_multi: bad argument");
    vie_solve_opts o = defaults(opts);
    vie_status st = check_solve_opts(o, dtype);
    if (st != VIE_OK) return st;
    size_t eb = dtype == VIE_C128 ? 16 : 8;
    for (int i = 0; i < count; ++i) {
        const vie_solve_instance& in = inst[i];
        if (!in.op || !in.eps_c || !in.b || !in.x || in.nrhs < 1) return fail(VIE_E_ARG, "vie_solve_multi: bad instance");
        const OpView& v = in.op->d.view;
        if (v.fam != 0) return fail(VIE_E_UNSUPPORTED, "vie_solve_multi: N operators only");
        size_t vb = (size_t)in.nrhs * 3 * v.n[0] * v.n[1] * v.n[2] * eb;
        const char* xb = (const char*)in.x;
        const char* bb = (const char*)in.b;
        if (!(xb + vb <= bb || bb + vb <= xb)) return fail(VIE_E_ARG, "vie_solve_multi: x and b overlap");
    }
    if (ws_bytes < multi_ws_bytes(inst, count, dtype, o)) return fail(VIE_E_ARG, "vie_solve_multi: workspace too small");
    return solve_instances(inst, count, dtype, o, o.adjoint ? MODE_AH : MODE_A, (char*)ws, (hipStream_t)stream);
}

size_t vie_matvec_multi_workspace_bytes(const vie_instance* inst, int count, int dtype)
{
    if (!inst || count < 1) return 0;
    size_t el = dtype == VIE_C128 ? 16 : 8;
    size_t tot = align256(sizeof(InstDev) * (size_t)count);
    for (int i = 0; i < count; ++i) {
        if (!inst[i].op || inst[i].nrhs < 1) return 0;
        tot += align256(matvec_ws_elems(inst[i].op->d, inst[i].nrhs) * el);
    }
    return tot;
}

vie_status vie_matvec_multi(const vie_instance* inst, int count, int kind, int adjoint, int dtype, void* ws,
                            size_t ws_bytes, void* stream)
{
    if (!inst || count < 1 || !ws) return fail(VIE_E_ARG, "vie_matvec_multi: bad argument");
    if (kind != VIE_OP_A && kind != VIE_OP_N) return fail(VIE_E_ARG, "vie_matvec_multi: bad kind");
    if (dtype != VIE_C64 && dtype != VIE_C128) return fail(VIE_E_ARG, "vie_matvec_multi: bad dtype");
    size_t need = vie_matvec_multi_workspace_bytes(inst, count, dtype);
    if (need == 0 || ws_bytes < need) return fail(VIE_E_ARG, "vie_matvec_multi: workspace too small");
    int mode = kind == VIE_OP_A ? (adjoint ? MODE_AH : MODE_A) : (adjoint ? MODE_NH : MODE_N);
    size_t eb = dtype == VIE_C128 ? 16 : 8;
    std::vector<InstHost> req(count);
    size_t off = align256(sizeof(InstDev) * (size_t)count);
    for (int i = 0; i < count; ++i) {
        const vie_instance& in = inst[i];
        if (!in.x || !in.y || (kind == VIE_OP_A && !in.eps_c)) return fail(VIE_E_ARG, "vie_matvec_multi: bad instance");
        if (in.op->d.nhat_source != 0) return fail(VIE_E_UNSUPPORTED, "vie_matvec_multi: Tucker operators only");
        if (in.op->d.view.fam != 0) return fail(VIE_E_UNSUPPORTED, "vie_matvec_multi: N operators only");
        const OpView& v = in.op->d.view;
        size_t vb = (size_t)in.nrhs * 3 * v.n[0] * v.n[1] * v.n[2] * eb;
        const char* xb = (const char*)in.x;
        const char* yb = (const char*)in.y;
        if (!(xb + vb <= yb || yb + vb <= xb)) return fail(VIE_E_ARG, "vie_matvec_multi: x and y overlap");
        req[i] = {&in.op->d, in.x, in.y, in.eps_c, nullptr, in.nrhs, (char*)ws + off};
        off += align256(matvec_ws_elems(in.op->d, in.nrhs) * eb);
    }
    std::string err;
    hipError_t e;
    if (dtype == VIE_C128)
        e = launch_batch<double, double>(req, mode, 0, (InstDev*)ws, (hipStream_t)stream, err);
    else
        e = launch_batch<float, float>(req, mode, 0, (InstDev*)ws, (hipStream_t)stream, err);
    if (e != hipSuccess) return err.empty() ? hip_fail(e, "vie_matvec_multi") : fail(VIE_E_UNSUPPORTED, "vie_matvec_multi: " + err);
    return VIE_OK;
}

}  // extern "C"
