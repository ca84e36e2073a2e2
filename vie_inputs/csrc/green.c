/*
 * Galerkin Green's tensor of the electric volume operator N for piecewise-
 * constant (pulse) current basis functions on a uniform cubic voxel grid.
 *
 * Problem data, not part of the compressed-matvec method: the paper defines
 * the entries as L2 inner products of a test pulse in voxel 0 with N applied
 * to a basis pulse in voxel Delta (Sec. II-B, eq. 8a-8b, with the operator N
 * of eq. 5 and the kernel of eq. 6) but leaves their evaluation to external
 * singular-integral routines.  This file evaluates them directly.
 *
 * Reading used (dimensionless coordinates x = r/h, kappa = k0*h):
 *   N u = u + (k0^2 + grad div) int g u      (curl curl = grad div - laplacian,
 *                                            and (lap + k0^2) g = -delta)
 *   The 6-D Galerkin integral of two unit pulses collapses to a 3-D integral
 *   against the pulse autocorrelation tau_D(x) = prod_i lam(x_i - D_i),
 *   lam(t) = max(1 - |t|, 0).  Rows are divided by the voxel volume, so the
 *   mass matrix is the identity and
 *     Nt_pq(D) = d_pq d_D0 + kappa^2 d_pq J0(D) + Jpq(D)
 *     J0(D)    = int g^(x) tau_D(x) dx
 *     Jpq(D)   = int g^(x) d_p d_q tau_D(x) dx        (distributional)
 *   with g^(x) = exp(-i kappa |x|) / (4 pi |x|).
 *   For max_i D_i >= 2 the kernel is smooth on the support and the classical
 *   form Nt_pq(D) = int Gd_pq(x) tau_D(x) dx is used, with the dyadic
 *   Gd_pq = (kappa^2 d_pq + d_p d_q) g^.
 *   For max_i D_i <= 1 the support touches the singularity: J0 and Jpq
 *   (p != q, where d_p d_q tau = lam' lam' lam) are volume integrals over the
 *   8 cells cut by the kinks of tau, with a Duffy transform on cells that have
 *   the origin at a corner; Jpp uses lam'' = delta(t+1) - 2 delta(t) +
 *   delta(t-1), i.e. three plane integrals per component, with a 2-D Duffy
 *   transform on the plane through the origin.
 *
 * Output layout: out[((c*n3 + k)*n2 + j)*n1 + i] (complex128 interleaved),
 * components c = xx, yy, zz, xy, xz, yz, entry = Nt_c(D = (i, j, k)).
 *
 * The same machinery gives the entries of the magnetic operator K of eq. 5
 * (vie_green_k_fill, below).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define QMAX 40
static double gl_x[QMAX + 1][QMAX];
static double gl_w[QMAX + 1][QMAX];
static int gl_ready = 0;

/* Gauss-Legendre nodes and weights on [0, 1] by Newton iteration on the
 * Legendre polynomial P_q (three-term recurrence). */
static void legendre(int q, double z, double *p, double *dp)
{
    double p0 = 1.0, p1 = 0.0;
    for (int j = 1; j <= q; ++j) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
    }
    *p = p0;
    *dp = q * (z * p0 - p1) / (z * z - 1.0);
}

static void gl_init(void)
{
    if (gl_ready) return;
    for (int q = 1; q <= QMAX; ++q) {
        for (int i = 0; i < q; ++i) {
            double z = cos(M_PI * (i + 0.75) / (q + 0.5)), p, dp;
            for (int it = 0; it < 100; ++it) {
                legendre(q, z, &p, &dp);
                double dz = p / dp;
                z -= dz;
                if (fabs(dz) < 1e-15) break;
            }
            legendre(q, z, &p, &dp);
            gl_x[q][i] = 0.5 * (1.0 - z);
            gl_w[q][i] = 1.0 / ((1.0 - z * z) * dp * dp);
        }
    }
    gl_ready = 1;
}

static const int comp_p[6] = {0, 1, 2, 0, 0, 1};
static const int comp_q[6] = {0, 1, 2, 1, 2, 2};

/* scalar kernel g^(x) = exp(-i kappa r) / (4 pi r) */
static inline cplx ghat(double r, double kappa)
{
    return cexp(-I * kappa * r) / (4.0 * M_PI * r);
}

/* lam(t) and its derivative on the open cell containing t */
static inline double lam(double t) { double a = 1.0 - fabs(t); return a > 0 ? a : 0.0; }

/* ---------------- far field: smooth dyadic against tau_D ---------------- */
static void far_entry(const int D[3], double kappa, int q, cplx out[6])
{
    cplx acc[6] = {0, 0, 0, 0, 0, 0};
    const double *gx = gl_x[q], *gw = gl_w[q];
    /* 8 cells: per axis t in [-1,0] or [0,1] around D, tent weight 1-|t| */
    for (int cell = 0; cell < 8; ++cell) {
        double lo[3];
        for (int a = 0; a < 3; ++a) lo[a] = ((cell >> a) & 1) ? 0.0 : -1.0;
        for (int ia = 0; ia < q; ++ia) {
            double t0 = lo[0] + gx[ia];
            double w0 = gw[ia] * (1.0 - fabs(t0));
            double x0 = D[0] + t0;
            for (int ib = 0; ib < q; ++ib) {
                double t1 = lo[1] + gx[ib];
                double w1 = w0 * gw[ib] * (1.0 - fabs(t1));
                double x1 = D[1] + t1;
                for (int ic = 0; ic < q; ++ic) {
                    double t2 = lo[2] + gx[ic];
                    double w = w1 * gw[ic] * (1.0 - fabs(t2));
                    double x2 = D[2] + t2;
                    double r2 = x0 * x0 + x1 * x1 + x2 * x2;
                    double r = sqrt(r2);
                    cplx g = ghat(r, kappa);
                    cplx ikr = I * kappa * r;
                    cplx diag = g * (kappa * kappa - (1.0 + ikr) / r2);
                    cplx radial = g * (3.0 + 3.0 * ikr - kappa * kappa * r2) / (r2 * r2);
                    double xs[3] = {x0, x1, x2};
                    for (int c = 0; c < 6; ++c) {
                        int p = comp_p[c], qq = comp_q[c];
                        cplx v = radial * xs[p] * xs[qq];
                        if (p == qq) v += diag;
                        acc[c] += w * v;
                    }
                }
            }
        }
    }
    for (int c = 0; c < 6; ++c) out[c] = acc[c];
}

/* ---------------- near field helpers ---------------- */

/* integrand weight for the volume integrals J0 and Jpq (p != q) at x:
 * returns tau_D(x) in w[0] and lam' lam' lam for the 3 off-diagonal pairs
 * (xy, xz, yz) in w[1..3].  x must lie strictly inside a cell. */
static inline void vol_weights(const double x[3], const int D[3], double w[4])
{
    double l[3], d[3];
    for (int a = 0; a < 3; ++a) {
        double t = x[a] - D[a];
        l[a] = lam(t);
        d[a] = (fabs(t) < 1.0) ? (t > 0 ? -1.0 : 1.0) : 0.0;
    }
    w[0] = l[0] * l[1] * l[2];
    w[1] = d[0] * d[1] * l[2];
    w[2] = d[0] * d[2] * l[1];
    w[3] = d[1] * d[2] * l[0];
}

/* weights of the K entries at x: -lam'(x_s - D_s) prod_{i != s} lam(x_i - D_i)
 * for s = x, y, z in w[0..2] (w[3] = 0), so that the volume integral of
 * g^ * w[s] is F_s(D) = -int g^ d_s tau_D.  x must lie strictly inside a cell. */
static inline void vol_weights_k(const double x[3], const int D[3], double w[4])
{
    double l[3], d[3];
    for (int a = 0; a < 3; ++a) {
        double t = x[a] - D[a];
        l[a] = lam(t);
        d[a] = (fabs(t) < 1.0) ? (t > 0 ? -1.0 : 1.0) : 0.0;
    }
    w[0] = -d[0] * l[1] * l[2];
    w[1] = -d[1] * l[0] * l[2];
    w[2] = -d[2] * l[0] * l[1];
    w[3] = 0.0;
}

static inline void cell_weights(int kind, const double x[3], const int D[3], double w[4])
{
    if (kind == 0) vol_weights(x, D, w);
    else vol_weights_k(x, D, w);
}

/* volume integral of g^ * {tau, lam'lam'lam (3 pairs)} (kind 0) or of the
 * K weights (kind 1) over a unit cell [lo, lo+1]^3 that does not contain the
 * origin in its closure */
static void vol_cell_regular(int kind, const double lo[3], const int D[3], double kappa, int q, cplx acc[4])
{
    const double *gx = gl_x[q], *gw = gl_w[q];
    for (int ia = 0; ia < q; ++ia)
        for (int ib = 0; ib < q; ++ib)
            for (int ic = 0; ic < q; ++ic) {
                double x[3] = {lo[0] + gx[ia], lo[1] + gx[ib], lo[2] + gx[ic]};
                double w = gw[ia] * gw[ib] * gw[ic];
                double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                cplx g = ghat(r, kappa) * w;
                double wt[4];
                cell_weights(kind, x, D, wt);
                for (int m = 0; m < 4; ++m) acc[m] += g * wt[m];
            }
}

/* same over a unit cell with the origin at one corner: the cell is
 * {sigma_a * y_a, y in [0,1]^3}; Duffy split into three pyramids with apex
 * at the origin, each mapped to [0,1]^3 with Jacobian s^2, which cancels
 * the 1/r singularity of g^. */
static void vol_cell_corner(int kind, const double sigma[3], const int D[3], double kappa, int q, cplx acc[4])
{
    const double *gx = gl_x[q], *gw = gl_w[q];
    for (int face = 0; face < 3; ++face) {
        int a1 = (face + 1) % 3, a2 = (face + 2) % 3;
        for (int is = 0; is < q; ++is) {
            double s = gx[is];
            for (int ib = 0; ib < q; ++ib)
                for (int ic = 0; ic < q; ++ic) {
                    double y[3];
                    y[face] = s;
                    y[a1] = s * gx[ib];
                    y[a2] = s * gx[ic];
                    double x[3] = {sigma[0] * y[0], sigma[1] * y[1], sigma[2] * y[2]};
                    double r = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
                    double w = gw[is] * gw[ib] * gw[ic] * s * s;
                    cplx g = ghat(r, kappa) * w;
                    double wt[4];
                    cell_weights(kind, x, D, wt);
                    for (int m = 0; m < 4; ++m) acc[m] += g * wt[m];
                }
        }
    }
}

/* plane integral over the unit square [lo_a, lo_a+1] x [lo_b, lo_b+1] in the
 * plane x_p = c of g^ * lam(x_a - D_a) * lam(x_b - D_b) */
static cplx plane_cell(int p, double c, const double lo2[2], const double sig2[2], int corner,
                       const int D[3], double kappa, int q)
{
    const double *gx = gl_x[q], *gw = gl_w[q];
    int a = (p + 1) % 3, b = (p + 2) % 3;
    cplx acc = 0;
    if (!corner) {
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j) {
                double xa = lo2[0] + gx[i], xb = lo2[1] + gx[j];
                double r = sqrt(c * c + xa * xa + xb * xb);
                acc += gw[i] * gw[j] * lam(xa - D[a]) * lam(xb - D[b]) * ghat(r, kappa);
            }
    } else {
        /* origin at a corner of the square and c == 0: two triangles */
        for (int tri = 0; tri < 2; ++tri)
            for (int i = 0; i < q; ++i) {
                double s = gx[i];
                for (int j = 0; j < q; ++j) {
                    double ya = tri == 0 ? s : s * gx[j];
                    double yb = tri == 0 ? s * gx[j] : s;
                    double xa = sig2[0] * ya, xb = sig2[1] * yb;
                    double r = sqrt(ya * ya + yb * yb);
                    acc += gw[i] * gw[j] * s * lam(xa - D[a]) * lam(xb - D[b]) * ghat(r, kappa);
                }
            }
    }
    return acc;
}

/* volume integrals over the 8 unit cells of the support of tau_D, with a
 * Duffy transform on a cell that has the origin at a corner */
static void near_volume(int kind, const int D[3], double kappa, int q, cplx vol[4])
{
    for (int cell = 0; cell < 8; ++cell) {
        double lo[3];
        int corner = 1;
        double sigma[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = D[a] + (((cell >> a) & 1) ? 0.0 : -1.0);
            if (lo[a] == 0.0) sigma[a] = 1.0;
            else if (lo[a] == -1.0) sigma[a] = -1.0;
            else corner = 0;
        }
        if (corner) vol_cell_corner(kind, sigma, D, kappa, q, vol);
        else vol_cell_regular(kind, lo, D, kappa, q, vol);
    }
}

static void near_entry(const int D[3], double kappa, int q, cplx out[6])
{
    /* volume part: J0 and the three off-diagonal Jpq */
    cplx vol[4] = {0, 0, 0, 0};
    near_volume(0, D, kappa, q, vol);
    /* plane part: Jpp = sum_s c_s * plane integral at x_p = D_p + s */
    cplx jpp[3];
    for (int p = 0; p < 3; ++p) {
        int a = (p + 1) % 3, b = (p + 2) % 3;
        cplx acc = 0;
        for (int sft = -1; sft <= 1; ++sft) {
            double c = D[p] + sft;
            double coef = (sft == 0) ? -2.0 : 1.0;
            for (int cell = 0; cell < 4; ++cell) {
                double lo2[2] = {D[a] + ((cell & 1) ? 0.0 : -1.0), D[b] + ((cell & 2) ? 0.0 : -1.0)};
                int corner = (c == 0.0);
                double sig2[2];
                for (int m = 0; m < 2; ++m) {
                    if (lo2[m] == 0.0) sig2[m] = 1.0;
                    else if (lo2[m] == -1.0) sig2[m] = -1.0;
                    else corner = 0;
                }
                acc += coef * plane_cell(p, c, lo2, sig2, corner, D, kappa, q);
            }
        }
        jpp[p] = acc;
    }
    int self = (D[0] == 0 && D[1] == 0 && D[2] == 0);
    for (int p = 0; p < 3; ++p) out[p] = (self ? 1.0 : 0.0) + kappa * kappa * vol[0] + jpp[p];
    out[3] = vol[1];
    out[4] = vol[2];
    out[5] = vol[3];
}

static int far_order(int d, int boost)
{
    int q;
    if (d <= 2) q = 10;
    else if (d == 3) q = 8;
    else if (d <= 5) q = 6;
    else if (d <= 11) q = 4;
    else if (d <= 31) q = 3;
    else q = 2;
    q += boost;
    return q > QMAX ? QMAX : q;
}

/* Fill the dense defining tensor.  near_q: Gauss order of the singular
 * (Duffy) integrals; boost: extra order on every far-field shell.  Only
 * entries with offset index in [lo_lin, hi_lin) of the linear (i fastest)
 * offset order are computed, so callers can split work. */
int vie_green_fill(int n1, int n2, int n3, double kappa, int near_q, int boost,
                   double *out, long lo_lin, long hi_lin)
{
    gl_init();
    if (near_q < 2 || near_q > QMAX) return -1;
    long V = (long)n1 * n2 * n3;
    if (hi_lin > V) hi_lin = V;
#pragma omp parallel for schedule(dynamic, 64)
    for (long lin = lo_lin; lin < hi_lin; ++lin) {
        int D[3] = {(int)(lin % n1), (int)((lin / n1) % n2), (int)(lin / ((long)n1 * n2))};
        int d = D[0];
        if (D[1] > d) d = D[1];
        if (D[2] > d) d = D[2];
        cplx e[6];
        if (d <= 1) near_entry(D, kappa, near_q, e);
        else far_entry(D, kappa, far_order(d, boost), e);
        for (int c = 0; c < 6; ++c) {
            out[2 * (c * V + lin)] = creal(e[c]);
            out[2 * (c * V + lin) + 1] = cimag(e[c]);
        }
    }
    return 0;
}

/* Entries of one component at arbitrary offsets: out[2 t], out[2 t + 1] =
 * Nt_comp(D = idx[3 t .. 3 t + 2]) for t < count, computed exactly as
 * vie_green_fill computes them (same per-offset quadrature), so the values
 * equal the dense tensor's bit for bit.  Offsets must be non-negative.
 * Used by fiber-sampling (cross) compressions, which never form the dense
 * tensor. */
int vie_green_entries(double kappa, int near_q, int boost, int comp, long count, const int *idx, double *out)
{
    gl_init();
    if (near_q < 2 || near_q > QMAX || comp < 0 || comp > 5 || count < 0) return -1;
    /* the 8 offsets with every D_i in {0, 1} (the singular shell) are
     * evaluated once here and looked up below: fibers meet them often */
    cplx nearv[8][6];
#pragma omp parallel for schedule(static, 1)
    for (int b = 0; b < 8; ++b) {
        int D[3] = {b & 1, (b >> 1) & 1, (b >> 2) & 1};
        near_entry(D, kappa, near_q, nearv[b]);
    }
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(|: bad)
    for (long t = 0; t < count; ++t) {
        int D[3] = {idx[3 * t], idx[3 * t + 1], idx[3 * t + 2]};
        if (D[0] < 0 || D[1] < 0 || D[2] < 0) {
            bad = 1;
            continue;
        }
        int d = D[0];
        if (D[1] > d) d = D[1];
        if (D[2] > d) d = D[2];
        cplx e[6];
        const cplx *src = e;
        if (d <= 1) src = nearv[D[0] | (D[1] << 1) | (D[2] << 2)];
        else far_entry(D, kappa, far_order(d, boost), e);
        out[2 * t] = creal(src[comp]);
        out[2 * t + 1] = cimag(src[comp]);
    }
    return bad ? -2 : 0;
}

/* The same as a callback of the shape the VIE library's cross compression
 * takes: ctx points at {double kappa; int near_q; int boost;}. */
typedef struct {
    double kappa;
    int near_q;
    int boost;
} vie_green_ctx;

int vie_green_entry_cb(void *ctx, int comp, long count, const int *idx, double *out)
{
    const vie_green_ctx *g = (const vie_green_ctx *)ctx;
    return vie_green_entries(g->kappa, g->near_q, g->boost, comp, count, idx, out);
}

/* ---------------- the K operator (curl of the single-layer potential) ----------------
 * Entries Kt_pq(D) = <P_D e_p, K P_0 e_q> / vol: observation voxel D, source
 * voxel 0, so that (K u)_p(m) = sum_m' Kt_pq(m - m') u_q(m') is a
 * convolution.  With (curl (g e_q))_p = eps_psq d_s g,
 *   Kt_pq(D) = eps_psq F_s(D),  F_s(D) = int d_s g^(x) tau_D(x) dx
 *                                      = -int g^(x) d_s tau_D(x) dx,
 * the second form (integrable 1/r kernel, piecewise constant lam') on the
 * near shells, the first (smooth kernel d_s g^ = -x_s (1 + i kappa r) g^ / r^2)
 * on the far ones.  Stored components xy, xz, yz:
 *   Kt_xy = -F_z, Kt_xz = F_y, Kt_yz = -F_x   (Kt_qp = -Kt_pq, diagonal 0).
 * Dimensionless: the physical entries are h Kt (the curl brings 1/h, the
 * kernel and the two volume integrals h^5, the row normalisation 1/h^3). */
static void k_far_entry(const int D[3], double kappa, int q, cplx F[3])
{
    cplx acc[3] = {0, 0, 0};
    const double *gx = gl_x[q], *gw = gl_w[q];
    for (int cell = 0; cell < 8; ++cell) {
        double lo[3];
        for (int a = 0; a < 3; ++a) lo[a] = ((cell >> a) & 1) ? 0.0 : -1.0;
        for (int ia = 0; ia < q; ++ia) {
            double t0 = lo[0] + gx[ia];
            double w0 = gw[ia] * (1.0 - fabs(t0));
            double x0 = D[0] + t0;
            for (int ib = 0; ib < q; ++ib) {
                double t1 = lo[1] + gx[ib];
                double w1 = w0 * gw[ib] * (1.0 - fabs(t1));
                double x1 = D[1] + t1;
                for (int ic = 0; ic < q; ++ic) {
                    double t2 = lo[2] + gx[ic];
                    double w = w1 * gw[ic] * (1.0 - fabs(t2));
                    double x2 = D[2] + t2;
                    double r2 = x0 * x0 + x1 * x1 + x2 * x2;
                    double r = sqrt(r2);
                    cplx dg = -ghat(r, kappa) * (1.0 + I * kappa * r) / r2;
                    acc[0] += w * dg * x0;
                    acc[1] += w * dg * x1;
                    acc[2] += w * dg * x2;
                }
            }
        }
    }
    for (int s = 0; s < 3; ++s) F[s] = acc[s];
}

/* Fill the K defining tensor: out[((c*n3 + k)*n2 + j)*n1 + i], c = xy, xz, yz,
 * complex128 interleaved; offsets [lo_lin, hi_lin) as in vie_green_fill. */
int vie_green_k_fill(int n1, int n2, int n3, double kappa, int near_q, int boost,
                     double *out, long lo_lin, long hi_lin)
{
    gl_init();
    if (near_q < 2 || near_q > QMAX) return -1;
    long V = (long)n1 * n2 * n3;
    if (hi_lin > V) hi_lin = V;
#pragma omp parallel for schedule(dynamic, 64)
    for (long lin = lo_lin; lin < hi_lin; ++lin) {
        int D[3] = {(int)(lin % n1), (int)((lin / n1) % n2), (int)(lin / ((long)n1 * n2))};
        int d = D[0];
        if (D[1] > d) d = D[1];
        if (D[2] > d) d = D[2];
        cplx F[3];
        if (d <= 1) {
            cplx vol[4] = {0, 0, 0, 0};
            near_volume(1, D, kappa, near_q, vol);
            for (int s = 0; s < 3; ++s) F[s] = vol[s];
        } else {
            k_far_entry(D, kappa, far_order(d, boost), F);
        }
        /* F_s is odd in D_s: exactly zero on the plane D_s = 0 */
        for (int s = 0; s < 3; ++s)
            if (D[s] == 0) F[s] = 0;
        cplx e[3] = {-F[2], F[1], -F[0]};
        for (int c = 0; c < 3; ++c) {
            out[2 * (c * V + lin)] = creal(e[c]);
            out[2 * (c * V + lin) + 1] = cimag(e[c]);
        }
    }
    return 0;
}

/* Dimensionless dyadic Gd_pq(x) = (kappa^2 d_pq + d_p d_q) g^(x) at points
 * x (npts x 3), all six components: used for point-sampled incident fields
 * of Hertzian dipoles.  out: npts x 6 complex interleaved. */
void vie_dyadic_points(long npts, const double *x, double kappa, double *out)
{
#pragma omp parallel for schedule(static)
    for (long m = 0; m < npts; ++m) {
        double x0 = x[3 * m], x1 = x[3 * m + 1], x2 = x[3 * m + 2];
        double r2 = x0 * x0 + x1 * x1 + x2 * x2;
        double r = sqrt(r2);
        cplx g = ghat(r, kappa);
        cplx ikr = I * kappa * r;
        cplx diag = g * (kappa * kappa - (1.0 + ikr) / r2);
        cplx radial = g * (3.0 + 3.0 * ikr - kappa * kappa * r2) / (r2 * r2);
        double xs[3] = {x0, x1, x2};
        for (int c = 0; c < 6; ++c) {
            cplx v = radial * xs[comp_p[c]] * xs[comp_q[c]];
            if (comp_p[c] == comp_q[c]) v += diag;
            out[2 * (6 * m + c)] = creal(v);
            out[2 * (6 * m + c) + 1] = cimag(v);
        }
    }
}

/* ================= piecewise-linear basis (eq. 7b) =================
 *
 * Per voxel four scalar functions: the pulse and the pulse times
 * (x_a - x_a,m)/h for a = x, y, z.  Per axis the test function of voxel 0 is
 * phi_al(t) and the basis function of voxel D is phi_be(t - D), with
 * phi_0 = pulse on [-1/2, 1/2] and phi_1 = t * pulse.  As for pulses, the
 * 6-D Galerkin integral of eq. 8a becomes a 3-D integral of g^ against the
 * product over the axes of the correlations
 *   c_{al be}(s) = int phi_al(t) phi_be(t + s) dt,   s = x - D,
 * which are (type = al + 2 be)
 *   type 0 (pulse test, pulse basis)    1 - |s|
 *   type 1 (linear test, pulse basis)  -s (1 - |s|) / 2
 *   type 2 (pulse test, linear basis)   s (1 - |s|) / 2
 *   type 3 (linear test, linear basis)  1/12 - |s|/4 + |s|^3 / 6
 * on |s| <= 1, zero outside.  With W_D(x) = prod_a c_{type_a}(x_a - D_a):
 *   Nt^{pl,ql'}(D) = d_pq d_ll' m_l d_D0 + kappa^2 d_pq int g^ W_D
 *                    + int g^ d_p d_q W_D                     (distributional)
 * with the self products m = (1, 1/12, 1/12, 1/12).  d_p d_q W (p != q) has
 * bounded first derivatives only; d_p^2 W has a regular part on the open
 * cells plus point masses of c'' at s_p = -1, 0, 1 (pwl_jump), which turn
 * into plane integrals.  Far from the singularity the smooth dyadic form
 * int Gd_pq W_D is used, as for pulses.
 *
 * The ten pairs l <= l' are stored; the others follow from
 * Nt^{(l',l)} = sigma Nt^{(l,l')}, sigma = -1 when exactly one of l, l' is
 * the pulse (c_{type 2} = -c_{type 1}).
 */
static const int pwl_pairs[10][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {1, 1}, {1, 2}, {1, 3}, {2, 2}, {2, 3}, {3, 3}};
/* coefficients of the point masses of c'' at s = -1, 0, 1 per type */
static const double pwl_jump[4][3] = {{1.0, -2.0, 1.0}, {0.5, 0.0, -0.5}, {-0.5, 0.0, 0.5}, {-0.25, -0.5, -0.25}};

static inline int pwl_type(int P, int a)
{
    return (pwl_pairs[P][0] == a + 1) + 2 * (pwl_pairs[P][1] == a + 1);
}

/* values, first derivatives and regular second derivatives of the four
 * correlation types at s (|s| < 1 and s != 0 on every quadrature point) */
static inline void pwl_axis(double s, double v[4], double d1[4], double d2[4])
{
    double a = fabs(s);
    if (a >= 1.0) {
        for (int t = 0; t < 4; ++t) v[t] = d1[t] = d2[t] = 0.0;
        return;
    }
    double sg = s > 0 ? 1.0 : (s < 0 ? -1.0 : 0.0);
    v[0] = 1.0 - a;
    d1[0] = -sg;
    d2[0] = 0.0;
    v[1] = -0.5 * s * (1.0 - a);
    d1[1] = a - 0.5;
    d2[1] = sg;
    v[2] = -v[1];
    d1[2] = -d1[1];
    d2[2] = -sg;
    v[3] = 1.0 / 12.0 - 0.25 * a + a * a * a / 6.0;
    d1[3] = sg * (0.5 * s * s - 0.25);
    d2[3] = a;
}

static int pwl_ty[10][3];
static int pwl_ty_ready = 0;
static void pwl_init(void)
{
    gl_init();
    if (pwl_ty_ready) return;
    for (int P = 0; P < 10; ++P)
        for (int a = 0; a < 3; ++a) pwl_ty[P][a] = pwl_type(P, a);
    pwl_ty_ready = 1;
}

/* far field: int Gd_pq(x) W_D(x) dx over the 8 unit cells around D */
static void pwl_far_entry(const int D[3], double kappa, int q, cplx out[60])
{
    cplx acc[60];
    for (int m = 0; m < 60; ++m) acc[m] = 0;
    const double *gx = gl_x[q], *gw = gl_w[q];
    for (int cell = 0; cell < 8; ++cell) {
        double lo[3];
        for (int a = 0; a < 3; ++a) lo[a] = ((cell >> a) & 1) ? 0.0 : -1.0;
        for (int ia = 0; ia < q; ++ia)
            for (int ib = 0; ib < q; ++ib)
                for (int ic = 0; ic < q; ++ic) {
                    double t[3] = {lo[0] + gx[ia], lo[1] + gx[ib], lo[2] + gx[ic]};
                    double w = gw[ia] * gw[ib] * gw[ic];
                    double x0 = D[0] + t[0], x1 = D[1] + t[1], x2 = D[2] + t[2];
                    double r2 = x0 * x0 + x1 * x1 + x2 * x2;
                    double r = sqrt(r2);
                    cplx g = ghat(r, kappa);
                    cplx ikr = I * kappa * r;
                    cplx diag = g * (kappa * kappa - (1.0 + ikr) / r2);
                    cplx radial = g * (3.0 + 3.0 * ikr - kappa * kappa * r2) / (r2 * r2);
                    double xs[3] = {x0, x1, x2};
                    cplx Gd[6];
                    for (int c = 0; c < 6; ++c) {
                        Gd[c] = radial * xs[comp_p[c]] * xs[comp_q[c]];
                        if (comp_p[c] == comp_q[c]) Gd[c] += diag;
                    }
                    double v[3][4], d1[4], d2[4];
                    for (int a = 0; a < 3; ++a) pwl_axis(t[a], v[a], d1, d2);
                    for (int P = 0; P < 10; ++P) {
                        double wt = w * v[0][pwl_ty[P][0]] * v[1][pwl_ty[P][1]] * v[2][pwl_ty[P][2]];
                        for (int c = 0; c < 6; ++c) acc[P * 6 + c] += wt * Gd[c];
                    }
                }
    }
    for (int m = 0; m < 60; ++m) out[m] = acc[m];
}

/* volume weights at x (s = x - D) for all pairs: per pair
 * [0] W, [1..3] d_p W d_q for xy, xz, yz, [4..6] regular d_p^2 W */
static inline void pwl_vol_point(const double x[3], const int D[3], cplx g, cplx acc[70])
{
    double v[3][4], d1[3][4], d2[3][4];
    for (int a = 0; a < 3; ++a) pwl_axis(x[a] - D[a], v[a], d1[a], d2[a]);
    for (int P = 0; P < 10; ++P) {
        const int t0 = pwl_ty[P][0], t1 = pwl_ty[P][1], t2 = pwl_ty[P][2];
        cplx *o = acc + 7 * P;
        o[0] += g * (v[0][t0] * v[1][t1] * v[2][t2]);
        o[1] += g * (d1[0][t0] * d1[1][t1] * v[2][t2]);
        o[2] += g * (d1[0][t0] * v[1][t1] * d1[2][t2]);
        o[3] += g * (v[0][t0] * d1[1][t1] * d1[2][t2]);
        o[4] += g * (d2[0][t0] * v[1][t1] * v[2][t2]);
        o[5] += g * (v[0][t0] * d2[1][t1] * v[2][t2]);
        o[6] += g * (v[0][t0] * v[1][t1] * d2[2][t2]);
    }
}

static void pwl_near_volume(const int D[3], double kappa, int q, cplx acc[70])
{
    const double *gx = gl_x[q], *gw = gl_w[q];
    for (int cell = 0; cell < 8; ++cell) {
        double lo[3], sigma[3];
        int corner = 1;
        for (int a = 0; a < 3; ++a) {
            lo[a] = D[a] + (((cell >> a) & 1) ? 0.0 : -1.0);
            if (lo[a] == 0.0) sigma[a] = 1.0;
            else if (lo[a] == -1.0) sigma[a] = -1.0;
            else corner = 0;
        }
        if (!corner) {
            for (int ia = 0; ia < q; ++ia)
                for (int ib = 0; ib < q; ++ib)
                    for (int ic = 0; ic < q; ++ic) {
                        double x[3] = {lo[0] + gx[ia], lo[1] + gx[ib], lo[2] + gx[ic]};
                        double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                        pwl_vol_point(x, D, ghat(r, kappa) * (gw[ia] * gw[ib] * gw[ic]), acc);
                    }
        } else {
            /* Duffy: three pyramids with apex at the origin, Jacobian s^2 */
            for (int face = 0; face < 3; ++face) {
                int a1 = (face + 1) % 3, a2 = (face + 2) % 3;
                for (int is = 0; is < q; ++is) {
                    double s = gx[is];
                    for (int ib = 0; ib < q; ++ib)
                        for (int ic = 0; ic < q; ++ic) {
                            double y[3];
                            y[face] = s;
                            y[a1] = s * gx[ib];
                            y[a2] = s * gx[ic];
                            double x[3] = {sigma[0] * y[0], sigma[1] * y[1], sigma[2] * y[2]};
                            double r = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
                            pwl_vol_point(x, D, ghat(r, kappa) * (gw[is] * gw[ib] * gw[ic] * s * s), acc);
                        }
                }
            }
        }
    }
}

/* plane integrals over x_p = c (the unit squares of the support in the
 * other two axes) of g^ * c_{type_a}(x_a - D_a) c_{type_b}(x_b - D_b), all
 * pairs: acc[P] */
static void pwl_plane(int p, double c, const int D[3], double kappa, int q, cplx acc[10])
{
    const double *gx = gl_x[q], *gw = gl_w[q];
    int a = (p + 1) % 3, b = (p + 2) % 3;
    for (int cell = 0; cell < 4; ++cell) {
        double lo2[2] = {D[a] + ((cell & 1) ? 0.0 : -1.0), D[b] + ((cell & 2) ? 0.0 : -1.0)};
        int corner = (c == 0.0);
        double sig2[2];
        for (int m = 0; m < 2; ++m) {
            if (lo2[m] == 0.0) sig2[m] = 1.0;
            else if (lo2[m] == -1.0) sig2[m] = -1.0;
            else corner = 0;
        }
        int npts = corner ? 2 * q * q : q * q;
        for (int e = 0; e < npts; ++e) {
            double xa, xb, r, w;
            if (!corner) {
                int i = e / q, j = e % q;
                xa = lo2[0] + gx[i];
                xb = lo2[1] + gx[j];
                r = sqrt(c * c + xa * xa + xb * xb);
                w = gw[i] * gw[j];
            } else {
                /* origin at a corner of the square in the plane through it:
                 * two triangles with apex at the origin, Jacobian s */
                int tri = e / (q * q), i = (e / q) % q, j = e % q;
                double s = gx[i];
                double ya = tri == 0 ? s : s * gx[j];
                double yb = tri == 0 ? s * gx[j] : s;
                xa = sig2[0] * ya;
                xb = sig2[1] * yb;
                r = sqrt(ya * ya + yb * yb);
                w = gw[i] * gw[j] * s;
            }
            cplx g = ghat(r, kappa) * w;
            double va[4], vb[4], d1[4], d2[4];
            pwl_axis(xa - D[a], va, d1, d2);
            pwl_axis(xb - D[b], vb, d1, d2);
            for (int P = 0; P < 10; ++P) acc[P] += g * (va[pwl_ty[P][a]] * vb[pwl_ty[P][b]]);
        }
    }
}

/* distributional form, valid at every offset (the Duffy maps take care of
 * cells and squares that have the origin at a corner) */
static void pwl_near_entry(const int D[3], double kappa, int q, cplx out[60])
{
    cplx vol[70];
    for (int m = 0; m < 70; ++m) vol[m] = 0;
    pwl_near_volume(D, kappa, q, vol);
    cplx diag[10][3];
    for (int P = 0; P < 10; ++P)
        for (int p = 0; p < 3; ++p) diag[P][p] = 0;
    for (int p = 0; p < 3; ++p)
        for (int sft = -1; sft <= 1; ++sft) {
            cplx pl[10];
            for (int P = 0; P < 10; ++P) pl[P] = 0;
            pwl_plane(p, (double)(D[p] + sft), D, kappa, q, pl);
            for (int P = 0; P < 10; ++P) diag[P][p] += pwl_jump[pwl_ty[P][p]][sft + 1] * pl[P];
        }
    const int self = (D[0] == 0 && D[1] == 0 && D[2] == 0);
    for (int P = 0; P < 10; ++P) {
        const int l = pwl_pairs[P][0], lp = pwl_pairs[P][1];
        const double mass = (self && l == lp) ? (l == 0 ? 1.0 : 1.0 / 12.0) : 0.0;
        const cplx *v = vol + 7 * P;
        for (int p = 0; p < 3; ++p) out[P * 6 + p] = mass + kappa * kappa * v[0] + v[4 + p] + diag[P][p];
        out[P * 6 + 3] = v[1];
        out[P * 6 + 4] = v[2];
        out[P * 6 + 5] = v[3];
    }
}

/* Dense PWL defining tensors: out[(((P * 6 + c) * n3 + k) * n2 + j) * n1 + i]
 * (complex128 interleaved) = Nt^{(l,l')}_c(D = (i, j, k)) for the pairs
 * P = (0,0), (0,1), (0,2), (0,3), (1,1), (1,2), (1,3), (2,2), (2,3), (3,3)
 * (test index l, basis index l'; 0 = pulse, 1..3 = linear in x, y, z) and
 * c = xx, yy, zz, xy, xz, yz.  Offsets with every D_i <= 1 use the
 * distributional form at Gauss order near_q, the others the smooth dyadic
 * form at the pulse orders plus one (the weights are cubic per axis).
 * Entries with linear offset index in [lo_lin, hi_lin) only. */
int vie_green_pwl_fill(int n1, int n2, int n3, double kappa, int near_q, int boost, double *out, long lo_lin,
                       long hi_lin)
{
    pwl_init();
    if (near_q < 2 || near_q > QMAX) return -1;
    long V = (long)n1 * n2 * n3;
    if (hi_lin > V) hi_lin = V;
#pragma omp parallel for schedule(dynamic, 16)
    for (long lin = lo_lin; lin < hi_lin; ++lin) {
        int D[3] = {(int)(lin % n1), (int)((lin / n1) % n2), (int)(lin / ((long)n1 * n2))};
        int d = D[0];
        if (D[1] > d) d = D[1];
        if (D[2] > d) d = D[2];
        cplx e[60];
        if (d <= 1) pwl_near_entry(D, kappa, near_q, e);
        else {
            int q = far_order(d, boost) + 1;
            pwl_far_entry(D, kappa, q > QMAX ? QMAX : q, e);
        }
        for (int m = 0; m < 60; ++m) {
            out[2 * (m * V + lin)] = creal(e[m]);
            out[2 * (m * V + lin) + 1] = cimag(e[m]);
        }
    }
    return 0;
}

/* All 60 entries at one offset D (any signs allowed) by one method at Gauss
 * order q: method 0 = distributional form (any D), 1 = smooth dyadic form
 * (needs max |D_i| >= 2).  out: 60 complex interleaved, index P * 6 + c. */
int vie_green_pwl_entry(const int D[3], double kappa, int q, int method, double *out)
{
    pwl_init();
    if (q < 2 || q > QMAX || (method != 0 && method != 1)) return -1;
    int d = abs(D[0]);
    if (abs(D[1]) > d) d = abs(D[1]);
    if (abs(D[2]) > d) d = abs(D[2]);
    if (method == 1 && d < 2) return -1;
    cplx e[60];
    if (method == 0) pwl_near_entry(D, kappa, q, e);
    else pwl_far_entry(D, kappa, q, e);
    for (int m = 0; m < 60; ++m) {
        out[2 * m] = creal(e[m]);
        out[2 * m + 1] = cimag(e[m]);
    }
    return 0;
}

/* One PWL component (pair P, dyadic c) at an offset with max |D_i| >= 2 by
 * the smooth dyadic form: the terms of pwl_far_entry for that component
 * only, in the same order. */
static cplx pwl_far_one(const int D[3], double kappa, int q, int P, int c)
{
    cplx acc = 0;
    const double *gx = gl_x[q], *gw = gl_w[q];
    const int t0 = pwl_ty[P][0], t1 = pwl_ty[P][1], t2 = pwl_ty[P][2];
    const int p = comp_p[c], qq = comp_q[c];
    for (int cell = 0; cell < 8; ++cell) {
        double lo[3];
        for (int a = 0; a < 3; ++a) lo[a] = ((cell >> a) & 1) ? 0.0 : -1.0;
        for (int ia = 0; ia < q; ++ia)
            for (int ib = 0; ib < q; ++ib)
                for (int ic = 0; ic < q; ++ic) {
                    double t[3] = {lo[0] + gx[ia], lo[1] + gx[ib], lo[2] + gx[ic]};
                    double w = gw[ia] * gw[ib] * gw[ic];
                    double x0 = D[0] + t[0], x1 = D[1] + t[1], x2 = D[2] + t[2];
                    double r2 = x0 * x0 + x1 * x1 + x2 * x2;
                    double r = sqrt(r2);
                    cplx g = ghat(r, kappa);
                    cplx ikr = I * kappa * r;
                    double xs[3] = {x0, x1, x2};
                    cplx Gd = g * (3.0 + 3.0 * ikr - kappa * kappa * r2) / (r2 * r2) * xs[p] * xs[qq];
                    if (p == qq) Gd += g * (kappa * kappa - (1.0 + ikr) / r2);
                    double v[3][4], d1[4], d2[4];
                    for (int a = 0; a < 3; ++a) pwl_axis(t[a], v[a], d1, d2);
                    acc += (w * v[0][t0] * v[1][t1] * v[2][t2]) * Gd;
                }
    }
    return acc;
}

/* Entries of one PWL component comp = 6 P + c (0..59) at offsets idx[3 t ..
 * 3 t + 2] >= 0, as vie_green_pwl_fill computes them up to rounding order:
 * the 8 offsets with every D_i in {0, 1} by the distributional form (all
 * sixty at once, evaluated once here), the others by the dyadic form of
 * that component alone.  For fiber-sampling (cross) compressions. */
int vie_green_pwl_entries(double kappa, int near_q, int boost, int comp, long count, const int *idx, double *out)
{
    pwl_init();
    if (near_q < 2 || near_q > QMAX || comp < 0 || comp > 59 || count < 0) return -1;
    const int P = comp / 6, c = comp % 6;
    cplx nearv[8];
#pragma omp parallel for schedule(static, 1)
    for (int b = 0; b < 8; ++b) {
        int D[3] = {b & 1, (b >> 1) & 1, (b >> 2) & 1};
        cplx e[60];
        pwl_near_entry(D, kappa, near_q, e);
        nearv[b] = e[comp];
    }
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(|: bad)
    for (long t = 0; t < count; ++t) {
        int D[3] = {idx[3 * t], idx[3 * t + 1], idx[3 * t + 2]};
        if (D[0] < 0 || D[1] < 0 || D[2] < 0) {
            bad = 1;
            continue;
        }
        int d = D[0];
        if (D[1] > d) d = D[1];
        if (D[2] > d) d = D[2];
        cplx e;
        if (d <= 1) e = nearv[D[0] | (D[1] << 1) | (D[2] << 2)];
        else {
            int q = far_order(d, boost) + 1;
            e = pwl_far_one(D, kappa, q > QMAX ? QMAX : q, P, c);
        }
        out[2 * t] = creal(e);
        out[2 * t + 1] = cimag(e);
    }
    return bad ? -2 : 0;
}

int vie_green_pwl_k_entries(double kappa, int near_q, int boost, int comp, long count, const int *idx,
                            double *out);

/* The same as an entry callback (ctx as vie_green_entry_cb's): comp 0..59
 * the N components 6 P + c, 60..89 the K components 60 + 3 P + c */
int vie_green_pwl_entry_cb(void *ctx, int comp, long count, const int *idx, double *out)
{
    const vie_green_ctx *g = (const vie_green_ctx *)ctx;
    if (comp >= 60) return vie_green_pwl_k_entries(g->kappa, g->near_q, g->boost, comp - 60, count, idx, out);
    return vie_green_pwl_entries(g->kappa, g->near_q, g->boost, comp, count, idx, out);
}

/* ============ the K operator in the piecewise-linear basis ============
 * Kt^{(l,l')}_pq(D) = <C^l_D e_p, K C^l'_0 e_q> / vol: test function l in
 * the observation voxel D, basis function l' in the source voxel 0, as for
 * the pulse K above.  The offset x = r - r' then carries the weight
 * W^K_D(x) = prod_a c_{type}(x_a - D_a) with the roles of test and basis
 * exchanged against N (type = [l' = a + 1] + 2 [l = a + 1]), and
 *   Kt_pq = eps_psq F_s,  F_s(D) = int d_s g^ W^K_D = -int g^ d_s W^K_D,
 * the first form on the far shells, the second (bounded first derivatives of
 * the correlations, no point masses) on the near ones.  Stored as the pulse K:
 * xy = -F_z, xz = F_y, yz = -F_x, for the ten pairs l <= l' (the others:
 * Kt^(l',l) = sigma Kt^(l,l') with the sigma of N).  A component vanishes on
 * D_a = 0 when it is odd along a: [s = a] + [type_a odd] odd. */
static int pwlk_ty[10][3];
static int pwlk_ready = 0;
static void pwlk_init(void)
{
    pwl_init();
    if (pwlk_ready) return;
    for (int P = 0; P < 10; ++P)
        for (int a = 0; a < 3; ++a)
            pwlk_ty[P][a] = (pwl_pairs[P][1] == a + 1) + 2 * (pwl_pairs[P][0] == a + 1);
    pwlk_ready = 1;
}

static void pwlk_far(const int D[3], double kappa, int q, cplx F[30])
{
    for (int m = 0; m < 30; ++m) F[m] = 0;
    const double *gx = gl_x[q], *gw = gl_w[q];
    for (int cell = 0; cell < 8; ++cell) {
        double lo[3];
        for (int a = 0; a < 3; ++a) lo[a] = ((cell >> a) & 1) ? 0.0 : -1.0;
        for (int ia = 0; ia < q; ++ia)
            for (int ib = 0; ib < q; ++ib)
                for (int ic = 0; ic < q; ++ic) {
                    double t[3] = {lo[0] + gx[ia], lo[1] + gx[ib], lo[2] + gx[ic]};
                    double w = gw[ia] * gw[ib] * gw[ic];
                    double xs[3] = {D[0] + t[0], D[1] + t[1], D[2] + t[2]};
                    double r2 = xs[0] * xs[0] + xs[1] * xs[1] + xs[2] * xs[2];
                    double r = sqrt(r2);
                    cplx dg = -ghat(r, kappa) * (1.0 + I * kappa * r) / r2;
                    double v[3][4], d1[4], d2[4];
                    for (int a = 0; a < 3; ++a) pwl_axis(t[a], v[a], d1, d2);
                    for (int P = 0; P < 10; ++P) {
                        cplx wd = (w * v[0][pwlk_ty[P][0]] * v[1][pwlk_ty[P][1]] * v[2][pwlk_ty[P][2]]) * dg;
                        for (int s = 0; s < 3; ++s) F[P * 3 + s] += wd * xs[s];
                    }
                }
    }
}

static inline void pwlk_vol_point(const double x[3], const int D[3], cplx g, cplx acc[30])
{
    double v[3][4], d1[3][4], d2[3][4];
    for (int a = 0; a < 3; ++a) pwl_axis(x[a] - D[a], v[a], d1[a], d2[a]);
    for (int P = 0; P < 10; ++P) {
        const int t0 = pwlk_ty[P][0], t1 = pwlk_ty[P][1], t2 = pwlk_ty[P][2];
        cplx *o = acc + 3 * P;
        o[0] -= g * (d1[0][t0] * v[1][t1] * v[2][t2]);
        o[1] -= g * (v[0][t0] * d1[1][t1] * v[2][t2]);
        o[2] -= g * (v[0][t0] * v[1][t1] * d1[2][t2]);
    }
}

/* -int g^ d_s W^K_D over the 8 unit cells (Duffy on cells with the origin
 * at a corner): F for all pairs, valid at every offset */
static void pwlk_near(const int D[3], double kappa, int q, cplx F[30])
{
    for (int m = 0; m < 30; ++m) F[m] = 0;
    const double *gx = gl_x[q], *gw = gl_w[q];
    for (int cell = 0; cell < 8; ++cell) {
        double lo[3], sigma[3];
        int corner = 1;
        for (int a = 0; a < 3; ++a) {
            lo[a] = D[a] + (((cell >> a) & 1) ? 0.0 : -1.0);
            if (lo[a] == 0.0) sigma[a] = 1.0;
            else if (lo[a] == -1.0) sigma[a] = -1.0;
            else corner = 0;
        }
        if (!corner) {
            for (int ia = 0; ia < q; ++ia)
                for (int ib = 0; ib < q; ++ib)
                    for (int ic = 0; ic < q; ++ic) {
                        double x[3] = {lo[0] + gx[ia], lo[1] + gx[ib], lo[2] + gx[ic]};
                        double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                        pwlk_vol_point(x, D, ghat(r, kappa) * (gw[ia] * gw[ib] * gw[ic]), F);
                    }
        } else {
            for (int face = 0; face < 3; ++face) {
                int a1 = (face + 1) % 3, a2 = (face + 2) % 3;
                for (int is = 0; is < q; ++is) {
                    double s = gx[is];
                    for (int ib = 0; ib < q; ++ib)
                        for (int ic = 0; ic < q; ++ic) {
                            double y[3];
                            y[face] = s;
                            y[a1] = s * gx[ib];
                            y[a2] = s * gx[ic];
                            double x[3] = {sigma[0] * y[0], sigma[1] * y[1], sigma[2] * y[2]};
                            double r = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
                            pwlk_vol_point(x, D, ghat(r, kappa) * (gw[is] * gw[ib] * gw[ic] * s * s), F);
                        }
                }
            }
        }
    }
}

/* F (pairs x s) into the stored components (pairs x {xy, xz, yz}), with the
 * exact zero planes of the odd components */
static void pwlk_store(const int D[3], const cplx F[30], cplx e[30])
{
    for (int P = 0; P < 10; ++P) {
        cplx f[3];
        for (int s = 0; s < 3; ++s) {
            int zero = 0;
            for (int a = 0; a < 3; ++a)
                if (D[a] == 0 && (((s == a) + (pwlk_ty[P][a] == 1 || pwlk_ty[P][a] == 2)) & 1)) zero = 1;
            f[s] = zero ? 0 : F[P * 3 + s];
        }
        e[P * 3 + 0] = -f[2];
        e[P * 3 + 1] = f[1];
        e[P * 3 + 2] = -f[0];
    }
}

/* Dense PWL K tensors: out[(((P * 3 + c) * n3 + k) * n2 + j) * n1 + i]
 * (complex128 interleaved), pairs as vie_green_pwl_fill, c = xy, xz, yz;
 * near form at order near_q on the shell max D_i <= 1, far form at the
 * pulse orders plus one elsewhere.  Dimensionless (the physical entries are
 * h times these). */
int vie_green_pwl_k_fill(int n1, int n2, int n3, double kappa, int near_q, int boost, double *out, long lo_lin,
                         long hi_lin)
{
    pwlk_init();
    if (near_q < 2 || near_q > QMAX) return -1;
    long V = (long)n1 * n2 * n3;
    if (hi_lin > V) hi_lin = V;
#pragma omp parallel for schedule(dynamic, 16)
    for (long lin = lo_lin; lin < hi_lin; ++lin) {
        int D[3] = {(int)(lin % n1), (int)((lin / n1) % n2), (int)(lin / ((long)n1 * n2))};
        int d = D[0];
        if (D[1] > d) d = D[1];
        if (D[2] > d) d = D[2];
        cplx F[30], e[30];
        if (d <= 1) pwlk_near(D, kappa, near_q, F);
        else {
            int q = far_order(d, boost) + 1;
            pwlk_far(D, kappa, q > QMAX ? QMAX : q, F);
        }
        pwlk_store(D, F, e);
        for (int m = 0; m < 30; ++m) {
            out[2 * (m * V + lin)] = creal(e[m]);
            out[2 * (m * V + lin) + 1] = cimag(e[m]);
        }
    }
    return 0;
}

/* All 30 PWL K entries at one offset D (any signs), method 0 = near form
 * (any D), 1 = far form (max |D_i| >= 2), Gauss order q; no zero planes
 * imposed.  out: 30 complex, index P * 3 + c. */
int vie_green_pwl_k_entry(const int D[3], double kappa, int q, int method, double *out)
{
    pwlk_init();
    if (q < 2 || q > QMAX || (method != 0 && method != 1)) return -1;
    int d = abs(D[0]);
    if (abs(D[1]) > d) d = abs(D[1]);
    if (abs(D[2]) > d) d = abs(D[2]);
    if (method == 1 && d < 2) return -1;
    cplx F[30];
    if (method == 0) pwlk_near(D, kappa, q, F);
    else pwlk_far(D, kappa, q, F);
    for (int P = 0; P < 10; ++P) {
        cplx e[3] = {-F[P * 3 + 2], F[P * 3 + 1], -F[P * 3 + 0]};
        for (int c = 0; c < 3; ++c) {
            out[2 * (P * 3 + c)] = creal(e[c]);
            out[2 * (P * 3 + c) + 1] = cimag(e[c]);
        }
    }
    return 0;
}

/* Entries of one PWL K component comp = 3 P + c (0..29) at offsets >= 0, as
 * vie_green_pwl_k_fill computes them up to rounding order */
int vie_green_pwl_k_entries(double kappa, int near_q, int boost, int comp, long count, const int *idx, double *out)
{
    pwlk_init();
    if (near_q < 2 || near_q > QMAX || comp < 0 || comp > 29 || count < 0) return -1;
    const int P = comp / 3, c = comp % 3;
    const int s = 2 - c;                       /* xy <- F_z, xz <- F_y, yz <- F_x */
    const double sg = (c == 1) ? 1.0 : -1.0;
    cplx nearv[8];
#pragma omp parallel for schedule(static, 1)
    for (int b = 0; b < 8; ++b) {
        int D[3] = {b & 1, (b >> 1) & 1, (b >> 2) & 1};
        cplx F[30], e[30];
        pwlk_near(D, kappa, near_q, F);
        pwlk_store(D, F, e);
        nearv[b] = e[comp];
    }
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(|: bad)
    for (long t = 0; t < count; ++t) {
        int D[3] = {idx[3 * t], idx[3 * t + 1], idx[3 * t + 2]};
        if (D[0] < 0 || D[1] < 0 || D[2] < 0) {
            bad = 1;
            continue;
        }
        int d = D[0];
        if (D[1] > d) d = D[1];
        if (D[2] > d) d = D[2];
        cplx e = 0;
        if (d <= 1) e = nearv[D[0] | (D[1] << 1) | (D[2] << 2)];
        else {
            int zero = 0;
            for (int a = 0; a < 3; ++a)
                if (D[a] == 0 && (((s == a) + (pwlk_ty[P][a] == 1 || pwlk_ty[P][a] == 2)) & 1)) zero = 1;
            if (!zero) {
                int q = far_order(d, boost) + 1;
                if (q > QMAX) q = QMAX;
                const double *gx = gl_x[q], *gw = gl_w[q];
                const int t0 = pwlk_ty[P][0], t1 = pwlk_ty[P][1], t2 = pwlk_ty[P][2];
                cplx acc = 0;
                for (int cell = 0; cell < 8; ++cell) {
                    double lo[3];
                    for (int a = 0; a < 3; ++a) lo[a] = ((cell >> a) & 1) ? 0.0 : -1.0;
                    for (int ia = 0; ia < q; ++ia)
                        for (int ib = 0; ib < q; ++ib)
                            for (int ic = 0; ic < q; ++ic) {
                                double tt[3] = {lo[0] + gx[ia], lo[1] + gx[ib], lo[2] + gx[ic]};
                                double w = gw[ia] * gw[ib] * gw[ic];
                                double xs[3] = {D[0] + tt[0], D[1] + tt[1], D[2] + tt[2]};
                                double r2 = xs[0] * xs[0] + xs[1] * xs[1] + xs[2] * xs[2];
                                double r = sqrt(r2);
                                cplx dg = -ghat(r, kappa) * (1.0 + I * kappa * r) / r2;
                                double v[3][4], d1[4], d2[4];
                                for (int a = 0; a < 3; ++a) pwl_axis(tt[a], v[a], d1, d2);
                                acc += ((w * v[0][t0] * v[1][t1] * v[2][t2]) * dg) * xs[s];
                            }
                }
                e = sg * acc;
            }
        }
        out[2 * t] = creal(e);
        out[2 * t + 1] = cimag(e);
    }
    return bad ? -2 : 0;
}
