// Tucker cross approximation of a defining tensor from its entries (FP64,
// host): the fiber-sampling alternative to the HOSVD that Sec. IV-A names
// (cross-Tucker after Oseledets, Savostyanov, Tyrtyshnikov; Rakhuba,
// Oseledets), at a cost linear in n instead of the HOSVD's O(n^3): the
// dense tensor is never formed, only the fibers the scheme asks for.
//
// Scheme (alternating fiber selection):
//  * index sets J1, J2, J3 start as s evenly spaced indices floor((t+1/2) n/s);
//  * a sweep visits the modes m = 1, 2, 3: the mode-m fibers through every
//    pair of the other two sets form C_m (n_m x |J_a||J_b|); its SVD gives
//    the rank r_m by the HOSVD's truncation rule (relative to ||C_m||_F;
//    above 96 columns and rows only the 96 leading singular triplets are
//    computed, by randomized subspace iteration, with the norm of the rest
//    formed explicitly),
//    and J_m becomes the maxvol rows of its leading min(r_m + p, numerical
//    rank) left singular vectors U_m (p = 8 by default: enough fibers through
//    the smooth far field for the interpolation to match the HOSVD's
//    accuracy there);
//  * sweeps stop when one leaves every set unchanged;
//  * interpolation form A ~= A(J1, J2, J3) x_m U_m U_m[J_m]^{-1};
//  * recompression: QR of each B_m = U_m U_m[J_m]^{-1}, the small core
//    times the R factors, its HOSVD at the same tolerance (Alg. 1), factors
//    Q_m V_m.
// maxvol: pivots of a column-pivoted QR of U^T (largest residual row norm,
// first on ties), then row swaps while an entry of U U[J]^{-1} exceeds
// 1 + 0.05 in modulus (the largest, first in row-major order on ties).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "host_compress.h"
#include "host_cross.h"

namespace vie {

using cd = std::complex<double>;

namespace {

// Inverse of a k x k row-major matrix by Gauss-Jordan with partial pivoting;
// false if a pivot is exactly zero.
bool invert(std::vector<cd>& M, int k)
{
    std::vector<cd> I((size_t)k * k, cd(0));
    for (int i = 0; i < k; ++i) I[(size_t)i * k + i] = 1.0;
    for (int col = 0; col < k; ++col) {
        int p = col;
        double best = std::abs(M[(size_t)col * k + col]);
        for (int r = col + 1; r < k; ++r) {
            const double v = std::abs(M[(size_t)r * k + col]);
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (best == 0.0) return false;
        if (p != col)
            for (int c = 0; c < k; ++c) {
                std::swap(M[(size_t)p * k + c], M[(size_t)col * k + c]);
                std::swap(I[(size_t)p * k + c], I[(size_t)col * k + c]);
            }
        const cd inv = 1.0 / M[(size_t)col * k + col];
        for (int c = 0; c < k; ++c) {
            M[(size_t)col * k + c] *= inv;
            I[(size_t)col * k + c] *= inv;
        }
        for (int r = 0; r < k; ++r) {
            if (r == col) continue;
            const cd f = M[(size_t)r * k + col];
            if (f == cd(0)) continue;
            for (int c = 0; c < k; ++c) {
                M[(size_t)r * k + c] -= f * M[(size_t)col * k + c];
                I[(size_t)r * k + c] -= f * I[(size_t)col * k + c];
            }
        }
    }
    M.swap(I);
    return true;
}

// C = A B (A: n x k, B: k x m, row-major)
void matmul(const std::vector<cd>& A, const std::vector<cd>& B, int n, int k, int m, std::vector<cd>& C)
{
    C.assign((size_t)n * m, cd(0));
    for (int i = 0; i < n; ++i)
        for (int t = 0; t < k; ++t) {
            const cd a = A[(size_t)i * k + t];
            if (a == cd(0)) continue;
            for (int j = 0; j < m; ++j) C[(size_t)i * m + j] += a * B[(size_t)t * m + j];
        }
}

// Thin QR of an n x k row-major matrix (n >= k) by classical Gram-Schmidt
// with one re-orthogonalisation pass: Q n x k, R k x k upper triangular.
void thin_qr(const std::vector<cd>& A, int n, int k, std::vector<cd>& Q, std::vector<cd>& R)
{
    Q = A;
    R.assign((size_t)k * k, cd(0));
    std::vector<cd> h(k);
    for (int j = 0; j < k; ++j) {
        for (int pass = 0; pass < 2; ++pass) {
            for (int i = 0; i < j; ++i) {
                cd acc = 0;
                for (int t = 0; t < n; ++t) acc += std::conj(Q[(size_t)t * k + i]) * Q[(size_t)t * k + j];
                h[i] = acc;
            }
            for (int i = 0; i < j; ++i) {
                R[(size_t)i * k + j] += h[i];
                for (int t = 0; t < n; ++t) Q[(size_t)t * k + j] -= h[i] * Q[(size_t)t * k + i];
            }
        }
        double nrm = 0;
        for (int t = 0; t < n; ++t) nrm += std::norm(Q[(size_t)t * k + j]);
        nrm = std::sqrt(nrm);
        R[(size_t)j * k + j] = nrm;
        if (nrm > 0)
            for (int t = 0; t < n; ++t) Q[(size_t)t * k + j] /= nrm;
    }
}

// Thin QR of an n x k row-major matrix (n >= k) by Householder reflections,
// stable also when the columns are (nearly) linearly dependent, as fiber
// matrices of a low-rank tensor are: Q n x k with orthonormal columns to
// working precision, R k x k upper triangular.
void householder_qr(const std::vector<cd>& A, int n, int k, std::vector<cd>& Q, std::vector<cd>& R)
{
    std::vector<cd> M = A;
    std::vector<std::vector<cd>> vs(k);
    for (int j = 0; j < k; ++j) {
        double nx = 0;
        for (int t = j; t < n; ++t) nx += std::norm(M[(size_t)t * k + j]);
        nx = std::sqrt(nx);
        std::vector<cd>& v = vs[j];
        v.assign((size_t)(n - j), cd(0));
        if (nx == 0.0) continue;
        const cd x0 = M[(size_t)j * k + j];
        const cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0);
        const cd alpha = -ph * nx;
        for (int t = j; t < n; ++t) v[t - j] = M[(size_t)t * k + j];
        v[0] -= alpha;
        double nv = 0;
        for (const cd& e : v) nv += std::norm(e);
        nv = std::sqrt(nv);
        if (nv == 0.0) {
            v.assign(v.size(), cd(0));
            continue;
        }
        for (cd& e : v) e /= nv;
        // M[j:, j:] -= 2 v (v^H M[j:, j:])
        for (int c = j; c < k; ++c) {
            cd d = 0;
            for (int t = j; t < n; ++t) d += std::conj(v[t - j]) * M[(size_t)t * k + c];
            d *= 2.0;
            for (int t = j; t < n; ++t) M[(size_t)t * k + c] -= d * v[t - j];
        }
    }
    R.assign((size_t)k * k, cd(0));
    for (int i = 0; i < k; ++i)
        for (int c = i; c < k; ++c) R[(size_t)i * k + c] = M[(size_t)i * k + c];
    // Q = H_0 H_1 ... H_{k-1} applied to the first k columns of the identity
    Q.assign((size_t)n * k, cd(0));
    for (int i = 0; i < k; ++i) Q[(size_t)i * k + i] = 1.0;
    for (int j = k - 1; j >= 0; --j) {
        const std::vector<cd>& v = vs[j];
        for (int c = 0; c < k; ++c) {
            cd d = 0;
            for (int t = j; t < n; ++t) d += std::conj(v[t - j]) * Q[(size_t)t * k + c];
            d *= 2.0;
            for (int t = j; t < n; ++t) Q[(size_t)t * k + c] -= d * v[t - j];
        }
    }
}

// Left singular vectors (n x q, q = min(n, K), descending) and singular
// values of the row-major n x K matrix C.
void left_svd(const std::vector<cd>& C, int n, int K, std::vector<cd>& U, int& q, std::vector<double>& s)
{
    if (n <= K) {
        std::vector<cd> Uf;
        svd_left(C.data(), n, K, Uf, s, true);
        q = n;
        U = Uf;
        return;
    }
    // n > K: C = Q R, then the left singular vectors of R (K x K)
    std::vector<cd> Q, R, Ur;
    householder_qr(C, n, K, Q, R);
    svd_left(R.data(), K, K, Ur, s, true);
    q = K;
    matmul(Q, Ur, n, K, K, U);
}

// C (n x K) times M (K x m), or C^H (K x n) times M (n x m) with `herm`;
// rows of the product on the host threads.
void mat_apply(const std::vector<cd>& C, int n, int K, const std::vector<cd>& M, int m, bool herm,
               std::vector<cd>& out)
{
    const int rows = herm ? K : n;
    out.assign((size_t)rows * m, cd(0));
    parallel_rows(rows, [&](long b, long e) {
        for (long r = b; r < e; ++r) {
            cd* o = &out[(size_t)r * m];
            if (!herm) {
                for (int t = 0; t < K; ++t) {
                    const cd a = C[(size_t)r * K + t];
                    const cd* mm = &M[(size_t)t * m];
                    for (int c = 0; c < m; ++c) o[c] += a * mm[c];
                }
            } else {
                for (int t = 0; t < n; ++t) {
                    const cd a = std::conj(C[(size_t)t * K + r]);
                    const cd* mm = &M[(size_t)t * m];
                    for (int c = 0; c < m; ++c) o[c] += a * mm[c];
                }
            }
        }
    });
}

uint64_t splitmix(uint64_t& x);

// The m leading left singular vectors (n x m) and values of C (n x K) and
// the squared Frobenius norm resid2 of what they leave out, by randomized
// subspace iteration (Halko, Martinsson, Tropp): a K x m test matrix of
// unit-modulus entries with splitmix64 phases (fixed seed), two power steps,
// orthonormalised after every product, then the exact SVD of the m x K
// projection Q^H C and resid2 = ||C - Q Q^H C||_F^2 formed explicitly (no
// cancellation).  When min(n, K) <= m every singular value is computed
// exactly instead and resid2 = 0.
void leading_svd(const std::vector<cd>& C, int n, int K, int m, std::vector<cd>& U, int& q, std::vector<double>& s,
                 double& resid2)
{
    resid2 = 0;
    if (std::min(n, K) <= m) {
        left_svd(C, n, K, U, q, s);
        return;
    }
    std::vector<cd> Om((size_t)K * m);
    uint64_t st = 0x2545F4914F6CDD1Dull;
    const double two_pi = 6.283185307179586476925286766559;
    for (auto& v : Om) v = std::polar(1.0, two_pi * (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0));
    std::vector<cd> Y, Q, R, Z, Qz;
    mat_apply(C, n, K, Om, m, false, Y);
    householder_qr(Y, n, m, Q, R);
    for (int it = 0; it < 2; ++it) {
        mat_apply(C, n, K, Q, m, true, Z);
        householder_qr(Z, K, m, Qz, R);
        mat_apply(C, n, K, Qz, m, false, Y);
        householder_qr(Y, n, m, Q, R);
    }
    // B = Q^H C (m x K) as (C^H Q)^H
    mat_apply(C, n, K, Q, m, true, Z);
    std::vector<cd> B((size_t)m * K);
    for (int k = 0; k < K; ++k)
        for (int c = 0; c < m; ++c) B[(size_t)c * K + k] = std::conj(Z[(size_t)k * m + c]);
    std::vector<cd> Ub;
    svd_left(B.data(), m, K, Ub, s, true);
    matmul(Q, Ub, n, m, m, U);
    q = m;
    // resid2 = ||C - Q B||_F^2
    std::vector<double> part(n, 0.0);
    parallel_rows(n, [&](long b, long e) {
        for (long i = b; i < e; ++i) {
            double acc = 0;
            for (int k = 0; k < K; ++k) {
                cd v = C[(size_t)i * K + k];
                for (int c = 0; c < m; ++c) v -= Q[(size_t)i * m + c] * B[(size_t)c * K + k];
                acc += std::norm(v);
            }
            part[i] = acc;
        }
    });
    for (int i = 0; i < n; ++i) resid2 += part[i];
}

// Greedy row pivots of U (n x r): r times the row of largest residual norm
// (first on ties), then its direction removed from every row.
std::vector<int> greedy_rows(const std::vector<cd>& U, int n, int r)
{
    std::vector<cd> Rm = U;
    std::vector<int> rows;
    std::vector<char> taken(n, 0);
    std::vector<cd> qv(r);
    for (int step = 0; step < r; ++step) {
        int best = -1;
        double bn = -1.0;
        for (int i = 0; i < n; ++i) {
            if (taken[i]) continue;
            double v = 0;
            for (int c = 0; c < r; ++c) v += std::norm(Rm[(size_t)i * r + c]);
            if (v > bn) {
                bn = v;
                best = i;
            }
        }
        rows.push_back(best);
        taken[best] = 1;
        const double nr = std::sqrt(bn);
        for (int c = 0; c < r; ++c) qv[c] = nr > 0 ? Rm[(size_t)best * r + c] / nr : cd(0);
        for (int i = 0; i < n; ++i) {
            cd d = 0;
            for (int c = 0; c < r; ++c) d += Rm[(size_t)i * r + c] * std::conj(qv[c]);
            for (int c = 0; c < r; ++c) Rm[(size_t)i * r + c] -= d * qv[c];
        }
    }
    return rows;
}

std::vector<int> maxvol(const std::vector<cd>& U, int n, int r)
{
    std::vector<int> rows = greedy_rows(U, n, r);
    for (int swap = 0; swap < 1000; ++swap) {
        std::vector<cd> S((size_t)r * r);
        for (int a = 0; a < r; ++a)
            for (int c = 0; c < r; ++c) S[(size_t)a * r + c] = U[(size_t)rows[a] * r + c];
        if (!invert(S, r)) break;
        std::vector<cd> B;
        matmul(U, S, n, r, r, B);
        int bi = 0, bj = 0;
        double bv = -1.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < r; ++j) {
                const double v = std::abs(B[(size_t)i * r + j]);
                if (v > bv) {
                    bv = v;
                    bi = i;
                    bj = j;
                }
            }
        if (bv <= 1.05) break;
        rows[bj] = bi;
    }
    std::sort(rows.begin(), rows.end());
    return rows;
}

// Leading singular triplets computed per fiber matrix (above every rank the
// device takes, 64, plus the oversampling)
constexpr int kLead = 96;

// Truncation rank from the leading singular values s and the squared norm
// resid2 of everything beyond them: rule 0, the smallest r whose tail
// resid2 + sum_{k >= r} s_k^2 is at most (tol / sqrt 3)^2 ||C||_F^2; rule 1,
// the count of s_k >= tol / sqrt(3) s_0.
int cross_rank(const std::vector<double>& s, double resid2, double tol, int rule, double fro)
{
    if (rule == 1 || resid2 == 0.0) return truncation_rank(s, tol, rule, fro);
    const int m = (int)s.size();
    double thr2 = tol / std::sqrt(3.0) * fro;
    thr2 *= thr2;
    double tail = resid2;
    std::vector<double> tails(m + 1);
    tails[m] = resid2;
    for (int k = m - 1; k >= 0; --k) tails[k] = tails[k + 1] + s[k] * s[k];
    (void)tail;
    for (int r = 1; r <= m; ++r)
        if (tails[r] <= thr2) return r;
    return m;
}

std::vector<int> start_indices(int n, int s)
{
    s = std::min(n, s);
    std::vector<int> J(s);
    for (int t = 0; t < s; ++t) J[t] = (int)(((2L * t + 1) * n) / (2L * s));
    return J;
}

struct Sampler {
    vie_entry_fn fn;
    void* ctx;
    int comp;
    int odd[3];
    long evals = 0;
    bool failed = false;
    bool nonfinite = false;
    // values at the index triples (count x 3, (i, j, k)), with the parity zeros
    void eval(const std::vector<int>& idx, std::vector<cd>& out)
    {
        const long count = (long)idx.size() / 3;
        std::vector<double> raw((size_t)2 * count);
        out.assign((size_t)count, cd(0));
        if (count == 0) return;
        if (fn(ctx, comp, count, idx.data(), raw.data()) != 0) failed = true;
        evals += count;
        for (long t = 0; t < count; ++t) {
            const double re = raw[2 * t], im = raw[2 * t + 1];
            if (!std::isfinite(re) || !std::isfinite(im)) nonfinite = true;
            bool zero = false;
            for (int a = 0; a < 3; ++a)
                if (odd[a] && idx[3 * t + a] == 0) zero = true;
            out[t] = zero ? cd(0) : cd(re, im);
        }
    }
};

// mode-m fibers through every (Ja x Jb) pair: n_m x (|Ja||Jb|), row-major,
// columns with the later set fastest
void fibers(Sampler& S, const int n[3], int m, const std::vector<int>& Ja, const std::vector<int>& Jb,
            std::vector<cd>& C)
{
    int a = m == 0 ? 1 : 0, b = m == 2 ? 1 : 2;
    const int K = (int)(Ja.size() * Jb.size());
    std::vector<int> idx((size_t)3 * n[m] * K);
    for (int t = 0; t < n[m]; ++t)
        for (size_t pa = 0; pa < Ja.size(); ++pa)
            for (size_t pb = 0; pb < Jb.size(); ++pb) {
                int* e = &idx[3 * ((size_t)t * K + pa * Jb.size() + pb)];
                e[m] = t;
                e[a] = Ja[pa];
                e[b] = Jb[pb];
            }
    S.eval(idx, C);
}

uint64_t splitmix(uint64_t& x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

int tucker_cross(vie_entry_fn fn, void* ctx, int comp, const int odd[3], const int n[3], const CrossParams& p,
                 TuckerComponent& out, CrossStats& st, std::string& err)
{
    Sampler S{fn, ctx, comp, {odd[0], odd[1], odd[2]}};
    std::vector<int> J[3];
    for (int m = 0; m < 3; ++m) J[m] = start_indices(n[m], p.start + p.oversample);
    std::vector<cd> U[3];
    int k[3] = {1, 1, 1};
    st.sweeps = 0;
    for (int sweep = 0; sweep < p.max_sweeps; ++sweep) {
        st.sweeps = sweep + 1;
        std::vector<int> old[3] = {J[0], J[1], J[2]};
        for (int m = 0; m < 3; ++m) {
            const int a = m == 0 ? 1 : 0, b = m == 2 ? 1 : 2;
            std::vector<cd> C;
            fibers(S, n, m, J[a], J[b], C);
            if (S.failed) {
                err = "the entry callback returned an error";
                return -1;
            }
            if (S.nonfinite) {
                err = "the entry callback returned a non-finite value";
                return -4;
            }
            const int K = (int)(J[a].size() * J[b].size());
            std::vector<cd> Uc;
            std::vector<double> s;
            int q = 0;
            double resid2 = 0;
            leading_svd(C, n[m], K, kLead, Uc, q, s, resid2);
            double fro = 0;
            for (const cd& v : C) fro += std::norm(v);
            fro = std::sqrt(fro);
            const int r = fro > 0 ? cross_rank(s, resid2, p.tol, p.rule, fro) : 1;
            int numerical = 0;
            for (int t = 0; t < q; ++t)
                if (s[0] > 0 && s[t] > s[0] * 1e-14) ++numerical;
            numerical = std::max(1, numerical);
            k[m] = std::max(1, std::min(r + p.oversample, numerical));
            k[m] = std::min(k[m], 64 + p.oversample);
            st.cross_ranks[m] = r;
            U[m].assign((size_t)n[m] * k[m], cd(0));
            for (int i = 0; i < n[m]; ++i)
                for (int c = 0; c < k[m]; ++c) U[m][(size_t)i * k[m] + c] = Uc[(size_t)i * q + c];
            J[m] = maxvol(U[m], n[m], k[m]);
        }
        if (sweep > 0 && old[0] == J[0] && old[1] == J[1] && old[2] == J[2]) break;
    }
    // interpolation form: core A(J1, J2, J3), factors U_m U_m[J_m]^{-1}
    std::vector<int> idx((size_t)3 * k[0] * k[1] * k[2]);
    for (int a = 0; a < k[0]; ++a)
        for (int b = 0; b < k[1]; ++b)
            for (int c = 0; c < k[2]; ++c) {
                int* e = &idx[3 * (((size_t)a * k[1] + b) * k[2] + c)];
                e[0] = J[0][a];
                e[1] = J[1][b];
                e[2] = J[2][c];
            }
    std::vector<cd> core;   // [a][b][c], c fastest
    S.eval(idx, core);
    if (S.failed) {
        err = "the entry callback returned an error";
        return -1;
    }
    if (S.nonfinite) {
        err = "the entry callback returned a non-finite value";
        return -4;
    }
    std::vector<cd> Q[3];
    for (int m = 0; m < 3; ++m) {
        std::vector<cd> Sm((size_t)k[m] * k[m]);
        for (int a = 0; a < k[m]; ++a)
            for (int c = 0; c < k[m]; ++c) Sm[(size_t)a * k[m] + c] = U[m][(size_t)J[m][a] * k[m] + c];
        if (!invert(Sm, k[m])) {
            err = "singular cross submatrix";
            return -5;
        }
        std::vector<cd> B, R;
        matmul(U[m], Sm, n[m], k[m], k[m], B);
        thin_qr(B, n[m], k[m], Q[m], R);
        // core x_m R: contract the mode-m index of the core with R's columns
        std::vector<cd> nc(core.size(), cd(0));
        for (int a = 0; a < k[0]; ++a)
            for (int b = 0; b < k[1]; ++b)
                for (int c = 0; c < k[2]; ++c) {
                    const int e[3] = {a, b, c};
                    cd acc = 0;
                    for (int t = 0; t < k[m]; ++t) {
                        int f[3] = {a, b, c};
                        f[m] = t;
                        acc += R[(size_t)e[m] * k[m] + t] * core[((size_t)f[0] * k[1] + f[1]) * k[2] + f[2]];
                    }
                    nc[((size_t)a * k[1] + b) * k[2] + c] = acc;
                }
        core.swap(nc);
    }
    // HOSVD of the small core (storage with the first mode fastest)
    std::vector<cd> cs(core.size());
    for (int a = 0; a < k[0]; ++a)
        for (int b = 0; b < k[1]; ++b)
            for (int c = 0; c < k[2]; ++c)
                cs[((size_t)c * k[1] + b) * k[0] + a] = core[((size_t)a * k[1] + b) * k[2] + c];
    TuckerComponent small;
    const int kk[3] = {k[0], k[1], k[2]};
    const int rc = hosvd_component(cs.data(), kk, p.tol, p.rule, p.max_rank, small);
    if (rc != 0) {
        err = "max_rank too small for tol";
        return -5;
    }
    out = TuckerComponent();
    for (int m = 0; m < 3; ++m) {
        out.r[m] = small.r[m];
        matmul(Q[m], small.U[m], n[m], k[m], small.r[m], out.U[m]);
        // the parity zeros hold exactly in the factors' row 0
        if (odd[m])
            for (int c = 0; c < out.r[m]; ++c) out.U[m][c] = 0.0;
        out.sv[m] = small.sv[m];
    }
    out.G = small.G;
    out.fro = small.fro;
    out.tail_rel = small.tail_rel;
    st.evals = S.evals;
    // a-posteriori estimate of the relative Frobenius error from seeded
    // random entries
    st.sample_rel_err = 0;
    if (p.n_sample > 0) {
        uint64_t x = p.seed ^ (0x5851F42D4C957F2Dull * (uint64_t)(comp + 1));
        std::vector<int> sidx((size_t)3 * p.n_sample);
        for (int t = 0; t < p.n_sample; ++t)
            for (int a = 0; a < 3; ++a) sidx[3 * t + a] = (int)(splitmix(x) % (uint64_t)n[a]);
        std::vector<cd> ref;
        S.eval(sidx, ref);
        double num = 0, den = 0;
        const int r1 = out.r[0], r2 = out.r[1], r3 = out.r[2];
        for (int t = 0; t < p.n_sample; ++t) {
            const int i = sidx[3 * t], j = sidx[3 * t + 1], kz = sidx[3 * t + 2];
            cd v = 0;
            for (int a = 0; a < r1; ++a)
                for (int b = 0; b < r2; ++b) {
                    const cd ab = out.U[0][(size_t)i * r1 + a] * out.U[1][(size_t)j * r2 + b];
                    for (int c = 0; c < r3; ++c)
                        v += out.G[((size_t)a * r2 + b) * r3 + c] * ab * out.U[2][(size_t)kz * r3 + c];
                }
            num += std::norm(v - ref[t]);
            den += std::norm(ref[t]);
        }
        // ||A - A~||_F^2 is estimated by V times the mean squared error at
        // the samples, and ||A~||_F is the core's norm (orthonormal factors)
        (void)den;
        double gn = 0;
        for (const cd& g : out.G) gn += std::norm(g);
        const double V = (double)n[0] * n[1] * n[2];
        st.sample_rel_err = gn > 0 ? std::sqrt(V * num / p.n_sample / gn) : 0.0;
        st.evals_sample = p.n_sample;
    }
    return 0;
}

}  // namespace vie
