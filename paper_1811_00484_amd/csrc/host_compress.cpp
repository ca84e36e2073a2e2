// Host-side HOSVD compression of the Green's defining tensors (FP64).
//
// Implements the compression of Sec. IV-A (Alg. 1): for each unfolding A^(i)
// of a defining tensor, its left singular vectors and singular values; the
// truncation rank r_i; the core G = A x1 U1^* x2 U2^* x3 U3^*.  Then the
// circulant embedding and DFT of the factor columns (Sec. V-A), keeping only
// rows 0..n_i of each transformed factor (the rest follow from the parity of
// the component along that axis).
//
// SVD of an unfolding Y (m x N, m <= N): Gram matrix Y Y^H, cyclic two-sided
// Jacobi on it (cheap, m x m), then one-sided Jacobi sweeps on the rows of
// Z = Q^H Y until they are orthogonal to working precision, which restores
// the accuracy of the small singular values that the Gram matrix squares
// away.  Left singular vectors are the columns of the accumulated Q,
// singular values the row norms of Z.
#include "host_compress.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <thread>
#include <vector>

namespace vie {

using cd = std::complex<double>;

int host_threads()
{
    const char* e = std::getenv("VIE_NUM_THREADS");
    int n = e ? std::atoi(e) : 0;
    if (n <= 0) {
        n = (int)std::thread::hardware_concurrency();
        if (n <= 0) n = 1;
        if (n > 16) n = 16;
    }
    return n;
}

// Set on the threads of parallel_jobs: work inside a job runs serially.
static thread_local bool tl_serial = false;

// Run f(begin, end) over [0, n) split into contiguous chunks on host threads.
template <class F>
static void parallel_for(long n, F f, long min_chunk = 1)
{
    int nt = tl_serial ? 1 : host_threads();
    long chunks = std::min<long>(nt, std::max<long>(1, n / std::max<long>(1, min_chunk)));
    if (chunks <= 1) {
        f(0L, n);
        return;
    }
    std::vector<std::thread> th;
    long per = (n + chunks - 1) / chunks;
    for (long c = 0; c < chunks; ++c) {
        long b = c * per, e = std::min(n, b + per);
        if (b >= e) break;
        th.emplace_back([=]() { f(b, e); });
    }
    for (auto& t : th) t.join();
}

void parallel_rows(long n, const std::function<void(long, long)>& f)
{
    parallel_for(n, [&](long b, long e) { f(b, e); });
}

void parallel_jobs(int count, const std::function<void(int)>& job)
{
    const int nt = std::min(host_threads(), count);
    if (nt <= 1 || tl_serial) {
        for (int i = 0; i < count; ++i) job(i);
        return;
    }
    std::atomic<int> next(0);
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&]() {
            tl_serial = true;
            for (int i; (i = next.fetch_add(1)) < count;) job(i);
        });
    for (auto& t : th) t.join();
}

// Jacobi rotation parameters diagonalising [[a, c], [conj(c), b]] (a, b
// real): returns cs, sn and the phase e^{i phi} of c.  The transform is
// J = [[cs, sn], [-ph* sn, ph* cs]], J^H M J diagonal.
static inline void jacobi_params(double a, double b, cd c, double& cs, double& sn, cd& ph)
{
    double ac = std::abs(c);
    ph = c / ac;
    double zeta = (b - a) / (2.0 * ac);
    double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
    cs = 1.0 / std::sqrt(1.0 + t * t);
    sn = t * cs;
}

// Round-robin tournament (circle method): m players, padded to even M;
// round r pairs position i with position M-1-i, where position 0 holds
// player 0 and position i >= 1 holds player 1 + (i - 1 + r) mod (M - 1).
// Every pair meets exactly once over the M - 1 rounds; pairs of one round
// are disjoint, so they can be rotated in parallel.
static void tournament_pairs(int m, int r, std::vector<std::pair<int, int>>& out)
{
    int M = m + (m & 1);
    out.clear();
    auto at = [&](int i) { return i == 0 ? 0 : 1 + ((i - 1 + r) % (M - 1)); };
    for (int i = 0; i < M / 2; ++i) {
        int p = at(i), q = at(M - 1 - i);
        if (p >= m || q >= m) continue;
        out.emplace_back(std::min(p, q), std::max(p, q));
    }
}

// Left singular vectors (columns of U, m x m, row-major U[i*m + col]) and
// singular values (descending) of Y (m x N row-major).  `refine` selects the
// one-sided Jacobi pass on Z = Q^H Y after the Gram eigen-decomposition.
void svd_left(const cd* Y, int m, long N, std::vector<cd>& U, std::vector<double>& s, bool refine, double floor)
{
    // Gram matrix G = Y Y^H.  The columns are cut into chunks of CH and the
    // chunks into NG contiguous groups whose count does not depend on the
    // thread count; each group is summed chunk by chunk in order into its
    // own m x m accumulator (upper triangle) by one thread, and the groups
    // are then added in group order.  The rounding is therefore the same
    // for any number of threads.
    const long CH = 512;
    long nch = (N + CH - 1) / CH;
    const int NG = (int)std::min<long>(16, nch);
    std::vector<std::vector<cd>> part(NG, std::vector<cd>((size_t)m * m, cd(0)));
    parallel_for(NG, [&](long gb, long ge) {
        for (long g = gb; g < ge; ++g) {
            std::vector<cd>& P = part[g];
            const long c0 = g * nch / NG, c1 = (g + 1) * nch / NG;
            for (long c = c0; c < c1; ++c) {
                long b = c * CH, e = std::min(N, b + CH);
                for (int i = 0; i < m; ++i) {
                    const cd* yi = Y + (size_t)i * N;
                    for (int j = i; j < m; ++j) {
                        const cd* yj = Y + (size_t)j * N;
                        double re = 0, im = 0;
                        for (long n = b; n < e; ++n) {
                            double ar = yi[n].real(), ai = yi[n].imag();
                            double br = yj[n].real(), bi = yj[n].imag();
                            re += ar * br + ai * bi;
                            im += ai * br - ar * bi;
                        }
                        P[(size_t)i * m + j] += cd(re, im);
                    }
                }
            }
        }
    });
    std::vector<cd> G((size_t)m * m);
    for (int i = 0; i < m; ++i)
        for (int j = i; j < m; ++j) {
            cd acc = 0;
            for (int g = 0; g < NG; ++g) acc += part[g][(size_t)i * m + j];
            G[(size_t)i * m + j] = acc;
            G[(size_t)j * m + i] = std::conj(acc);
        }
    part.clear();
    // cyclic two-sided Jacobi on G, accumulate Q (columns = eigenvectors)
    std::vector<cd> Q((size_t)m * m, cd(0));
    for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
    double gnorm = 0;
    for (auto& v : G) gnorm += std::norm(v);
    gnorm = std::sqrt(gnorm);
    for (int sweep = 0; sweep < 60 && m > 1; ++sweep) {
        double off = 0;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) off += std::norm(G[(size_t)p * m + q]);
        if (std::sqrt(off) <= 1e-15 * gnorm) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                cd c = G[(size_t)p * m + q];
                if (std::abs(c) <= 1e-300) continue;
                double a = G[(size_t)p * m + p].real(), b = G[(size_t)q * m + q].real();
                double cs, sn;
                cd ph;
                jacobi_params(a, b, c, cs, sn, ph);
                // G <- J^H G J : columns then rows
                for (int k = 0; k < m; ++k) {
                    cd gp = G[(size_t)k * m + p], gq = G[(size_t)k * m + q];
                    G[(size_t)k * m + p] = cs * gp - std::conj(ph) * sn * gq;
                    G[(size_t)k * m + q] = sn * gp + std::conj(ph) * cs * gq;
                }
                for (int k = 0; k < m; ++k) {
                    cd gp = G[(size_t)p * m + k], gq = G[(size_t)q * m + k];
                    G[(size_t)p * m + k] = cs * gp - ph * sn * gq;
                    G[(size_t)q * m + k] = sn * gp + ph * cs * gq;
                }
                for (int k = 0; k < m; ++k) {
                    cd vp = Q[(size_t)k * m + p], vq = Q[(size_t)k * m + q];
                    Q[(size_t)k * m + p] = cs * vp - std::conj(ph) * sn * vq;
                    Q[(size_t)k * m + q] = sn * vp + std::conj(ph) * cs * vq;
                }
            }
    }
    std::vector<double> nrm(m);
    if (!refine) {
        for (int i = 0; i < m; ++i) nrm[i] = std::max(0.0, G[(size_t)i * m + i].real());
    } else {
        // Z = Q^H Y (column chunks in parallel)
        std::vector<cd> Z((size_t)m * N);
        parallel_for(nch, [&](long cb, long ce) {
            for (long c = cb; c < ce; ++c) {
                long b = c * CH, e = std::min(N, b + CH);
                for (int i = 0; i < m; ++i) {
                    cd* zi = &Z[(size_t)i * N];
                    for (long n = b; n < e; ++n) zi[n] = 0;
                    for (int k = 0; k < m; ++k) {
                        cd q = std::conj(Q[(size_t)k * m + i]);
                        const cd* yk = Y + (size_t)k * N;
                        for (long n = b; n < e; ++n) zi[n] += q * yk[n];
                    }
                }
            }
        });
        // one-sided Jacobi on the rows of Z (tournament order, pairs in parallel)
        parallel_for(m, [&](long b, long e) {
            for (long i = b; i < e; ++i) {
                double acc = 0;
                const cd* z = &Z[(size_t)i * N];
                for (long n = 0; n < N; ++n) acc += std::norm(z[n]);
                nrm[i] = acc;
            }
        });
        // pairs whose rows both carry less than 1e-12 of the largest singular
        // value are left alone: they cannot change any rank decision
        double amax = 0;
        for (int i = 0; i < m; ++i) amax = std::max(amax, nrm[i]);
        const double negligible = 1e-24 * amax;
        // rows count as orthogonal once their cosine is within the rounding
        // of a length-N dot product (a fixed 4e-16 never settles on long rows)
        const double rot_eps = 4e-16 * std::max(1.0, std::sqrt((double)N) / 8.0);
        const double skip_one = floor * amax;
        std::vector<std::pair<int, int>> pairs;
        for (int sweep = 0; sweep < 30 && m > 1; ++sweep) {
            std::atomic<int> rotated(0);
            int M = m + (m & 1);
            for (int r = 0; r < M - 1; ++r) {
                tournament_pairs(m, r, pairs);
                // the pairs of a round touch disjoint rows, so their order
                // does not matter; short rows are not worth a thread each
                const long serial_below = N < (1L << 14) ? (long)pairs.size() + 1 : 1;
                parallel_for((long)pairs.size(), [&](long b, long e) {
                    for (long t = b; t < e; ++t) {
                        int p = pairs[t].first, q = pairs[t].second;
                        double a = nrm[p], bb = nrm[q];
                        if (a < negligible && bb < negligible) continue;
                        if (a < skip_one || bb < skip_one) continue;
                        cd* zp = &Z[(size_t)p * N];
                        cd* zq = &Z[(size_t)q * N];
                        cd c = 0;
                        for (long n = 0; n < N; ++n) c += zp[n] * std::conj(zq[n]);
                        if (std::abs(c) <= rot_eps * std::sqrt(a * bb) || std::abs(c) == 0.0) continue;
                        rotated.fetch_add(1);
                        double cs, sn;
                        cd ph;
                        jacobi_params(a, bb, c, cs, sn, ph);
                        double na = 0, nb = 0;
                        for (long n = 0; n < N; ++n) {
                            cd x = zp[n], y = zq[n];
                            cd xp = cs * x - ph * sn * y;
                            cd yp = sn * x + ph * cs * y;
                            zp[n] = xp;
                            zq[n] = yp;
                            na += std::norm(xp);
                            nb += std::norm(yp);
                        }
                        nrm[p] = na;
                        nrm[q] = nb;
                        for (int k = 0; k < m; ++k) {
                            cd vp = Q[(size_t)k * m + p], vq = Q[(size_t)k * m + q];
                            Q[(size_t)k * m + p] = cs * vp - std::conj(ph) * sn * vq;
                            Q[(size_t)k * m + q] = sn * vp + std::conj(ph) * cs * vq;
                        }
                    }
                }, serial_below);
            }
            if (rotated.load() == 0) break;
        }
    }
    // sort by singular value, descending
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nrm[a] > nrm[b]; });
    U.assign((size_t)m * m, 0);
    s.resize(m);
    for (int c = 0; c < m; ++c) {
        s[c] = std::sqrt(std::max(0.0, nrm[order[c]]));
        for (int k = 0; k < m; ++k) U[(size_t)k * m + c] = Q[(size_t)k * m + order[c]];
    }
}

int truncation_rank(const std::vector<double>& s, double tol, int rule, double fro)
{
    int m = (int)s.size();
    if (m == 0 || s[0] == 0.0) return 1;
    if (rule == 1) {
        int r = 0;
        for (int k = 0; k < m; ++k)
            if (s[k] >= tol / std::sqrt(3.0) * s[0]) ++r;
        return std::max(1, r);
    }
    double thr2 = tol / std::sqrt(3.0) * fro;
    thr2 *= thr2;
    std::vector<double> tail(m + 1, 0.0);
    for (int k = m - 1; k >= 0; --k) tail[k] = tail[k + 1] + s[k] * s[k];
    for (int r = 1; r <= m; ++r)
        if (tail[r] <= thr2) return r;
    return m;
}

// Unfolding of A (storage [k][j][i], i fastest) along `mode` (1, 2, 3) into
// a row-major m x N matrix.
static void unfold(const cd* A, int n1, int n2, int n3, int mode, std::vector<cd>& Y)
{
    long V = (long)n1 * n2 * n3;
    Y.resize(V);
    if (mode == 1) {            // rows i, columns (j, k)
        parallel_for(n1, [&](long b, long e) {
            for (long i = b; i < e; ++i)
                for (long k = 0; k < n3; ++k)
                    for (long j = 0; j < n2; ++j)
                        Y[(size_t)i * n2 * n3 + k * n2 + j] = A[(k * n2 + j) * n1 + i];
        });
    } else if (mode == 2) {     // rows j, columns (i, k)
        parallel_for(n2, [&](long b, long e) {
            for (long j = b; j < e; ++j)
                for (long k = 0; k < n3; ++k)
                    for (long i = 0; i < n1; ++i)
                        Y[(size_t)j * n1 * n3 + k * n1 + i] = A[(k * n2 + j) * n1 + i];
        });
    } else {                    // rows k, columns (i, j)
        parallel_for(n3, [&](long b, long e) {
            for (long k = b; k < e; ++k)
                for (long j = 0; j < n2; ++j)
                    for (long i = 0; i < n1; ++i)
                        Y[(size_t)k * n1 * n2 + j * n1 + i] = A[(k * n2 + j) * n1 + i];
        });
    }
}

int hosvd_component(const cd* A, const int n[3], double tol, int rule, int max_rank,
                    TuckerComponent& out)
{
    int n1 = n[0], n2 = n[1], n3 = n[2];
    double fro = 0;
    long V = (long)n1 * n2 * n3;
    for (long t = 0; t < V; ++t) fro += std::norm(A[t]);
    fro = std::sqrt(fro);
    out.fro = fro;
    std::vector<cd> Y, Ufull;
    double tail2 = 0;
    for (int mode = 1; mode <= 3; ++mode) {
        int m = n[mode - 1];
        unfold(A, n1, n2, n3, mode, Y);
        std::vector<double> s;
        // the Gram eigenvectors resolve singular values down to ~1e-8 sigma_max;
        // the Jacobi refinement restores full accuracy when a tight tolerance
        // needs it, and always on unfoldings up to 2^24 entries times m, so
        // that the factors there agree with an exact SVD to ~1e-14 (without
        // it a 40 x 24 x 64 K tensor's agree to ~1e-10 only); it costs about
        // 0.7 s per 60^3 tensor
        const bool small = (long)m * V <= (long)1 << 24;
        bool refine = tol < 1e-7 || small;
        // on very large unfoldings (more than 2^28 entries times m), rows far
        // below the truncation level (squared norm under (1e-3 tol)^2 of the
        // largest: together less than 1e-6 of the allowed tail) are left out
        // of the rotations; the error bound is unchanged, the kept subspace
        // then differs from the exact SVD's by far less than tol
        const double floor = (long)m * V > (long)1 << 28 ? (1e-3 * tol) * (1e-3 * tol) : 0.0;
        svd_left(Y.data(), m, V / m, Ufull, s, refine, floor);
        int r = truncation_rank(s, tol, rule, fro);
        int status = 0;
        if (max_rank > 0 && r > max_rank) {
            r = max_rank;
            status = 1;
        }
        for (int k = r; k < m; ++k) tail2 += s[k] * s[k];
        out.r[mode - 1] = r;
        out.sv[mode - 1] = s;
        out.U[mode - 1].assign((size_t)m * r, 0);
        for (int i = 0; i < m; ++i)
            for (int c = 0; c < r; ++c) out.U[mode - 1][(size_t)i * r + c] = Ufull[(size_t)i * m + c];
        if (status && std::sqrt(tail2) > tol * fro) return 1;
    }
    out.tail_rel = fro > 0 ? std::sqrt(tail2) / fro : 0.0;
    // core G[a][b][c] = sum_{ijk} A[k][j][i] conj(U1[i][a]) conj(U2[j][b]) conj(U3[k][c])
    int r1 = out.r[0], r2 = out.r[1], r3 = out.r[2];
    std::vector<cd> B1((size_t)n3 * n2 * r1);      // [k][j][a]
    parallel_for((long)n3 * n2, [&](long b, long e) {
        for (long kj = b; kj < e; ++kj)
            for (int a = 0; a < r1; ++a) {
                cd acc = 0;
                for (int i = 0; i < n1; ++i) acc += A[kj * n1 + i] * std::conj(out.U[0][(size_t)i * r1 + a]);
                B1[(size_t)kj * r1 + a] = acc;
            }
    });
    std::vector<cd> B2((size_t)n3 * r2 * r1);      // [k][b][a]
    parallel_for(n3, [&](long b0, long e0) {
        for (long k = b0; k < e0; ++k)
            for (int bb = 0; bb < r2; ++bb)
                for (int a = 0; a < r1; ++a) {
                    cd acc = 0;
                    for (int j = 0; j < n2; ++j)
                        acc += B1[((size_t)k * n2 + j) * r1 + a] * std::conj(out.U[1][(size_t)j * r2 + bb]);
                    B2[((size_t)k * r2 + bb) * r1 + a] = acc;
                }
    });
    out.G.assign((size_t)r1 * r2 * r3, 0);         // [a][b][c], c fastest
    parallel_for(r1, [&](long b0, long e0) {
        for (long a = b0; a < e0; ++a)
            for (int bb = 0; bb < r2; ++bb)
                for (int c = 0; c < r3; ++c) {
                    cd acc = 0;
                    for (int k = 0; k < n3; ++k)
                        acc += B2[((size_t)k * r2 + bb) * r1 + a] * std::conj(out.U[2][(size_t)k * r3 + c]);
                    out.G[((size_t)a * r2 + bb) * r3 + c] = acc;
                }
    });
    return 0;
}

// Rows 0..n of the DFT (length 2n, exp(-2 pi i m k / 2n)) of the embedded
// columns e[m] = U[m] (m < n), e[n] = 0, e[2n - m] = s U[m] (1 <= m < n).
// element (a, b, c) of the core, math order, r3 fastest
static inline cd core_at(const std::vector<cd>& G, const int r[3], int a, int b, int c)
{
    return G[((size_t)a * r[1] + b) * r[2] + c];
}

// Mode-`mode` unfolding of the core with the column order (other axes in
// increasing axis order, the later one fastest): rows r_mode, columns
// r_p r_q with (p, q) the other two axes.
static void core_unfold(const std::vector<cd>& G, const int r[3], int mode, std::vector<cd>& Y)
{
    const int p = mode == 0 ? 1 : 0, q = mode == 2 ? 1 : 2;
    const int nr = r[mode], np = r[p], nq = r[q];
    Y.assign((size_t)nr * np * nq, 0);
    for (int i = 0; i < nr; ++i)
        for (int x = 0; x < np; ++x)
            for (int y = 0; y < nq; ++y) {
                int idx[3];
                idx[mode] = i;
                idx[p] = x;
                idx[q] = y;
                Y[((size_t)i * np + x) * nq + y] = core_at(G, r, idx[0], idx[1], idx[2]);
            }
}

// Solve X M = B for X (rows x R) with M (R x R): Gauss-Jordan with partial
// pivoting on M^T; a (near) singular pivot is replaced by a tiny ridge.
static void solve_right(std::vector<cd>& B, int rows, const std::vector<cd>& M, int R)
{
    std::vector<cd> A((size_t)R * R);   // A = M^T
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < R; ++j) A[(size_t)i * R + j] = M[(size_t)j * R + i];
    // right-hand sides: columns of B^T, i.e. rows of B
    std::vector<cd> Bt((size_t)R * rows);
    for (int t = 0; t < rows; ++t)
        for (int l = 0; l < R; ++l) Bt[(size_t)l * rows + t] = B[(size_t)t * R + l];
    double scale = 0;
    for (int i = 0; i < R; ++i) scale = std::max(scale, std::abs(A[(size_t)i * R + i]));
    for (int k = 0; k < R; ++k) {
        int piv = k;
        for (int i = k + 1; i < R; ++i)
            if (std::abs(A[(size_t)i * R + k]) > std::abs(A[(size_t)piv * R + k])) piv = i;
        if (piv != k) {
            for (int j = 0; j < R; ++j) std::swap(A[(size_t)k * R + j], A[(size_t)piv * R + j]);
            for (int t = 0; t < rows; ++t) std::swap(Bt[(size_t)k * rows + t], Bt[(size_t)piv * rows + t]);
        }
        cd d = A[(size_t)k * R + k];
        if (std::abs(d) <= 1e-14 * scale) d = A[(size_t)k * R + k] = cd(1e-14 * (scale > 0 ? scale : 1.0));
        for (int i = 0; i < R; ++i) {
            if (i == k) continue;
            const cd f = A[(size_t)i * R + k] / d;
            if (f == cd(0)) continue;
            for (int j = k; j < R; ++j) A[(size_t)i * R + j] -= f * A[(size_t)k * R + j];
            for (int t = 0; t < rows; ++t) Bt[(size_t)i * rows + t] -= f * Bt[(size_t)k * rows + t];
        }
    }
    for (int k = 0; k < R; ++k) {
        const cd d = A[(size_t)k * R + k];
        for (int t = 0; t < rows; ++t) B[(size_t)t * R + k] = Bt[(size_t)k * rows + t] / d;
    }
}

double cp_als(const std::vector<cd>& G, const int r[3], int R, int iters, std::vector<cd> V[3])
{
    std::vector<cd> Y;
    double gn = 0;
    for (const cd& g : G) gn += std::norm(g);
    gn = std::sqrt(gn);
    // start: leading R left singular vectors of each unfolding
    for (int m = 0; m < 3; ++m) {
        core_unfold(G, r, m, Y);
        std::vector<cd> U;
        std::vector<double> s;
        const long cols = (long)r[(m + 1) % 3] * r[(m + 2) % 3];
        if (r[m] <= cols) {
            svd_left(Y.data(), r[m], cols, U, s, true);
        } else {
            U.assign((size_t)r[m] * r[m], 0);
            for (int i = 0; i < r[m]; ++i) U[(size_t)i * r[m] + i] = 1.0;
        }
        // columns beyond the r_m singular vectors (a CP rank above this
        // mode's Tucker rank): generic deterministic phases
        // exp(2 pi i frac(g (i + 1) (l + 1))) / sqrt(r_m), g = (sqrt 5 - 1) / 2
        const double g = (std::sqrt(5.0) - 1.0) / 2.0;
        const double two_pi = 6.283185307179586476925286766559;
        V[m].assign((size_t)r[m] * R, 0);
        for (int i = 0; i < r[m]; ++i)
            for (int l = 0; l < R; ++l) {
                if (l < r[m]) {
                    V[m][(size_t)i * R + l] = U[(size_t)i * r[m] + l];
                } else {
                    const double t = g * (double)(i + 1) * (double)(l + 1);
                    const double ph = t - std::floor(t);
                    V[m][(size_t)i * R + l] = std::polar(1.0 / std::sqrt((double)r[m]), two_pi * ph);
                }
            }
    }
    auto fit_error = [&]() {
        double e = 0;
        for (int a = 0; a < r[0]; ++a)
            for (int b = 0; b < r[1]; ++b)
                for (int c = 0; c < r[2]; ++c) {
                    cd acc = 0;
                    for (int l = 0; l < R; ++l)
                        acc += V[0][(size_t)a * R + l] * V[1][(size_t)b * R + l] * V[2][(size_t)c * R + l];
                    e += std::norm(core_at(G, r, a, b, c) - acc);
                }
        return gn > 0 ? std::sqrt(e) / gn : 0.0;
    };
    std::vector<cd> K, M((size_t)R * R), B;
    for (int it = 0; it < iters; ++it) {
        for (int m = 0; m < 3; ++m) {
            const int p = m == 0 ? 1 : 0, q = m == 2 ? 1 : 2;
            const int np = r[p], nq = r[q];
            // K[x nq + y, l] = V_p[x, l] V_q[y, l]
            K.assign((size_t)np * nq * R, 0);
            for (int x = 0; x < np; ++x)
                for (int y = 0; y < nq; ++y)
                    for (int l = 0; l < R; ++l)
                        K[((size_t)x * nq + y) * R + l] = V[p][(size_t)x * R + l] * V[q][(size_t)y * R + l];
            // M = (V_p^T conj V_p) * (V_q^T conj V_q)
            for (int l = 0; l < R; ++l)
                for (int k = 0; k < R; ++k) {
                    cd gp = 0, gq = 0;
                    for (int x = 0; x < np; ++x) gp += V[p][(size_t)x * R + l] * std::conj(V[p][(size_t)x * R + k]);
                    for (int y = 0; y < nq; ++y) gq += V[q][(size_t)y * R + l] * std::conj(V[q][(size_t)y * R + k]);
                    M[(size_t)l * R + k] = gp * gq;
                }
            // B = G^(m) conj(K)
            core_unfold(G, r, m, Y);
            const long cols = (long)np * nq;
            B.assign((size_t)r[m] * R, 0);
            for (int i = 0; i < r[m]; ++i)
                for (long t = 0; t < cols; ++t) {
                    const cd y = Y[(size_t)i * cols + t];
                    if (y == cd(0)) continue;
                    for (int l = 0; l < R; ++l) B[(size_t)i * R + l] += y * std::conj(K[(size_t)t * R + l]);
                }
            solve_right(B, r[m], M, R);
            V[m] = B;
        }
    }
    return fit_error();
}

cd twiddle(long m, long L)
{
    m %= L;
    if (m < 0) m += L;
    if ((4 * m) % L == 0) {
        switch ((4 * m) / L) {
        case 0: return cd(1.0, 0.0);
        case 1: return cd(0.0, -1.0);
        case 2: return cd(-1.0, 0.0);
        default: return cd(0.0, 1.0);
        }
    }
    const double ang = -2.0 * M_PI * (double)m / (double)L;
    return cd(std::cos(ang), std::sin(ang));
}

void fourier_factor(const std::vector<cd>& U, int n, int r, int s, std::vector<cd>& Uh)
{
    int L = 2 * n;
    std::vector<cd> w(L);
    for (int m = 0; m < L; ++m) w[m] = twiddle(m, L);
    Uh.assign((size_t)(n + 1) * r, 0);
    for (int k = 0; k <= n; ++k)
        for (int c = 0; c < r; ++c) {
            cd acc = 0;
            for (int m = 0; m < n; ++m) {
                const cd& wk = w[((long)m * k) % L];
                cd u = U[(size_t)m * r + c];
                acc += u * wk;
                if (m >= 1) acc += (double)s * u * std::conj(wk);
            }
            Uh[(size_t)k * r + c] = acc;
        }
}

}  // namespace vie
