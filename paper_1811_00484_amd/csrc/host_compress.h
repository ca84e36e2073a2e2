// Host-side HOSVD compression (FP64) of the Green's defining tensors.
#pragma once
#include <complex>
#include <functional>
#include <vector>

namespace vie {

struct TuckerComponent {
    int r[3] = {0, 0, 0};
    std::vector<std::complex<double>> U[3];   // U[a]: n_a x r_a row-major (left singular vectors)
    std::vector<std::complex<double>> G;      // core [r1][r2][r3], r3 fastest
    std::vector<double> sv[3];                // all singular values of each unfolding
    double fro = 0;                           // ||A||_F
    double tail_rel = 0;                      // sqrt(sum of discarded sigma^2) / ||A||_F
};

int host_threads();

// f(begin, end) over [0, n) in contiguous chunks on the host threads; each
// index is handled by exactly one call, so results written per index do not
// depend on the thread count.
void parallel_rows(long n, const std::function<void(long, long)>& f);

// job(0) .. job(count - 1) on the host threads, each job on one thread with
// every parallel loop inside it serial (results do not depend on which
// thread runs a job, as the loops' results do not depend on the thread count)
void parallel_jobs(int count, const std::function<void(int)>& job);

// Left singular vectors (U, m x m row-major, columns by descending singular
// value) and singular values of a row-major m x N matrix, m <= N.  With
// `refine`, one-sided Jacobi sweeps on Z = Q^H Y restore full accuracy;
// floor > 0 leaves out every rotation that involves a row of squared norm
// below floor * (largest), whose value then stays the row norm (used where
// such rows cannot change a rank decision).
void svd_left(const std::complex<double>* Y, int m, long N, std::vector<std::complex<double>>& U,
              std::vector<double>& s, bool refine, double floor = 0.0);

// Truncation rank for one unfolding (rule 0: Frobenius tail; rule 1: sigma cut).
int truncation_rank(const std::vector<double>& s, double tol, int rule, double fro);

// HOSVD (Alg. 1) of one defining tensor stored [k][j][i].  Returns 0, or 1 if
// max_rank forces a tail above tol.
int hosvd_component(const std::complex<double>* A, const int n[3], double tol, int rule,
                    int max_rank, TuckerComponent& out);

// CP of a Tucker core G [r1][r2][r3] (r3 fastest) with R <= min r_i terms by
// alternating least squares (the CP step of Alg. 2): start from the leading R
// left singular vectors of the core's unfoldings, then `iters` sweeps over
// modes 1, 2, 3, each the least-squares update V_i = G^(i) conj(K) M^{-1}
// (K the Khatri-Rao product of the other two factors, M the element-wise
// product of their Gram matrices).  V[a]: r_a x R row-major.  Returns the
// relative Frobenius error of the fit.
double cp_als(const std::vector<std::complex<double>>& G, const int r[3], int R, int iters,
              std::vector<std::complex<double>> V[3]);

// exp(-2 pi i m / L), exact (0, +-1) at the multiples of a quarter turn.
std::complex<double> twiddle(long m, long L);

// Rows 0..n of the length-2n DFT of the parity-s embedded columns of U (n x r).
void fourier_factor(const std::vector<std::complex<double>>& U, int n, int r, int s,
                    std::vector<std::complex<double>>& Uh);

}  // namespace vie
