// Host-side eigenvalues of the tridiagonal projected matrix T_k (ritz.cpp).
#pragma once

namespace tslov {

// Eigenvalues of the k x k complex tridiagonal T with (0-based rows)
//   T[j][j] = alpha[j],  T[j][j-1] = beta[j] (real),  T[j-1][j] = gamma[j]   (j >= 1),
// alpha and gamma as interleaved (re, im) pairs; beta[0] and gamma[0] are not read.
// out: 2k doubles (re, im).  Returns the sweeps used (>= 0), or -1 when some
// eigenvalue did not settle to rounding level (out still holds the last iterates).
// nthreads > 1 runs the divide-and-conquer halves of a large matrix on threads of their own.
int tridiag_eigvals(int k, const double* alpha, const double* beta, const double* gamma, double* out,
                    int nthreads = 1);

struct RitzSummary {
    double min_abs_re = 0.0;   // min_i |Re theta_i|
    double norm_T = 0.0;       // infinity norm of T
    int sweeps = 0;            // as tridiag_eigvals
};
RitzSummary ritz_summary(int k, const double* alpha, const double* beta, const double* gamma, int nthreads = 1);

}  // namespace tslov
