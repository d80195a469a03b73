// Eigenvalues of the projected matrix T_k (the Ritz values) on the host, for the
// diagnostics of a call: the smallest |Re theta| (the sign function is undefined
// on Re z = 0, Sec. 2 after eq. spectral_form) and the matrix norm it is compared
// with.  T_k is complex tridiagonal and non-Hermitian; its characteristic
// polynomial and the polynomial's logarithmic derivative follow from the
// three-term recurrence of the leading minors, so the simultaneous Ehrlich-Aberth
// iteration finds all k eigenvalues in O(k^2) work per sweep without forming a
// dense matrix (the approach of D. A. Bini, L. Gemignani and F. Tisseur, "The
// Ehrlich-Aberth method for the nonsymmetric tridiagonal eigenvalue problem",
// SIAM J. Matrix Anal. Appl. 27 (2005)).  Host code only.
#include "ritz.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace tslov {

namespace {

using C = std::complex<double>;

// Newton correction p(z)/p'(z) of p(z) = det(z - T) from the ratios
// rho_j = d_j / d_{j-1} of the leading minors d_j = (z - a_j) d_{j-1} - w_j d_{j-2}
// and the logarithmic derivatives sig_j = d_j' / d_j.  A vanishing ratio is moved
// off zero by a relative rounding-size amount (the minor recurrence is then still
// accurate to first order).
C newton_correction(const C* a, const C* w, int k, C z, double tiny) {
    C rho = z - a[0];
    if (rho == C(0.0)) rho = C(tiny, 0.0);
    C sig_prev = C(0.0), sig = C(1.0) / rho;
    for (int j = 1; j < k; ++j) {
        const C zr = z - a[j];
        const C q = w[j] / rho;                       // w_j d_{j-2} / d_{j-1}
        C rho_n = zr - q;
        if (rho_n == C(0.0)) rho_n = C(tiny, 0.0);
        const C sig_n = (C(1.0) + zr * sig - q * sig_prev) / rho_n;
        sig_prev = sig;
        sig = sig_n;
        rho = rho_n;
    }
    return C(1.0) / sig;
}

// Ehrlich-Aberth sweeps on the n x n scaled matrix (a, w) from the starting
// points z; a root stops moving once its correction is at rounding level,
// or once a correction below 1e-10 fails to halve (an ill-conditioned eigenvalue
// at its attainable accuracy).  Returns the sweeps used, or -1 if some root never
// settled.
int aberth(const C* a, const C* w, int n, C* z) {
    const double tol = 4.0 * 2.220446049250313e-16;
    const double tiny = 1e-300;
    std::vector<char> done(n, 0);
    std::vector<double> prev(n, INFINITY);
    int left = n, sweeps = 0;
    for (; sweeps < 500 && left > 0; ++sweeps) {
        for (int i = 0; i < n; ++i) {
            if (done[i]) continue;
            const C N = newton_correction(a, w, n, z[i], tiny);
            C sum = 0.0;
            for (int m = 0; m < n; ++m)
                if (m != i) sum += C(1.0) / (z[i] - z[m]);
            const C step = N / (C(1.0) - N * sum);
            if (!std::isfinite(step.real()) || !std::isfinite(step.imag())) {
                done[i] = 1;
                --left;
                continue;
            }
            z[i] -= step;
            const double st = std::abs(step), sc = std::max(1.0, std::abs(z[i]));
            if (st <= tol * sc || (st < 1e-10 * sc && st > 0.5 * prev[i])) {
                done[i] = 1;
                --left;
            }
            prev[i] = st;
        }
    }
    return left == 0 ? sweeps : -1;
}

// Roots of the rows [0, n) by divide and conquer: the eigenvalues of the two
// diagonal halves (the coupling entry dropped) start the iteration on the whole,
// which then needs only a few sweeps; small blocks start from a circle holding
// their Gershgorin discs.
int eig_rec(const C* a, const C* w, int n, C* z) {
    constexpr int kLeaf = 24;
    if (n == 1) {
        z[0] = a[0];
        return 0;
    }
    if (n <= kLeaf) {
        C centre = 0.0;
        for (int j = 0; j < n; ++j) centre += a[j];
        centre /= (double)n;
        double radius = 0.0;
        for (int j = 0; j < n; ++j) {
            // |T_{j,j-1} T_{j-1,j}|^(1/2) bounds the off-diagonal part after a diagonal similarity
            double r = std::abs(a[j] - centre);
            if (j > 0) r += std::sqrt(std::abs(w[j]));
            if (j + 1 < n) r += std::sqrt(std::abs(w[j + 1]));
            radius = std::max(radius, r);
        }
        if (!(radius > 0.0)) radius = 1.0;
        const double kPi = 3.14159265358979323846;
        for (int i = 0; i < n; ++i) z[i] = centre + radius * std::polar(1.0, 2.0 * kPi * (i + 0.25) / n + 0.4);
    } else {
        const int h = n / 2;
        std::vector<C> w2(w + h, w + n);
        w2[0] = 0.0;   // the second half's first row has no coupling to the first half
        // (a half whose roots did not all settle still gives starting points: the
        // sweeps on the whole refine every root)
        (void)eig_rec(a, w, h, z);
        (void)eig_rec(a + h, w2.data(), n - h, z + h);
        // equal starting points would make the Aberth sum singular
        for (int i = h; i < n; ++i)
            for (int m = 0; m < h; ++m)
                if (z[i] == z[m]) z[i] += C(1e-8 * std::max(1.0, std::abs(z[i])), 1e-8);
    }
    return aberth(a, w, n, z);
}

}  // namespace

int tridiag_eigvals(int k, const double* alpha, const double* beta, const double* gamma, double* out) {
    if (k <= 0) return 0;
    // scale to unit size: the iteration's stopping rule is then absolute
    double scale = 0.0;
    for (int j = 0; j < k; ++j) scale = std::max(scale, std::abs(C(alpha[2 * j], alpha[2 * j + 1])));
    for (int j = 1; j < k; ++j) {
        scale = std::max(scale, std::fabs(beta[j]));
        scale = std::max(scale, std::abs(C(gamma[2 * j], gamma[2 * j + 1])));
    }
    if (!(scale > 0.0) || !std::isfinite(scale)) {
        for (int j = 0; j < k; ++j) out[2 * j] = out[2 * j + 1] = scale > 0.0 ? NAN : 0.0;
        return scale > 0.0 ? -1 : 0;
    }
    std::vector<C> a(k), w(k, C(0.0)), z(k);
    for (int j = 0; j < k; ++j) a[j] = C(alpha[2 * j], alpha[2 * j + 1]) / scale;
    // w_j = T_{j,j-1} T_{j-1,j} (row j >= 1): the characteristic polynomial depends
    // on the off-diagonal entries only through these products
    for (int j = 1; j < k; ++j) w[j] = beta[j] * C(gamma[2 * j], gamma[2 * j + 1]) / (scale * scale);
    const int sweeps = eig_rec(a.data(), w.data(), k, z.data());
    for (int i = 0; i < k; ++i) {
        out[2 * i] = z[i].real() * scale;
        out[2 * i + 1] = z[i].imag() * scale;
    }
    return sweeps;
}

RitzSummary ritz_summary(int k, const double* alpha, const double* beta, const double* gamma) {
    RitzSummary r;
    if (k <= 0) return r;
    std::vector<double> ev((size_t)2 * k);
    r.sweeps = tridiag_eigvals(k, alpha, beta, gamma, ev.data());
    double mn = INFINITY;
    for (int i = 0; i < k; ++i) mn = std::min(mn, std::fabs(ev[2 * i]));
    r.min_abs_re = mn;
    // infinity norm of T_k (largest absolute row sum)
    double nt = 0.0;
    for (int j = 0; j < k; ++j) {
        double row = std::hypot(alpha[2 * j], alpha[2 * j + 1]);
        if (j > 0) row += std::fabs(beta[j]);
        if (j + 1 < k) row += std::hypot(gamma[2 * (j + 1)], gamma[2 * (j + 1) + 1]);
        nt = std::max(nt, row);
    }
    r.norm_T = nt;
    return r;
}

}  // namespace tslov
