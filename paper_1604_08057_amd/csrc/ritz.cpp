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
#include <thread>
#include <vector>

namespace tslov {

namespace {

using C = std::complex<double>;

// Newton corrections p(z)/p'(z) of p(z) = det(z - T) at B points at once, from the
// ratios rho_j = d_j / d_{j-1} of the leading minors d_j = (z - a_j) d_{j-1} - w_j d_{j-2}
// and the logarithmic derivatives sig_j = d_j' / d_j:
//   rho_j = (z - a_j) - w_j / rho_{j-1},
//   sig_j = (1 + (z - a_j) sig_{j-1} - w_j sig_{j-2} / rho_{j-1}) / rho_j.
// The B recurrences are independent, so they run interleaved (the division of one
// overlaps the others').  A vanishing ratio is moved off zero by a rounding-size
// amount (the matrix is scaled to unit size; the recurrence is then still accurate
// to first order).
constexpr int kB = 8;
void newton_batch(const double* ar, const double* ai, const double* wr, const double* wi, int k, const double* zr,
                  const double* zi, double* nr, double* ni) {
    constexpr double tiny = 1e-18;
    double ir[kB], ii[kB], sr[kB], si[kB], pr[kB], pi[kB];
    for (int b = 0; b < kB; ++b) {
        double rr = zr[b] - ar[0], ri = zi[b] - ai[0];
        if (rr == 0.0 && ri == 0.0) rr = tiny;
        const double d = 1.0 / (rr * rr + ri * ri);
        ir[b] = rr * d;
        ii[b] = -ri * d;
        sr[b] = ir[b];
        si[b] = ii[b];
        pr[b] = pi[b] = 0.0;
    }
    for (int j = 1; j < k; ++j) {
        const double aj = ar[j], bj = ai[j], wjr = wr[j], wji = wi[j];
        for (int b = 0; b < kB; ++b) {
            const double xr = zr[b] - aj, xi = zi[b] - bj;
            const double qr = wjr * ir[b] - wji * ii[b], qi = wjr * ii[b] + wji * ir[b];   // w_j / rho_{j-1}
            double rr = xr - qr, ri = xi - qi;
            if (rr == 0.0 && ri == 0.0) rr = tiny;
            const double d = 1.0 / (rr * rr + ri * ri);
            const double nir = rr * d, nii = -ri * d;
            const double tr = 1.0 + (xr * sr[b] - xi * si[b]) - (qr * pr[b] - qi * pi[b]);
            const double ti = (xr * si[b] + xi * sr[b]) - (qr * pi[b] + qi * pr[b]);
            pr[b] = sr[b];
            pi[b] = si[b];
            sr[b] = tr * nir - ti * nii;
            si[b] = tr * nii + ti * nir;
            ir[b] = nir;
            ii[b] = nii;
        }
    }
    for (int b = 0; b < kB; ++b) {
        const double d = 1.0 / (sr[b] * sr[b] + si[b] * si[b]);
        nr[b] = sr[b] * d;
        ni[b] = -si[b] * d;
    }
}

// Ehrlich-Aberth sweeps on the n x n scaled matrix (a, w) from the starting
// points z: each sweep takes the unsettled roots in groups of kB, forms their
// Newton corrections together, and moves each by
//   N / (1 - N sum_{m != i} 1/(z_i - z_m))
// with the current positions of the others.  A root stops once its step is at
// rounding level, or once a step below 1e-10 fails to halve (an ill-conditioned
// eigenvalue at its attainable accuracy).  Returns the sweeps used, or -1 if some
// root never settled.
int aberth(const double* ar, const double* ai, const double* wr, const double* wi, int n, C* z) {
    const double tol = 4.0 * 2.220446049250313e-16;
    std::vector<char> done(n, 0);
    std::vector<double> prev(n, INFINITY);
    std::vector<int> act;
    int sweeps = 0;
    double zr[kB], zi[kB], nr[kB], ni[kB];
    for (; sweeps < 500; ++sweeps) {
        act.clear();
        for (int i = 0; i < n; ++i)
            if (!done[i]) act.push_back(i);
        if (act.empty()) break;
        for (size_t g = 0; g < act.size(); g += kB) {
            const int m = (int)std::min<size_t>(kB, act.size() - g);
            for (int b = 0; b < kB; ++b) {
                const C zz = z[act[g + std::min(b, m - 1)]];
                zr[b] = zz.real();
                zi[b] = zz.imag();
            }
            newton_batch(ar, ai, wr, wi, n, zr, zi, nr, ni);
            for (int b = 0; b < m; ++b) {
                const int i = act[g + b];
                const C N(nr[b], ni[b]);
                const C zi_ = z[i];
                double sr = 0.0, si = 0.0;
                for (int q = 0; q < n; ++q) {
                    if (q == i) continue;
                    const double dr = zi_.real() - z[q].real(), di = zi_.imag() - z[q].imag();
                    const double d = 1.0 / (dr * dr + di * di);
                    sr += dr * d;
                    si -= di * d;
                }
                const C den = C(1.0, 0.0) - N * C(sr, si);
                const C step = N / den;
                if (!std::isfinite(step.real()) || !std::isfinite(step.imag())) {
                    done[i] = 1;
                    continue;
                }
                z[i] = zi_ - step;
                const double st = std::abs(step), sc = std::max(1.0, std::abs(z[i]));
                if (st <= tol * sc || (st < 1e-10 * sc && st > 0.5 * prev[i])) done[i] = 1;
                prev[i] = st;
            }
        }
    }
    for (int i = 0; i < n; ++i)
        if (!done[i]) return -1;
    return sweeps;
}

// Roots of the rows [0, n) by divide and conquer: the eigenvalues of the two
// diagonal halves (the coupling entry dropped) start the iteration on the whole,
// which then needs only a few sweeps; small blocks start from a circle holding
// their Gershgorin discs.  The halves of a large block run on two threads.
void eig_rec(const double* ar, const double* ai, const double* wr, const double* wi, int n, C* z, int depth,
             int* sweeps_top) {
    constexpr int kLeaf = 24;
    if (n == 1) {
        z[0] = C(ar[0], ai[0]);
        if (sweeps_top) *sweeps_top = 0;
        return;
    }
    if (n <= kLeaf) {
        C centre = 0.0;
        for (int j = 0; j < n; ++j) centre += C(ar[j], ai[j]);
        centre /= (double)n;
        double radius = 0.0;
        for (int j = 0; j < n; ++j) {
            // |T_{j,j-1} T_{j-1,j}|^(1/2) bounds the off-diagonal part after a diagonal similarity
            double r = std::abs(C(ar[j], ai[j]) - centre);
            if (j > 0) r += std::sqrt(std::hypot(wr[j], wi[j]));
            if (j + 1 < n) r += std::sqrt(std::hypot(wr[j + 1], wi[j + 1]));
            radius = std::max(radius, r);
        }
        if (!(radius > 0.0)) radius = 1.0;
        const double kPi = 3.14159265358979323846;
        for (int i = 0; i < n; ++i) z[i] = centre + radius * std::polar(1.0, 2.0 * kPi * (i + 0.25) / n + 0.4);
    } else {
        const int h = n / 2;
        // the second half's first row has no coupling to the first half
        std::vector<double> w2r(wr + h, wr + n), w2i(wi + h, wi + n);
        w2r[0] = w2i[0] = 0.0;
        // (a half whose roots did not all settle still gives starting points: the
        // sweeps on the whole refine every root)
        if (depth < 3 && n >= 96) {
            std::thread t([&] { eig_rec(ar, ai, wr, wi, h, z, depth + 1, nullptr); });
            eig_rec(ar + h, ai + h, w2r.data(), w2i.data(), n - h, z + h, depth + 1, nullptr);
            t.join();
        } else {
            eig_rec(ar, ai, wr, wi, h, z, depth + 1, nullptr);
            eig_rec(ar + h, ai + h, w2r.data(), w2i.data(), n - h, z + h, depth + 1, nullptr);
        }
        // equal starting points would make the Aberth sum singular
        for (int i = h; i < n; ++i)
            for (int m = 0; m < h; ++m)
                if (z[i] == z[m]) z[i] += C(1e-8 * std::max(1.0, std::abs(z[i])), 1e-8);
    }
    const int sw = aberth(ar, ai, wr, wi, n, z);
    if (sweeps_top) *sweeps_top = sw;
}

}  // namespace

int tridiag_eigvals(int k, const double* alpha, const double* beta, const double* gamma, double* out,
                    int nthreads) {
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
    std::vector<double> ar(k), ai(k), wr(k, 0.0), wi(k, 0.0);
    std::vector<C> z(k);
    for (int j = 0; j < k; ++j) {
        ar[j] = alpha[2 * j] / scale;
        ai[j] = alpha[2 * j + 1] / scale;
    }
    // w_j = T_{j,j-1} T_{j-1,j} (row j >= 1): the characteristic polynomial depends
    // on the off-diagonal entries only through these products
    for (int j = 1; j < k; ++j) {
        wr[j] = beta[j] * gamma[2 * j] / (scale * scale);
        wi[j] = beta[j] * gamma[2 * j + 1] / (scale * scale);
    }
    int sweeps = 0;
    eig_rec(ar.data(), ai.data(), wr.data(), wi.data(), k, z.data(), nthreads > 1 ? 0 : 99, &sweeps);
    for (int i = 0; i < k; ++i) {
        out[2 * i] = z[i].real() * scale;
        out[2 * i + 1] = z[i].imag() * scale;
    }
    return sweeps;
}

RitzSummary ritz_summary(int k, const double* alpha, const double* beta, const double* gamma, int nthreads) {
    RitzSummary r;
    if (k <= 0) return r;
    std::vector<double> ev((size_t)2 * k);
    r.sweeps = tridiag_eigvals(k, alpha, beta, gamma, ev.data(), nthreads);
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
