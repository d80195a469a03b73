// Host-side launchers of the tslov kernels (internal interface between the
// kernel translation units and the C ABI in api.hip).
#pragma once

#include "common.h"

namespace tslov {

inline int grid_for(int n, int blk = kBlock) { return (n + blk - 1) / blk; }

// Optional event pair recorded by the dispatch of one launch (kernel timing).
struct Timing {
    hipEvent_t a = nullptr;
    hipEvent_t b = nullptr;
};

// ---------------------------------------------------------------- layout
// Also stores 1 into *bad (device int) if some link element is not finite.
void launch_links_to_soa(const ZD* Ucanon, ZD* U64, Z<float>* U32, const Geom& g, int antiperiodic, int* bad,
                         hipStream_t st);
template <typename R>
void launch_spinor_to_soa(const ZD* in, Z<R>* out, const Geom& g, double* part_norm, hipStream_t st);
template <typename R>
void launch_spinor_from_soa(const Z<R>* in, ZD* out, const Geom& g, hipStream_t st);

// ---------------------------------------------------------------- operator
// out = G5out * (G5in in - kappa * hop_{mu}(G5in in))
template <typename R, typename RL>
void launch_apply(const Z<RL>* U, const Z<R>* in, Z<R>* out, const Geom& g, double kappa, double mu,
                  int g5_in, int g5_out, hipStream_t st, Timing t = {}, int tm_T = 0);
// The t-slices per chunk the t-march operator can run this lattice with (each
// gives the same result), at most maxn of them into T; 0 when it does not apply.
// launch_apply's tm_T picks one (0: the built-in choice).
int tmarch_chunks(const Geom& g, int* T, int maxn);

// ---------------------------------------------------------------- batch workspace
// Per-source lattice fields of a batch in the working precision.  Sources sit in
// batch slots; every per-step array holds kcap fields per slot (step j at j - 1).
constexpr int kNF = 8;   // per-slot fields: 0 psi, 1 eta, 2 r, 3 s, 4 vbar, 5 wbar, 6/7 rbar ring
constexpr int kNP = 4;   // per-slot partial-sum arrays

template <typename R>
struct Work {
    Z<R>* V;    // v_j
    Z<R>* W;    // w_j
    Z<R>* A;    // a_j = H v_j
    Z<R>* B;    // b_j = H^dag w_j
    Z<R>* AB;   // abar_j (reverse pass)
    Z<R>* SB;   // sbar_j (reverse pass)
    Z<R>* F;    // [slot][kNF] fields
    double* part;  // [slot][kNP][pstride]
    size_t fe;     // complex elements per field (12 ldv)
    int kcap;      // steps held per slot
    int pstride;
    int ring;      // 0: step j at index j - 1; 1: at (j - 1) mod kcap (vectors regenerated in segments)
    __host__ __device__ size_t step(int slot, int j) const {
        int i = j - 1;
        if (ring) {
            i %= kcap;
#if defined(__HIP_DEVICE_COMPILE__)
            // the index is uniform; the division runs on the vector unit, and without
            // this every address derived from it would leave the scalar registers
            i = __builtin_amdgcn_readfirstlane(i);
#endif
        }
        return ((size_t)slot * kcap + i) * fe;
    }
    __host__ __device__ Z<R>* v(int slot, int j) const { return V + step(slot, j); }
    __host__ __device__ Z<R>* w(int slot, int j) const { return W + step(slot, j); }
    __host__ __device__ Z<R>* a(int slot, int j) const { return A + step(slot, j); }
    __host__ __device__ Z<R>* b(int slot, int j) const { return B + step(slot, j); }
    __host__ __device__ Z<R>* ab(int slot, int j) const { return AB + step(slot, j); }
    __host__ __device__ Z<R>* sb(int slot, int j) const { return SB + step(slot, j); }
    __host__ __device__ Z<R>* f(int slot, int i) const { return F + ((size_t)slot * kNF + i) * fe; }
    __host__ __device__ double* p(int slot, int i) const { return part + ((size_t)slot * kNP + i) * pstride; }
};

// ---------------------------------------------------------------- forward Lanczos
// Partials: forward pair writes 5 doubles per block (alpha re/im, |a|^2, h re/im);
// recurrence writes 4 (omega re/im, |r|^2, |s|^2).
constexpr int kNvPair = 5;
constexpr int kNvRecur = 4;

// Batched canonical -> SoA copy of field `which` (0 psi, 1 eta), times g5 if g5 = 1,
// for every list entry (source src[e] of the canonical array); for psi also the
// |x|^2 partials.
template <typename R>
void launch_sources_to_soa(const ZD* canon, int which, int g5, const Work<R>& wk, const SrcList& L, const Geom& g,
                           hipStream_t st);
// Step j of the Lanczos process for every list entry (k[e] = the entry's target size).
// ns: entries per workgroup on the colour-split layout (1, 2 or 4), which share the
// link loads; an entry's results do not depend on it.
template <typename R, typename RL>
void launch_fwd_pair(const Z<RL>* U, const Geom& g, double kappa, double mu, const Work<R>& wk, const SrcList& L,
                     Coef coef, int j, int has_eta, int ns, hipStream_t st, Timing t = {});
template <typename R>
void launch_recur(const Geom& g, const Work<R>& wk, const SrcList& L, Coef coef, int j, hipStream_t st);
// Replay of step j for regeneration: the step's own kernels (one entry per
// workgroup) with the recorded coefficients (beta_j, gamma_j; alpha_j) in place of
// their reductions, rewriting v_j, w_j, a_j, b_j (fwd) and the residuals of step j
// for entries with j < k[e] (recur) bit for bit, and no partial sums, flags or
// coefficient records.
template <typename R, typename RL>
void launch_fwd_replay(const Z<RL>* U, const Geom& g, double kappa, double mu, const Work<R>& wk, const SrcList& L,
                       Coef coef, int j, hipStream_t st);
template <typename R>
void launch_recur_replay(const Geom& g, const Work<R>& wk, const SrcList& L, Coef coef, int j, hipStream_t st);
// out[src] (canonical) = [psi[src] +] g5^{overlap} |x| sum_j c_j v_j over j = 1..k_used.
// With j1 > 0 only the steps j0..min(j1, k_used) are summed (one recompute segment,
// whose basis vectors sit in the ring): an entry whose k_used <= j1 (its top
// segment) writes out, every lower segment adds to it.
template <typename R>
void launch_assemble(const Geom& g, const Work<R>& wk, const SrcList& L, Coef coef, const ZD* psi_canon,
                     int overlap, ZD* out, hipStream_t st, int j0 = 1, int j1 = 0);

// Biorthogonality probe of every entry after its forward pass: block partials
// (x^H v_k re, im, w_k^H x re, im), k = k_used (zeros below 2), in wk.p(slot, 3).
// Returns the number of blocks.
template <typename R>
int launch_biorth(const Geom& g, const Work<R>& wk, const SrcList& L, Coef coef, hipStream_t st);

// ---------------------------------------------------------------- backward
constexpr int kNvRA = 8;   // P1..P4 complex
constexpr int kNvRB = 3;   // Re(vbar^H v), (wbar^H w) re/im

// Reverse step j: k[e] = k_used of the entry.  bwd_ra for entries with j < k_used,
// bwd_rb for entries with j <= k_used (last = 1: j == k_used for every entry).
template <typename R>
void launch_bwd_ra(const Geom& g, const Work<R>& wk, const SrcList& L, Coef coef, int j, hipStream_t st);
template <typename R, typename RL>
void launch_bwd_rb(const Z<RL>* U, const Geom& g, double kappa, double mu, const Work<R>& wk, const SrcList& L,
                   Coef coef, int j, int last, int ns, hipStream_t st, Timing t = {});
// Per-link force partials gpart[slot][chunk][36 planes] over the steps j of
// [jlo, min(jhi, k[e])] of each entry (jhi = 0: every step), stored, or added to
// the partials already there (accumulate = 1).
template <typename R>
void launch_force(const Geom& g, double kappa, double mu, const Work<R>& wk, const SrcList& L, int nchunk, ZD* gpart,
                  hipStream_t st, int jlo = 1, int jhi = 0, int accumulate = 0);
// dU[src] (canonical) from the chunk partials, boundary sign undone.
void launch_force_reduce(const Geom& g, const ZD* gpart, int nchunk, const SrcList& L, int antiperiodic, ZD* dU,
                         hipStream_t st);
// U(1) projections g_e(x, nu) = -Im tr(G^H U) of every entry, into gsrc[slot][4][ldv]
// (nullable) and, summed over the entries in list order, into jsum[nu][V]
// (accumulate = 1: added to its contents).
void launch_force_current(const Geom& g, const ZD* gpart, int nchunk, const SrcList& L, const ZD* U64,
                          double* gsrc, double* jsum, int accumulate, hipStream_t st);
template <typename R>
void launch_source_grad(const Geom& g, const Work<R>& wk, const SrcList& L, Coef coef, ZD* dpsi, hipStream_t st);
// Fill n doubles with zero (kernel, not a memset node).
void launch_zero(double* p, size_t n, hipStream_t st);

// ---------------------------------------------------------------- current estimator
// div(x) = scale sum_nu [j_nu(x) - j_nu(x - nu)], tot(x) = scale sum_nu [j_nu(x) + j_nu(x - nu)]
// (either nullable), then j <- scale j.
void launch_current_finish(const Geom& g, double* j, double scale, double* div, double* tot, hipStream_t st);
// Per-entry Ward residuals of the local U(1) symmetry for eta = g5 psi, block
// maxima in part[e][block][2]: max |lhs - rhs| and max |g|, where
// lhs(x) = sum_nu [g(x, nu) - g(x - nu, nu)], rhs(x) = -Im eta^H y (x) + Im dpsi^H psi (x).
// psi is indexed by src[e], y and dpsi by e.  Returns the number of blocks.
int launch_ward(const Geom& g, const double* gsrc, const SrcList& L, const ZD* psi, const ZD* y, const ZD* dpsi,
                double* part, hipStream_t st);

// ---------------------------------------------------------------- deflation / error estimate
void launch_defl_coeffs(const ZD* L, const ZD* psi, int V, int l, double* part, ZD* c, hipStream_t st);
void launch_defl_project(const ZD* R, const ZD* psi, const ZD* c, int V, int l, ZD* out, hipStream_t st);
void launch_defl_finish(const ZD* R, const ZD* c, const double* sgn, const ZD* yp, const ZD* psi, int V, int l,
                        int overlap, ZD* out, hipStream_t st);
int launch_diff_norm(const ZD* a, const ZD* b, size_t n, double* part, hipStream_t st);
// out = [a +] g5^{g5} b on canonical spinors of V sites (a nullable; out may alias a or b).
// overlap solve: y += a x, y = x + b y (n complex values, a and b real), out = f g5 in
void launch_caxpy(const ZD* x, double a, ZD* y, size_t n, hipStream_t st);
void launch_cxpby(const ZD* x, double b, ZD* y, size_t n, hipStream_t st);
void launch_g5_scale(const ZD* in, ZD f, int V, ZD* out, hipStream_t st);
void launch_combine(const ZD* a, const ZD* b, int g5, int V, ZD* out, hipStream_t st);

// ---------------------------------------------------------------- deflated derivative
// Batched CGNR for (sigma_e - H(m_e mu)) x_e = b_e, one system per grid row e.
struct CgRhs {
    ZD sigma;        // shift
    double msign;    // +1: H(mu); -1: H(-mu) = H(mu)^dag
    double bnorm2;   // |b|^2
    double zeta[2];  // |A^dag r|^2, double-buffered by iteration parity
    double rr;       // |r|^2 at the last check
    int done;        // converged (frozen)
    int pad;
};
constexpr int kCgX = 0, kCgR = 1, kCgP = 2, kCgW = 3, kCgZ = 4, kCgFields = 5;
// Operator forms of the shifted solves (all give the same hop sums; the partial sums
// of |A p|^2 differ in their summation order): multi-right-hand-side site per thread
// (default), colour split with two systems per block.
constexpr int kCgOpMulti = 0, kCgOpColour = 1, kCgOpMfma = 2, kCgOpTmarch = 3;
struct CgWork {
    ZD* f;        // [e][kCgFields] float64 SoA fields
    double* part; // [e][4][pstride]
    CgRhs* st;    // [e]
    size_t fe;
    int pstride;
    int op;       // kCgOp*
    __host__ __device__ ZD* field(int e, int i) const { return f + ((size_t)e * kCgFields + i) * fe; }
    __host__ __device__ double* p(int e, int i) const { return part + ((size_t)e * 4 + i) * pstride; }
};
// right-hand sides of the 2l systems (Z_i psi, Z_i^H a_i), r = b, x = 0, |b|^2
void launch_cg_rhs(const Geom& g, const ZD* psi, const ZD* eta, const ZD* pbar, const ZD* R, const ZD* L, const ZD* c,
                   const ZD* q, const double* sgn, int l, const CgWork& cw, hipStream_t st);
// right-hand sides from canonical vectors (e < la: rhs_a + e 12 V; e >= la: rhs_b), r = b, x = 0, |b|^2
void launch_cg_load(const Geom& g, const ZD* rhs_a, int la, const ZD* rhs_b, int nr, const CgWork& cw,
                    hipStream_t st);
// solutions x_e into out + e 12 V (canonical)
void launch_cg_store(const Geom& g, int nr, const CgWork& cw, ZD* out, hipStream_t st);
void launch_cg_start(const ZD* U, const Geom& g, double kappa, double mu, int nr, const CgWork& cw, hipStream_t st);
// one CGNR iteration (check = 1: evaluate convergence afterwards)
void launch_cg_iteration(const ZD* U, const Geom& g, double kappa, double mu, int nr, int it, int check, double tol,
                         const CgWork& cw, hipStream_t st);
// projections (1 - Pi_i) / (1 - Pi_i^H) of the solutions and the conj(c_i) scaling
void launch_cg_finish(const Geom& g, const ZD* R, const ZD* L, const ZD* c, int l, const CgWork& cw, hipStream_t st);
// U(1) projections -Im tr(G_e^H U) of nsrc canonical link gradients dU[e] into gsrc[e][4][ldv]
// (nullable) and summed over e into jsum[4][V] (accumulate: added to its contents)
void launch_u1_projection(const Geom& g, const ZD* U64, const ZD* dU, int nsrc, int antiperiodic, double* gsrc,
                          double* jsum, int accumulate, hipStream_t st);
// dU += eigenpair-motion terms (canonical dU, boundary sign undone)
void launch_defl_force(const Geom& g, double kappa, double mu, const ZD* R, const ZD* L, const ZD* q, int l,
                       const CgWork& cw, int antiperiodic, ZD* dU, hipStream_t st);

// ---------------------------------------------------------------- projected-matrix step
struct DenseWork {
    ZD* X;        // iterate                     [slot][kk]
    ZD* Y;        // Frechet iterate
    ZD* Wk;       // in-place inversion workspace
    ZD* Xinv;     // inverse (columns un-permuted)
    ZD* Zt;       // GEMM temporary
    ZD* Y2;       // second temporary (inverse-free steps with the Frechet block)
    ZD* P2;       // third and fourth temporaries (the same steps' split products)
    ZD* Y3;
    int* rowperm; // [slot][2 kcap]: row permutation, then pivot rows
    double* part; // [slot][pstride]: update partials, scatter partials, mu, residual partials,
                  // column-norm partials
    double* delta;  // [slot][4]: |X_new - X|^2, |X_new|^2 of the last step, |I - X_new^2|_F^2, unused
    size_t kk;    // kcap^2
    int kcap;
    int npart_max;  // partial blocks per slot (= blocks over kcap^2)
    int pstride;
    __host__ __device__ DenseWork at(int slot) const {
        DenseWork o = *this;
        const size_t d = (size_t)slot * kk;
        o.X += d; o.Y += d; o.Wk += d; o.Xinv += d; o.Zt += d; o.Y2 += d; o.P2 += d; o.Y3 += d;
        o.rowperm += (size_t)slot * 2 * kcap;
        o.part += (size_t)slot * pstride;
        o.delta += (size_t)slot * 4;
        return o;
    }
};
inline int dense_colnorm_blocks(int k) { return (k + 15) / 16; }
inline int dense_pstride(int kcap) { return 5 * grid_for(kcap * kcap, 256) + 8 + 2 * dense_colnorm_blocks(kcap); }

// Build X = T_k (tridiagonal from coef) and, if grad, Y = e_1 cbar^H with cbar = |x| conj(h),
// for every list entry (k[e] = k_used, sorted in decreasing order).
void launch_dense_build(Coef coef, const SrcList& L, int grad, const DenseWork& w, hipStream_t st);
// X and Y from caller matrices (test entry point, slot 0).
void launch_dense_load(const ZD* T, const ZD* E, int k, const DenseWork& w, hipStream_t st);
// One Newton step X <- (mu X + X^{-1}/mu)/2 (and Y) for every entry; flag[e] = 1
// turns the entry's norm scaling on.  Leaves delta[slot] for the host.
// tridiag: X is tridiagonal (the first step from T_k); its inverse then comes from a
// banded elimination instead of the Gauss-Jordan sweep.
void dense_newton_step(const SrcList& L, int grad, int nb, size_t lds_bytes, const DenseWork& w, hipStream_t st,
                       int tridiag);
// One inverse-free (Newton-Schulz) step X <- X (3 - X^2)/2 and, if grad, the
// Frechet block Y <- [Y (3 - X^2) - X (X Y + Y X)]/2; leaves delta[slot].
void dense_ns_step(const SrcList& L, int grad, const DenseWork& w, hipStream_t st);
// |I - X^2|_F^2 of every entry into delta[2] (one GEMM into Zt and a reduction).
void dense_residual(const SrcList& L, const DenseWork& w, hipStream_t st);
// X^{-1} of the tridiagonal X (Gaussian elimination on the band) into Xinv, and
// C = A B for workspace matrices A, B, C (indices: 0 X, 1 Y, 2 Wk, 3 Xinv, 4 Zt,
// 5 Y2, 6 P2, 7 Y3), for every list entry.
void launch_tridiag_inverse(const SrcList& L, const DenseWork& w, hipStream_t st);
void launch_dense_gemm(const SrcList& L, const DenseWork& w, int ia, int ib, int ic, hipStream_t st);

// ---------------------------------------------------------------- block-matrix process
// One link parameter: U_nu(site) -> exp(i t X) U_nu(site), X as [a][b][re, im].
struct BlockTangent {
    int nu, site;
    double X[3][3][2];
};
// Float64 SoA fields of the block process, [0] upper and [1] lower half: the source
// x, the current and previous vectors, the products (then the residuals), and the
// basis (step j at basis[h] + (j - 1) 12 ldv).
struct BlockFields {
    ZD* x[2];
    ZD* v[2];
    ZD* w[2];
    ZD* vp[2];
    ZD* wp[2];
    ZD* a[2];
    ZD* b[2];
    ZD* basis[2];
};
int blk_blocks(const Geom& g);   // partial-sum blocks of the block-process kernels
// out_a += dH in_a, out_b += dH^dag in_b (either pair null) for the tangent t.
void launch_blk_tangent(const ZD* U, const BlockTangent& t, const Geom& g, double kappa, double mu, const ZD* in_a,
                        ZD* out_a, const ZD* in_b, ZD* out_b, hipStream_t st);
// v_1 = w_1 = x / |x| (|x| in coef.misc[0]; a zero source stops with k_used = 0).
void launch_blk_start(const BlockFields& f, const Geom& g, Coef coef, double* part, hipStream_t st);
// The recursion of step j after the products a = B v_j, b = B^H w_j (p0, p1: partials).
void launch_blk_step(const BlockFields& f, const Geom& g, Coef coef, double* p0, double* p1, int j, int k,
                     hipStream_t st);

// ---------------------------------------------------------------- nested step
// Inner two-sided Lanczos process of the nested projected-matrix step (nested.hip)
// on W = (T^2)^{-1} (in Zt of the outer dense workspace, slot 0), from e_1.
struct NestWork {
    ZD* Vb;       // inner right basis V', column j at Vb + j k
    ZD* vec;      // six vectors of length k: v, w, a = W v, b = W^H w, v_prev, w_prev
    ZD* alpha;    // inner coefficients, 0-based step j: alpha[j], beta[j], gamma[j] (j >= 1)
    double* beta;
    ZD* gamma;
    int* status;  // [0] stopped, [1] steps taken (m_used), [2] serious breakdown
};
// Y2 = W^T (so that both products of a step read the matrix with unit stride).
void nest_prepare(const DenseWork& w, int k, hipStream_t st);
void nest_init(const NestWork& nw, int k, hipStream_t st);
// Inner step j of m (0-based).
void nest_step(const DenseWork& w, const NestWork& nw, int k, int j, int m, hipStream_t st);
// X = Wk = [[0, T'], [I, 0]] (2m x 2m) in w2 (slot 0), for the principal square root.
void nest_block(const NestWork& nw, const DenseWork& w2, int m, hipStream_t st);
// coef.c[1..k] = T V' (T')^{1/2} e_1 from X = sgn([[0, T'], [I, 0]]).
void nest_finish(const NestWork& nw, const DenseWork& w2, Coef coef, int k, int m, hipStream_t st);

// c = X e_1, adjoint seeds from Y, S = |x| Re sum_j c_j h_j.
void launch_dense_extract(Coef coef, const SrcList& L, int grad, const DenseWork& w, hipStream_t st);

}  // namespace tslov
