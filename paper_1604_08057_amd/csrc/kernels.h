// Host-side launchers of the tslov kernels (internal interface between the
// kernel translation units and the C ABI in api.hip).
#pragma once

#include "common.h"

namespace tslov {

inline int grid_for(int n, int blk = kBlock) { return (n + blk - 1) / blk; }

// ---------------------------------------------------------------- layout
void launch_links_to_soa(const ZD* Ucanon, ZD* U64, Z<float>* U32, const Geom& g, int antiperiodic,
                         hipStream_t st);
template <typename R>
void launch_spinor_to_soa(const ZD* in, Z<R>* out, const Geom& g, double* part_norm, hipStream_t st);
template <typename R>
void launch_spinor_from_soa(const Z<R>* in, ZD* out, const Geom& g, hipStream_t st);

// ---------------------------------------------------------------- operator
// out = G5out * (G5in in - kappa * hop_{mu}(G5in in))
template <typename R>
void launch_apply(const Z<R>* U, const Z<R>* in, Z<R>* out, const Geom& g, double kappa, double mu,
                  int g5_in, int g5_out, hipStream_t st);

// ---------------------------------------------------------------- forward Lanczos
// Partials: forward pair writes 5 doubles per block (alpha re/im, |a|^2, h re/im);
// recurrence writes 4 (omega re/im, |r|^2, |s|^2).
constexpr int kNvPair = 5;
constexpr int kNvRecur = 4;

template <typename R>
void launch_fwd_pair(const Z<R>* U, const Geom& g, double kappa, double mu, const Z<R>* rin,
                     const Z<R>* sin, const double* part_in, int npart_in, int first, Coef coef, int j,
                     Z<R>* vout, Z<R>* wout, Z<R>* aout, Z<R>* bout, const Z<R>* eta, double* part_out,
                     hipStream_t st);
template <typename R>
void launch_recur(const Geom& g, const Z<R>* a, const Z<R>* b, const Z<R>* v, const Z<R>* w, const Z<R>* vp,
                  const Z<R>* wp, const double* part_in, int npart_in, Coef coef, int j, int last,
                  Z<R>* rout, Z<R>* sout, double* part_out, hipStream_t st);
// out (canonical) = [psi +] g5^{overlap} |x| sum_j c_j v_j
template <typename R>
void launch_assemble(const Geom& g, const Z<R>* basis, size_t field_stride, Coef coef, const ZD* psi_canon,
                     int overlap, ZD* out, hipStream_t st);

// ---------------------------------------------------------------- backward
constexpr int kNvRA = 8;   // P1..P4 complex
constexpr int kNvRB = 3;   // Re(vbar^H v), (wbar^H w) re/im

template <typename R>
void launch_bwd_ra(const Geom& g, const Z<R>* vbar, const Z<R>* wbar, const Z<R>* v_next, const Z<R>* w_next,
                   const Z<R>* v_j, const Z<R>* w_j, const Z<R>* v_prev, const Z<R>* w_prev,
                   const double* part_in, int npart_in, Coef coef, int j, Z<R>* rbar_out, Z<R>* sbar_out,
                   double* part_out, hipStream_t st);
template <typename R>
void launch_bwd_rb(const Z<R>* U, const Geom& g, double kappa, double mu, const double* part_in, int npart_in,
                   Coef coef, int j, int k_used, const Z<R>* rbar_j, const Z<R>* rbar_next,
                   const Z<R>* sbar_j, const Z<R>* sbar_next, const Z<R>* v_j, const Z<R>* w_j,
                   const Z<R>* a_j, const Z<R>* b_j, const Z<R>* eta, Z<R>* vbar_out, Z<R>* wbar_out,
                   Z<R>* abar_out, double* part_out, hipStream_t st);
template <typename R>
void launch_force(const Geom& g, double kappa, double mu, const Z<R>* abar, const Z<R>* sbar, const Z<R>* vb,
                  const Z<R>* wb, size_t field_stride, const int* status, int nchunk, ZD* gpart, hipStream_t st);
void launch_force_reduce(const Geom& g, const ZD* gpart, int nchunk, int antiperiodic, ZD* out, hipStream_t st);
template <typename R>
void launch_source_grad(const Geom& g, const Z<R>* vbar, const Z<R>* wbar, const Z<R>* x, Coef coef,
                        double* part, ZD* out, hipStream_t st);

// ---------------------------------------------------------------- deflation / error estimate
void launch_defl_coeffs(const ZD* L, const ZD* psi, int V, int l, double* part, ZD* c, hipStream_t st);
void launch_defl_project(const ZD* R, const ZD* psi, const ZD* c, int V, int l, ZD* out, hipStream_t st);
void launch_defl_finish(const ZD* R, const ZD* c, const double* sgn, const ZD* yp, const ZD* psi, int V, int l,
                        int overlap, ZD* out, hipStream_t st);
int launch_diff_norm(const ZD* a, const ZD* b, size_t n, double* part, hipStream_t st);

// ---------------------------------------------------------------- projected-matrix step
struct DenseWork {
    ZD* X;        // iterate
    ZD* Y;        // Frechet iterate
    ZD* Wk;       // in-place inversion workspace
    ZD* Xinv;     // inverse (columns un-permuted)
    ZD* Zt;       // GEMM temporary
    int* rowperm;
    double* logpiv;
    double* part;
    int npart_max;
};
// Build X = T_k (tridiagonal from coef) and, if grad, Y = e_1 cbar^H with cbar = |x| conj(h).
void launch_dense_build(Coef coef, int k, int grad, DenseWork w, hipStream_t st);
// X and Y from caller matrices (test entry point).
void launch_dense_load(const ZD* T, const ZD* E, int k, DenseWork w, hipStream_t st);
// One Newton step X <- (mu X + X^{-1}/mu)/2 (and Y); returns host-readable partials count.
int dense_newton_step(int k, int grad, int scaling, int nb, size_t lds_bytes, DenseWork w, hipStream_t st);
// c = X e_1, adjoint seeds from Y, S = |x| Re sum_j c_j h_j.
void launch_dense_extract(Coef coef, int k, int grad, DenseWork w, hipStream_t st);

}  // namespace tslov
