// Two-sided Lanczos process on the block matrix B = [[H, dH], [0, H]] of Theorem 1
// (Sec. 2, eq. func_derivative_1): f(B) (0, x) = (d f(H) x, f(H) x), the paper's
// derivative of sgn(H) x along one link parameter, U_nu(x0) -> exp(i t X) U_nu(x0).
// Block vectors are pairs of float64 SoA fields (upper, lower); the products
// B v = (H v1 + dH v2, H v2) and B^H w = (H^H w1, dH^H w1 + H^H w2) take the
// operator launches of fields.hip plus the two-site tangent term below; the inner
// products run over both halves.  The recursion is that of the plain process
// (both Krylov spaces from the source, v_1 = w_1 = x / |x|, no re-biorthogonalisation).
#include "kernels.h"

namespace tslov {

namespace {

constexpr int kBT = 256;   // threads per block of the elementwise kernels

// Per-block partial sums over both halves of a block vector, in part[b * NV + i];
// the consumer re-reduces them in a fixed order.
template <int NV>
__device__ __forceinline__ void blk_partials(double* part, double (&v)[NV]) {
    write_partials<NV, kBT>(part, v);
}

}  // namespace

// The tangent term at its two sites: with dU = i X U_nu(x0) (boundary sign folded
// into U as for the stencil),
//   dD_w psi (x0)        = -kappa e^{+mu d} (1 + g_nu) dU       psi(x0 + nu),
//   dD_w psi (x0 + nu)   = -kappa e^{-mu d} (1 - g_nu) dU^dag   psi(x0),
// and dH = g5 dD_w; dH^dag is the same at -mu.  out_a += dH in_a; out_b += dH^dag in_b
// (either pair may be null).  One thread.
template <int NU>
__device__ void tangent_one(const ZD (&u)[3][3], const BlockTangent& t, const Geom& g, double kappa, double emu,
                            const ZD* in_a, ZD* out_a, const ZD* in_b, ZD* out_b, int s0, int s1) {
    const double ef = NU == 3 ? emu : 1.0, eb = NU == 3 ? 1.0 / emu : 1.0;
    for (int which = 0; which < 2; ++which) {
        const ZD* in = which ? in_b : in_a;
        ZD* out = which ? out_b : out_a;
        if (!in) continue;
        // H(+mu) for the product, H(-mu) = H^dag for its adjoint
        const double cf = which ? eb : ef, cb = which ? ef : eb;
        Spinor<double> p1, p0, acc0, acc1;
        load_spinor(p1, in, g.ldv, s1);
        load_spinor(p0, in, g.ldv, s0);
        zero_spinor(acc0);
        zero_spinor(acc1);
        hop_fwd<NU>(acc0, u, p1, cf);
        hop_bwd<NU>(acc1, u, p0, cb);
        Spinor<double> o0, o1;
        load_spinor(o0, out, g.ldv, s0);
        load_spinor(o1, out, g.ldv, s1);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
            const double sg = sp < 2 ? -kappa : kappa;   // -kappa, then g5
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                o0.c[sp][c] = o0.c[sp][c] + sg * acc0.c[sp][c];
                o1.c[sp][c] = o1.c[sp][c] + sg * acc1.c[sp][c];
            }
        }
        store_spinor(out, g.ldv, s0, o0);
        store_spinor(out, g.ldv, s1, o1);
    }
    (void)t;
}

__global__ __launch_bounds__(64) void k_blk_tangent(const ZD* __restrict__ U, BlockTangent t, Geom g, double kappa,
                                                    double emu, const ZD* in_a, ZD* out_a, const ZD* in_b,
                                                    ZD* out_b) {
    if (threadIdx.x != 0) return;
    const Nbr n = neighbours(g, t.site);
    const int s0 = t.site, s1 = n.fwd[t.nu];
    // dU = i X U_nu(x0)
    ZD u0[3][3], du[3][3];
    load_link(u0, U, g.ldv, t.nu, s0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            ZD acc = mk<double>(0, 0);
#pragma unroll
            for (int c = 0; c < 3; ++c) acc = acc + mk<double>(t.X[a][c][0], t.X[a][c][1]) * u0[c][b];
            du[a][b] = timesI(acc);
        }
    switch (t.nu) {
        case 0: tangent_one<0>(du, t, g, kappa, emu, in_a, out_a, in_b, out_b, s0, s1); break;
        case 1: tangent_one<1>(du, t, g, kappa, emu, in_a, out_a, in_b, out_b, s0, s1); break;
        case 2: tangent_one<2>(du, t, g, kappa, emu, in_a, out_a, in_b, out_b, s0, s1); break;
        default: tangent_one<3>(du, t, g, kappa, emu, in_a, out_a, in_b, out_b, s0, s1); break;
    }
}

// |x|^2 partials of the source (both halves); v = w = x / |x| follows in k_blk_start.
__global__ __launch_bounds__(kBT) void k_blk_norm(BlockFields f, Geom g, double* part) {
    const int s = blockIdx.x * kBT + threadIdx.x;
    double v[1] = {0.0};
    if (s < g.V)
        for (int h = 0; h < 2; ++h)
            for (int p = 0; p < 12; ++p) v[0] += norm2(f.x[h][(size_t)p * g.ldv + s]);
    blk_partials<1>(part, v);
}

// v_1 = w_1 = x / |x| into the basis and the working fields; |x| into misc[0]
// (zero source: k_used = 0 and the stop flag).
__global__ __launch_bounds__(kBT) void k_blk_start(BlockFields f, Geom g, Coef coef, const double* part, int np) {
    double r[1];
    reduce_partials<1, kBT>(part, np, r);
    const double nx = sqrt(r[0]);
    const int s = blockIdx.x * kBT + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        coef.misc[0] = nx;
        coef.beta[1] = nx;
        coef.gamma[1] = mk<double>(nx, 0.0);
        coef.status[0] = nx > 0.0 && std::isfinite(nx) ? 0 : 1;
        coef.status[1] = 0;
        coef.status[2] = nx > 0.0 ? (std::isfinite(nx) ? 0 : 3) : 1;
    }
    if (!(nx > 0.0) || !std::isfinite(nx) || s >= g.V) return;
    const double inv = 1.0 / nx;
    for (int h = 0; h < 2; ++h)
        for (int p = 0; p < 12; ++p) {
            const size_t i = (size_t)p * g.ldv + s;
            const ZD v = inv * f.x[h][i];
            f.v[h][i] = v;
            f.w[h][i] = v;
            f.vp[h][i] = mk<double>(0, 0);
            f.wp[h][i] = mk<double>(0, 0);
            f.basis[h][i] = v;   // step 1
        }
}

// alpha_j = w^H a over both halves and |a|^2: partials (4 doubles per block).
__global__ __launch_bounds__(kBT) void k_blk_alpha(BlockFields f, Geom g, const Coef coef, double* part) {
    if (*(volatile const int*)coef.status) return;
    const int s = blockIdx.x * kBT + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (s < g.V)
        for (int h = 0; h < 2; ++h)
            for (int p = 0; p < 12; ++p) {
                const size_t i = (size_t)p * g.ldv + s;
                const ZD t = cjmul(f.w[h][i], f.a[h][i]);
                v[0] += t.re;
                v[1] += t.im;
                v[2] += norm2(f.a[h][i]);
            }
    blk_partials<3>(part, v);
}

// Step j's residuals r = a - alpha v - gamma_j v_prev and s = b - conj(alpha) w -
// beta_j w_prev (in place of a, b), alpha_j recorded, partials of s^H r, |r|^2,
// |s|^2.  At j = k (the last step) only alpha_j is recorded.
__global__ __launch_bounds__(kBT) void k_blk_recur(BlockFields f, Geom g, Coef coef, const double* pin, int np,
                                                   double* pout, int j, int k) {
    if (*(volatile const int*)coef.status) return;
    double r3[3];
    reduce_partials<3, kBT>(pin, np, r3);
    const ZD al = mk<double>(r3[0], r3[1]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        coef.alpha[j] = al;
        coef.anorm2[j] = r3[2];
    }
    if (j == k) return;
    const ZD gj = j > 1 ? coef.gamma[j] : mk<double>(0, 0);
    const double bj = j > 1 ? coef.beta[j] : 0.0;
    const int s = blockIdx.x * kBT + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (s < g.V)
        for (int h = 0; h < 2; ++h)
            for (int p = 0; p < 12; ++p) {
                const size_t i = (size_t)p * g.ldv + s;
                const ZD r = f.a[h][i] - al * f.v[h][i] - gj * f.vp[h][i];
                const ZD q = f.b[h][i] - cj(al) * f.w[h][i] - bj * f.wp[h][i];
                f.a[h][i] = r;
                f.b[h][i] = q;
                const ZD t = cjmul(q, r);
                v[0] += t.re;
                v[1] += t.im;
                v[2] += norm2(r);
                v[3] += norm2(q);
            }
    blk_partials<4>(pout, v);
}

// Breakdown decisions (lucky: |r| <= tau |a|; serious: |s^H r| <= tau' |r||s| or a
// non-finite omega), else beta_{j+1} = |omega|^{1/2}, gamma_{j+1} = omega / beta,
// v <- r / beta, w <- s / conj(gamma) (the previous ones kept), stored as basis
// step j + 1.
__global__ __launch_bounds__(kBT) void k_blk_next(BlockFields f, Geom g, Coef coef, const double* pin, int np,
                                                  int j, int k) {
    if (*(volatile const int*)coef.status) return;
    if (j == k) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            coef.status[1] = k;
            *(volatile int*)coef.status = 1;
        }
        return;
    }
    double r4[4];
    reduce_partials<4, kBT>(pin, np, r4);
    const ZD om = mk<double>(r4[0], r4[1]);
    const double aom = sqrt(norm2(om));
    const bool lucky = r4[2] <= kTauLucky * kTauLucky * coef.anorm2[j];
    const bool finite = std::isfinite(om.re) && std::isfinite(om.im);
    const bool serious = !lucky && (!finite || aom <= kTauSerious * sqrt(r4[2] * r4[3]));
    if (lucky || serious) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            coef.status[1] = j;
            coef.status[2] = lucky ? 1 : 2;
            coef.status[3] = j + 1;
            *(volatile int*)coef.status = 1;
        }
        return;
    }
    const double be = sqrt(aom);
    const ZD ga = (1.0 / be) * om;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        coef.beta[j + 1] = be;
        coef.gamma[j + 1] = ga;
    }
    const int s = blockIdx.x * kBT + threadIdx.x;
    if (s >= g.V) return;
    const double ib = 1.0 / be;
    const ZD icg = zdiv(mk<double>(1.0, 0.0), cj(ga));
    for (int h = 0; h < 2; ++h)
        for (int p = 0; p < 12; ++p) {
            const size_t i = (size_t)p * g.ldv + s;
            const ZD vn = ib * f.a[h][i];
            const ZD wn = icg * f.b[h][i];
            f.vp[h][i] = f.v[h][i];
            f.wp[h][i] = f.w[h][i];
            f.v[h][i] = vn;
            f.w[h][i] = wn;
            f.basis[h][(size_t)j * 12 * g.ldv + i] = vn;   // step j + 1
        }
}

int blk_blocks(const Geom& g) { return grid_for(g.V, kBT); }

void launch_blk_tangent(const ZD* U, const BlockTangent& t, const Geom& g, double kappa, double mu, const ZD* in_a,
                        ZD* out_a, const ZD* in_b, ZD* out_b, hipStream_t st) {
    hipLaunchKernelGGL(k_blk_tangent, dim3(1), dim3(64), 0, st, U, t, g, kappa, std::exp(mu), in_a, out_a, in_b,
                       out_b);
}

void launch_blk_start(const BlockFields& f, const Geom& g, Coef coef, double* part, hipStream_t st) {
    const int nb = blk_blocks(g);
    hipLaunchKernelGGL(k_blk_norm, dim3(nb), dim3(kBT), 0, st, f, g, part);
    hipLaunchKernelGGL(k_blk_start, dim3(nb), dim3(kBT), 0, st, f, g, coef, part, nb);
}

void launch_blk_step(const BlockFields& f, const Geom& g, Coef coef, double* p0, double* p1, int j, int k,
                     hipStream_t st) {
    const int nb = blk_blocks(g);
    hipLaunchKernelGGL(k_blk_alpha, dim3(nb), dim3(kBT), 0, st, f, g, coef, p0);
    hipLaunchKernelGGL(k_blk_recur, dim3(nb), dim3(kBT), 0, st, f, g, coef, p0, nb, p1, j, k);
    hipLaunchKernelGGL(k_blk_next, dim3(nb), dim3(kBT), 0, st, f, g, coef, p1, nb, j, k);
}

}  // namespace tslov
