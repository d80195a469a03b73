// Derivative of the deflated sign function: eigenpair motion (Sec. 3 with
// App. E).  For a simple deflated eigenvalue lambda_i with spectral projector
// Pi_i = R_i L_i^H the first-order change is
//     dPi_i = Z_i dH Pi_i + Pi_i dH Z_i,   Z_i = (lambda_i - H)^{-1} (1 - Pi_i),
// so for a_i = s_i eta - psibar_p (psibar_p the TSL source gradient) the link
// derivative gains, per eigenpair, the rank-one terms
//     Re [c_i (Z_i^H a_i)]^H dH R_i  +  Re [(R_i^H a_i) L_i]^H dH (Z_i psi),   c_i = L_i^H psi.
// Z_i psi and Z_i^H a_i solve the consistent singular systems
//     (lambda_i - H) z = (1 - Pi_i) psi,          then z <- (1 - Pi_i) z,
//     (conj lambda_i - H^dag) z' = (1 - Pi_i^H) a_i,  then z' <- (1 - Pi_i^H) z',
// by conjugate gradients on the normal equations (CGNR), all 2l systems in one
// lockstep batch (grid dimension y over the right-hand sides, per-system shift
// and chemical-potential sign, scalars on the device, frozen once converged).
// Fields are float64 structure-of-arrays planes; R, L and the sources are
// canonical [V][4][3] arrays of the caller.
#include "kernels.h"

#include <cmath>

namespace tslov {

namespace {

__device__ __forceinline__ int block_flag_cg(const int* p) {
    __shared__ int f;
    if (threadIdx.x == 0) f = *(volatile const int*)p;
    __syncthreads();
    const int r = f;
    __syncthreads();
    return r;
}

// (1 + S g) hops of one colour for NS systems e0 .. e0 + NS - 1: each link row is loaded
// once and applied to every live system's field, with the system's own
// chemical-potential factors (ep, em) on the temporal hops.
template <int NU, int NS>
__device__ __forceinline__ void cg_hop(ZD (&acc)[NS][4], const ZD* __restrict__ U, const CgWork& cw, int e0,
                                       int field, const int (&live)[NS], const Geom& g, int s, int a, const Nbr& n,
                                       const double (&ep)[NS], const double (&em)[NS]) {
    ZD u[3];
    Spinor<double> p;
    load_row(u, U, g.ldv, NU, a, s);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        if (!live[i]) continue;
        load_spinor(p, cw.field(e0 + i, field), g.ldv, n.fwd[NU]);
        hop1<NU, +1>(acc[i], u, p, (NU == 3) ? ep[i] : 1.0);
    }
    load_col_conj(u, U, g.ldv, NU, a, n.bwd[NU]);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        if (!live[i]) continue;
        load_spinor(p, cw.field(e0 + i, field), g.ldv, n.bwd[NU]);
        hop1<NU, -1>(acc[i], u, p, (NU == 3) ? em[i] : 1.0);
    }
}

}  // namespace

// out_e = A_e in_e for the NS systems e = e0 .. e0 + NS - 1 of this block (e0 = NS y),
// with A_e = sigma_e - H(m_e mu) (adj = 0) or its adjoint conj(sigma_e) - H(-m_e mu)
// (adj = 1); H = g5 (1 - kappa hop).  Partials of |out_e|^2.  The systems share each
// link load (the links are the same for all of them); frozen systems keep their fields
// and partials.  Each system's arithmetic is that of a block of its own.
template <int NS>
__global__ __launch_bounds__(kCBlock) void k_cg_apply(const ZD* __restrict__ U, Geom g, double kappa, double emu,
                                                      CgWork cw, int adj, int in_field, int out_field, int preg) {
    const int e0 = blockIdx.y * NS;
    __shared__ int live_s[NS];
    if (threadIdx.x < NS) live_s[threadIdx.x] = !*(volatile const int*)&cw.st[e0 + threadIdx.x].done;
    __syncthreads();
    int live[NS], any = 0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        live[i] = live_s[i];
        any |= live[i];
    }
    if (!any) return;
    ZD sig[NS];
    double ep[NS], em[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const CgRhs* st = cw.st + e0 + i;
        sig[i] = adj ? cj(st->sigma) : st->sigma;
        const double m = adj ? -st->msign : st->msign;
        ep[i] = m > 0 ? emu : 1.0 / emu;
        em[i] = 1.0 / ep[i];
    }
    const int a = wave_colour();
    const int s = blockIdx.x * kSites + threadIdx.x % kSites;
    double pv[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) pv[i] = 0.0;
    if (s < g.V) {
        const Nbr n = neighbours(g, s);
        ZD acc[NS][4];
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) acc[i][sp] = mk<double>(0, 0);
#pragma unroll 1
        for (int nu = 0; nu < 4; ++nu) {
            switch (nu) {
                case 0: cg_hop<0, NS>(acc, U, cw, e0, in_field, live, g, s, a, n, ep, em); break;
                case 1: cg_hop<1, NS>(acc, U, cw, e0, in_field, live, g, s, a, n, ep, em); break;
                case 2: cg_hop<2, NS>(acc, U, cw, e0, in_field, live, g, s, a, n, ep, em); break;
                default: cg_hop<3, NS>(acc, U, cw, e0, in_field, live, g, s, a, n, ep, em); break;
            }
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            if (!live[i]) continue;
            const FieldBase fi = field_base(cw.field(e0 + i, in_field)), fo = field_base(cw.field(e0 + i, out_field));
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                const int pl = sp * 3 + a;
                const ZD x = fload<double>(fi, g.ldv, pl, (unsigned)s);
                const double g5 = sp < 2 ? 1.0 : -1.0;
                const ZD o = sig[i] * x - g5 * (x - kappa * acc[i][sp]);
                fstore<double>(fo, g.ldv, pl, (unsigned)s, o);
                pv[i] += norm2(o);
            }
        }
    }
    block_sum<NS, kCBlock>(pv);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NS; ++i)
            if (live[i]) cw.p(e0 + i, preg)[blockIdx.x] = pv[i];
}

namespace {

// the operator launch over the nr systems, two per block when nr is even (measured at
// 16^4 with 40 systems: 1, 2 and 4 per block took 8.00, 7.97 and 8.92 s per derivative:
// the kernel waits on latency, not on link bytes, and more systems per block lengthen
// each block's chain)
void cg_apply(const ZD* U, const Geom& g, double kappa, double emu, int nr, const CgWork& cw, int adj, int in_field,
              int out_field, int preg, hipStream_t st) {
    if (nr % 2 == 0)
        hipLaunchKernelGGL(k_cg_apply<2>, dim3(np_stencil(g.V), nr / 2), dim3(kCBlock), 0, st, U, g, kappa, emu, cw,
                           adj, in_field, out_field, preg);
    else
        hipLaunchKernelGGL(k_cg_apply<1>, dim3(np_stencil(g.V), nr), dim3(kCBlock), 0, st, U, g, kappa, emu, cw, adj,
                           in_field, out_field, preg);
}

}  // namespace

// Right-hand sides: e < l: b = psi - c_e R_e;  e >= l (i = e - l):
// b = s_i eta - pbar - q_i L_i with q_i = R_i^H (s_i eta - pbar).  r = b, x = 0,
// partials of |b|^2.
__global__ __launch_bounds__(kBlock) void k_cg_rhs(Geom g, const ZD* __restrict__ psi, const ZD* __restrict__ eta,
                                                   const ZD* __restrict__ pbar, const ZD* __restrict__ R,
                                                   const ZD* __restrict__ L, const ZD* __restrict__ c,
                                                   const ZD* __restrict__ q, const double* __restrict__ sgn, int l,
                                                   CgWork cw) {
    const int e = blockIdx.y;
    const int i = e < l ? e : e - l;
    const int s = blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (s < g.V) {
        const size_t n12 = (size_t)12 * g.V, o = (size_t)s * 12;
        ZD* __restrict__ r = cw.field(e, kCgR);
        ZD* __restrict__ x = cw.field(e, kCgX);
#pragma unroll
        for (int p = 0; p < 12; ++p) {
            ZD b;
            if (e < l) b = psi[o + p] - c[i] * R[(size_t)i * n12 + o + p];
            else b = sgn[i] * eta[o + p] - pbar[o + p] - q[i] * L[(size_t)i * n12 + o + p];
            r[(size_t)p * g.ldv + s] = b;
            x[(size_t)p * g.ldv + s] = mk<double>(0, 0);
            v[0] += norm2(b);
        }
    }
    write_partials<1, kBlock>(cw.p(e, 0), v);
}

__global__ __launch_bounds__(kBlock) void k_cg_bnorm(CgWork cw, int npart) {
    const int e = blockIdx.y;
    double red[1];
    reduce_partials<1, kBlock>(cw.p(e, 0), npart, red);
    if (threadIdx.x == 0) {
        cw.st[e].bnorm2 = red[0];
        cw.st[e].rr = red[0];
        cw.st[e].done = red[0] > 0.0 ? 0 : 1;
    }
}

// p = z, zeta_0 = |z|^2 (after z = A^dag r).
__global__ __launch_bounds__(kPBlock) void k_cg_init_p(Geom g, CgWork cw, int npart) {
    const int e = blockIdx.z;
    CgRhs* st = cw.st + e;
    if (block_flag_cg(&st->done)) return;
    double red[1];
    reduce_partials<1, kPBlock>(cw.p(e, 2), npart, red);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) st->zeta[0] = red[0];
    const int s = blockIdx.x * kPBlock + threadIdx.x;
    if (s >= g.V) return;
    const size_t i = (size_t)blockIdx.y * g.ldv + s;
    cw.field(e, kCgP)[i] = cw.field(e, kCgZ)[i];
}

// alpha = zeta / |A p|^2;  x += alpha p;  r -= alpha w;  partials of |r|^2.
__global__ __launch_bounds__(kPBlock) void k_cg_update_xr(Geom g, CgWork cw, int npart, int par) {
    const int e = blockIdx.z;
    CgRhs* st = cw.st + e;
    if (block_flag_cg(&st->done)) return;
    double red[1];
    reduce_partials<1, kPBlock>(cw.p(e, 0), npart, red);
    const double alpha = red[0] > 0.0 ? st->zeta[par] / red[0] : 0.0;
    const int s = blockIdx.x * kPBlock + threadIdx.x;
    double v[1] = {0.0};
    if (s < g.V) {
        const size_t i = (size_t)blockIdx.y * g.ldv + s;
        ZD* x = cw.field(e, kCgX);
        ZD* r = cw.field(e, kCgR);
        x[i] = x[i] + alpha * cw.field(e, kCgP)[i];
        const ZD rn = r[i] - alpha * cw.field(e, kCgW)[i];
        r[i] = rn;
        v[0] = norm2(rn);
    }
    write_partials_at<1, kPBlock>(cw.p(e, 1), blockIdx.y * gridDim.x + blockIdx.x, v);
}

// beta = |z_new|^2 / zeta;  p = z + beta p;  zeta_next = |z_new|^2.
__global__ __launch_bounds__(kPBlock) void k_cg_update_p(Geom g, CgWork cw, int npart, int par) {
    const int e = blockIdx.z;
    CgRhs* st = cw.st + e;
    if (block_flag_cg(&st->done)) return;
    double red[1];
    reduce_partials<1, kPBlock>(cw.p(e, 2), npart, red);
    const double zo = st->zeta[par];
    const double beta = zo > 0.0 ? red[0] / zo : 0.0;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) st->zeta[par ^ 1] = red[0];
    const int s = blockIdx.x * kPBlock + threadIdx.x;
    if (s >= g.V) return;
    const size_t i = (size_t)blockIdx.y * g.ldv + s;
    ZD* p = cw.field(e, kCgP);
    p[i] = cw.field(e, kCgZ)[i] + beta * p[i];
}

// |r|^2 of every system; converged (|r| <= tol |b|) or stalled systems freeze.
__global__ __launch_bounds__(kPBlock) void k_cg_check(CgWork cw, int npart, double tol2) {
    const int e = blockIdx.y;
    CgRhs* st = cw.st + e;
    if (block_flag_cg(&st->done)) return;
    double red[1];
    reduce_partials<1, kPBlock>(cw.p(e, 1), npart, red);
    if (threadIdx.x == 0) {
        st->rr = red[0];
        if (red[0] <= tol2 * st->bnorm2) st->done = 1;
    }
}

// Projection after the solve: e < l: x -= R_i (L_i^H x);  e >= l: x -= L_i (R_i^H x),
// then x *= conj(c_i).  Two phases: per-block partials of the dot, then the update.
__global__ __launch_bounds__(kBlock) void k_cg_proj_dot(Geom g, const ZD* __restrict__ R, const ZD* __restrict__ L,
                                                        int l, CgWork cw) {
    const int e = blockIdx.y;
    const int i = e < l ? e : e - l;
    const ZD* __restrict__ P = e < l ? L : R;
    const int s = blockIdx.x * kBlock + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (s < g.V) {
        const size_t n12 = (size_t)12 * g.V, o = (size_t)s * 12;
        const ZD* x = cw.field(e, kCgX);
#pragma unroll
        for (int p = 0; p < 12; ++p) {
            const ZD t = cjmul(P[(size_t)i * n12 + o + p], x[(size_t)p * g.ldv + s]);
            v[0] += t.re;
            v[1] += t.im;
        }
    }
    write_partials<2, kBlock>(cw.p(e, 3), v);
}

__global__ __launch_bounds__(kBlock) void k_cg_proj_apply(Geom g, const ZD* __restrict__ R, const ZD* __restrict__ L,
                                                          const ZD* __restrict__ c, int l, CgWork cw, int npart) {
    const int e = blockIdx.y;
    const int i = e < l ? e : e - l;
    const ZD* __restrict__ P = e < l ? R : L;
    double red[2];
    reduce_partials<2, kBlock>(cw.p(e, 3), npart, red);
    const ZD d = mk<double>(red[0], red[1]);
    const ZD sc = e < l ? mk<double>(1.0, 0.0) : cj(c[i]);
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const size_t n12 = (size_t)12 * g.V, o = (size_t)s * 12;
    ZD* x = cw.field(e, kCgX);
#pragma unroll
    for (int p = 0; p < 12; ++p) {
        const size_t k = (size_t)p * g.ldv + s;
        x[k] = sc * (x[k] - d * P[(size_t)i * n12 + o + p]);
    }
}

// dU[nu][x] += boundary sign * (-kappa) sum_i [force(X1_i, R_i) + force(q_i L_i, Z_i psi)]
// with X1_i = conj(c_i) Z_i^H a_i (solution e = l + i) and Z_i psi (solution e = i).
// Pair (p, q) adds the coefficient of dU in Re p^H dH q (the same contraction as the
// Krylov force); p, q read from canonical (R, L) or SoA (solutions) storage.
template <int NU>
__device__ void defl_force_body(const Geom& g, double kappa, double emu, const ZD* __restrict__ R,
                                const ZD* __restrict__ L, const ZD* __restrict__ q, int l, const CgWork& cw, int s,
                                int antiperiodic, ZD* __restrict__ dU) {
    const Nbr n = neighbours(g, s);
    const int y = n.fwd[NU];
    const double ef = (NU == 3) ? emu : 1.0, eb = (NU == 3) ? 1.0 / emu : 1.0;
    const size_t n12 = (size_t)12 * g.V;
    ZD G[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) G[a][b] = mk<double>(0, 0);
    auto canon = [&](Spinor<double>& sp, const ZD* f, int site, ZD scale) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) sp.c[a][b] = scale * f[(size_t)site * 12 + a * 3 + b];
    };
    for (int i = 0; i < l; ++i) {
        Spinor<double> px, qx, py, qy;
        // pair 1: p = conj(c_i) Z_i^H a_i (SoA), q = R_i (canonical)
        load_spinor(px, cw.field(l + i, kCgX), g.ldv, s);
        load_spinor(py, cw.field(l + i, kCgX), g.ldv, y);
        canon(qx, R + (size_t)i * n12, s, mk<double>(1.0, 0.0));
        canon(qy, R + (size_t)i * n12, y, mk<double>(1.0, 0.0));
        force_pair<NU>(G, px, qx, py, qy, ef, eb);
        // pair 2: p = q_i L_i (canonical), q = Z_i psi (SoA)
        canon(px, L + (size_t)i * n12, s, q[i]);
        canon(py, L + (size_t)i * n12, y, q[i]);
        load_spinor(qx, cw.field(i, kCgX), g.ldv, s);
        load_spinor(qy, cw.field(i, kCgX), g.ldv, y);
        force_pair<NU>(G, px, qx, py, qy, ef, eb);
    }
    const double sign = (NU == 3 && antiperiodic && s / (g.nx * g.ny * g.nz) == g.nt - 1) ? -1.0 : 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            ZD& o = dU[((size_t)NU * g.V + s) * 9 + a * 3 + b];
            o = o + (-kappa * sign) * G[a][b];
        }
}

__global__ __launch_bounds__(kBlock) void k_defl_force(Geom g, double kappa, double emu, const ZD* __restrict__ R,
                                                       const ZD* __restrict__ L, const ZD* __restrict__ q, int l,
                                                       CgWork cw, int antiperiodic, ZD* __restrict__ dU) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.V) return;
    switch (blockIdx.y) {
        case 0: defl_force_body<0>(g, kappa, emu, R, L, q, l, cw, s, antiperiodic, dU); break;
        case 1: defl_force_body<1>(g, kappa, emu, R, L, q, l, cw, s, antiperiodic, dU); break;
        case 2: defl_force_body<2>(g, kappa, emu, R, L, q, l, cw, s, antiperiodic, dU); break;
        default: defl_force_body<3>(g, kappa, emu, R, L, q, l, cw, s, antiperiodic, dU); break;
    }
}

// ---------------------------------------------------------------- launchers
void launch_cg_rhs(const Geom& g, const ZD* psi, const ZD* eta, const ZD* pbar, const ZD* R, const ZD* L, const ZD* c,
                   const ZD* q, const double* sgn, int l, const CgWork& cw, hipStream_t st) {
    const int nb = grid_for(g.V);
    hipLaunchKernelGGL(k_cg_rhs, dim3(nb, 2 * l), dim3(kBlock), 0, st, g, psi, eta, pbar, R, L, c, q, sgn, l, cw);
    hipLaunchKernelGGL(k_cg_bnorm, dim3(1, 2 * l), dim3(kBlock), 0, st, cw, nb);
}

void launch_cg_start(const ZD* U, const Geom& g, double kappa, double mu, int nr, const CgWork& cw, hipStream_t st) {
    const double emu = std::exp(mu);
    cg_apply(U, g, kappa, emu, nr, cw, 1, kCgR, kCgZ, 2, st);
    dim3 gp((g.V + kPBlock - 1) / kPBlock, 12, nr);
    hipLaunchKernelGGL(k_cg_init_p, gp, dim3(kPBlock), 0, st, g, cw, np_stencil(g.V));
}

void launch_cg_iteration(const ZD* U, const Geom& g, double kappa, double mu, int nr, int it, int check, double tol,
                         const CgWork& cw, hipStream_t st) {
    const double emu = std::exp(mu);
    const int par = it & 1;
    const dim3 gp((g.V + kPBlock - 1) / kPBlock, 12, nr);
    cg_apply(U, g, kappa, emu, nr, cw, 0, kCgP, kCgW, 0, st);
    hipLaunchKernelGGL(k_cg_update_xr, gp, dim3(kPBlock), 0, st, g, cw, np_stencil(g.V), par);
    if (check) hipLaunchKernelGGL(k_cg_check, dim3(1, nr), dim3(kPBlock), 0, st, cw, np_point(g.V), tol * tol);
    cg_apply(U, g, kappa, emu, nr, cw, 1, kCgR, kCgZ, 2, st);
    hipLaunchKernelGGL(k_cg_update_p, gp, dim3(kPBlock), 0, st, g, cw, np_stencil(g.V), par);
}

void launch_cg_finish(const Geom& g, const ZD* R, const ZD* L, const ZD* c, int l, const CgWork& cw, hipStream_t st) {
    const int nb = grid_for(g.V);
    hipLaunchKernelGGL(k_cg_proj_dot, dim3(nb, 2 * l), dim3(kBlock), 0, st, g, R, L, l, cw);
    hipLaunchKernelGGL(k_cg_proj_apply, dim3(nb, 2 * l), dim3(kBlock), 0, st, g, R, L, c, l, cw, nb);
}

void launch_defl_force(const Geom& g, double kappa, double mu, const ZD* R, const ZD* L, const ZD* q, int l,
                       const CgWork& cw, int antiperiodic, ZD* dU, hipStream_t st) {
    hipLaunchKernelGGL(k_defl_force, dim3(grid_for(g.V), 4), dim3(kBlock), 0, st, g, kappa, std::exp(mu), R, L, q, l,
                       cw, antiperiodic, dU);
}

}  // namespace tslov
