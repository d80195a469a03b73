// Lattice-field kernels of the TSL hot path: layout conversion, the Wilson
// stencil (App. A, eq. WD_op/WD_G), the fused two-sided Lanczos step (Sec. 2),
// output assembly (eq. overlap), the reverse-mode recursion and the per-link
// force contraction for dS/dU.
#include "kernels.h"

#include <cmath>

namespace tslov {

namespace {

// Launch with the timing events recorded by the dispatch itself when given.
template <typename K, typename... Args>
void timed_launch(K kernel, dim3 grid, dim3 block, hipStream_t st, Timing t, Args... args) {
    if (t.a && t.b) hipExtLaunchKernelGGL(kernel, grid, block, 0, st, t.a, t.b, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

// Compiler barrier for memory operations: keeps the epilogue's own-site loads from
// being hoisted above the hopping loop, where they would stay live (and spill).
__device__ __forceinline__ void mem_fence_compiler() { asm volatile("" ::: "memory"); }

// One direction of the hopping sum for a single field.
template <int NU, typename R, typename RL>
__device__ __forceinline__ void hop_dir(Spinor<R>& acc, const Z<RL>* __restrict__ U, const Z<R>* __restrict__ in,
                                        const Geom& g, int s, const Nbr& n, R cf, R cb, int g5_in) {
    Z<R> u[3][3];
    Spinor<R> p;
    load_link(u, U, g.ldv, NU, s);
    load_spinor(p, in, g.ldv, n.fwd[NU]);
    if (g5_in) g5_inplace(p);
    hop_fwd<NU>(acc, u, p, cf);
    load_link(u, U, g.ldv, NU, n.bwd[NU]);
    load_spinor(p, in, g.ldv, n.bwd[NU]);
    if (g5_in) g5_inplace(p);
    hop_bwd<NU>(acc, u, p, cb);
}

// One direction of the hopping sums of two fields sharing the link loads:
// field A with chemical potential +mu, field B with -mu.
template <int NU, typename R, typename RL>
__device__ __forceinline__ void hop_dir_pair(Spinor<R>& acca, Spinor<R>& accb, const Z<RL>* __restrict__ U,
                                             const Z<R>* __restrict__ fa, const Z<R>* __restrict__ fb,
                                             const Geom& g, int s, const Nbr& n, R ep, R em) {
    const R fa_f = (NU == 3) ? ep : R(1), fa_b = (NU == 3) ? em : R(1);
    Z<R> u[3][3];
    Spinor<R> p;
    load_link(u, U, g.ldv, NU, s);
    load_spinor(p, fa, g.ldv, n.fwd[NU]);
    hop_fwd<NU>(acca, u, p, fa_f);
    load_spinor(p, fb, g.ldv, n.fwd[NU]);
    hop_fwd<NU>(accb, u, p, fa_b);
    load_link(u, U, g.ldv, NU, n.bwd[NU]);
    load_spinor(p, fa, g.ldv, n.bwd[NU]);
    hop_bwd<NU>(acca, u, p, fa_b);
    load_spinor(p, fb, g.ldv, n.bwd[NU]);
    hop_bwd<NU>(accb, u, p, fa_f);
}

}  // namespace

// =============================================================== layout
// A thread that meets a non-finite link element stores 1 into *bad (a plain store:
// every writer writes the same value).
__global__ __launch_bounds__(kBlock) void k_links_to_soa(const ZD* __restrict__ Uc, ZD* __restrict__ U64,
                                                         Z<float>* __restrict__ U32, Geom g, int antiperiodic,
                                                         int* __restrict__ bad) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    const int nu = blockIdx.y;
    if (s >= g.V) return;
    double sign = 1.0;
    if (nu == 3 && antiperiodic && s / (g.nx * g.ny * g.nz) == g.nt - 1) sign = -1.0;
    bool finite = true;
#pragma unroll
    for (int ab = 0; ab < 9; ++ab) {
        const ZD u = sign * Uc[((size_t)nu * g.V + s) * 9 + ab];
        finite = finite && std::isfinite(u.re) && std::isfinite(u.im);
        U64[(size_t)(nu * 9 + ab) * g.ldv + s] = u;
        if (U32) U32[(size_t)(nu * 9 + ab) * g.ldv + s] = zcast<float>(u);
    }
    if (!finite) *bad = 1;
}

void launch_links_to_soa(const ZD* Ucanon, ZD* U64, Z<float>* U32, const Geom& g, int antiperiodic, int* bad,
                         hipStream_t st) {
    dim3 grid(grid_for(g.V), 4);
    hipLaunchKernelGGL(k_links_to_soa, grid, dim3(kBlock), 0, st, Ucanon, U64, U32, g, antiperiodic, bad);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_spinor_to_soa(const ZD* __restrict__ in, Z<R>* __restrict__ out, Geom g,
                                                          double* __restrict__ part) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    double v[kNvRecur] = {0.0, 0.0, 0.0, 0.0};
    if (s < g.V) {
        double n2 = 0.0;
#pragma unroll
        for (int p = 0; p < 12; ++p) {
            const ZD z = in[(size_t)s * 12 + p];
            const Z<R> zr = zcast<R>(z);
            out[(size_t)p * g.ldv + s] = zr;
            n2 += (double)zr.re * zr.re + (double)zr.im * zr.im;
        }
        // |x|^2 laid out as (omega re, omega im, |r|^2, |s|^2) so that the first
        // Lanczos step normalises with beta_1 = gamma_1 = |x|.
        v[0] = n2;
        v[2] = n2;
        v[3] = n2;
    }
    if (part) write_partials<kNvRecur, kBlock>(part, v);
}

template <typename R>
void launch_spinor_to_soa(const ZD* in, Z<R>* out, const Geom& g, double* part_norm, hipStream_t st) {
    hipLaunchKernelGGL(k_spinor_to_soa<R>, dim3(grid_for(g.V)), dim3(kBlock), 0, st, in, out, g, part_norm);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_spinor_from_soa(const Z<R>* __restrict__ in, ZD* __restrict__ out, Geom g) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.V) return;
#pragma unroll
    for (int p = 0; p < 12; ++p) out[(size_t)s * 12 + p] = zcast<double>(in[(size_t)p * g.ldv + s]);
}

template <typename R>
void launch_spinor_from_soa(const Z<R>* in, ZD* out, const Geom& g, hipStream_t st) {
    hipLaunchKernelGGL(k_spinor_from_soa<R>, dim3(grid_for(g.V)), dim3(kBlock), 0, st, in, out, g);
}

// =============================================================== stencil layouts
// One thread per (site, colour), 64 consecutive sites per wavefront, so that every
// load instruction touches 64 consecutive sites of one plane.  Colour grid (small
// lattices): single-wavefront blocks, block (a, b) handles colour a of site block b,
// which spreads the three colours of a site over three compute units.  Colour split
// (the Lanczos pair kernels on larger lattices): blocks of 3 wavefronts, wavefront a
// handles colour a.  The operator on larger lattices uses one thread per site
// (k_apply_site).
template <typename R>
__device__ __forceinline__ void load1(Z<R> (&p)[4], const Z<R>* __restrict__ f, int ldv, int a, int s) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) p[sp] = fload<R>(field_base(f), ldv, sp * 3 + a, (unsigned)s);
}
// load1 with the streaming hint, for a field this kernel reads once
template <typename R>
__device__ __forceinline__ void load1_nt(Z<R> (&p)[4], const Z<R>* __restrict__ f, int ldv, int a, int s) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) p[sp] = fload_nt<R>(field_base(f), ldv, sp * 3 + a, (unsigned)s);
}

template <typename R>
__device__ __forceinline__ void store1(Z<R>* __restrict__ f, int ldv, int a, int s, const Z<R> (&p)[4]) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) fstore<R>(field_base(f), ldv, sp * 3 + a, (unsigned)s, p[sp]);
}

template <typename R>
__device__ __forceinline__ void store1_nt(Z<R>* __restrict__ f, int ldv, int a, int s, const Z<R> (&p)[4]) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) fstore_nt<R>(field_base(f), ldv, sp * 3 + a, (unsigned)s, p[sp]);
}

template <typename R>
__device__ __forceinline__ void zero1(Z<R> (&p)[4]) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) p[sp] = mk<R>(0, 0);
}

// Both hops of direction NU for two fields sharing the link rows: field A at +mu,
// field B at -mu (the temporal factors swap).
template <int NU, typename R, typename RL>
__device__ __forceinline__ void hop_dir_pair1(Z<R> (&acca)[4], Z<R> (&accb)[4], const Z<RL>* __restrict__ U,
                                              const Z<R>* __restrict__ fa, const Z<R>* __restrict__ fb,
                                              const Geom& g, int s, int a, const Nbr& n, R ep, R em) {
    const R up = (NU == 3) ? ep : R(1), dn = (NU == 3) ? em : R(1);
    Z<R> u[3];
    Spinor<R> p;
    load_row(u, U, g.ldv, NU, a, s);
    load_spinor(p, fa, g.ldv, n.fwd[NU]);
    hop1<NU, +1>(acca, u, p, up);
    load_spinor(p, fb, g.ldv, n.fwd[NU]);
    hop1<NU, +1>(accb, u, p, dn);
    load_col_conj(u, U, g.ldv, NU, a, n.bwd[NU]);
    load_spinor(p, fa, g.ldv, n.bwd[NU]);
    hop1<NU, -1>(acca, u, p, dn);
    load_spinor(p, fb, g.ldv, n.bwd[NU]);
    hop1<NU, -1>(accb, u, p, up);
}

// Both hops of direction NU for one field (colour a):
//   acc += cf (1+g) U(x) f(x+nu) + cb (1-g) U(x-nu)^dag f(x-nu), f optionally g5-multiplied,
// with every load of the direction issued before any arithmetic (the compiler
// barrier keeps the scheduler from sinking the loads to their uses): one memory
// round trip per direction instead of one per loaded operand, at the cost of
// holding all operands of a direction in registers.  The pair version below does
// the same for two fields sharing the link rows.
template <int NU, typename R, typename RL>
__device__ __forceinline__ void hop_dir1_eager(Z<R> (&acc)[4], const Z<RL>* __restrict__ U,
                                               const Z<R>* __restrict__ f, const Geom& g, int s, int a, const Nbr& n,
                                               R cf, R cb, int g5_in) {
    Z<R> uf[3], ub[3];
    Spinor<R> pf, pb;
    load_row(uf, U, g.ldv, NU, a, s);
    load_spinor(pf, f, g.ldv, n.fwd[NU]);
    load_col_conj(ub, U, g.ldv, NU, a, n.bwd[NU]);
    load_spinor(pb, f, g.ldv, n.bwd[NU]);
    mem_fence_compiler();
    if (g5_in) {
        g5_inplace(pf);
        g5_inplace(pb);
    }
    hop1<NU, +1>(acc, uf, pf, cf);
    hop1<NU, -1>(acc, ub, pb, cb);
}

// All eight hops of two fields (colour a) sharing the link rows (A at +mu, B at
// -mu), a rolled loop over a wavefront-uniform switch: the colour split, with
// several wavefronts per SIMD, so one operand's loads in flight at a time and few
// registers.  (The colour grid's pair kernels use hop_two_dirs_pair_eager.)
template <int BLK, typename R, typename RL>
__device__ __forceinline__ void hop_all_pair(Z<R> (&acca)[4], Z<R> (&accb)[4], const Z<RL>* __restrict__ U,
                                             const Z<R>* __restrict__ fa, const Z<R>* __restrict__ fb,
                                             const Geom& g, int s, int a, const Nbr& n, R ep, R em) {
#pragma unroll 1
    for (int nu = 0; nu < 4; ++nu) {
        switch (nu) {
            case 0: hop_dir_pair1<0>(acca, accb, U, fa, fb, g, s, a, n, ep, em); break;
            case 1: hop_dir_pair1<1>(acca, accb, U, fa, fb, g, s, a, n, ep, em); break;
            case 2: hop_dir_pair1<2>(acca, accb, U, fa, fb, g, s, a, n, ep, em); break;
            default: hop_dir_pair1<3>(acca, accb, U, fa, fb, g, s, a, n, ep, em); break;
        }
    }
}

// Two directions at once for two fields sharing the link rows: all sixteen
// operands (four link rows, eight neighbour spinors) issued before any arithmetic,
// one memory round trip for both directions.  Needs more than 256 registers: for
// kernels whose grid leaves one wavefront per SIMD anyway (the colour grid).
template <int NU0, int NU1, typename R, typename RL>
__device__ __forceinline__ void hop_two_dirs_pair_eager(Z<R> (&acca)[4], Z<R> (&accb)[4], const Z<RL>* __restrict__ U,
                                                        const Z<R>* __restrict__ fa, const Z<R>* __restrict__ fb,
                                                        const Geom& g, int s, int a, const Nbr& n, R ep, R em) {
    const R up0 = (NU0 == 3) ? ep : R(1), dn0 = (NU0 == 3) ? em : R(1);
    const R up1 = (NU1 == 3) ? ep : R(1), dn1 = (NU1 == 3) ? em : R(1);
    Z<R> uf0[3], ub0[3], uf1[3], ub1[3];
    Spinor<R> paf0, pbf0, pab0, pbb0, paf1, pbf1, pab1, pbb1;
    load_row(uf0, U, g.ldv, NU0, a, s);
    load_spinor(paf0, fa, g.ldv, n.fwd[NU0]);
    load_spinor(pbf0, fb, g.ldv, n.fwd[NU0]);
    load_col_conj(ub0, U, g.ldv, NU0, a, n.bwd[NU0]);
    load_spinor(pab0, fa, g.ldv, n.bwd[NU0]);
    load_spinor(pbb0, fb, g.ldv, n.bwd[NU0]);
    load_row(uf1, U, g.ldv, NU1, a, s);
    load_spinor(paf1, fa, g.ldv, n.fwd[NU1]);
    load_spinor(pbf1, fb, g.ldv, n.fwd[NU1]);
    load_col_conj(ub1, U, g.ldv, NU1, a, n.bwd[NU1]);
    load_spinor(pab1, fa, g.ldv, n.bwd[NU1]);
    load_spinor(pbb1, fb, g.ldv, n.bwd[NU1]);
    mem_fence_compiler();
    hop1<NU0, +1>(acca, uf0, paf0, up0);
    hop1<NU0, +1>(accb, uf0, pbf0, dn0);
    hop1<NU0, -1>(acca, ub0, pab0, dn0);
    hop1<NU0, -1>(accb, ub0, pbb0, up0);
    hop1<NU1, +1>(acca, uf1, paf1, up1);
    hop1<NU1, +1>(accb, uf1, pbf1, dn1);
    hop1<NU1, -1>(acca, ub1, pab1, dn1);
    hop1<NU1, -1>(accb, ub1, pbb1, up1);
}

// Colour-grid pair kernels: hop wavefront h (0 or 1) takes directions 2h and 2h + 1,
// all their operands in one round trip.
template <typename R, typename RL>
__device__ __forceinline__ void hop_half_pair(Z<R> (&acca)[4], Z<R> (&accb)[4], const Z<RL>* __restrict__ U,
                                              const Z<R>* __restrict__ fa, const Z<R>* __restrict__ fb,
                                              const Geom& g, int s, int a, const Nbr& n, R ep, R em, int half) {
    if (half == 0)
        hop_two_dirs_pair_eager<0, 1>(acca, accb, U, fa, fb, g, s, a, n, ep, em);
    else
        hop_two_dirs_pair_eager<2, 3>(acca, accb, U, fa, fb, g, s, a, n, ep, em);
}

// Colour-split hops of NS entries of a batch (A_q at +mu, B_q at -mu) with the neighbour
// spinors shared through LDS.  Thread (a, l) loads only colour a of the four neighbour
// spinors of a direction (four spins each), projects it to its two half-spinor
// components and publishes them; after a barrier it reads the three colours of each
// half spinor of its own site and applies its link row.  A neighbour value thus passes
// the vector L1 once per block, not once per colour wavefront, and the link rows are
// loaded once for all NS entries (the entries whose bit is set in the block-uniform
// mask `live`).  Every half-spinor component, product and sum of an entry is formed by
// the same operations in the same order whatever NS (the link-row products by
// row_dot's fixed chain), so an entry gets the same bits in every shape.  All threads
// of the block must call it (`in` false for sites past the volume: no loads, their
// slots are not read).
template <typename R>
struct HopX {
    Z<R> h[4][2][3][kSites];   // hop (A forward, B forward, A backward, B backward), half spin, colour, site
};

template <int NU, int S, typename R>
__device__ __forceinline__ void hop1_x(Z<R> (&acc)[4], const Z<R> (&urow)[3], const Z<R> (&hx)[2][3][kSites], int l,
                                       R coef) {
    Z<R> h[2][3], o[2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) h[s][c] = hx[s][c][l];
#pragma unroll
    for (int s = 0; s < 2; ++s) o[s] = row_dot(urow, h[s][0], h[s][1], h[s][2]);
    recon1_add<NU, S>(acc, o, coef);
}

template <int NU, int NS, typename R, typename RL>
__device__ __forceinline__ void hop_dir_pair_x(Z<R> (&acca)[NS][4], Z<R> (&accb)[NS][4], const Z<RL>* __restrict__ U,
                                               const Z<R>* const (&fa)[NS], const Z<R>* const (&fb)[NS],
                                               unsigned live, const Geom& g, int s, int a, int l, bool in,
                                               const Nbr& n, R ep, R em, HopX<R> (&x)[NS]) {
    const R up = (NU == 3) ? ep : R(1), dn = (NU == 3) ? em : R(1);
    Z<R> uf[3], ub[3];
    if (in) {
        const unsigned yf = (unsigned)n.fwd[NU], yb = (unsigned)n.bwd[NU];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            if (!(live & (1u << q))) continue;
            if (q > 0) mem_fence_compiler();   // one entry's neighbour operands in flight at a time
            const FieldBase ra = field_base(fa[q]), rb = field_base(fb[q]);
            Z<R> p[4][4];   // colour a of A(x+nu), B(x+nu), A(x-nu), B(x-nu)
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                p[0][sp] = fload<R>(ra, g.ldv, sp * 3 + a, yf);
                p[1][sp] = fload<R>(rb, g.ldv, sp * 3 + a, yf);
                p[2][sp] = fload<R>(ra, g.ldv, sp * 3 + a, yb);
                p[3][sp] = fload<R>(rb, g.ldv, sp * 3 + a, yb);
            }
            if (q == NS - 1) {
                load_row(uf, U, g.ldv, NU, a, s);
                load_col_conj(ub, U, g.ldv, NU, a, n.bwd[NU]);
            }
            Z<R> h0, h1;
            project_col<NU, +1>(p[0][0], p[0][1], p[0][2], p[0][3], h0, h1);
            x[q].h[0][0][a][l] = h0;
            x[q].h[0][1][a][l] = h1;
            project_col<NU, +1>(p[1][0], p[1][1], p[1][2], p[1][3], h0, h1);
            x[q].h[1][0][a][l] = h0;
            x[q].h[1][1][a][l] = h1;
            project_col<NU, -1>(p[2][0], p[2][1], p[2][2], p[2][3], h0, h1);
            x[q].h[2][0][a][l] = h0;
            x[q].h[2][1][a][l] = h1;
            project_col<NU, -1>(p[3][0], p[3][1], p[3][2], p[3][3], h0, h1);
            x[q].h[3][0][a][l] = h0;
            x[q].h[3][1][a][l] = h1;
        }
        if (!(live & (1u << (NS - 1)))) {   // the last entry is stopped or past the list's end
            load_row(uf, U, g.ldv, NU, a, s);
            load_col_conj(ub, U, g.ldv, NU, a, n.bwd[NU]);
        }
    }
    __syncthreads();
    if (in) {
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            if (!(live & (1u << q))) continue;
            hop1_x<NU, +1>(acca[q], uf, x[q].h[0], l, up);
            hop1_x<NU, +1>(accb[q], uf, x[q].h[1], l, dn);
            hop1_x<NU, -1>(acca[q], ub, x[q].h[2], l, dn);
            hop1_x<NU, -1>(accb[q], ub, x[q].h[3], l, up);
        }
    }
    __syncthreads();   // the next direction overwrites the slots
}

template <int NS, typename R, typename RL>
__device__ __forceinline__ void hop_all_pair_x(Z<R> (&acca)[NS][4], Z<R> (&accb)[NS][4], const Z<RL>* __restrict__ U,
                                               const Z<R>* const (&fa)[NS], const Z<R>* const (&fb)[NS],
                                               unsigned live, const Geom& g, int s, int a, R ep, R em,
                                               HopX<R> (&x)[NS]) {
    const int l = threadIdx.x % kSites;
    const bool in = s < g.V;
    const Nbr n = neighbours(g, in ? s : 0);
#pragma unroll 1
    for (int nu = 0; nu < 4; ++nu) {
        switch (nu) {
            case 0: hop_dir_pair_x<0, NS>(acca, accb, U, fa, fb, live, g, s, a, l, in, n, ep, em, x); break;
            case 1: hop_dir_pair_x<1, NS>(acca, accb, U, fa, fb, live, g, s, a, l, in, n, ep, em, x); break;
            case 2: hop_dir_pair_x<2, NS>(acca, accb, U, fa, fb, live, g, s, a, l, in, n, ep, em, x); break;
            default: hop_dir_pair_x<3, NS>(acca, accb, U, fa, fb, live, g, s, a, l, in, n, ep, em, x); break;
        }
    }
}

// Block-uniform reads of the stop flags of NS entries (1 for an entry past the
// end of the list), with one pair of barriers for all of them.
template <int NS>
__device__ __forceinline__ unsigned block_live(const Coef& coef0, const SrcList& L, int e0) {
    __shared__ int f[NS];
    if (threadIdx.x < NS) {
        const int e = e0 + (int)threadIdx.x;
        f[threadIdx.x] = e < L.n ? *(volatile const int*)coef0.at(L.slot[e]).status : 1;
    }
    __syncthreads();
    unsigned live = 0;
#pragma unroll
    for (int q = 0; q < NS; ++q)
        if (!f[q]) live |= 1u << q;
    __syncthreads();
    return live;
}

// =============================================================== operator
// Colour grid (small lattices): block (a, b) forms colour a of site block b.
template <typename R, typename RL>
__global__ __launch_bounds__(kSites) void k_apply(const Z<RL>* __restrict__ U, const Z<R>* __restrict__ in,
                                                  Z<R>* __restrict__ out, Geom g, R kappa, R ep, R em, int g5_in,
                                                  int g5_out) {
    const int a = sten_colour<kSites>();
    const int s = sten_block<kSites>(g) * kSites + threadIdx.x;
    if (s >= g.V) return;
    const Nbr n = neighbours(g, s);
    Z<R> acc[4];
    zero1(acc);
#pragma unroll 1
    for (int nu = 0; nu < 4; ++nu) {
        switch (nu) {
            case 0: hop_dir1_eager<0>(acc, U, in, g, s, a, n, R(1), R(1), g5_in); break;
            case 1: hop_dir1_eager<1>(acc, U, in, g, s, a, n, R(1), R(1), g5_in); break;
            case 2: hop_dir1_eager<2>(acc, U, in, g, s, a, n, R(1), R(1), g5_in); break;
            default: hop_dir1_eager<3>(acc, U, in, g, s, a, n, ep, em, g5_in); break;
        }
    }
    mem_fence_compiler();
    Z<R> x[4];
    load1(x, in, g.ldv, a, s);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
        const R s_in = (g5_in && sp >= 2) ? R(-1) : R(1);
        const R s_out = (g5_out && sp >= 2) ? R(-1) : R(1);
        x[sp] = s_out * (s_in * x[sp] - kappa * acc[sp]);
    }
    store1(out, g.ldv, a, s, x);
}

// Site per thread (lattices above the colour grid's range): each thread forms all
// three colours of its site, so every neighbour spinor and link passes through the
// compute unit's L1 once per site instead of once per colour wavefront.  Blocks go
// out in XCD order: when the site blocks of a t-slice split evenly over the XCDs,
// each XCD takes the same run of them in every slice, slice after slice, so that a
// site's t-neighbours were read one run earlier on the same L2; otherwise each
// XCD takes a contiguous run of the lattice.
template <typename R, typename RL>
__global__ __launch_bounds__(kBlock) void k_apply_site(const Z<RL>* __restrict__ U, const Z<R>* __restrict__ in,
                                                       Z<R>* __restrict__ out, Geom g, R kappa, R ep, R em,
                                                       int g5_in, int g5_out, int slice_order) {
    int sb;
    if (slice_order) {
        // each XCD takes the same run of site blocks in every t-slice, t outermost:
        // a site's t-neighbours were touched one slice's run earlier on this XCD
        const int n3 = g.nx * g.ny * g.nz / kBlock, per = n3 / kXcd, m = blockIdx.x / kXcd;
        sb = (m / per) * n3 + (blockIdx.x % kXcd) * per + m % per;
    } else {
        sb = xcd_block(blockIdx.x, gridDim.x);
    }
    const int s = sb * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const Nbr n = neighbours(g, s);
    Spinor<R> acc;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc.c[sp][c] = mk<R>(0, 0);
#pragma unroll 1
    for (int nu = 0; nu < 4; ++nu) {
        Z<R> u[3][3];
        Spinor<R> p;
        switch (nu) {
            case 0:
                load_link(u, U, g.ldv, 0, s); load_spinor(p, in, g.ldv, n.fwd[0]); if (g5_in) g5_inplace(p);
                hop_fwd<0>(acc, u, p, R(1));
                load_link(u, U, g.ldv, 0, n.bwd[0]); load_spinor(p, in, g.ldv, n.bwd[0]); if (g5_in) g5_inplace(p);
                hop_bwd<0>(acc, u, p, R(1));
                break;
            case 1:
                load_link(u, U, g.ldv, 1, s); load_spinor(p, in, g.ldv, n.fwd[1]); if (g5_in) g5_inplace(p);
                hop_fwd<1>(acc, u, p, R(1));
                load_link(u, U, g.ldv, 1, n.bwd[1]); load_spinor(p, in, g.ldv, n.bwd[1]); if (g5_in) g5_inplace(p);
                hop_bwd<1>(acc, u, p, R(1));
                break;
            case 2:
                load_link(u, U, g.ldv, 2, s); load_spinor(p, in, g.ldv, n.fwd[2]); if (g5_in) g5_inplace(p);
                hop_fwd<2>(acc, u, p, R(1));
                load_link(u, U, g.ldv, 2, n.bwd[2]); load_spinor(p, in, g.ldv, n.bwd[2]); if (g5_in) g5_inplace(p);
                hop_bwd<2>(acc, u, p, R(1));
                break;
            default:
                load_link(u, U, g.ldv, 3, s); load_spinor(p, in, g.ldv, n.fwd[3]); if (g5_in) g5_inplace(p);
                hop_fwd<3>(acc, u, p, ep);
                load_link(u, U, g.ldv, 3, n.bwd[3]); load_spinor(p, in, g.ldv, n.bwd[3]); if (g5_in) g5_inplace(p);
                hop_bwd<3>(acc, u, p, em);
                break;
        }
    }
    mem_fence_compiler();
    Spinor<R> x;
    load_spinor(x, in, g.ldv, s);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
        const R s_in = (g5_in && sp >= 2) ? R(-1) : R(1);
        const R s_out = (g5_out && sp >= 2) ? R(-1) : R(1);
#pragma unroll
        for (int c = 0; c < 3; ++c) x.c[sp][c] = s_out * (s_in * x.c[sp][c] - kappa * acc.c[sp][c]);
    }
    // streaming stores: the result is not read again here and would only displace
    // neighbour spinors and links from L2
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            R* q = reinterpret_cast<R*>(out + (size_t)(sp * 3 + c) * g.ldv + s);
            __builtin_nontemporal_store(x.c[sp][c].re, q);
            __builtin_nontemporal_store(x.c[sp][c].im, q + 1);
        }
}

// Both hops of direction NU for a whole site, with the four operands' loads
// issued before any arithmetic (one memory round trip per direction).
template <int NU, typename R, typename RL>
__device__ __forceinline__ void tm_hops_eager(Spinor<R>& acc, const Z<RL>* __restrict__ U, const Z<R>* __restrict__ in,
                                              const Geom& g, int s, int sf, int sb, int g5_in) {
    Z<R> uf[3][3], ub[3][3];
    Spinor<R> pf, pb;
    load_link(uf, U, g.ldv, NU, s);
    load_spinor(pf, in, g.ldv, sf);
    load_link(ub, U, g.ldv, NU, sb);
    load_spinor(pb, in, g.ldv, sb);
    mem_fence_compiler();
    if (g5_in) {
        g5_inplace(pf);
        g5_inplace(pb);
    }
    hop_fwd<NU>(acc, uf, pf, R(1));
    hop_bwd<NU>(acc, ub, pb, R(1));
}

// Site per thread with a march along t: a thread owns one (x, y, z) site of a
// 128-site tile and runs through a chunk of T consecutive t-slices.  The forward
// t-hop's operands at slice t, psi(t+1) and U_t(t), are loaded once: psi(t+1) is
// the own spinor of slice t+1, and U_t(t)^dag P- psi(t) (the backward t-hop of
// slice t+1 before reconstruction) is carried in registers.  So along t every
// spinor and link is read once per chunk instead of up to three times.  The hop
// sum runs in the same order as k_apply_site (x, y, z, t; forward then backward),
// with the same operations, so the two kernels give identical results.  Block
// b works on tile (b mod 8) * per + (b / 8) mod per of chunk b / (8 per): each XCD
// takes the same run of tiles (a slab of z-planes) in every chunk.
template <typename R, typename RL>
__global__ __launch_bounds__(kBlock) void k_apply_tmarch(const Z<RL>* __restrict__ U, const Z<R>* __restrict__ in,
                                                         Z<R>* __restrict__ out, Geom g, R kappa, R ep, R em,
                                                         int g5_in, int g5_out, int T) {
    const int V3 = g.nx * g.ny * g.nz, per = V3 / kBlock / kXcd, m = blockIdx.x / kXcd;
    const int tile = (blockIdx.x % kXcd) * per + m % per, chunk = m / per;
    const int s3 = tile * kBlock + threadIdx.x;   // the (x, y, z) site; t = 0
    const int t0 = chunk * T;
    const Nbr n3 = neighbours(g, s3);
    const R s_in_lo = R(1), s_in_hi = g5_in ? R(-1) : R(1), s_out_hi = g5_out ? R(-1) : R(1);
    // the own spinor waits in a slot of LDS private to the thread (it is needed
    // only after the x, y, z hops, whose operands take the registers)
    __shared__ Z<R> stash[12][kBlock];
    __shared__ Z<R> hstash[6][kBlock];
    auto park = [&](const Spinor<R>& p) {
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) stash[sp * 3 + c][threadIdx.x] = p.c[sp][c];
    };
    {
        Spinor<R> own0;
        load_spinor(own0, in, g.ldv, s3 + t0 * V3);
        park(own0);
    }
    // the carried backward t-hop from slice t0 - 1 (also parked in LDS)
    auto park_h = [&](const Z<R> (&h)[2][3]) {
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) hstash[q * 3 + c][threadIdx.x] = h[q][c];
    };
    {
        Z<R> hb[2][3];
        const int sp = s3 + ((t0 + g.nt - 1) % g.nt) * V3;
        Z<R> u[3][3], h[2][3];
        Spinor<R> p;
        load_link(u, U, g.ldv, 3, sp);
        load_spinor(p, in, g.ldv, sp);
        if (g5_in) g5_inplace(p);
        project<3, -1>(p, h);
        adj_mat_vec(u, h, hb);
        park_h(hb);
    }
#pragma unroll 1
    for (int t = t0; t < t0 + T; ++t) {
        const int s = s3 + t * V3;
        Spinor<R> acc;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc.c[sp][c] = mk<R>(0, 0);
#pragma unroll 1
        for (int nu = 0; nu < 3; ++nu) {
            switch (nu) {
                case 0: tm_hops_eager<0>(acc, U, in, g, s, n3.fwd[0] + t * V3, n3.bwd[0] + t * V3, g5_in); break;
                case 1: tm_hops_eager<1>(acc, U, in, g, s, n3.fwd[1] + t * V3, n3.bwd[1] + t * V3, g5_in); break;
                default: tm_hops_eager<2>(acc, U, in, g, s, n3.fwd[2] + t * V3, n3.bwd[2] + t * V3, g5_in); break;
            }
        }
        // t: forward hop with psi(t+1), then the carried backward hop
        Spinor<R> own;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) own.c[sp][c] = stash[sp * 3 + c][threadIdx.x];
        Z<R> ut[3][3];
        Spinor<R> nxt;
        load_link(ut, U, g.ldv, 3, s);
        load_spinor(nxt, in, g.ldv, s3 + ((t + 1) % g.nt) * V3);
        {
            Spinor<R> p = nxt;
            if (g5_in) g5_inplace(p);
            hop_fwd<3>(acc, ut, p, ep);
        }
        {
            Z<R> hb[2][3];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) hb[q][c] = hstash[q * 3 + c][threadIdx.x];
            reconstruct_add<3, -1>(acc, hb, em);
        }
        // the next slice's backward t-hop: U_t(t)^dag P- psi(t)
        {
            Spinor<R> p = own;
            if (g5_in) g5_inplace(p);
            Z<R> h[2][3], hb[2][3];
            project<3, -1>(p, h);
            adj_mat_vec(ut, h, hb);
            park_h(hb);
        }
        mem_fence_compiler();
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
            const R s_in = sp >= 2 ? s_in_hi : s_in_lo;
            const R s_out = sp >= 2 ? s_out_hi : R(1);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const Z<R> x = s_out * (s_in * own.c[sp][c] - kappa * acc.c[sp][c]);
                R* q = reinterpret_cast<R*>(out + (size_t)(sp * 3 + c) * g.ldv + s);
                __builtin_nontemporal_store(x.re, q);
                __builtin_nontemporal_store(x.im, q + 1);
            }
        }
        park(nxt);
    }
}

// t-slices per chunk of the t-march: the largest divisor of nt that still gives
// 512 workgroups, i.e. one wavefront on every SIMD (the kernel's 256 registers
// allow one; measured at 32^4, 512 beat 256, 1024 and 2048); 0 when the tiles do
// not split evenly over the XCDs.
constexpr int kTmarchGroups = 512;
inline int tmarch_chunk(const Geom& g) {
    const int V3 = g.nx * g.ny * g.nz;
    if (V3 % (kBlock * kXcd) != 0) return 0;
    const int nb3 = V3 / kBlock;
    int T = 0;
    for (int c = 1; c <= g.nt; ++c)
        if (g.nt % c == 0 && (long long)nb3 * (g.nt / c) >= kTmarchGroups) T = c;
    return T > 0 ? T : 1;
}

int tmarch_chunks(const Geom& g, int* T, int maxn) {
    if (colour_grid(g.V) || tmarch_chunk(g) == 0) return 0;
    const long long nb3 = g.nx * g.ny * g.nz / kBlock;
    int n = 0;
    for (int c = 1; c <= g.nt && n < maxn; ++c)
        if (g.nt % c == 0 && nb3 * (g.nt / c) >= 128 && nb3 * (g.nt / c) <= 4096) T[n++] = c;
    return n;
}

template <typename R, typename RL>
void launch_apply(const Z<RL>* U, const Z<R>* in, Z<R>* out, const Geom& g, double kappa, double mu, int g5_in,
                  int g5_out, hipStream_t st, Timing t, int tm_T) {
    if (colour_grid(g.V)) {
        timed_launch(k_apply<R, RL>, dim3(np_sten(g.V)), dim3(kSites), st, t, U, in, out, g, (R)kappa,
                     (R)std::exp(mu), (R)std::exp(-mu), g5_in, g5_out);
    } else if (const int T = tmarch_chunk(g) ? (tm_T > 0 && g.nt % tm_T == 0 ? tm_T : tmarch_chunk(g)) : 0) {
        const int nb = g.nx * g.ny * g.nz / kBlock * (g.nt / T);
        timed_launch(k_apply_tmarch<R, RL>, dim3(nb), dim3(kBlock), st, t, U, in, out, g, (R)kappa, (R)std::exp(mu),
                     (R)std::exp(-mu), g5_in, g5_out, T);
    } else {
        const int nb = (grid_for(g.V) + kXcd - 1) / kXcd * kXcd;
        const int slice = (g.nx * g.ny * g.nz) % (kBlock * kXcd) == 0;   // t-slices split evenly over XCDs
        timed_launch(k_apply_site<R, RL>, dim3(nb), dim3(kBlock), st, t, U, in, out, g, (R)kappa, (R)std::exp(mu),
                     (R)std::exp(-mu), g5_in, g5_out, slice);
    }
}

// =============================================================== batched sources
// Grid dimension y (or z) runs over the entries of a SrcList; the entry's slot
// selects its workspace and coefficients.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_sources_to_soa(const ZD* __restrict__ canon, int which, int g5, Work<R> wk,
                                                           SrcList L, Geom g) {
    const int e = blockIdx.y, slot = L.slot[e];
    const ZD* in = canon + (size_t)L.src[e] * 12 * g.V;
    Z<R>* out = wk.f(slot, which);
    const int s = blockIdx.x * kBlock + threadIdx.x;
    double v[kNvRecur] = {0.0, 0.0, 0.0, 0.0};
    if (s < g.V) {
        double n2 = 0.0;
#pragma unroll
        for (int p = 0; p < 12; ++p) {
            const Z<R> zr = zcast<R>(((g5 && p >= 6) ? -1.0 : 1.0) * in[(size_t)s * 12 + p]);
            out[(size_t)p * g.ldv + s] = zr;
            n2 += (double)zr.re * zr.re + (double)zr.im * zr.im;
        }
        // |x|^2 laid out as (omega re, omega im, |r|^2, |s|^2) so that the first
        // Lanczos step normalises with beta_1 = gamma_1 = |x|.
        v[0] = n2;
        v[2] = n2;
        v[3] = n2;
    }
    if (which == 0) write_partials<kNvRecur, kBlock>(wk.p(slot, 1), v);
}

template <typename R>
void launch_sources_to_soa(const ZD* canon, int which, int g5, const Work<R>& wk, const SrcList& L, const Geom& g,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_sources_to_soa<R>, dim3(grid_for(g.V), L.n), dim3(kBlock), 0, st, canon, which, g5, wk, L,
                       g);
}

// =============================================================== forward Lanczos
// Step j: normalise the previous residuals (v_j = r/beta_j, w_j = s/conj(gamma_j)),
// apply a = H(mu) v_j and b = H(-mu) w_j = H^dag w_j with shared link loads, and
// emit per-block partial sums of alpha_j = w_j^H a, |a|^2 and eta^H v_j.  At
// j >= 2 the step first decides breakdown from the previous omega and norms.
// block_sum over a one-wavefront block without its barriers (0 + the wavefront's
// sum, as block_sum forms it), for a wavefront whose partner has left the block.
template <int NV>
__device__ __forceinline__ void wave_block_sum(double (&v)[NV]) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = 0.0 + wave_sum(v[i]);
}
template <int NV>
__device__ __forceinline__ void wave_partials_at(double* __restrict__ part, int slot, double (&v)[NV]) {
    wave_block_sum<NV>(v);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) part[slot * NV + i] = v[i];
}

// Epilogue of step j for one entry, after the hops: breakdown decisions from the
// block-summed previous (omega, |r|^2, |s|^2) in `red`, the coefficient records,
// the stores of v_j, w_j, a_j, b_j and the step's partial sums.  Every branch
// depends on block-uniform values only, so a block takes it as a whole.
// replay: the step's coefficients are the recorded beta_j, gamma_j, and nothing but
// the four fields is written (a runtime flag, so that a replayed step runs the
// very instructions of the original one).
template <typename R, int BLK>
__device__ __forceinline__ void fwd_pair_finish(const Geom& g, double kappa, const Work<R>& wk, const Coef& coef,
                                                int slot, int j, int pslot, int a, int s,
                                                const double (&red)[kNvRecur], const Z<R> (&acca)[4],
                                                const Z<R> (&accb)[4], const Z<R>* __restrict__ rin,
                                                const Z<R>* __restrict__ sin, int has_eta, int replay) {
    const int first = j == 1;
    double beta;
    ZD gam;
    if (replay) {
        beta = coef.beta[j];
        gam = coef.gamma[j];
    } else {
    const ZD om = mk<double>(red[0], red[1]);
    const double rn2 = red[2], sn2 = red[3];
    const double aom = std::sqrt(norm2(om));
    if (first && !(rn2 > 0.0 && std::isfinite(rn2))) {   // zero (or non-finite) source
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            coef.status[1] = 0;
            coef.status[2] = rn2 == 0.0 ? 1 : 3;   // 1: empty Krylov space, nothing to do; 3: not finite
            coef.status[3] = 1;
            coef.misc[0] = 0.0;
            *(volatile int*)coef.status = 1;
        }
        return;
    }
    if (!first) {
        const double an2 = coef.anorm2[j - 1];
        const bool lucky = rn2 <= kTauLucky * kTauLucky * an2;
        const bool finite = std::isfinite(om.re) && std::isfinite(om.im);
        const bool serious = !lucky && (!finite || aom <= kTauSerious * std::sqrt(rn2 * sn2));
        if (lucky || serious) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                coef.status[1] = j - 1;
                coef.status[2] = lucky ? 1 : 2;
                coef.status[3] = j;
                *(volatile int*)coef.status = 1;
            }
            return;
        }
    }
    beta = std::sqrt(aom);
    gam = (1.0 / beta) * om;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        coef.beta[j] = beta;
        coef.gamma[j] = gam;
        if (first) coef.misc[0] = beta;
    }
    }
    const R ib = (R)(1.0 / beta);
    const Z<R> icg = zcast<R>(zdiv(mk<double>(1.0, 0.0), cj(gam)));
    double pv[kNvPair] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (s < g.V) {
        Z<R> r0[4], s0[4], v[4], w[4], av[4], bv[4];
        load1(r0, rin, g.ldv, a, s);
        load1(s0, sin, g.ldv, a, s);
        const R kap = (R)kappa;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
            const R sg = sp < 2 ? R(1) : R(-1);
            v[sp] = ib * r0[sp];
            w[sp] = icg * s0[sp];
            av[sp] = (sg * ib) * (r0[sp] - kap * acca[sp]);
            bv[sp] = icg * (sg * (s0[sp] - kap * accb[sp]));
            const ZD wd = zcast<double>(w[sp]), ad = zcast<double>(av[sp]);
            const ZD wa = cjmul(wd, ad);
            pv[0] += wa.re;
            pv[1] += wa.im;
            pv[2] += norm2(ad);
        }
        store1_nt(wk.v(slot, j), g.ldv, a, s, v);
        store1_nt(wk.w(slot, j), g.ldv, a, s, w);
        store1_nt(wk.a(slot, j), g.ldv, a, s, av);
        store1_nt(wk.b(slot, j), g.ldv, a, s, bv);
        if (!replay && has_eta) {
            Z<R> e[4];
            load1_nt(e, wk.f(slot, 1), g.ldv, a, s);
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                const ZD ev = cjmul(zcast<double>(e[sp]), zcast<double>(v[sp]));
                pv[3] += ev.re;
                pv[4] += ev.im;
            }
        }
    }
    if (!replay) write_partials_at<kNvPair, BLK>(wk.p(slot, 0), pslot, pv);
}

// fwd_pair_finish on own-site operands loaded beforehand (r0 = r, s0 = s, e = eta at
// colour a), for the colour-grid kernel: its wavefront 0 runs it alone, so the sums
// are formed without barriers.
template <typename R>
__device__ __forceinline__ void fwd_pair_finish_pre(const Geom& g, double kappa, const Work<R>& wk, const Coef& coef,
                                                    int slot, int j, int pslot, int a, int s,
                                                    const double (&red)[kNvRecur], const Z<R> (&acca)[4],
                                                    const Z<R> (&accb)[4], const Z<R> (&r0)[4],
                                                    const Z<R> (&s0)[4], const Z<R> (&e)[4], int has_eta,
                                                    int replay) {
    const int first = j == 1;
    double beta;
    ZD gam;
    if (replay) {
        beta = coef.beta[j];
        gam = coef.gamma[j];
    } else {
    const ZD om = mk<double>(red[0], red[1]);
    const double rn2 = red[2], sn2 = red[3];
    const double aom = std::sqrt(norm2(om));
    if (first && !(rn2 > 0.0 && std::isfinite(rn2))) {   // zero (or non-finite) source
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            coef.status[1] = 0;
            coef.status[2] = rn2 == 0.0 ? 1 : 3;   // 1: empty Krylov space, nothing to do; 3: not finite
            coef.status[3] = 1;
            coef.misc[0] = 0.0;
            *(volatile int*)coef.status = 1;
        }
        return;
    }
    if (!first) {
        const double an2 = coef.anorm2[j - 1];
        const bool lucky = rn2 <= kTauLucky * kTauLucky * an2;
        const bool finite = std::isfinite(om.re) && std::isfinite(om.im);
        const bool serious = !lucky && (!finite || aom <= kTauSerious * std::sqrt(rn2 * sn2));
        if (lucky || serious) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                coef.status[1] = j - 1;
                coef.status[2] = lucky ? 1 : 2;
                coef.status[3] = j;
                *(volatile int*)coef.status = 1;
            }
            return;
        }
    }
    beta = std::sqrt(aom);
    gam = (1.0 / beta) * om;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        coef.beta[j] = beta;
        coef.gamma[j] = gam;
        if (first) coef.misc[0] = beta;
    }
    }
    const R ib = (R)(1.0 / beta);
    const Z<R> icg = zcast<R>(zdiv(mk<double>(1.0, 0.0), cj(gam)));
    double pv[kNvPair] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (s < g.V) {
        Z<R> v[4], w[4], av[4], bv[4];
        const R kap = (R)kappa;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
            const R sg = sp < 2 ? R(1) : R(-1);
            v[sp] = ib * r0[sp];
            w[sp] = icg * s0[sp];
            av[sp] = (sg * ib) * (r0[sp] - kap * acca[sp]);
            bv[sp] = icg * (sg * (s0[sp] - kap * accb[sp]));
            const ZD wd = zcast<double>(w[sp]), ad = zcast<double>(av[sp]);
            const ZD wa = cjmul(wd, ad);
            pv[0] += wa.re;
            pv[1] += wa.im;
            pv[2] += norm2(ad);
        }
        store1_nt(wk.v(slot, j), g.ldv, a, s, v);
        store1_nt(wk.w(slot, j), g.ldv, a, s, w);
        store1_nt(wk.a(slot, j), g.ldv, a, s, av);
        store1_nt(wk.b(slot, j), g.ldv, a, s, bv);
        if (!replay && has_eta) {
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                const ZD ev = cjmul(zcast<double>(e[sp]), zcast<double>(v[sp]));
                pv[3] += ev.re;
                pv[4] += ev.im;
            }
        }
    }
    if (!replay) wave_partials_at<kNvPair>(wk.p(slot, 0), pslot, pv);
}

// Step j: normalise the previous residuals (v_j = r/beta_j, w_j = s/conj(gamma_j)),
// apply a = H(mu) v_j and b = H(-mu) w_j = H^dag w_j with shared link loads, and
// emit per-block partial sums of alpha_j = w_j^H a, |a|^2 and eta^H v_j.  At
// j >= 2 the step first decides breakdown from the previous omega and norms.
// Colour grid: one entry per workgroup (grid.y = entry), three wavefronts per
// workgroup (kRBlock).  Wavefronts 1 and 2 apply directions 0, 1 and 2, 3 (one
// memory round trip each) and hand their sums over through LDS.  Wavefront 0
// meanwhile gathers the previous step's partial sums, reads the stop flag and loads
// the epilogue's own-site operands; after the one barrier it adds the halves
// (directions 0, 1 first) and runs the epilogue.  The hops do not depend on the sums
// or the flag (normalisation and breakdown act in the epilogue): a stopped entry's
// hops are discarded.
template <typename R, typename RL>
__global__ __launch_bounds__(kRBlock) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_fwd_pair(const Z<RL>* __restrict__ U, Geom g, double kappa, double emu, Work<R> wk, SrcList L, Coef coef0,
                int j, int npart_in, int has_eta, int replay) {
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kSites);
    const int slot = L.slot[blockIdx.y];
    const int first = j == 1;
    const Z<R>* rin = wk.f(slot, first ? 0 : 2);
    const Z<R>* sin = wk.f(slot, first ? 0 : 3);
    const int ncb = gridDim.x / 3;   // colour-major grid, as sten_block / sten_colour for the colour grid
    const int sb = blockIdx.x % ncb, a = blockIdx.x / ncb;
    const int l = threadIdx.x % kSites;
    const int s = sb * kSites + l;
    __shared__ Z<R> xa[2][4][kSites], xb[2][4][kSites];
    if (wv > 0) {
        Z<R> acca[4], accb[4];
        zero1(acca);
        zero1(accb);
        if (s < g.V) {
            hop_half_pair(acca, accb, U, rin, sin, g, s, a, neighbours(g, s), (R)emu, (R)(1.0 / emu), wv - 1);
            mem_fence_compiler();
        }
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
            xa[wv - 1][sp][l] = acca[sp];
            xb[wv - 1][sp][l] = accb[sp];
        }
        __syncthreads();
        return;
    }
    const Coef coef = coef0.at(slot);
    double red[kNvRecur] = {0.0, 0.0, 0.0, 0.0};
    if (!replay) gather_partials<kNvRecur, kSites>(wk.p(slot, 1), npart_in, red);
    // one load for the whole wavefront: every lane sees the same flag
    const int stop = replay ? 0 : __builtin_amdgcn_readfirstlane(*(volatile const int*)coef.status);
    Z<R> r0[4], s0[4], e[4];
    if (s < g.V) {
        load1(r0, rin, g.ldv, a, s);
        load1(s0, sin, g.ldv, a, s);
        if (!replay && has_eta) load1(e, wk.f(slot, 1), g.ldv, a, s);
    }
    if (!replay) wave_block_sum<kNvRecur>(red);
    __syncthreads();
    if (stop) return;
    Z<R> acca[4], accb[4];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
        acca[sp] = xa[0][sp][l] + xa[1][sp][l];
        accb[sp] = xb[0][sp][l] + xb[1][sp][l];
    }
    fwd_pair_finish_pre<R>(g, kappa, wk, coef, slot, j, (int)blockIdx.x, a, s, red, acca, accb, r0, s0, e, has_eta,
                           replay);
}

// Colour split: NS entries per workgroup (entries NS*blockIdx.y + q), which share
// every link load; the partial-sum slot is the site block.
template <typename R, int NS, typename RL>
__global__ __launch_bounds__(kCBlock) void k_fwd_pair_ms(const Z<RL>* __restrict__ U, Geom g, double kappa,
                                                         double emu, Work<R> wk, SrcList L, Coef coef0, int j,
                                                         int npart_in, int has_eta, int replay_arg) {
    const int replay = NS == 1 ? replay_arg : 0;   // regeneration runs one entry per workgroup
    const int e0 = (int)blockIdx.y * NS;
    const int first = j == 1;
    int slot[NS];
    const Z<R>* rin[NS];
    const Z<R>* sin[NS];
    double red[NS][kNvRecur];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        slot[q] = L.slot[min(e0 + q, L.n - 1)];
        rin[q] = wk.f(slot[q], first ? 0 : 2);
        sin[q] = wk.f(slot[q], first ? 0 : 3);
#pragma unroll
        for (int i = 0; i < kNvRecur; ++i) red[q][i] = 0.0;
        if (!replay) gather_partials<kNvRecur, kCBlock>(wk.p(slot[q], 1), npart_in, red[q]);
    }
    const int sb = sten_block<kCBlock>(g);
    if (sb < 0) return;   // padding workgroup (uniform over the block)
    unsigned live = 0;
    if (replay) {
#pragma unroll
        for (int q = 0; q < NS; ++q)
            if (e0 + q < L.n) live |= 1u << q;
    } else {
        live = block_live<NS>(coef0, L, e0);
    }
    if (!live) return;
    const int a = sten_colour<kCBlock>();
    const int s = sb * kSites + threadIdx.x % kSites;
    Z<R> acca[NS][4], accb[NS][4];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        zero1(acca[q]);
        zero1(accb[q]);
    }
    __shared__ HopX<R> x[NS];
    hop_all_pair_x<NS>(acca, accb, U, rin, sin, live, g, s, a, (R)emu, (R)(1.0 / emu), x);
    mem_fence_compiler();
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        if (live & (1u << q)) {
            if (!replay) block_sum<kNvRecur, kCBlock>(red[q]);
            fwd_pair_finish<R, kCBlock>(g, kappa, wk, coef0.at(slot[q]), slot[q], j, sb, a, s, red[q], acca[q],
                                        accb[q], rin[q], sin[q], has_eta, replay);
        }
    }
}

template <typename R, typename RL>
void fwd_pair_launch(const Z<RL>* U, const Geom& g, double kappa, double mu, const Work<R>& wk, const SrcList& L,
                     Coef coef, int j, int has_eta, int ns, int replay, hipStream_t st, Timing t) {
    const int npart_in = j == 1 ? grid_for(g.V) : np_point(g.V);
    const double emu = std::exp(mu);
    if (colour_grid(g.V)) {
        timed_launch(k_fwd_pair<R, RL>, dim3(np_colour(g.V), L.n), dim3(kRBlock), st, t, U, g, kappa, emu, wk,
                     L, coef, j, npart_in, has_eta, replay);
        return;
    }
    const dim3 block(kCBlock);
    switch (ns) {
        case 4:
            timed_launch(k_fwd_pair_ms<R, 4, RL>, dim3(g.nwg, (L.n + 3) / 4), block, st, t, U, g, kappa, emu, wk, L, coef,
                         j, npart_in, has_eta, replay);
            break;
        case 2:
            timed_launch(k_fwd_pair_ms<R, 2, RL>, dim3(g.nwg, (L.n + 1) / 2), block, st, t, U, g, kappa, emu, wk, L, coef,
                         j, npart_in, has_eta, replay);
            break;
        default:
            timed_launch(k_fwd_pair_ms<R, 1, RL>, dim3(g.nwg, L.n), block, st, t, U, g, kappa, emu, wk, L, coef, j,
                         npart_in, has_eta, replay);
    }
}

template <typename R, typename RL>
void launch_fwd_pair(const Z<RL>* U, const Geom& g, double kappa, double mu, const Work<R>& wk, const SrcList& L,
                     Coef coef, int j, int has_eta, int ns, hipStream_t st, Timing t) {
    fwd_pair_launch<R>(U, g, kappa, mu, wk, L, coef, j, has_eta, ns, 0, st, t);
}

// Replay of step j for regeneration: the step's own kernel with the replay flag,
// one entry per workgroup (the shape a single-source step runs with).
template <typename R, typename RL>
void launch_fwd_replay(const Z<RL>* U, const Geom& g, double kappa, double mu, const Work<R>& wk, const SrcList& L,
                       Coef coef, int j, hipStream_t st) {
    fwd_pair_launch<R>(U, g, kappa, mu, wk, L, coef, j, 0, 1, 1, st, Timing{});
}

// r = a - alpha_j v_j - gamma_j v_{j-1},  s = b - conj(alpha_j) w_j - beta_j w_{j-1},
// with per-block partials of omega = s^H r, |r|^2, |s|^2.  One thread per
// (plane, site): grid.y runs over the 12 spin-colour planes, grid.z over the
// entries.  At the entry's last step (j = k[e]) only alpha_j is recorded.
template <typename R>
__device__ __forceinline__ void recur_update(Z<R> a_i, Z<R> b_i, Z<R> v_i, Z<R> w_i, Z<R> vp_i, Z<R> wp_i, Z<R> al,
                                             Z<R> alc, Z<R> gj, R bj, bool has_prev, Z<R>& r, Z<R>& q) {
    r = a_i - al * v_i;
    q = b_i - alc * w_i;
    if (has_prev) {
        r = r - gj * vp_i;
        q = q - bj * wp_i;
    }
}

template <typename R>
__global__ __launch_bounds__(kPBlock) void k_recur(Geom g, Work<R> wk, SrcList L, Coef coef0, int j, int npart_in,
                                                   int replay) {
    const int e = blockIdx.z, slot = L.slot[e];
    const Coef coef = coef0.at(slot);
    const int s = blockIdx.x * kPBlock + threadIdx.x;
    const size_t i = (size_t)blockIdx.y * g.ldv + s;
    const bool has_prev = j > 1, live = s < g.V && j < L.k[e];
    // the site's operands, the step's scalars and the partial sums first: their
    // loads share one round trip with the flag read (a compiler fence keeps them
    // ahead of the flag test)
    const Z<R> gj = has_prev ? zcast<R>(coef.gamma[j]) : mk<R>(0, 0);
    const R bj = has_prev ? (R)coef.beta[j] : R(0);
    Z<R> a_i = mk<R>(0, 0), b_i = a_i, v_i = a_i, w_i = a_i, vp_i = a_i, wp_i = a_i;
    if (live) {
        a_i = wk.a(slot, j)[i];
        b_i = wk.b(slot, j)[i];
        v_i = wk.v(slot, j)[i];
        w_i = wk.w(slot, j)[i];
        if (has_prev) {
            vp_i = wk.v(slot, j - 1)[i];
            wp_i = wk.w(slot, j - 1)[i];
        }
    }
    double red[kNvPair] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (!replay) gather_partials<kNvPair, kPBlock>(wk.p(slot, 0), npart_in, red);
    mem_fence_compiler();
    // the flag is written by the forward pair only, never during this launch, so a
    // read per wavefront is uniform over the block
    if (!replay && __builtin_amdgcn_readfirstlane(*(volatile const int*)coef.status)) return;
    ZD alpha;
    if (replay) {   // regeneration: alpha_j as recorded, nothing written but r and s
        alpha = coef.alpha[j];
    } else {
        block_sum_last<kNvPair, kPBlock>(red);
        alpha = mk<double>(red[0], red[1]);
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
            coef.alpha[j] = alpha;
            coef.anorm2[j] = red[2];
            coef.h[j] = mk<double>(red[3], red[4]);
        }
    }
    if (j >= L.k[e]) return;
    const Z<R> al = zcast<R>(alpha), alc = zcast<R>(cj(alpha));
    double pv[kNvRecur] = {0.0, 0.0, 0.0, 0.0};
    if (live) {
        Z<R> r, q;
        recur_update(a_i, b_i, v_i, w_i, vp_i, wp_i, al, alc, gj, bj, has_prev, r, q);
        wk.f(slot, 2)[i] = r;
        wk.f(slot, 3)[i] = q;
        const double rr = r.re, ri = r.im, qr = q.re, qi = q.im;
        pv[0] = qr * rr + qi * ri;
        pv[1] = qr * ri - qi * rr;
        pv[2] = rr * rr + ri * ri;
        pv[3] = qr * qr + qi * qi;
    }
    if (!replay) write_partials_at_last<kNvRecur, kPBlock>(wk.p(slot, 1), blockIdx.y * gridDim.x + blockIdx.x, pv);
}

template <typename R>
void launch_recur(const Geom& g, const Work<R>& wk, const SrcList& L, Coef coef, int j, hipStream_t st) {
    dim3 grid((g.V + kPBlock - 1) / kPBlock, 12, L.n);
    hipLaunchKernelGGL(k_recur<R>, grid, dim3(kPBlock), 0, st, g, wk, L, coef, j, np_sten(g.V), 0);
}

template <typename R>
void launch_recur_replay(const Geom& g, const Work<R>& wk, const SrcList& L, Coef coef, int j, hipStream_t st) {
    dim3 grid((g.V + kPBlock - 1) / kPBlock, 12, L.n);
    hipLaunchKernelGGL(k_recur<R>, grid, dim3(kPBlock), 0, st, g, wk, L, coef, j, np_sten(g.V), 1);
}

// out(s) = [psi(s) +] g5^{overlap} |x| sum_{j <= k_used} c_j v_j(s), canonical layout;
// with j1 > 0 the sum runs over j0..min(j1, k_used) and adds to out below the
// entry's top segment (see launch_assemble).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_assemble(Geom g, Work<R> wk, SrcList L, Coef coef0,
                                                     const ZD* __restrict__ psi_base, int overlap,
                                                     ZD* __restrict__ out_base, int j0, int j1) {
    const int e = blockIdx.y, slot = L.slot[e];
    const Coef coef = coef0.at(slot);
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const size_t co = (size_t)L.src[e] * 12 * g.V;
    const int k = coef.status[1];
    const int jlast = j1 > 0 ? min(j1, k) : k;
    const bool add = j1 > 0 && k > j1;
    const double nx = coef.misc[0];
    ZD acc[12];
#pragma unroll
    for (int p = 0; p < 12; ++p) acc[p] = mk<double>(0, 0);
    for (int j = j0; j <= jlast; ++j) {
        const ZD c = coef.c[j];
        const Z<R>* f = wk.v(slot, j);
#pragma unroll
        for (int p = 0; p < 12; ++p) acc[p] = acc[p] + c * zcast<double>(f[(size_t)p * g.ldv + s]);
    }
#pragma unroll
    for (int p = 0; p < 12; ++p) {
        const double sg = (overlap && p >= 6) ? -nx : nx;
        ZD o = sg * acc[p];
        const size_t i = co + (size_t)s * 12 + p;
        if (add) o = o + out_base[i];
        else if (overlap) o = o + psi_base[i];
        out_base[i] = o;
    }
}

template <typename R>
void launch_assemble(const Geom& g, const Work<R>& wk, const SrcList& L, Coef coef, const ZD* psi_canon,
                     int overlap, ZD* out, hipStream_t st, int j0, int j1) {
    hipLaunchKernelGGL(k_assemble<R>, dim3(grid_for(g.V), L.n), dim3(kBlock), 0, st, g, wk, L, coef, psi_canon,
                       overlap, out, j0, j1);
}

// =============================================================== backward (reverse mode)
// Reverse of the normalisation and of omega = s^H r for step j < k_used:
// from vbar_{j+1}, wbar_{j+1} and the beta/gamma adjoints form
//   omegabar = gbar/beta + [bbar - Re(conj(gbar) omega)/beta^2] omega / (2 beta^3),
//   rbar_j = vbar_{j+1}/beta + omegabar conj(gamma) w_{j+1},
//   sbar_j = wbar_{j+1}/gamma + conj(omegabar) beta v_{j+1},
// and partials P1 = v_j^H rbar, P2 = sbar^H w_j, P3 = v_{j-1}^H rbar, P4 = w_{j-1}^H sbar.
template <typename R>
__global__ __launch_bounds__(kPBlock) void k_bwd_ra(Geom g, Work<R> wk, SrcList L, Coef coef0, int j, int npart_in) {
    const int e = blockIdx.z, slot = L.slot[e];
    const Coef coef = coef0.at(slot);
    const int s = blockIdx.x * kPBlock + threadIdx.x;
    const size_t i = (size_t)blockIdx.y * g.ldv + s;
    const bool has_prev = j > 1, live = s < g.V;
    // the site's operands first: their loads overlap the partial-sum reads below
    Z<R> vb_i = mk<R>(0, 0), wb_i = vb_i, vn_i = vb_i, wn_i = vb_i, vj_i = vb_i, wj_i = vb_i, vp_i = vb_i,
         wp_i = vb_i;
    if (live) {
        vb_i = wk.f(slot, 4)[i];
        wb_i = wk.f(slot, 5)[i];
        vn_i = wk.v(slot, j + 1)[i];
        wn_i = wk.w(slot, j + 1)[i];
        vj_i = wk.v(slot, j)[i];
        wj_i = wk.w(slot, j)[i];
        if (has_prev) {
            vp_i = wk.v(slot, j - 1)[i];
            wp_i = wk.w(slot, j - 1)[i];
        }
    }
    const double beta = coef.beta[j + 1];
    const ZD gam = coef.gamma[j + 1];
    const double bbar_n = coef.bbar_tot[j + 1];
    const ZD gbar_n = coef.gbar_tot[j + 1];
    double red[kNvRB];
    gather_partials<kNvRB, kPBlock>(wk.p(slot, 0), npart_in, red);   // its loads join the operands'
    block_sum_last<kNvRB, kPBlock>(red);
    const double D1 = red[0];
    const ZD D2 = mk<double>(red[1], red[2]);
    const ZD om = beta * gam;
    const double bbarR = bbar_n - D1 / beta;
    const ZD gbar = gbar_n - zdiv(D2, cj(gam));
    const ZD cgo = cjmul(gbar, om);   // conj(gbar) * omega
    const double K = (bbarR - cgo.re / (beta * beta)) / (2.0 * beta * beta * beta);
    const ZD ombar = (1.0 / beta) * gbar + K * om;
    const R c1 = (R)(1.0 / beta);
    const Z<R> c2 = zcast<R>(mulcj(ombar, gam));                 // omegabar conj(gamma)
    const Z<R> c3 = zcast<R>(zdiv(mk<double>(1.0, 0.0), gam));   // 1/gamma
    const Z<R> c4 = zcast<R>(beta * cj(ombar));                  // conj(omegabar) beta
    double pv[kNvRA] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (live) {
        const Z<R> r = c1 * vb_i + c2 * wn_i;
        const Z<R> q = c3 * wb_i + c4 * vn_i;
        wk.f(slot, 6 + (j & 1))[i] = r;
        wk.sb(slot, j)[i] = q;
        const ZD rd = zcast<double>(r), qd = zcast<double>(q);
        const ZD p1 = cjmul(zcast<double>(vj_i), rd);
        const ZD p2 = cjmul(qd, zcast<double>(wj_i));
        pv[0] = p1.re; pv[1] = p1.im;
        pv[2] = p2.re; pv[3] = p2.im;
        if (has_prev) {
            const ZD p3 = cjmul(zcast<double>(vp_i), rd);
            const ZD p4 = cjmul(zcast<double>(wp_i), qd);
            pv[4] = p3.re; pv[5] = p3.im;
            pv[6] = p4.re; pv[7] = p4.im;
        }
    }
    write_partials_at_last<kNvRA, kPBlock>(wk.p(slot, 1), blockIdx.y * gridDim.x + blockIdx.x, pv);
}

template <typename R>
void launch_bwd_ra(const Geom& g, const Work<R>& wk, const SrcList& L, Coef coef, int j, hipStream_t st) {
    dim3 grid((g.V + kPBlock - 1) / kPBlock, 12, L.n);
    hipLaunchKernelGGL(k_bwd_ra<R>, grid, dim3(kPBlock), 0, st, g, wk, L, coef, j, np_sten(g.V));
}

// Reverse of a_j = H v_j, b_j = H^dag w_j, alpha_j = w_j^H a_j and of the recurrence:
//   alphabar_j = conj(Gamma_jj) - v_j^H rbar_j - sbar_j^H w_j,   abar_j = rbar_j + alphabar_j w_j,
//   vbar_j = |x| conj(c_j) eta + H^dag rbar_j + alphabar_j b_j - conj(alpha_j) rbar_j - conj(gamma_{j+1}) rbar_{j+1},
//   wbar_j = H sbar_j + conj(alphabar_j) a_j - alpha_j sbar_j - beta_{j+1} sbar_{j+1},
// using the forward pass's a_j and b_j = H^dag w_j, so the stencil acts on rbar_j
// (at -mu) and sbar_j (at +mu) only.  Stores abar_j for the force and emits
// partials of Re vbar_j^H v_j and wbar_j^H w_j.  The last step (j = k_used) has
// no residual adjoints: abar = alphabar w, vbar = |x| conj(c) eta + alphabar b,
// wbar = conj(alphabar) a.
// The recorded scalars of reverse step j, read at the top of the kernel so that
// their loads share a round trip with the hops' instead of following the block sum.
struct BwdCoefs {
    ZD abar_T, gbar_T, alpha, etac, gnc;
    double bbar_T, bn;
};
__device__ __forceinline__ BwdCoefs bwd_coefs(const Coef& coef, int j, bool carry) {
    BwdCoefs c;
    c.abar_T = coef.abar_T[j];
    c.gbar_T = coef.gbar_T[j];
    c.bbar_T = coef.bbar_T[j];
    c.alpha = coef.alpha[j];
    c.etac = coef.misc[0] * cj(coef.c[j]);
    c.gnc = carry ? cj(coef.gamma[j + 1]) : mk<double>(0, 0);
    c.bn = carry ? coef.beta[j + 1] : 0.0;
    return c;
}

// Epilogue of reverse step j for one entry, after the hops: the coefficient
// adjoints from the block-summed partials `red` (not LAST), the adjoint fields'
// stores and the step's partial sums.
// The epilogue's own-site operands (colour a, four spins), loaded by bwd_rb_load.
template <typename R>
struct BwdRbIn {
    Z<R> w[4], v[4], a[4], b[4], e[4], r[4], sb[4], rn[4], sn[4];
};

template <typename R>
__device__ __forceinline__ void bwd_rb_load(const Geom& g, const Work<R>& wk, int slot, int j, int k_used, int a,
                                            int s, BwdRbIn<R>& in) {
    const bool carry = j + 1 < k_used;
    const FieldBase rw = field_base(wk.w(slot, j)), rv = field_base(wk.v(slot, j)), ra = field_base(wk.a(slot, j)),
                    rb = field_base(wk.b(slot, j)), re = field_base(wk.f(slot, 1));
    const FieldBase rr = field_base(wk.f(slot, 6 + (j & 1))), rs = field_base(wk.sb(slot, j));
    const FieldBase rrn = field_base(wk.f(slot, 6 + ((j + 1) & 1))), rsn = field_base(carry ? wk.sb(slot, j + 1)
                                                                                          : wk.sb(slot, j));
    const unsigned i = (unsigned)s;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
        const int pl = sp * 3 + a;
        in.w[sp] = fload<R>(rw, g.ldv, pl, i);
        in.v[sp] = fload<R>(rv, g.ldv, pl, i);
        in.a[sp] = fload<R>(ra, g.ldv, pl, i);
        in.b[sp] = fload<R>(rb, g.ldv, pl, i);
        in.e[sp] = fload<R>(re, g.ldv, pl, i);
        {
            in.r[sp] = fload<R>(rr, g.ldv, pl, i);
            in.sb[sp] = fload<R>(rs, g.ldv, pl, i);
            if (carry) {
                in.rn[sp] = fload<R>(rrn, g.ldv, pl, i);
                in.sn[sp] = fload<R>(rsn, g.ldv, pl, i);
            }
        }
    }
}

// The epilogue of bwd_rb_finish (not the last step) on operands loaded beforehand, for
// the colour-grid kernel: its wavefront 0 runs it alone, so the sums are formed
// without barriers.
template <typename R>
__device__ __forceinline__ void bwd_rb_finish_pre(const Geom& g, double kappa, const Work<R>& wk, const Coef& coef,
                                                  int slot, int j, int k_used, int pslot, int a, int s,
                                                  const double (&red)[kNvRA], const Z<R> (&accs)[4],
                                                  const Z<R> (&accr)[4], const BwdCoefs& cf, const BwdRbIn<R>& in) {
    constexpr bool LAST = false;
    const bool carry = j + 1 < k_used;
    ZD abar = cf.abar_T;
    if (!LAST) {
        abar = abar - mk<double>(red[0], red[1]) - mk<double>(red[2], red[3]);
        if (blockIdx.x == 0 && threadIdx.x == 0 && j >= 2) {
            coef.gbar_tot[j] = cf.gbar_T - mk<double>(red[4], red[5]);
            coef.bbar_tot[j] = cf.bbar_T - red[6];
        }
    }
    const Z<R> ca = zcast<R>(abar);
    const ZD alpha = cf.alpha;
    const Z<R> alr = zcast<R>(alpha), alc = zcast<R>(cj(alpha)), abc = zcast<R>(cj(abar));
    const Z<R> etac = zcast<R>(cf.etac);
    const Z<R> gnc = zcast<R>(cf.gnc);
    const R bn = (R)cf.bn;
    double pv[kNvRB] = {0.0, 0.0, 0.0};
    if (s < g.V) {
        const R kap = (R)kappa;
        Z<R> vbo[4], wbo[4], abo[4];
        double d1 = 0.0, d2r = 0.0, d2i = 0.0;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
            const R sg = sp < 2 ? R(1) : R(-1);
            const Z<R> w_s = in.w[sp];
            const Z<R> v_s = in.v[sp];
            const Z<R> a_s = in.a[sp];
            const Z<R> b_s = in.b[sp];
            Z<R> vb = etac * in.e[sp] + ca * b_s;
            Z<R> wb = abc * a_s;
            Z<R> ab_s = ca * w_s;
            if (!LAST) {
                const Z<R> r_s = in.r[sp];
                const Z<R> sb_s = in.sb[sp];
                ab_s = ab_s + r_s;
                vb = vb + sg * (r_s - kap * accr[sp]) - alc * r_s;
                wb = wb + sg * (sb_s - kap * accs[sp]) - alr * sb_s;
                if (carry) {
                    vb = vb - gnc * in.rn[sp];
                    wb = wb - bn * in.sn[sp];
                }
            }
            vbo[sp] = vb;
            wbo[sp] = wb;
            abo[sp] = ab_s;
            const ZD x1 = cjmul(zcast<double>(vb), zcast<double>(v_s));
            const ZD x2 = cjmul(zcast<double>(wb), zcast<double>(w_s));
            d1 += x1.re;
            d2r += x2.re;
            d2i += x2.im;
        }
        store1_nt(wk.f(slot, 4), g.ldv, a, s, vbo);
        store1_nt(wk.f(slot, 5), g.ldv, a, s, wbo);
        store1_nt(wk.ab(slot, j), g.ldv, a, s, abo);
        pv[0] = d1;
        pv[1] = d2r;
        pv[2] = d2i;
    }
    wave_partials_at<kNvRB>(wk.p(slot, 0), pslot, pv);
}

template <typename R, bool LAST, int BLK>
__device__ __forceinline__ void bwd_rb_finish(const Geom& g, double kappa, const Work<R>& wk, const Coef& coef,
                                              int slot, int j, int k_used, int pslot, int a, int s,
                                              const double (&red)[kNvRA], const Z<R> (&accs)[4],
                                              const Z<R> (&accr)[4], const BwdCoefs& cf) {
    const Z<R>* __restrict__ rbar_j = wk.f(slot, 6 + (j & 1));
    const Z<R>* __restrict__ rbar_n = wk.f(slot, 6 + ((j + 1) & 1));
    const Z<R>* __restrict__ sbar_j = wk.sb(slot, j);
    const bool carry = j + 1 < k_used;
    const Z<R>* __restrict__ sbar_n = carry ? wk.sb(slot, j + 1) : sbar_j;
    ZD abar = cf.abar_T;
    if (!LAST) {
        abar = abar - mk<double>(red[0], red[1]) - mk<double>(red[2], red[3]);
        if (blockIdx.x == 0 && threadIdx.x == 0 && j >= 2) {
            coef.gbar_tot[j] = cf.gbar_T - mk<double>(red[4], red[5]);
            coef.bbar_tot[j] = cf.bbar_T - red[6];
        }
    }
    const Z<R> ca = zcast<R>(abar);
    const ZD alpha = cf.alpha;
    const Z<R> alr = zcast<R>(alpha), alc = zcast<R>(cj(alpha)), abc = zcast<R>(cj(abar));
    const Z<R> etac = zcast<R>(cf.etac);
    const Z<R> gnc = zcast<R>(cf.gnc);
    const R bn = (R)cf.bn;
    double pv[kNvRB] = {0.0, 0.0, 0.0};
    if (s < g.V) {
        const R kap = (R)kappa;
        const FieldBase rw = field_base(wk.w(slot, j)), rv = field_base(wk.v(slot, j)),
                     ra = field_base(wk.a(slot, j)), rb = field_base(wk.b(slot, j)),
                     re = field_base(wk.f(slot, 1));
        Z<R> vbo[4], wbo[4], abo[4];
        double d1 = 0.0, d2r = 0.0, d2i = 0.0;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
            const int pl = sp * 3 + a;
            const unsigned i = (unsigned)s;
            const R sg = sp < 2 ? R(1) : R(-1);
            const Z<R> w_s = fload_nt<R>(rw, g.ldv, pl, i);
            const Z<R> v_s = fload_nt<R>(rv, g.ldv, pl, i);
            const Z<R> a_s = fload_nt<R>(ra, g.ldv, pl, i);
            const Z<R> b_s = fload_nt<R>(rb, g.ldv, pl, i);
            Z<R> vb = etac * fload_nt<R>(re, g.ldv, pl, i) + ca * b_s;
            Z<R> wb = abc * a_s;
            Z<R> ab_s = ca * w_s;
            if (!LAST) {
                const Z<R> r_s = fload<R>(field_base(rbar_j), g.ldv, pl, i);
                const Z<R> sb_s = fload<R>(field_base(sbar_j), g.ldv, pl, i);
                ab_s = ab_s + r_s;
                vb = vb + sg * (r_s - kap * accr[sp]) - alc * r_s;
                wb = wb + sg * (sb_s - kap * accs[sp]) - alr * sb_s;
                if (carry) {
                    vb = vb - gnc * fload_nt<R>(field_base(rbar_n), g.ldv, pl, i);
                    wb = wb - bn * fload_nt<R>(field_base(sbar_n), g.ldv, pl, i);
                }
            }
            vbo[sp] = vb;
            wbo[sp] = wb;
            abo[sp] = ab_s;
            const ZD x1 = cjmul(zcast<double>(vb), zcast<double>(v_s));
            const ZD x2 = cjmul(zcast<double>(wb), zcast<double>(w_s));
            d1 += x1.re;
            d2r += x2.re;
            d2i += x2.im;
        }
        store1_nt(wk.f(slot, 4), g.ldv, a, s, vbo);
        store1_nt(wk.f(slot, 5), g.ldv, a, s, wbo);
        store1_nt(wk.ab(slot, j), g.ldv, a, s, abo);
        pv[0] = d1;
        pv[1] = d2r;
        pv[2] = d2i;
    }
    write_partials_at<kNvRB, BLK>(wk.p(slot, 0), pslot, pv);
}

// Reverse step j (one entry per workgroup, grid.y = entry):
//   vbar_j = |x| conj(c_j) eta + H^dag rbar_j + alphabar_j b_j - conj(alpha_j) rbar_j - conj(gamma_{j+1}) rbar_{j+1},
//   wbar_j = H sbar_j + conj(alphabar_j) a_j - alpha_j sbar_j - beta_{j+1} sbar_{j+1},
// using the forward pass's a_j and b_j = H^dag w_j, so the stencil acts on rbar_j
// (at -mu) and sbar_j (at +mu) only.  Stores abar_j for the force and emits
// partials of Re vbar_j^H v_j and wbar_j^H w_j.  The last step (j = k_used) has
// no residual adjoints: abar = alphabar w, vbar = |x| conj(c) eta + alphabar b,
// wbar = conj(alphabar) a.
template <typename R, bool LAST, int BLK, typename RL>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(1, 8)))
void k_bwd_rb(const Z<RL>* __restrict__ U, Geom g, double kappa, double emu,
                                                    Work<R> wk, SrcList L, Coef coef0, int j, int npart_in) {
    const int e = blockIdx.y, slot = L.slot[e];
    const Coef coef = coef0.at(slot);
    const int sb = sten_block<BLK>(g);
    if (sb < 0) return;   // padding workgroup (uniform over the block)
    const int a = sten_colour<BLK>();
    const int s = sb * kSites + threadIdx.x % kSites;
    const BwdCoefs cf = bwd_coefs(coef, j, j + 1 < L.k[e]);
    // the partial sums' loads go out with the hops' loads; only the epilogue needs
    // the sums, so they are combined after the hops
    double red[kNvRA];
    Z<R> accs[4], accr[4];   // field A = sbar_j at +mu, field B = rbar_j at -mu
    zero1(accs);
    zero1(accr);
    if (!LAST) {
        gather_partials<kNvRA, BLK>(wk.p(slot, 1), npart_in, red);
        if (s < g.V) {
            const Z<R>* fs = wk.sb(slot, j);
            const Z<R>* fr = wk.f(slot, 6 + (j & 1));
            const Nbr n = neighbours(g, s);
            hop_all_pair<BLK>(accs, accr, U, fs, fr, g, s, a, n, (R)emu, (R)(1.0 / emu));
            mem_fence_compiler();
        }
        block_sum<kNvRA, BLK>(red);
    }
    bwd_rb_finish<R, LAST, BLK>(g, kappa, wk, coef, slot, j, L.k[e], BLK == kSites ? (int)blockIdx.x : sb, a, s,
                                red, accs, accr, cf);
}

// Colour grid, not the last step: blocks of three wavefronts (kRBlock).  Wavefronts 1 and 2
// run the hops of directions 0, 1 and 2, 3, each pair in one memory round trip (up
// to 512 registers at one wavefront per SIMD), and hand their sums over through
// LDS.  Wavefront 0 meanwhile gathers the partial sums and loads the epilogue's nine
// own-site fields, so that round trip overlaps the hops; after the one barrier it
// adds the two halves (directions 0, 1 first) and runs the epilogue.
template <typename R, typename RL>
__global__ __launch_bounds__(kRBlock) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_bwd_rb_cg(const Z<RL>* __restrict__ U, Geom g, double kappa, double emu, Work<R> wk, SrcList L, Coef coef0,
                 int j, int npart_in) {
    const int e = blockIdx.y, slot = L.slot[e];
    const int ncb = gridDim.x / 3;   // colour-major grid, as sten_block / sten_colour for the colour grid
    const int sb = blockIdx.x % ncb, a = blockIdx.x / ncb;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kSites);
    const int l = threadIdx.x % kSites;
    const int s = sb * kSites + l;
    __shared__ Z<R> xs[2][4][kSites], xr[2][4][kSites];
    if (wv > 0) {
        Z<R> accs[4], accr[4];   // field A = sbar_j at +mu, field B = rbar_j at -mu
        zero1(accs);
        zero1(accr);
        if (s < g.V) {
            const Z<R>* fs = wk.sb(slot, j);
            const Z<R>* fr = wk.f(slot, 6 + (j & 1));
            const Nbr n = neighbours(g, s);
            if (wv == 1)
                hop_two_dirs_pair_eager<0, 1>(accs, accr, U, fs, fr, g, s, a, n, (R)emu, (R)(1.0 / emu));
            else
                hop_two_dirs_pair_eager<2, 3>(accs, accr, U, fs, fr, g, s, a, n, (R)emu, (R)(1.0 / emu));
            mem_fence_compiler();
        }
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
            xs[wv - 1][sp][l] = accs[sp];
            xr[wv - 1][sp][l] = accr[sp];
        }
        __syncthreads();
        return;
    }
    const Coef coef = coef0.at(slot);
    const BwdCoefs cf = bwd_coefs(coef, j, j + 1 < L.k[e]);
    double red[kNvRA];
    gather_partials<kNvRA, kSites>(wk.p(slot, 1), npart_in, red);
    BwdRbIn<R> in;
    if (s < g.V) bwd_rb_load<R>(g, wk, slot, j, L.k[e], a, s, in);
    wave_block_sum<kNvRA>(red);
    __syncthreads();
    Z<R> accs[4], accr[4];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
        accs[sp] = xs[0][sp][l] + xs[1][sp][l];
        accr[sp] = xr[0][sp][l] + xr[1][sp][l];
    }
    bwd_rb_finish_pre<R>(g, kappa, wk, coef, slot, j, L.k[e], (int)blockIdx.x, a, s, red, accs, accr, cf, in);
}

// Colour split, not the last step: NS entries per workgroup sharing the link loads.
template <typename R, int NS, typename RL>
__global__ __launch_bounds__(kCBlock) void k_bwd_rb_ms(const Z<RL>* __restrict__ U, Geom g, double kappa,
                                                       double emu, Work<R> wk, SrcList L, Coef coef0, int j,
                                                       int npart_in) {
    const int e0 = (int)blockIdx.y * NS;
    const int sb = sten_block<kCBlock>(g);
    if (sb < 0) return;   // padding workgroup (uniform over the block)
    unsigned live = 0;
    int slot[NS];
    const Z<R>* fs[NS];
    const Z<R>* fr[NS];
    double red[NS][kNvRA];
    BwdCoefs cf[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int e = min(e0 + q, L.n - 1);
        if (e0 + q < L.n) live |= 1u << q;
        slot[q] = L.slot[e];
        fs[q] = wk.sb(slot[q], j);
        fr[q] = wk.f(slot[q], 6 + (j & 1));
        cf[q] = bwd_coefs(coef0.at(slot[q]), j, j + 1 < L.k[e]);
        gather_partials<kNvRA, kCBlock>(wk.p(slot[q], 1), npart_in, red[q]);
    }
    const int a = sten_colour<kCBlock>();
    const int s = sb * kSites + threadIdx.x % kSites;
    Z<R> accs[NS][4], accr[NS][4];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        zero1(accs[q]);
        zero1(accr[q]);
    }
    __shared__ HopX<R> x[NS];
    hop_all_pair_x<NS>(accs, accr, U, fs, fr, live, g, s, a, (R)emu, (R)(1.0 / emu), x);
    mem_fence_compiler();
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        if (live & (1u << q)) {
            block_sum<kNvRA, kCBlock>(red[q]);
            bwd_rb_finish<R, false, kCBlock>(g, kappa, wk, coef0.at(slot[q]), slot[q], j, L.k[e0 + q], sb, a, s,
                                             red[q], accs[q], accr[q], cf[q]);
        }
    }
}

template <typename R, typename RL>
void launch_bwd_rb(const Z<RL>* U, const Geom& g, double kappa, double mu, const Work<R>& wk, const SrcList& L,
                   Coef coef, int j, int last, int ns, hipStream_t st, Timing t) {
    const int np = np_point(g.V);
    const bool cg = colour_grid(g.V);
    const double emu = std::exp(mu);
    const dim3 grid(cg ? np_colour(g.V) : g.nwg, L.n);
    if (last && cg)
        timed_launch(k_bwd_rb<R, true, kSites, RL>, grid, dim3(kSites), st, t, U, g, kappa, emu, wk, L, coef, j, np);
    else if (last)
        timed_launch(k_bwd_rb<R, true, kCBlock, RL>, grid, dim3(kCBlock), st, t, U, g, kappa, emu, wk, L, coef, j, np);
    else if (cg)
        timed_launch(k_bwd_rb_cg<R, RL>, grid, dim3(kRBlock), st, t, U, g, kappa, emu, wk, L, coef, j, np);
    else if (ns == 4)
        timed_launch(k_bwd_rb_ms<R, 4, RL>, dim3(g.nwg, (L.n + 3) / 4), dim3(kCBlock), st, t, U, g, kappa, emu, wk, L,
                     coef, j, np);
    else if (ns == 2)
        timed_launch(k_bwd_rb_ms<R, 2, RL>, dim3(g.nwg, (L.n + 1) / 2), dim3(kCBlock), st, t, U, g, kappa, emu, wk, L,
                     coef, j, np);
    else
        timed_launch(k_bwd_rb_ms<R, 1, RL>, dim3(g.nwg, L.n), dim3(kCBlock), st, t, U, g, kappa, emu, wk, L, coef, j, np);
}

// =============================================================== force contraction
// dS = sum_j Re(abar_j^H dH v_j) + Re(w_j^H dH sbar_j) with H = g5 D_w(mu).
// For the link U_nu(x) and a pair (p, q) the coefficient of dU is
//   G_ab += -kappa sum_{s=0,1} [ e_f hP[s][a] conj(hQ[s][b]) + e_b hQ2[s][a] conj(hP2[s][b]) ]
// with hP = P+(g5 p(x)), hQ = P+(q(x+nu)), hP2 = P-(g5 p(x+nu)), hQ2 = P-(q(x)) the
// half spinors of the (1 +- g_nu) projectors, e_f = e^{+mu}, e_b = e^{-mu} for nu = t.
template <int NU, typename R>
__device__ void force_body(const Geom& g, double kappa, double emu, const Work<R>& wk, int slot, int k, int j0,
                           int j1, int s, ZD* __restrict__ gout, int accumulate) {
    const Nbr n = neighbours(g, s);
    const int y = n.fwd[NU];
    const double ef = (NU == 3) ? emu : 1.0, eb = (NU == 3) ? 1.0 / emu : 1.0;
    ZD G[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) G[a][b] = mk<double>(0, 0);
    for (int j = j0; j < j1; ++j) {
        Spinor<R> px, qx, py, qy;
        load_spinor(px, wk.ab(slot, j), g.ldv, s);
        load_spinor(qx, wk.v(slot, j), g.ldv, s);
        load_spinor(py, wk.ab(slot, j), g.ldv, y);
        load_spinor(qy, wk.v(slot, j), g.ldv, y);
        force_pair<NU>(G, px, qx, py, qy, ef, eb);
        if (j < k) {
            load_spinor(px, wk.w(slot, j), g.ldv, s);
            load_spinor(qx, wk.sb(slot, j), g.ldv, s);
            load_spinor(py, wk.w(slot, j), g.ldv, y);
            load_spinor(qy, wk.sb(slot, j), g.ldv, y);
            force_pair<NU>(G, px, qx, py, qy, ef, eb);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            ZD& o = gout[(size_t)(NU * 9 + a * 3 + b) * g.ldv + s];
            o = accumulate ? o + (-kappa) * G[a][b] : (-kappa) * G[a][b];
        }
}

// Blocks of 64 sites x 4 directions, one wavefront per direction: the four links of
// a site read its spinors at nearly the same time on one compute unit (from L1/L2
// rather than from memory four times over), and the blocks go out in XCD order so
// that neighbour spinors are mostly still in L2.
template <typename R>
__global__ __launch_bounds__(4 * kSites) void k_force(Geom g, double kappa, double emu, Work<R> wk, SrcList L,
                                                      int nchunk, ZD* __restrict__ gpart, int jlo, int jhi,
                                                      int accumulate) {
    const int nu = __builtin_amdgcn_readfirstlane(threadIdx.x / kSites);
    const int sb = g.sbmap ? g.sbmap[blockIdx.x] : (int)blockIdx.x;
    const int s = sb * kSites + threadIdx.x % kSites;
    if (sb < 0 || s >= g.V) return;
    const int e = blockIdx.z, slot = L.slot[e];
    const int k = L.k[e];
    const int top = jhi > 0 ? min(jhi, k) : k;   // steps jlo..top
    const int n = top - jlo + 1;
    const int chunk = blockIdx.y;
    const int j0 = jlo + (int)((long long)n * chunk / nchunk);
    const int j1 = jlo + (int)((long long)n * (chunk + 1) / nchunk);
    ZD* out = gpart + ((size_t)slot * nchunk + chunk) * 36 * g.ldv;
    switch (nu) {
        case 0: force_body<0>(g, kappa, emu, wk, slot, k, j0, j1, s, out, accumulate); break;
        case 1: force_body<1>(g, kappa, emu, wk, slot, k, j0, j1, s, out, accumulate); break;
        case 2: force_body<2>(g, kappa, emu, wk, slot, k, j0, j1, s, out, accumulate); break;
        default: force_body<3>(g, kappa, emu, wk, slot, k, j0, j1, s, out, accumulate); break;
    }
}

template <typename R>
void launch_force(const Geom& g, double kappa, double mu, const Work<R>& wk, const SrcList& L, int nchunk, ZD* gpart,
                  hipStream_t st, int jlo, int jhi, int accumulate) {
    dim3 grid(g.sbmap ? g.nwg : np_stencil(g.V), nchunk, L.n);
    hipLaunchKernelGGL(k_force<R>, grid, dim3(4 * kSites), 0, st, g, kappa, std::exp(mu), wk, L, nchunk, gpart, jlo,
                       jhi, accumulate);
}

__device__ __forceinline__ double boundary_sign(const Geom& g, int nu, int s, int antiperiodic) {
    return (nu == 3 && antiperiodic && s / (g.nx * g.ny * g.nz) == g.nt - 1) ? -1.0 : 1.0;
}

__global__ __launch_bounds__(kBlock) void k_force_reduce(Geom g, const ZD* __restrict__ gpart, int nchunk, SrcList L,
                                                         int antiperiodic, ZD* __restrict__ dU) {
    // one thread per (site, direction, colour entry): the chunks' loads all go out at
    // once and are summed in chunk order
    const int s = blockIdx.x * kBlock + threadIdx.x;
    const int nu = blockIdx.y / 9, ab = blockIdx.y % 9, e = blockIdx.z, slot = L.slot[e];
    if (s >= g.V) return;
    // gradient with respect to the caller's link: undo the folded boundary sign
    const double sign = boundary_sign(g, nu, s, antiperiodic);
    const ZD* gp = gpart + (size_t)slot * nchunk * 36 * g.ldv + (size_t)(nu * 9 + ab) * g.ldv + s;
    ZD* out = dU + (size_t)L.src[e] * 36 * g.V;
    ZD acc = mk<double>(0, 0);
#pragma unroll 16
    for (int c = 0; c < nchunk; ++c) acc = acc + gp[(size_t)c * 36 * g.ldv];
    out[((size_t)nu * g.V + s) * 9 + ab] = sign * acc;
}

void launch_force_reduce(const Geom& g, const ZD* gpart, int nchunk, const SrcList& L, int antiperiodic, ZD* dU,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_force_reduce, dim3(grid_for(g.V), 36, L.n), dim3(kBlock), 0, st, g, gpart, nchunk, L,
                       antiperiodic, dU);
}

// U(1) projection of the link gradient: with G the gradient for the caller's link
// U_c = sign U (sign the folded boundary factor), -Im tr(G^H U_c) = -Im tr(acc^H U)
// for the unsigned accumulator acc and the stored (signed) link U.
__global__ __launch_bounds__(kBlock) void k_force_current(Geom g, const ZD* __restrict__ gpart, int nchunk, SrcList L,
                                                          const ZD* __restrict__ U, double* __restrict__ gsrc,
                                                          double* __restrict__ jsum, int accumulate) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    const int nu = blockIdx.y;
    if (s >= g.V) return;
    ZD u[9];
#pragma unroll
    for (int ab = 0; ab < 9; ++ab) u[ab] = U[(size_t)(nu * 9 + ab) * g.ldv + s];
    double tot = accumulate ? jsum[(size_t)nu * g.V + s] : 0.0;
    for (int e = 0; e < L.n; ++e) {
        const int slot = L.slot[e];
        const ZD* gp = gpart + (size_t)slot * nchunk * 36 * g.ldv;
        double im = 0.0;
#pragma unroll
        for (int ab = 0; ab < 9; ++ab) {
            ZD acc = mk<double>(0, 0);
            for (int c = 0; c < nchunk; ++c) acc = acc + gp[(size_t)c * 36 * g.ldv + (size_t)(nu * 9 + ab) * g.ldv + s];
            im += cjmul(acc, u[ab]).im;
        }
        if (gsrc) gsrc[((size_t)slot * 4 + nu) * g.ldv + s] = -im;
        tot += -im;
    }
    jsum[(size_t)nu * g.V + s] = tot;
}

void launch_force_current(const Geom& g, const ZD* gpart, int nchunk, const SrcList& L, const ZD* U64,
                          double* gsrc, double* jsum, int accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_force_current, dim3(grid_for(g.V), 4), dim3(kBlock), 0, st, g, gpart, nchunk, L, U64, gsrc,
                       jsum, accumulate);
}

__global__ __launch_bounds__(kBlock) void k_zero(double* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) p[i] = 0.0;
}

void launch_zero(double* p, size_t n, hipStream_t st) {
    if (n == 0) return;
    size_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)nb), dim3(kBlock), 0, st, p, n);
}

// =============================================================== current estimator
__global__ __launch_bounds__(kBlock) void k_current_div(Geom g, const double* __restrict__ j, double scale,
                                                        double* __restrict__ div, double* __restrict__ tot) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const Nbr n = neighbours(g, s);
    double d = 0.0, t = 0.0;
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        const double out = j[(size_t)nu * g.V + s], in = j[(size_t)nu * g.V + n.bwd[nu]];
        d += out - in;
        t += out + in;
    }
    if (div) div[s] = scale * d;
    if (tot) tot[s] = scale * t;
}

__global__ __launch_bounds__(kBlock) void k_scale(double* __restrict__ p, size_t n, double scale) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] *= scale;
}

void launch_current_finish(const Geom& g, double* j, double scale, double* div, double* tot, hipStream_t st) {
    if (div || tot)
        hipLaunchKernelGGL(k_current_div, dim3(grid_for(g.V)), dim3(kBlock), 0, st, g, j, scale, div, tot);
    hipLaunchKernelGGL(k_scale, dim3(grid_for(4 * g.V)), dim3(kBlock), 0, st, j, (size_t)4 * g.V, scale);
}

// Ward identity of the local U(1) symmetry (phase rotation of U_nu(x) for all
// outgoing links, of U_nu(x - nu) for all incoming ones and of psi(x), eta(x)),
// per entry, for eta = g5 psi: the link derivatives' divergence equals the
// source terms.  psi is indexed by the entry's source, y and dpsi by the entry.
__global__ __launch_bounds__(kBlock) void k_ward(Geom g, const double* __restrict__ gsrc, SrcList L,
                                                 const ZD* __restrict__ psi, const ZD* __restrict__ y,
                                                 const ZD* __restrict__ dpsi, double* __restrict__ part) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    const int e = blockIdx.y, slot = L.slot[e];
    double mx[2] = {0.0, 0.0};
    if (s < g.V) {
        const Nbr n = neighbours(g, s);
        const double* gs = gsrc + (size_t)slot * 4 * g.ldv;
        double lhs = 0.0;
#pragma unroll
        for (int nu = 0; nu < 4; ++nu) {
            const double o = gs[(size_t)nu * g.ldv + s], i = gs[(size_t)nu * g.ldv + n.bwd[nu]];
            lhs += o - i;
            mx[1] = fmax(mx[1], fabs(o));
        }
        const size_t co = (size_t)L.src[e] * 12 * g.V + (size_t)s * 12;
        const size_t cy = (size_t)e * 12 * g.V + (size_t)s * 12;
        double rhs = 0.0;
#pragma unroll
        for (int p = 0; p < 12; ++p) {   // eta = g5 psi
            const double g5 = p < 6 ? 1.0 : -1.0;
            rhs -= g5 * cjmul(psi[co + p], y[cy + p]).im;
            rhs += cjmul(dpsi[cy + p], psi[co + p]).im;
        }
        mx[0] = fabs(lhs - rhs);
    }
    // block maxima (wave shuffle tree, then waves in order)
    __shared__ double red[kBlock / kWave][2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) mx[q] = fmax(mx[q], __shfl_down(mx[q], off, kWave));
    if (threadIdx.x % kWave == 0) {
        red[threadIdx.x / kWave][0] = mx[0];
        red[threadIdx.x / kWave][1] = mx[1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) {
            a = fmax(a, red[w][0]);
            b = fmax(b, red[w][1]);
        }
        part[((size_t)e * gridDim.x + blockIdx.x) * 2] = a;
        part[((size_t)e * gridDim.x + blockIdx.x) * 2 + 1] = b;
    }
}

int launch_ward(const Geom& g, const double* gsrc, const SrcList& L, const ZD* psi, const ZD* y, const ZD* dpsi,
                double* part, hipStream_t st) {
    const int nb = grid_for(g.V);
    hipLaunchKernelGGL(k_ward, dim3(nb, L.n), dim3(kBlock), 0, st, g, gsrc, L, psi, y, dpsi, part);
    return nb;
}

// =============================================================== source gradient
// x = |x| v_1 with v_1 = w_1 = x/|x|:  xbar = u/|x| + [S/|x| - Re(u^H x)/|x|^2] x/|x|, u = vbar_1 + wbar_1.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_sgrad_dot(Geom g, Work<R> wk, SrcList L) {
    const int slot = L.slot[blockIdx.y];
    const Z<R>* __restrict__ vbar = wk.f(slot, 4);
    const Z<R>* __restrict__ wbar = wk.f(slot, 5);
    const Z<R>* __restrict__ x = wk.f(slot, 0);
    const int s = blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (s < g.V) {
#pragma unroll
        for (int p = 0; p < 12; ++p) {
            const size_t i = (size_t)p * g.ldv + s;
            const ZD u = zcast<double>(vbar[i]) + zcast<double>(wbar[i]);
            v[0] += cjmul(u, zcast<double>(x[i])).re;
        }
    }
    write_partials<1, kBlock>(wk.p(slot, 2), v);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_sgrad_out(Geom g, Work<R> wk, SrcList L, Coef coef0, int npart,
                                                      ZD* __restrict__ out_base) {
    const int e = blockIdx.y, slot = L.slot[e];
    const Coef coef = coef0.at(slot);
    double red[1];
    reduce_partials<1, kBlock>(wk.p(slot, 2), npart, red);
    const double nx = coef.misc[0], S = coef.misc[1];
    const double c2 = (S / nx - red[0] / (nx * nx)) / nx;
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const Z<R>* __restrict__ vbar = wk.f(slot, 4);
    const Z<R>* __restrict__ wbar = wk.f(slot, 5);
    const Z<R>* __restrict__ x = wk.f(slot, 0);
    ZD* out = out_base + (size_t)L.src[e] * 12 * g.V;
#pragma unroll
    for (int p = 0; p < 12; ++p) {
        const size_t i = (size_t)p * g.ldv + s;
        const ZD u = zcast<double>(vbar[i]) + zcast<double>(wbar[i]);
        out[(size_t)s * 12 + p] = (1.0 / nx) * u + c2 * zcast<double>(x[i]);
    }
}

template <typename R>
void launch_source_grad(const Geom& g, const Work<R>& wk, const SrcList& L, Coef coef, ZD* dpsi, hipStream_t st) {
    const int nb = grid_for(g.V);
    hipLaunchKernelGGL(k_sgrad_dot<R>, dim3(nb, L.n), dim3(kBlock), 0, st, g, wk, L);
    hipLaunchKernelGGL(k_sgrad_out<R>, dim3(nb, L.n), dim3(kBlock), 0, st, g, wk, L, coef, nb, dpsi);
}

// =============================================================== biorthogonality probe
// After the forward pass, with k = k_used read on the device: block partials of
// x^H v_k and w_k^H x for the entry's source x = f(slot, 0) (so that with
// v_1 = w_1 = x/|x| they give w_1^H v_k and w_k^H v_1 up to the factor 1/|x|),
// zeros for k_used < 2, into wk.p(slot, 3)[block * 4].
template <typename R>
__global__ __launch_bounds__(kBlock) void k_biorth(Geom g, Work<R> wk, SrcList L, Coef coef0) {
    const int e = blockIdx.y, slot = L.slot[e];
    const int ku = coef0.at(slot).status[1];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (ku >= 2 && s < g.V) {
        const Z<R>* x = wk.f(slot, 0);
        const Z<R>* vk = wk.v(slot, ku);
        const Z<R>* wkk = wk.w(slot, ku);
#pragma unroll
        for (int p = 0; p < 12; ++p) {
            const ZD xs = zcast<double>(x[(size_t)p * g.ldv + s]);
            const ZD xv = cjmul(xs, zcast<double>(vk[(size_t)p * g.ldv + s]));
            const ZD wx = cjmul(zcast<double>(wkk[(size_t)p * g.ldv + s]), xs);
            v[0] += xv.re;
            v[1] += xv.im;
            v[2] += wx.re;
            v[3] += wx.im;
        }
    }
    write_partials_at<4, kBlock>(wk.p(slot, 3), blockIdx.x, v);
}

template <typename R>
int launch_biorth(const Geom& g, const Work<R>& wk, const SrcList& L, Coef coef, hipStream_t st) {
    const int nb = grid_for(g.V);
    hipLaunchKernelGGL(k_biorth<R>, dim3(nb, L.n), dim3(kBlock), 0, st, g, wk, L, coef);
    return nb;
}

// =============================================================== instantiations
#define TSLOV_INST(R)                                                                                           \
    template void launch_spinor_to_soa<R>(const ZD*, Z<R>*, const Geom&, double*, hipStream_t);                 \
    template void launch_spinor_from_soa<R>(const Z<R>*, ZD*, const Geom&, hipStream_t);                        \
    template void launch_sources_to_soa<R>(const ZD*, int, int, const Work<R>&, const SrcList&, const Geom&,    \
                                           hipStream_t);                                                        \
    template void launch_recur<R>(const Geom&, const Work<R>&, const SrcList&, Coef, int, hipStream_t);         \
    template void launch_recur_replay<R>(const Geom&, const Work<R>&, const SrcList&, Coef, int, hipStream_t);  \
    template void launch_assemble<R>(const Geom&, const Work<R>&, const SrcList&, Coef, const ZD*, int, ZD*,    \
                                     hipStream_t, int, int);                                                    \
    template void launch_bwd_ra<R>(const Geom&, const Work<R>&, const SrcList&, Coef, int, hipStream_t);        \
    template void launch_force<R>(const Geom&, double, double, const Work<R>&, const SrcList&, int, ZD*,        \
                                  hipStream_t, int, int, int);                                                  \
    template void launch_source_grad<R>(const Geom&, const Work<R>&, const SrcList&, Coef, ZD*, hipStream_t);   \
    template int launch_biorth<R>(const Geom&, const Work<R>&, const SrcList&, Coef, hipStream_t);

// The stencil launchers for fields of type R and links of type RL.
#define TSLOV_INST_STENCIL(R, RL)                                                                               \
    template void launch_apply<R, RL>(const Z<RL>*, const Z<R>*, Z<R>*, const Geom&, double, double, int, int,  \
                                      hipStream_t, Timing, int);                                                \
    template void launch_fwd_pair<R, RL>(const Z<RL>*, const Geom&, double, double, const Work<R>&,             \
                                         const SrcList&, Coef, int, int, int, hipStream_t, Timing);             \
    template void launch_fwd_replay<R, RL>(const Z<RL>*, const Geom&, double, double, const Work<R>&,           \
                                           const SrcList&, Coef, int, hipStream_t);                             \
    template void launch_bwd_rb<R, RL>(const Z<RL>*, const Geom&, double, double, const Work<R>&,               \
                                       const SrcList&, Coef, int, int, int, hipStream_t, Timing);

TSLOV_INST(double)
TSLOV_INST(float)
TSLOV_INST_STENCIL(double, double)
TSLOV_INST_STENCIL(float, float)
TSLOV_INST_STENCIL(double, float)

}  // namespace tslov
