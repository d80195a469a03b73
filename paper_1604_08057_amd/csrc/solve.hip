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

// Compiler barrier for memory operations: keeps the epilogue's own-site loads from
// being hoisted above the hops, where they would stay live.
__device__ __forceinline__ void cg_fence_compiler() { asm volatile("" ::: "memory"); }

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

// Spinor of one site for the lane's own system: the plane base is that of the
// wavefront's first system (scalar registers) and the lane adds its system's
// distance from it, off = (e - e0) * kCgFields * fe * 16 + site * 16 bytes, a 32-bit
// offset (the launcher checks that it fits).
__device__ __forceinline__ void load_spinor_off(Spinor<double>& p, FieldBase f, int ldv, unsigned off) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const TSLOV_GLOBAL char* plane = uniform_ptr(f.p + (size_t)(sp * 3 + c) * (size_t)ldv * sizeof(ZD));
            const TSLOV_GLOBAL double* q = (const TSLOV_GLOBAL double*)(plane + (size_t)off);
            p.c[sp][c] = mk<double>(q[0], q[1]);
        }
}

// Both hops of direction NU for a whole site (forward, then backward: the hop sum of
// the colour split per colour row, so both forms give the same acc).
template <int NU>
__device__ __forceinline__ void mr_hops(Spinor<double>& acc, const ZD* __restrict__ U, FieldBase in, unsigned sysoff,
                                        const Geom& g, int s, const Nbr& n, double ep, double em) {
    ZD u[3][3];
    Spinor<double> p;
    load_link(u, U, g.ldv, NU, s);
    load_spinor_off(p, in, g.ldv, sysoff + (unsigned)n.fwd[NU] * (unsigned)sizeof(ZD));
    hop_fwd<NU>(acc, u, p, NU == 3 ? ep : 1.0);
    load_link(u, U, g.ldv, NU, n.bwd[NU]);
    load_spinor_off(p, in, g.ldv, sysoff + (unsigned)n.bwd[NU] * (unsigned)sizeof(ZD));
    hop_bwd<NU>(acc, u, p, NU == 3 ? em : 1.0);
}

// Both hops of direction NU for a whole site of the t-march form, the four operands'
// loads issued before any arithmetic (one memory round trip per direction).
template <int NU>
__device__ __forceinline__ void tm_cg_hops(Spinor<double>& acc, const ZD* __restrict__ U, const ZD* __restrict__ in,
                                           const Geom& g, int s, int sf, int sb) {
    ZD uf[3][3], ub[3][3];
    Spinor<double> pf, pb;
    load_link(uf, U, g.ldv, NU, s);
    load_spinor(pf, in, g.ldv, sf);
    load_link(ub, U, g.ldv, NU, sb);
    load_spinor(pb, in, g.ldv, sb);
    cg_fence_compiler();
    hop_fwd<NU>(acc, uf, pf, 1.0);
    hop_bwd<NU>(acc, ub, pb, 1.0);
}


}  // namespace

// Multi-right-hand-side form of out_e = A_e in_e (A_e as for k_cg_apply): one
// wavefront per block, lane l serving system e = 8 blockIdx.y + l / 8 at site offset
// l % 8 of an eight-site chunk; the block walks the eight chunks of its 64-site block
// (site blocks in XCD order).  The eight systems read a chunk's link elements in one
// load instruction (one address per site), and each thread forms all three colours of
// its site (one neighbour spinor load per hop instead of one per colour).  Partials of
// |out_e|^2 per site block, summed over the chunks in order and over the eight lanes of
// a system by a fixed butterfly.  The register budget is left to the compiler (210
// registers, two wavefronts per SIMD): capped at 164 registers (three per SIMD) the
// loads go out later and the derivative takes 8.02 instead of 7.69 s.  (Measured at
// 16^4 with 40 systems: blocks of one, two, four and five such wavefronts, the latter
// sharing each link among all 40 systems through L1, took 7.69, 8.04, 8.16 and 8.14 s
// per deflated derivative, the colour split 7.82 s: the operator is not limited by its
// link loads.)
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_cg_apply_mr(const ZD* __restrict__ U, Geom g, double kappa,
                                                            double emu, CgWork cw, int nr, int adj, int in_field,
                                                            int out_field, int preg) {
    const int lane = threadIdx.x % kWave;
    const int e0 = 8 * (int)blockIdx.y;
    const int e = e0 + lane / 8;
    const int sb = xcd_block(blockIdx.x, gridDim.x);
    const bool live = e < nr && sb < np_stencil(g.V) && !*(volatile const int*)&cw.st[e].done;
    double pv = 0.0;
    if (live) {
        const CgRhs* st = cw.st + e;
        const ZD sig = adj ? cj(st->sigma) : st->sigma;
        const double m = adj ? -st->msign : st->msign;
        const double ep = m > 0 ? emu : 1.0 / emu, em = 1.0 / ep;
        const FieldBase in = field_base(cw.field(e0, in_field)), out = field_base(cw.field(e0, out_field));
        const unsigned sysoff = (unsigned)(lane / 8) * (unsigned)(kCgFields * cw.fe * sizeof(ZD));
#pragma unroll 1
        for (int ch = 0; ch < kSites / 8; ++ch) {
            const int s = sb * kSites + ch * 8 + lane % 8;
            if (s >= g.V) break;
            const Nbr n = neighbours(g, s);
            Spinor<double> acc;
            zero_spinor(acc);
            mr_hops<0>(acc, U, in, sysoff, g, s, n, ep, em);
            mr_hops<1>(acc, U, in, sysoff, g, s, n, ep, em);
            mr_hops<2>(acc, U, in, sysoff, g, s, n, ep, em);
            mr_hops<3>(acc, U, in, sysoff, g, s, n, ep, em);
            cg_fence_compiler();
            const unsigned off = sysoff + (unsigned)s * (unsigned)sizeof(ZD);
            Spinor<double> x;
            load_spinor_off(x, in, g.ldv, off);
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                const double g5 = sp < 2 ? 1.0 : -1.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const ZD o = sig * x.c[sp][c] - g5 * (x.c[sp][c] - kappa * acc.c[sp][c]);
                    TSLOV_GLOBAL char* plane = uniform_ptr(out.p + (size_t)(sp * 3 + c) * (size_t)g.ldv * sizeof(ZD));
                    TSLOV_GLOBAL double* q = (TSLOV_GLOBAL double*)(plane + (size_t)off);
                    q[0] = o.re;
                    q[1] = o.im;
                    pv += norm2(o);
                }
            }
        }
    }
    // the eight lanes of a system hold the same sum after these three steps
    pv = pv + dpp_d<kDppSwap1>(pv);
    pv = pv + dpp_d<kDppSwap2>(pv);
    pv = pv + dpp_d<kDppHalfMirror>(pv);
    if (live && lane % 8 == 0) cw.p(e, preg)[sb] = pv;
}

// ---------------------------------------------------------------- t-march form
// The operator with a march along t (the t-march of the plain operator, per system): a
// block of kBlock threads owns a tile of kBlock (x, y, z) sites of one system and runs
// through a chunk of T consecutive t-slices.  psi(t+1), loaded for the forward t-hop of
// slice t, is the own spinor of slice t+1, and the backward t-hop of slice t+1 before
// reconstruction, U_t(t)^dag P- psi(t), is carried: along t every spinor and link is
// read once per chunk.  Both wait in LDS slots private to the thread while the x, y, z
// hops hold the registers.  The blocks of one (tile, chunk) for all systems run
// back to back on one XCD (block b: XCD b % 8; system (b / 8) % nr; then tile and chunk,
// each XCD taking the same run of tiles, a slab of z-planes, in every chunk), so the
// systems read the tile's links from that XCD's L2.  Each x, y, z direction issues its
// four operands before any arithmetic (one round trip; loading the backward hop's after
// the forward hop's arithmetic took 7.62 instead of 7.50 s per 16^4 derivative).  Hop
// sum in the order of the other forms (x, y, z, t; forward then backward).  Partials of
// |out_e|^2 per (tile, chunk).
__global__ __launch_bounds__(kBlock) void k_cg_apply_tm(const ZD* __restrict__ U, Geom g, double kappa, double emu,
                                                        CgWork cw, int nr, int adj, int in_field, int out_field,
                                                        int preg, int T) {
    const int V3 = g.nx * g.ny * g.nz, per = V3 / kBlock / kXcd;
    const int m = blockIdx.x / kXcd, e = m % nr, rest = m / nr;
    const int tile = (blockIdx.x % kXcd) * per + rest % per, chunk = rest / per;
    if (*(volatile const int*)&cw.st[e].done) return;   // uniform over the block
    const CgRhs* st = cw.st + e;
    const ZD sig = adj ? cj(st->sigma) : st->sigma;
    const double msg = adj ? -st->msign : st->msign;
    const double ep = msg > 0 ? emu : 1.0 / emu, em = 1.0 / ep;
    const ZD* __restrict__ in = cw.field(e, in_field);
    ZD* __restrict__ out = cw.field(e, out_field);
    const int s3 = tile * kBlock + threadIdx.x;   // the (x, y, z) site; t = 0
    const int t0 = chunk * T;
    const Nbr n3 = neighbours(g, s3);
    __shared__ ZD stash[12][kBlock];
    __shared__ ZD hstash[6][kBlock];
    auto park = [&](const Spinor<double>& p) {
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) stash[sp * 3 + c][threadIdx.x] = p.c[sp][c];
    };
    auto park_h = [&](const ZD (&h)[2][3]) {
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) hstash[q * 3 + c][threadIdx.x] = h[q][c];
    };
    {
        Spinor<double> own0;
        load_spinor(own0, in, g.ldv, s3 + t0 * V3);
        park(own0);
    }
    {
        const int sp = s3 + ((t0 + g.nt - 1) % g.nt) * V3;
        ZD u[3][3], h[2][3], hb[2][3];
        Spinor<double> p;
        load_link(u, U, g.ldv, 3, sp);
        load_spinor(p, in, g.ldv, sp);
        project<3, -1>(p, h);
        adj_mat_vec(u, h, hb);
        park_h(hb);
    }
    double pv = 0.0;
#pragma unroll 1
    for (int t = t0; t < t0 + T; ++t) {
        const int s = s3 + t * V3;
        Spinor<double> acc;
        zero_spinor(acc);
#pragma unroll 1
        for (int nu = 0; nu < 3; ++nu) {
            switch (nu) {
                case 0: tm_cg_hops<0>(acc, U, in, g, s, n3.fwd[0] + t * V3, n3.bwd[0] + t * V3); break;
                case 1: tm_cg_hops<1>(acc, U, in, g, s, n3.fwd[1] + t * V3, n3.bwd[1] + t * V3); break;
                default: tm_cg_hops<2>(acc, U, in, g, s, n3.fwd[2] + t * V3, n3.bwd[2] + t * V3); break;
            }
        }
        Spinor<double> own;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) own.c[sp][c] = stash[sp * 3 + c][threadIdx.x];
        ZD ut[3][3];
        Spinor<double> nxt;
        load_link(ut, U, g.ldv, 3, s);
        load_spinor(nxt, in, g.ldv, s3 + ((t + 1) % g.nt) * V3);
        hop_fwd<3>(acc, ut, nxt, ep);
        {
            ZD hb[2][3];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) hb[q][c] = hstash[q * 3 + c][threadIdx.x];
            reconstruct_add<3, -1>(acc, hb, em);
        }
        {
            ZD h[2][3], hb[2][3];
            project<3, -1>(own, h);
            adj_mat_vec(ut, h, hb);
            park_h(hb);
        }
        cg_fence_compiler();
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
            const double g5 = sp < 2 ? 1.0 : -1.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const ZD x = own.c[sp][c];
                const ZD o = sig * x - g5 * (x - kappa * acc.c[sp][c]);
                out[(size_t)(sp * 3 + c) * g.ldv + s] = o;
                pv += norm2(o);
            }
        }
        park(nxt);
    }
    double red[1] = {pv};
    block_sum_last<1, kBlock>(red);
    if (threadIdx.x == 0) cw.p(e, preg)[tile * (g.nt / T) + chunk] = red[0];
}

// ---------------------------------------------------------------- matrix-core form
// The same operator with the link times half-spinor products on the matrix cores
// (v_mfma_f64_16x16x4f64, D = A B + C with A 16x4, B 4x16 in float64).  One wavefront
// serves eight systems at the eight sites of a chunk (lane = 8 system + site, as the
// multi-right-hand-side form).  For a hop and a site j the product is one real GEMM
//     D[(e, s')][n] = sum_k A[(e, s')][k] B[k][n],
// rows (system e, half-spinor spin s'), k over (Re, Im) x colour of the half spinor,
// n over (Re, Im) x colour of the result, B the real 6x6 form of the 3x3 link:
//     Re o = Re U Re h - Im U Im h,   Im o = Im U Re h + Re U Im h,
// two steps of K = 4 (six of eight k used) and six of sixteen columns.  The half
// spinors pass through LDS from the lane that projected them to the lanes of the
// A operand, and the results back to the lane that reconstructs its four spins.
// Register layout of the instruction (lane l): A[l % 16][l / 16], B[l / 16][l % 16],
// D[l / 16 + 4 r][l % 16] in the r-th element of the result (checked on the device).
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

// Real-form link element B[k][n] of the hop's 3x3 matrix M (M = U for a forward hop,
// U^dag for a backward one), k = 3 pin + b, n = 3 pout + c, zero outside 6 x 6.
template <int DIR>
__device__ __forceinline__ double link_real_form(const ZD* __restrict__ U, int ldv, int nu, int site, int k, int n) {
    if (k >= 6 || n >= 6) return 0.0;
    const int pin = k / 3, b = k % 3, pout = n / 3, c = n % 3;
    // M[c][b]: forward U[c][b]; backward conj(U[b][c])
    const ZD m = DIR > 0 ? U[(size_t)(nu * 9 + c * 3 + b) * ldv + site] : cj(U[(size_t)(nu * 9 + b * 3 + c) * ldv + site]);
    if (pin == 0) return pout == 0 ? m.re : m.im;     // Re h -> (Re M, Im M)
    return pout == 0 ? -m.im : m.re;                  // Im h -> (-Im M, Re M)
}

template <int NU, int DIR>
__device__ __forceinline__ void mfma_hop(Spinor<double>& acc, const ZD* __restrict__ U, FieldBase in, unsigned sysoff,
                                         const Geom& g, int nb_site, int link_site, bool valid, double coef,
                                         double (*hs)[8][2][3][2], double (*ds)[16][6], int* lsite) {
    const int lane = threadIdx.x % kWave;
    const int e = lane / 8, j = lane % 8;
    // project the neighbour spinor (zero for lanes without a site or system)
    ZD h[2][3];
    if (valid) {
        Spinor<double> p;
        load_spinor_off(p, in, g.ldv, sysoff + (unsigned)nb_site * (unsigned)sizeof(ZD));
        project<NU, DIR>(p, h);
    } else {
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) h[sp][c] = mk<double>(0, 0);
    }
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            hs[j][e][sp][c][0] = coef * h[sp][c].re;
            hs[j][e][sp][c][1] = coef * h[sp][c].im;
        }
    if (e == 0) lsite[j] = link_site;
    __syncthreads();
    const int i = lane % 16, kk = lane / 16, n = lane % 16;
    // A operand: K-step 0 holds k = kk (Re h colour kk for kk < 3, Im h colour 0 for kk = 3),
    // K-step 1 holds k = 4 + kk (Im h colours 1, 2; zero beyond)
    const int k0 = kk, k1 = 4 + kk;
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
        const double a0 = hs[jj][i / 2][i % 2][k0 % 3][k0 / 3];
        const double a1 = k1 < 6 ? hs[jj][i / 2][i % 2][k1 % 3][k1 / 3] : 0.0;
        const int ls = lsite[jj];
        const double b0 = link_real_form<DIR>(U, g.ldv, NU, ls, k0, n);
        const double b1 = link_real_form<DIR>(U, g.ldv, NU, ls, k1, n);
        mfma_d4 d = {0.0, 0.0, 0.0, 0.0};
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, d, 0, 0, 0);
        if (n < 6) {
#pragma unroll
            for (int r = 0; r < 4; ++r) ds[jj][kk + 4 * r][n] = d[r];
        }
    }
    __syncthreads();
    ZD o[2][3];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) o[sp][c] = mk<double>(ds[j][2 * e + sp][c], ds[j][2 * e + sp][3 + c]);
    __syncthreads();   // hs, ds and lsite are rewritten by the next hop
    if (valid) reconstruct_add<NU, DIR>(acc, o, 1.0);
}

// Matrix-core form of out_e = A_e in_e (A_e as for k_cg_apply), one wavefront per
// block serving systems 8 blockIdx.y .. + 7; partials as k_cg_apply_mr.
__global__ __launch_bounds__(kWave) void k_cg_apply_mfma(const ZD* __restrict__ U, Geom g, double kappa, double emu,
                                                         CgWork cw, int nr, int adj, int in_field, int out_field,
                                                         int preg) {
    __shared__ double hs[8][8][2][3][2];
    __shared__ double ds[8][16][6];
    __shared__ int lsite[8];
    const int lane = threadIdx.x % kWave;
    const int e0 = 8 * (int)blockIdx.y;
    const int e = e0 + lane / 8;
    const int sb = xcd_block(blockIdx.x, gridDim.x);
    if (e0 >= nr || sb >= np_stencil(g.V)) return;   // uniform over the block
    const bool live = e < nr && !*(volatile const int*)&cw.st[e].done;
    ZD sig = mk<double>(0, 0);
    double ep = 1.0, em = 1.0;
    if (live) {
        const CgRhs* st = cw.st + e;
        sig = adj ? cj(st->sigma) : st->sigma;
        const double m = adj ? -st->msign : st->msign;
        ep = m > 0 ? emu : 1.0 / emu;
        em = 1.0 / ep;
    }
    const FieldBase in = field_base(cw.field(e0, in_field)), out = field_base(cw.field(e0, out_field));
    const unsigned sysoff = (unsigned)(lane / 8) * (unsigned)(kCgFields * cw.fe * sizeof(ZD));
    double pv = 0.0;
#pragma unroll 1
    for (int ch = 0; ch < kSites / 8; ++ch) {
        const int s = sb * kSites + ch * 8 + lane % 8;
        const bool valid = live && s < g.V;
        const int sv = s < g.V ? s : 0;   // a site in range for the address arithmetic
        const Nbr n = neighbours(g, sv);
        Spinor<double> acc;
        zero_spinor(acc);
        mfma_hop<0, +1>(acc, U, in, sysoff, g, n.fwd[0], sv, valid, 1.0, hs, ds, lsite);
        mfma_hop<0, -1>(acc, U, in, sysoff, g, n.bwd[0], n.bwd[0], valid, 1.0, hs, ds, lsite);
        mfma_hop<1, +1>(acc, U, in, sysoff, g, n.fwd[1], sv, valid, 1.0, hs, ds, lsite);
        mfma_hop<1, -1>(acc, U, in, sysoff, g, n.bwd[1], n.bwd[1], valid, 1.0, hs, ds, lsite);
        mfma_hop<2, +1>(acc, U, in, sysoff, g, n.fwd[2], sv, valid, 1.0, hs, ds, lsite);
        mfma_hop<2, -1>(acc, U, in, sysoff, g, n.bwd[2], n.bwd[2], valid, 1.0, hs, ds, lsite);
        mfma_hop<3, +1>(acc, U, in, sysoff, g, n.fwd[3], sv, valid, ep, hs, ds, lsite);
        mfma_hop<3, -1>(acc, U, in, sysoff, g, n.bwd[3], n.bwd[3], valid, em, hs, ds, lsite);
        if (valid) {
            const unsigned off = sysoff + (unsigned)s * (unsigned)sizeof(ZD);
            Spinor<double> x;
            load_spinor_off(x, in, g.ldv, off);
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                const double g5 = sp < 2 ? 1.0 : -1.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const ZD o = sig * x.c[sp][c] - g5 * (x.c[sp][c] - kappa * acc.c[sp][c]);
                    TSLOV_GLOBAL char* plane = uniform_ptr(out.p + (size_t)(sp * 3 + c) * (size_t)g.ldv * sizeof(ZD));
                    TSLOV_GLOBAL double* q = (TSLOV_GLOBAL double*)(plane + (size_t)off);
                    q[0] = o.re;
                    q[1] = o.im;
                    pv += norm2(o);
                }
            }
        }
    }
    pv = pv + dpp_d<kDppSwap1>(pv);
    pv = pv + dpp_d<kDppSwap2>(pv);
    pv = pv + dpp_d<kDppHalfMirror>(pv);
    if (live && lane % 8 == 0) cw.p(e, preg)[sb] = pv;
}

namespace {

// t-slices per chunk of the t-march form: the whole time extent when the tiles and systems
// give at least 512 workgroups, else the largest divisor of nt that does; 0 when the
// (x, y, z) volume does not split into tiles of kBlock sites evenly over the XCDs.
int cg_tm_chunk(const Geom& g, int nr) {
    const int V3 = g.nx * g.ny * g.nz;
    if (V3 % (kBlock * kXcd) != 0) return 0;
    const long long nb = (long long)V3 / kBlock * nr;
    int T = 1;
    for (int c = 1; c <= g.nt; ++c)
        if (g.nt % c == 0 && nb * (g.nt / c) >= 512) T = c;
    return T;
}

// Partial sums per system written by one operator launch.
int cg_apply_parts(const Geom& g, int nr, int op) {
    if (op == kCgOpTmarch && cg_tm_chunk(g, nr) > 0) return g.nx * g.ny * g.nz / kBlock * (g.nt / cg_tm_chunk(g, nr));
    return np_stencil(g.V);
}

// The operator launch over the nr systems.  Forms (measured at 16^4 with 40 systems, per
// deflated derivative): t-march 7.50 s, multi-right-hand-side 7.70 s, colour split
// 7.82 s, matrix-core 14.2 s.  The t-march form needs (x, y, z) volumes in multiples of
// 1024 sites and otherwise runs the multi-right-hand-side form; the eight-system forms
// address a wavefront's systems with 32-bit offsets from the first one's planes and
// otherwise run the colour split (two systems per block when nr is even; 1, 2 and 4 per
// block took 8.00, 7.97 and 8.92 s).
void cg_apply(const ZD* U, const Geom& g, double kappa, double emu, int nr, const CgWork& cw, int adj, int in_field,
              int out_field, int preg, hipStream_t st) {
    const bool fits = (7.0 * kCgFields * cw.fe + g.ldv) * sizeof(ZD) < 4294967296.0;
    const int nb = (np_stencil(g.V) + kXcd - 1) / kXcd * kXcd;
    if (cw.op == kCgOpTmarch && cg_tm_chunk(g, nr) > 0) {
        const int T = cg_tm_chunk(g, nr);
        const int units = g.nx * g.ny * g.nz / kBlock * (g.nt / T);
        hipLaunchKernelGGL(k_cg_apply_tm, dim3(units * nr), dim3(kBlock), 0, st, U, g, kappa, emu, cw, nr, adj,
                           in_field, out_field, preg, T);
        return;
    }
    if (cw.op == kCgOpMfma && fits) {
        hipLaunchKernelGGL(k_cg_apply_mfma, dim3(nb, (nr + 7) / 8), dim3(kWave), 0, st, U, g, kappa, emu, cw, nr, adj,
                           in_field, out_field, preg);
        return;
    }
    if ((cw.op == kCgOpMulti || cw.op == kCgOpTmarch) && fits) {
        hipLaunchKernelGGL(k_cg_apply_mr, dim3(nb, (nr + 7) / 8), dim3(kWave), 0, st, U, g, kappa, emu, cw, nr, adj,
                           in_field, out_field, preg);
        return;
    }
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

// Right-hand sides given as canonical vectors: e < la: b = rhs_a[e]; e >= la: b = rhs_b
// (shared).  r = b, x = 0, partials of |b|^2.
__global__ __launch_bounds__(kBlock) void k_cg_load(Geom g, const ZD* __restrict__ rhs_a, int la,
                                                    const ZD* __restrict__ rhs_b, CgWork cw) {
    const int e = blockIdx.y;
    const int s = blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (s < g.V) {
        const ZD* __restrict__ b = e < la ? rhs_a + (size_t)e * 12 * g.V : rhs_b;
        ZD* __restrict__ r = cw.field(e, kCgR);
        ZD* __restrict__ x = cw.field(e, kCgX);
#pragma unroll
        for (int p = 0; p < 12; ++p) {
            const ZD z = b[(size_t)s * 12 + p];
            r[(size_t)p * g.ldv + s] = z;
            x[(size_t)p * g.ldv + s] = mk<double>(0, 0);
            v[0] += norm2(z);
        }
    }
    write_partials<1, kBlock>(cw.p(e, 0), v);
}

// Solution x of system e into a canonical vector.
__global__ __launch_bounds__(kBlock) void k_cg_store(Geom g, CgWork cw, ZD* __restrict__ out) {
    const int e = blockIdx.y;
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.V) return;
    const ZD* __restrict__ x = cw.field(e, kCgX);
#pragma unroll
    for (int p = 0; p < 12; ++p) out[(size_t)e * 12 * g.V + (size_t)s * 12 + p] = x[(size_t)p * g.ldv + s];
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

// U(1) projections g_e(x, nu) = -Im tr(G_e^H U_nu(x)) of canonical link gradients
// dU[e][nu][x][3][3] (the boundary sign undone, so U is the caller's field: U64 times
// the folded sign), into gsrc[e][nu][ldv] (nullable) and, summed over the sources in
// order, into jsum[nu][V] (added to its contents with accumulate).
__global__ __launch_bounds__(kBlock) void k_u1_projection(Geom g, const ZD* __restrict__ U64, const ZD* __restrict__ dU,
                                                          int nsrc, int antiperiodic, double* __restrict__ gsrc,
                                                          double* __restrict__ jsum, int accumulate) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    const int nu = blockIdx.y;
    if (s >= g.V) return;
    const double sign = (nu == 3 && antiperiodic && s / (g.nx * g.ny * g.nz) == g.nt - 1) ? -1.0 : 1.0;
    ZD u[9];
#pragma unroll
    for (int ab = 0; ab < 9; ++ab) u[ab] = sign * U64[(size_t)(nu * 9 + ab) * g.ldv + s];
    double tot = accumulate ? jsum[(size_t)nu * g.V + s] : 0.0;
    for (int e = 0; e < nsrc; ++e) {
        const ZD* G = dU + (((size_t)e * 4 + nu) * g.V + s) * 9;
        double im = 0.0;
#pragma unroll
        for (int ab = 0; ab < 9; ++ab) im += cjmul(G[ab], u[ab]).im;
        if (gsrc) gsrc[((size_t)e * 4 + nu) * g.ldv + s] = -im;
        tot += -im;
    }
    jsum[(size_t)nu * g.V + s] = tot;
}

// ---------------------------------------------------------------- launchers
void launch_u1_projection(const Geom& g, const ZD* U64, const ZD* dU, int nsrc, int antiperiodic, double* gsrc,
                          double* jsum, int accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_u1_projection, dim3(grid_for(g.V), 4), dim3(kBlock), 0, st, g, U64, dU, nsrc, antiperiodic,
                       gsrc, jsum, accumulate);
}

void launch_cg_rhs(const Geom& g, const ZD* psi, const ZD* eta, const ZD* pbar, const ZD* R, const ZD* L, const ZD* c,
                   const ZD* q, const double* sgn, int l, const CgWork& cw, hipStream_t st) {
    const int nb = grid_for(g.V);
    hipLaunchKernelGGL(k_cg_rhs, dim3(nb, 2 * l), dim3(kBlock), 0, st, g, psi, eta, pbar, R, L, c, q, sgn, l, cw);
    hipLaunchKernelGGL(k_cg_bnorm, dim3(1, 2 * l), dim3(kBlock), 0, st, cw, nb);
}

void launch_cg_load(const Geom& g, const ZD* rhs_a, int la, const ZD* rhs_b, int nr, const CgWork& cw,
                    hipStream_t st) {
    const int nb = grid_for(g.V);
    hipLaunchKernelGGL(k_cg_load, dim3(nb, nr), dim3(kBlock), 0, st, g, rhs_a, la, rhs_b, cw);
    hipLaunchKernelGGL(k_cg_bnorm, dim3(1, nr), dim3(kBlock), 0, st, cw, nb);
}

void launch_cg_store(const Geom& g, int nr, const CgWork& cw, ZD* out, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_store, dim3(grid_for(g.V), nr), dim3(kBlock), 0, st, g, cw, out);
}

void launch_cg_start(const ZD* U, const Geom& g, double kappa, double mu, int nr, const CgWork& cw, hipStream_t st) {
    const double emu = std::exp(mu);
    cg_apply(U, g, kappa, emu, nr, cw, 1, kCgR, kCgZ, 2, st);
    dim3 gp((g.V + kPBlock - 1) / kPBlock, 12, nr);
    hipLaunchKernelGGL(k_cg_init_p, gp, dim3(kPBlock), 0, st, g, cw, cg_apply_parts(g, nr, cw.op));
}

void launch_cg_iteration(const ZD* U, const Geom& g, double kappa, double mu, int nr, int it, int check, double tol,
                         const CgWork& cw, hipStream_t st) {
    const double emu = std::exp(mu);
    const int par = it & 1;
    const dim3 gp((g.V + kPBlock - 1) / kPBlock, 12, nr);
    const int npa = cg_apply_parts(g, nr, cw.op);
    cg_apply(U, g, kappa, emu, nr, cw, 0, kCgP, kCgW, 0, st);
    hipLaunchKernelGGL(k_cg_update_xr, gp, dim3(kPBlock), 0, st, g, cw, npa, par);
    if (check) hipLaunchKernelGGL(k_cg_check, dim3(1, nr), dim3(kPBlock), 0, st, cw, np_point(g.V), tol * tol);
    cg_apply(U, g, kappa, emu, nr, cw, 1, kCgR, kCgZ, 2, st);
    hipLaunchKernelGGL(k_cg_update_p, gp, dim3(kPBlock), 0, st, g, cw, npa, par);
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
