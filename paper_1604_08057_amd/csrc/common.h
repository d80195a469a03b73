// Internal device helpers shared by the tslov HIP kernels: complex arithmetic,
// lattice geometry, structure-of-arrays field access, deterministic block
// reductions and the spin-projected Wilson hopping term (App. A, eq. WD_op/WD_G).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstdint>

namespace tslov {

constexpr int kWave = 64;      // CDNA wavefront
constexpr int kBlock = 128;    // threads per block of the simple per-site kernels
constexpr int kSites = 64;     // sites per wavefront (and site block) of the colour-layout stencil kernels
constexpr int kCBlock = 3 * kSites;   // colour split: one wavefront per colour
constexpr int kRBlock = 3 * kSites;   // colour grid, pair kernels: two hop wavefronts and an epilogue wavefront
constexpr int kPBlock = 256;   // pointwise kernels: sites per block, grid.y = 12 planes

constexpr int kXcd = 8;        // accelerator complex dies; workgroups go to them round robin

// Number of per-block partial sums written by each kernel family.
__host__ __device__ inline int np_stencil(int V) { return (V + kSites - 1) / kSites; }
__host__ __device__ inline int np_point(int V) { return 12 * ((V + kPBlock - 1) / kPBlock); }
// Colour-grid stencil kernels: one single-wavefront block per (colour, 64 sites),
// colour-major, the site blocks padded to a multiple of the XCD count so that the
// three colours of a site block run on one XCD and share its L2.
__host__ __device__ inline int nsb_pad(int V) { return (np_stencil(V) + kXcd - 1) / kXcd * kXcd; }
__host__ __device__ inline int np_colour(int V) { return 3 * nsb_pad(V); }
__host__ __device__ inline int np_max(int V) { return np_colour(V) > np_point(V) ? np_colour(V) : np_point(V); }
// Layout of the stencil kernels, a function of the lattice alone (so that a source
// gives the same bits in any batch): the colour grid while the lattice has too few
// site blocks to occupy the chip with three-wavefront blocks, the colour-split
// blocks (kCBlock threads, colour = wavefront) above that, with the site blocks
// padded to a multiple of the XCD count and dealt out to the XCDs by Geom::sbmap.
constexpr int kColourGridMaxBlocks = 128;
__host__ __device__ inline bool colour_grid(int V) { return np_stencil(V) <= kColourGridMaxBlocks; }
// Blocks (= partial sums) of one stencil launch per source.
__host__ __device__ inline int np_sten(int V) { return colour_grid(V) ? np_colour(V) : nsb_pad(V); }
// Block b of a grid of nb blocks (nb a multiple of kXcd) -> the b-th block in XCD
// order: XCD b % kXcd takes the contiguous run of nb / kXcd blocks.
__host__ __device__ inline int xcd_block(int b, int nb) { return (b % kXcd) * (nb / kXcd) + b / kXcd; }

// ------------------------------------------------------------------ complex
template <typename R>
struct __align__(2 * sizeof(R)) Z {
    R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ Z<R> mk(R a, R b) { Z<R> z; z.re = a; z.im = b; return z; }
template <typename R>
__host__ __device__ __forceinline__ Z<R> operator+(Z<R> a, Z<R> b) { return mk<R>(a.re + b.re, a.im + b.im); }
template <typename R>
__host__ __device__ __forceinline__ Z<R> operator-(Z<R> a, Z<R> b) { return mk<R>(a.re - b.re, a.im - b.im); }
template <typename R>
__host__ __device__ __forceinline__ Z<R> operator-(Z<R> a) { return mk<R>(-a.re, -a.im); }
template <typename R>
__host__ __device__ __forceinline__ Z<R> operator*(Z<R> a, Z<R> b) {
    return mk<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R>
__host__ __device__ __forceinline__ Z<R> operator*(R s, Z<R> a) { return mk<R>(s * a.re, s * a.im); }
template <typename R>
__host__ __device__ __forceinline__ Z<R> cj(Z<R> a) { return mk<R>(a.re, -a.im); }
// conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ Z<R> cjmul(Z<R> a, Z<R> b) {
    return mk<R>(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
// a * conj(b)
template <typename R>
__host__ __device__ __forceinline__ Z<R> mulcj(Z<R> a, Z<R> b) {
    return mk<R>(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
template <typename R>
__host__ __device__ __forceinline__ Z<R> timesI(Z<R> a) { return mk<R>(-a.im, a.re); }
template <typename R>
__host__ __device__ __forceinline__ Z<R> timesMinusI(Z<R> a) { return mk<R>(a.im, -a.re); }
template <typename R>
__host__ __device__ __forceinline__ R norm2(Z<R> a) { return a.re * a.re + a.im * a.im; }

template <typename To, typename From>
__host__ __device__ __forceinline__ Z<To> zcast(Z<From> a) { return mk<To>((To)a.re, (To)a.im); }

__host__ __device__ __forceinline__ Z<double> zdiv(Z<double> a, Z<double> b) {
    double d = b.re * b.re + b.im * b.im;
    return mk<double>((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}

using ZD = Z<double>;

// ------------------------------------------------------------------ geometry
struct Geom {
    int nx, ny, nz, nt;
    int V;      // sites
    int ldv;    // plane stride (V rounded up to 64)
    // Site-block order of the colour-split and force kernels on larger lattices:
    // workgroup i works on site block sbmap[i] (-1: nothing).  Workgroup i runs on
    // XCD i % 8, so the map decides which site blocks share an L2 and in what order.
    const int* sbmap;
    int nwg;    // workgroups per entry (a multiple of 8, >= nsb_pad(V))
};

struct Nbr {
    int fwd[4];
    int bwd[4];
};

__device__ __forceinline__ Nbr neighbours(const Geom& g, int s) {
    const int x = s % g.nx;
    const int r1 = s / g.nx;
    const int y = r1 % g.ny;
    const int r2 = r1 / g.ny;
    const int z = r2 % g.nz;
    const int t = r2 / g.nz;
    const int sy = g.nx, sz = g.nx * g.ny, st = g.nx * g.ny * g.nz;
    Nbr n;
    n.fwd[0] = (x + 1 == g.nx) ? s - (g.nx - 1) : s + 1;
    n.bwd[0] = (x == 0) ? s + (g.nx - 1) : s - 1;
    n.fwd[1] = (y + 1 == g.ny) ? s - (g.ny - 1) * sy : s + sy;
    n.bwd[1] = (y == 0) ? s + (g.ny - 1) * sy : s - sy;
    n.fwd[2] = (z + 1 == g.nz) ? s - (g.nz - 1) * sz : s + sz;
    n.bwd[2] = (z == 0) ? s + (g.nz - 1) * sz : s - sz;
    n.fwd[3] = (t + 1 == g.nt) ? s - (g.nt - 1) * st : s + st;
    n.bwd[3] = (t == 0) ? s + (g.nt - 1) * st : s - st;
    return n;
}

// ------------------------------------------------------------------ fields
// Spinor field: 12 complex planes (index spin*3 + colour) of stride ldv.
// Gauge field: 4 directions x 9 complex planes (index a*3 + b) of stride ldv.
template <typename R>
struct Spinor {
    Z<R> c[4][3];
};

// Field access: the plane base is wavefront-uniform (scalar registers) and the
// site offset is one 32-bit vector register shared by every load of a thread,
// so the compiler emits the scalar-base form of the global load/store
// instructions (one VGPR of address per thread instead of a 64-bit pointer per
// plane).  Accesses are in range by construction (sites s < V).
struct FieldBase {
    char* p;
};

template <typename R>
__device__ __forceinline__ FieldBase field_base(const Z<R>* base) {
    return FieldBase{reinterpret_cast<char*>(const_cast<Z<R>*>(base))};
}

// The plane address passes through readfirstlane: it is uniform by
// construction, and the intrinsic keeps the compiler from folding the site
// offset into a per-load 64-bit vector address.  The result is a pointer into the
// global address space, so that loads and stores are global instructions (scalar
// base, 32-bit vector offset) rather than flat ones: a flat access takes a 64-bit
// vector address and is counted with the LDS accesses, so a wait for LDS data
// would also wait for it.
#define TSLOV_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ TSLOV_GLOBAL char* uniform_ptr(char* p) {
    const unsigned long long v = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (TSLOV_GLOBAL char*)(((unsigned long long)hi << 32) | lo);
}

template <typename R>
__device__ __forceinline__ Z<R> fload(FieldBase f, int ldv, int pl, unsigned s) {
    const TSLOV_GLOBAL char* plane = uniform_ptr(f.p + (size_t)pl * (size_t)ldv * sizeof(Z<R>));
    const TSLOV_GLOBAL R* q = (const TSLOV_GLOBAL R*)(plane + (size_t)(unsigned)(s * (unsigned)sizeof(Z<R>)));
    return mk<R>(q[0], q[1]);   // one 2-element load
}

// Streaming load: for operands this kernel reads once (an epilogue's own-site
// fields), so that they do not displace from L2 the neighbour spinors and links
// that other blocks of the launch still read.
template <typename R>
__device__ __forceinline__ Z<R> fload_nt(FieldBase f, int ldv, int pl, unsigned s) {
    const TSLOV_GLOBAL char* plane = uniform_ptr(f.p + (size_t)pl * (size_t)ldv * sizeof(Z<R>));
    const TSLOV_GLOBAL R* q = (const TSLOV_GLOBAL R*)(plane + (size_t)(unsigned)(s * (unsigned)sizeof(Z<R>)));
    return mk<R>(__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1));
}

template <typename R>
__device__ __forceinline__ void fstore(FieldBase f, int ldv, int pl, unsigned s, Z<R> v) {
    TSLOV_GLOBAL char* plane = uniform_ptr(f.p + (size_t)pl * (size_t)ldv * sizeof(Z<R>));
    TSLOV_GLOBAL R* q = (TSLOV_GLOBAL R*)(plane + (size_t)(unsigned)(s * (unsigned)sizeof(Z<R>)));
    q[0] = v.re;   // one 2-element store
    q[1] = v.im;
}

// Streaming store: for results that the next reader, a kernel whose blocks sit on
// other XCDs, takes from memory anyway; they then do not displace operands that
// this kernel's neighbouring blocks still read from L2.
template <typename R>
__device__ __forceinline__ void fstore_nt(FieldBase f, int ldv, int pl, unsigned s, Z<R> v) {
    TSLOV_GLOBAL char* plane = uniform_ptr(f.p + (size_t)pl * (size_t)ldv * sizeof(Z<R>));
    TSLOV_GLOBAL R* q = (TSLOV_GLOBAL R*)(plane + (size_t)(unsigned)(s * (unsigned)sizeof(Z<R>)));
    __builtin_nontemporal_store(v.re, q);
    __builtin_nontemporal_store(v.im, q + 1);
}

template <typename R>
__device__ __forceinline__ void load_spinor(Spinor<R>& p, const Z<R>* __restrict__ f, int ldv, int s) {
    const FieldBase r = field_base(f);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) p.c[sp][c] = fload<R>(r, ldv, sp * 3 + c, (unsigned)s);
}

template <typename R>
__device__ __forceinline__ void store_spinor(Z<R>* __restrict__ f, int ldv, int s, const Spinor<R>& p) {
    const FieldBase r = field_base(f);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) fstore<R>(r, ldv, sp * 3 + c, (unsigned)s, p.c[sp][c]);
}

template <typename R>
__device__ __forceinline__ void zero_spinor(Spinor<R>& p) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) p.c[sp][c] = mk<R>(0, 0);
}

// Links may be stored in a narrower type RL than the arithmetic type R (float
// links with double fields); they are widened as they are loaded.
template <typename R, typename RL>
__device__ __forceinline__ void load_link(Z<R> (&u)[3][3], const Z<RL>* __restrict__ U, int ldv, int nu, int s) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) u[a][b] = zcast<R>(fload<RL>(field_base(U), ldv, nu * 9 + a * 3 + b, (unsigned)s));
}

// ------------------------------------------------------------------ spin projection
// Chiral basis: g_k = [[0, -i s_k], [i s_k, 0]], g_4 = [[0, 1], [1, 0]].
// (1 + S g_nu) psi has rank 2: it equals [h; L h] with the half spinor
// h = psi_up + S * (-i s_k or 1) psi_dn and L the lower-block map.  PROJ<NU, S>
// gives h from psi and the two lower spin components from h.
// One colour: (h0, h1) from the spin components (p0, p1, p2, p3).
template <int NU, int S, typename R>
__device__ __forceinline__ void project_col(Z<R> p0, Z<R> p1, Z<R> p2, Z<R> p3, Z<R>& h0, Z<R>& h1) {
    if (NU == 0) {          // -i s_1 psi_dn = (-i p3, -i p2)
        h0 = (S > 0) ? p0 + timesMinusI(p3) : p0 + timesI(p3);
        h1 = (S > 0) ? p1 + timesMinusI(p2) : p1 + timesI(p2);
    } else if (NU == 1) {   // -i s_2 psi_dn = (-p3, p2)
        h0 = (S > 0) ? p0 - p3 : p0 + p3;
        h1 = (S > 0) ? p1 + p2 : p1 - p2;
    } else if (NU == 2) {   // -i s_3 psi_dn = (-i p2, i p3)
        h0 = (S > 0) ? p0 + timesMinusI(p2) : p0 + timesI(p2);
        h1 = (S > 0) ? p1 + timesI(p3) : p1 + timesMinusI(p3);
    } else {                // g_4: psi_dn
        h0 = (S > 0) ? p0 + p2 : p0 - p2;
        h1 = (S > 0) ? p1 + p3 : p1 - p3;
    }
}

template <int NU, int S, typename R>
__device__ __forceinline__ void project(const Spinor<R>& p, Z<R> (&h)[2][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) project_col<NU, S>(p.c[0][c], p.c[1][c], p.c[2][c], p.c[3][c], h[0][c], h[1][c]);
}

// acc += coef * [h; L h]
template <int NU, int S, typename R>
__device__ __forceinline__ void reconstruct_add(Spinor<R>& acc, const Z<R> (&h)[2][3], R coef) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const Z<R> h0 = coef * h[0][c], h1 = coef * h[1][c];
        acc.c[0][c] = acc.c[0][c] + h0;
        acc.c[1][c] = acc.c[1][c] + h1;
        Z<R> l2, l3;
        if (NU == 0) {          // lower = S * i s_1 h = S (i h1, i h0)
            l2 = timesI(h1); l3 = timesI(h0);
        } else if (NU == 1) {   // S * i s_2 h = S (h1, -h0)
            l2 = h1; l3 = -h0;
        } else if (NU == 2) {   // S * i s_3 h = S (i h0, -i h1)
            l2 = timesI(h0); l3 = timesMinusI(h1);
        } else {                // S * h
            l2 = h0; l3 = h1;
        }
        if (S > 0) {
            acc.c[2][c] = acc.c[2][c] + l2;
            acc.c[3][c] = acc.c[3][c] + l3;
        } else {
            acc.c[2][c] = acc.c[2][c] - l2;
            acc.c[3][c] = acc.c[3][c] - l3;
        }
    }
}

template <typename R>
__device__ __forceinline__ void mat_vec(const Z<R> (&u)[3][3], const Z<R> (&h)[2][3], Z<R> (&o)[2][3]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) o[s][a] = u[a][0] * h[s][0] + u[a][1] * h[s][1] + u[a][2] * h[s][2];
}

template <typename R>
__device__ __forceinline__ void adj_mat_vec(const Z<R> (&u)[3][3], const Z<R> (&h)[2][3], Z<R> (&o)[2][3]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) o[s][a] = cjmul(u[0][a], h[s][0]) + cjmul(u[1][a], h[s][1]) + cjmul(u[2][a], h[s][2]);
}

// Forward hop of direction NU into acc:  acc += coef * (1 + g_NU) u psi
template <int NU, typename R>
__device__ __forceinline__ void hop_fwd(Spinor<R>& acc, const Z<R> (&u)[3][3], const Spinor<R>& psi, R coef) {
    Z<R> h[2][3], o[2][3];
    project<NU, +1>(psi, h);
    mat_vec(u, h, o);
    reconstruct_add<NU, +1>(acc, o, coef);
}

// Backward hop of direction NU into acc:  acc += coef * (1 - g_NU) u^dag psi
template <int NU, typename R>
__device__ __forceinline__ void hop_bwd(Spinor<R>& acc, const Z<R> (&u)[3][3], const Spinor<R>& psi, R coef) {
    Z<R> h[2][3], o[2][3];
    project<NU, -1>(psi, h);
    adj_mat_vec(u, h, o);
    reconstruct_add<NU, -1>(acc, o, coef);
}

// ------------------------------------------------------------------ one colour
// Colour layouts: a thread owns colour a of a site.  For a hop it needs the
// neighbour's full half spinor h[2][3] and one row of the (adjoint) link.
template <int NU, int S, typename R>
__device__ __forceinline__ void recon1_add(Z<R> (&acc)[4], const Z<R> (&o)[2], R coef) {
    const Z<R> h0 = coef * o[0], h1 = coef * o[1];
    acc[0] = acc[0] + h0;
    acc[1] = acc[1] + h1;
    Z<R> l2, l3;
    if (NU == 0) { l2 = timesI(h1); l3 = timesI(h0); }
    else if (NU == 1) { l2 = h1; l3 = -h0; }
    else if (NU == 2) { l2 = timesI(h0); l3 = timesMinusI(h1); }
    else { l2 = h0; l3 = h1; }
    if (S > 0) { acc[2] = acc[2] + l2; acc[3] = acc[3] + l3; }
    else { acc[2] = acc[2] - l2; acc[3] = acc[3] - l3; }
}

__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// u . h for one link row and the colour vector of one half spin, as a fixed chain
// of fused multiply-adds.  Written out so that the result does not depend on how
// the compiler would contract a plain expression, which varies with the code that
// produced h (in registers from the projection, or read back from LDS): every hop
// form that uses it gives the same bits.
template <typename R>
__device__ __forceinline__ Z<R> row_dot(const Z<R> (&u)[3], Z<R> h0, Z<R> h1, Z<R> h2) {
    R re = u[0].re * h0.re, im = u[0].re * h0.im;
    re = fmadd(-u[0].im, h0.im, re);
    im = fmadd(u[0].im, h0.re, im);
    re = fmadd(u[1].re, h1.re, re);
    im = fmadd(u[1].re, h1.im, im);
    re = fmadd(-u[1].im, h1.im, re);
    im = fmadd(u[1].im, h1.re, im);
    re = fmadd(u[2].re, h2.re, re);
    im = fmadd(u[2].re, h2.im, im);
    re = fmadd(-u[2].im, h2.im, re);
    im = fmadd(u[2].im, h2.re, im);
    return mk<R>(re, im);
}

// acc += coef * [(1 + S g_NU) u psi]_a with u given by its row a (forward hop,
// u = U_nu(x)) or by conj of its column a (backward hop, u = U_nu(x-nu)^dag).
template <int NU, int S, typename R>
__device__ __forceinline__ void hop1(Z<R> (&acc)[4], const Z<R> (&urow)[3], const Spinor<R>& psi, R coef) {
    Z<R> h[2][3], o[2];
    project<NU, S>(psi, h);
#pragma unroll
    for (int s = 0; s < 2; ++s) o[s] = row_dot(urow, h[s][0], h[s][1], h[s][2]);
    recon1_add<NU, S>(acc, o, coef);
}

template <typename R, typename RL>
__device__ __forceinline__ void load_row(Z<R> (&u)[3], const Z<RL>* __restrict__ U, int ldv, int nu, int a, int s) {
#pragma unroll
    for (int b = 0; b < 3; ++b) u[b] = zcast<R>(fload<RL>(field_base(U), ldv, nu * 9 + a * 3 + b, (unsigned)s));
}

template <typename R, typename RL>
__device__ __forceinline__ void load_col_conj(Z<R> (&u)[3], const Z<RL>* __restrict__ U, int ldv, int nu, int a,
                                              int s) {
#pragma unroll
    for (int b = 0; b < 3; ++b) u[b] = cj(zcast<R>(fload<RL>(field_base(U), ldv, nu * 9 + b * 3 + a, (unsigned)s)));
}

// Colour handled by this thread in the colour split: one wavefront per colour,
// made explicit as a scalar so plane addresses stay uniform.
__device__ __forceinline__ int wave_colour() { return __builtin_amdgcn_readfirstlane(threadIdx.x / kSites); }

// Colour and site block of this thread in a stencil kernel of BLK threads per block:
// BLK = kSites is the colour grid (grid.x = np_colour, colour-major), BLK = kCBlock
// the colour split (grid.x = Geom::nwg, colour = wavefront, site block from
// Geom::sbmap, -1 for a padding workgroup).  A block's partial-sum slot is its
// grid index in the colour grid and its site block in the colour split.
template <int BLK>
__device__ __forceinline__ int sten_colour() {
    if (BLK != kCBlock) return blockIdx.x / (gridDim.x / 3);
    return wave_colour();
}
template <int BLK>
__device__ __forceinline__ int sten_block(const Geom& g) {
    if (BLK != kCBlock) return blockIdx.x % (gridDim.x / 3);
    return g.sbmap[blockIdx.x];
}

// ------------------------------------------------------------------ force contraction
template <typename R>
__device__ __forceinline__ void g5_inplace(Spinor<R>& p) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        p.c[2][c] = -p.c[2][c];
        p.c[3][c] = -p.c[3][c];
    }
}

// Coefficient of dU_nu(x) in Re p^H dH q, H = g5 D_w (both hops of the link):
//   G_ab += sum_{s=0,1} [ e_f hP[s][a] conj(hQ[s][b]) + e_b hQ2[s][a] conj(hP2[s][b]) ]
// with hP = P+(g5 p(x)), hQ = P+(q(x+nu)), hP2 = P-(g5 p(x+nu)), hQ2 = P-(q(x)) the
// half spinors of the (1 +- g_nu) projectors; the caller multiplies by -kappa and
// the boundary sign.
template <int NU, typename R>
__device__ __forceinline__ void force_pair(ZD (&G)[3][3], const Spinor<R>& p_x, const Spinor<R>& q_x,
                                           const Spinor<R>& p_y, const Spinor<R>& q_y, double ef, double eb) {
    Spinor<R> gp_x = p_x, gp_y = p_y;
    g5_inplace(gp_x);
    g5_inplace(gp_y);
    Z<R> hP[2][3], hQ[2][3], hP2[2][3], hQ2[2][3];
    project<NU, +1>(gp_x, hP);
    project<NU, +1>(q_y, hQ);
    project<NU, -1>(gp_y, hP2);
    project<NU, -1>(q_x, hQ2);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            ZD t = mk<double>(0, 0);
#pragma unroll
            for (int sp = 0; sp < 2; ++sp) {
                t = t + ef * mulcj(zcast<double>(hP[sp][a]), zcast<double>(hQ[sp][b]));
                t = t + eb * mulcj(zcast<double>(hQ2[sp][a]), zcast<double>(hP2[sp][b]));
            }
            G[a][b] = G[a][b] + t;
        }
}

// ------------------------------------------------------------------ reductions
// Cross-lane moves of a double: DPP within rows of 16 lanes, lane reads across rows.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __hiloint2double(hi, lo);
}

constexpr int kDppSwap1 = 0xB1;       // quad_perm [1, 0, 3, 2]
constexpr int kDppSwap2 = 0x4E;       // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // lane j <-> 7 - j within 8
constexpr int kDppMirror = 0x140;     // lane j <-> 15 - j within 16

// Wavefront sum, the same bits in every lane and a fixed order: butterflies within
// rows of 16 lanes (both lanes of a pair add the same two operands, so they agree
// exactly), then the four row sums in row order.
__device__ __forceinline__ double wave_sum(double v) {
    v = v + dpp_d<kDppSwap1>(v);
    v = v + dpp_d<kDppSwap2>(v);
    v = v + dpp_d<kDppHalfMirror>(v);
    v = v + dpp_d<kDppMirror>(v);
    return ((readlane_d(v, 0) + readlane_d(v, 16)) + readlane_d(v, 32)) + readlane_d(v, 48);
}

// Block sum of NV values per thread; result valid in every thread.
template <int NV, int BLK>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    __shared__ double red[BLK / kWave][NV];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) red[wave][i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < BLK / kWave; ++w) s += red[w][i];
        v[i] = s;
    }
    __syncthreads();
}

// block_sum for the last use of its LDS slots in a kernel (no other call with the
// same NV follows): the same sums, without the barrier that guards the slots' reuse.
template <int NV, int BLK>
__device__ __forceinline__ void block_sum_last(double (&v)[NV]) {
    __shared__ double red[BLK / kWave][NV];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) red[wave][i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < BLK / kWave; ++w) s += red[w][i];
        v[i] = s;
    }
}

// Sum of per-block partials part[b*NV + i], b < nparts, in a fixed order; every
// block that calls this gets bit-identical results.  gather_partials is the first
// half (each thread's strided share, no barrier), so that a kernel can issue these
// loads together with others and finish the sum with block_sum later.
template <int NV, int BLK>
__device__ __forceinline__ void gather_partials(const double* __restrict__ part, int nparts, double (&out)[NV]) {
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = 0.0;
    for (int b = threadIdx.x; b < nparts; b += BLK)
#pragma unroll
        for (int i = 0; i < NV; ++i) out[i] += part[b * NV + i];
}

template <int NV, int BLK>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nparts, double (&out)[NV]) {
    gather_partials<NV, BLK>(part, nparts, out);
    block_sum<NV, BLK>(out);
}

template <int NV, int BLK>
__device__ __forceinline__ void write_partials(double* __restrict__ part, double (&v)[NV]) {
    block_sum<NV, BLK>(v);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) part[blockIdx.x * NV + i] = v[i];
}

// write_partials_at with block_sum_last (the kernel's last sum with this NV).
template <int NV, int BLK>
__device__ __forceinline__ void write_partials_at_last(double* __restrict__ part, int slot, double (&v)[NV]) {
    block_sum_last<NV, BLK>(v);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) part[slot * NV + i] = v[i];
}

// Same with the partial slot given explicitly (2-D grids).
template <int NV, int BLK>
__device__ __forceinline__ void write_partials_at(double* __restrict__ part, int slot, double (&v)[NV]) {
    block_sum<NV, BLK>(v);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) part[slot * NV + i] = v[i];
}

// Accumulate conj(a) . b over a spinor into (re, im) in double.
template <typename R>
__device__ __forceinline__ void acc_dot(double& re, double& im, const Spinor<R>& a, const Spinor<R>& b) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double ar = a.c[sp][c].re, ai = a.c[sp][c].im, br = b.c[sp][c].re, bi = b.c[sp][c].im;
            re += ar * br + ai * bi;
            im += ar * bi - ai * br;
        }
}

template <typename R>
__device__ __forceinline__ double spinor_norm2(const Spinor<R>& a) {
    double n = 0.0;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) n += (double)a.c[sp][c].re * a.c[sp][c].re + (double)a.c[sp][c].im * a.c[sp][c].im;
    return n;
}

// ------------------------------------------------------------------ scalars
// Device-resident Lanczos coefficients (1-based step index j).
struct Coef {
    ZD* alpha;      // alpha_j = w_j^H H v_j
    double* beta;   // beta_j (beta_1 = |x|)
    ZD* gamma;      // gamma_j (gamma_1 = |x|)
    double* anorm2; // |H v_j|^2
    ZD* h;          // eta^H v_j (derivative mode)
    ZD* c;          // sgn(T) e_1
    ZD* abar_T;     // adjoints seeded by the Frechet step
    double* bbar_T;
    ZD* gbar_T;
    double* bbar_tot;  // beta/gamma adjoints including the recursion's contributions
    ZD* gbar_tot;
    int* status;    // [0] stop flag, [1] k_used, [2] breakdown code, [3] breakdown step
    double* misc;   // [0] |x|, [1] S, [2] mu (Newton scaling), [3] scratch
    int n;          // entries per source of every per-step array (sources are stacked)

    // The coefficient set of batch slot `slot` (per-step arrays of n entries,
    // status and misc of 16 entries per source).
    __host__ __device__ Coef at(int slot) const {
        Coef o = *this;
        const size_t d = (size_t)slot * n, m = (size_t)slot * 16;
        o.alpha += d; o.beta += d; o.gamma += d; o.anorm2 += d; o.h += d; o.c += d;
        o.abar_T += d; o.bbar_T += d; o.gbar_T += d; o.bbar_tot += d; o.gbar_tot += d;
        o.status += m; o.misc += m;
        return o;
    }
};

// Sources of one batched launch: entry e (a grid index) is batch slot slot[e],
// the caller's source src[e], with per-entry size k[e] (a Krylov size) and flag[e].
constexpr int kMaxBatch = 64;
struct SrcList {
    int n;
    int slot[kMaxBatch];
    int src[kMaxBatch];
    int k[kMaxBatch];
    int flag[kMaxBatch];
};

constexpr double kTauLucky = 1e-11;
constexpr double kTauSerious = 1e-14;

}  // namespace tslov
