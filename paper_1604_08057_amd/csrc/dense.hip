// Projected-matrix step on the GPU: sgn(T_k) of the k x k Lanczos matrix by the
// scaled Newton iteration X <- (mu X + X^{-1}/mu)/2, and the Frechet derivative
// L_sgn(T_k, E) from Theorem 1 (the upper-right block of sgn([[T, E], [0, T]])):
// Newton on the block-triangular matrix keeps the form [[X, Y], [0, X]] and
// updates Y <- (mu Y - X^{-1} Y X^{-1} / mu)/2.  The inverse comes from an
// in-place, blocked Gauss-Jordan elimination with partial pivoting: one block
// factors a panel of nb columns in LDS, then all blocks apply the panel's
// transform to the remaining columns; the row permutation is undone by a
// column scatter.  Once the iterate is close to its limit (X^2 ~ 1) the
// inverse-free Newton-Schulz step X <- X (3 - X^2)/2 takes over (quadratically
// convergent there, GEMMs only); on the block matrix it updates
// Y <- [Y (3 - X^2) - X (X Y + Y X)]/2.  All arithmetic is float64 complex.  Every kernel serves a list
// of independent matrices (one per batch entry, sizes k[e] in decreasing order);
// grid dimension z runs over the entries.
#include "kernels.h"

#include <cfloat>
#include <cmath>

namespace tslov {

constexpr int kDB = 256;   // threads per block of the dense kernels

__global__ __launch_bounds__(kDB) void k_dense_build(Coef coef0, SrcList L, int grad, DenseWork w0) {
    const int e = blockIdx.z, slot = L.slot[e], k = L.k[e];
    const Coef coef = coef0.at(slot);
    const DenseWork w = w0.at(slot);
    const int idx = blockIdx.x * kDB + threadIdx.x;
    if (idx >= k * k) return;
    const int i = idx / k, c = idx % k;   // 0-based; Lanczos index j = i + 1
    ZD v = mk<double>(0, 0);
    if (i == c) v = coef.alpha[i + 1];
    else if (i == c + 1) v = mk<double>(coef.beta[i + 1], 0.0);   // T_{j+1,j} = beta_{j+1}
    else if (c == i + 1) v = coef.gamma[c + 1];                   // T_{j,j+1} = gamma_{j+1}
    w.X[idx] = v;
    w.Wk[idx] = v;
    if (grad) w.Y[idx] = (i == 0) ? coef.misc[0] * coef.h[c + 1] : mk<double>(0, 0);  // E = e_1 cbar^H
}

void launch_dense_build(Coef coef, const SrcList& L, int grad, const DenseWork& w, hipStream_t st) {
    const int k = L.k[0];
    hipLaunchKernelGGL(k_dense_build, dim3(grid_for(k * k, kDB), 1, L.n), dim3(kDB), 0, st, coef, L, grad, w);
}

__global__ __launch_bounds__(kDB) void k_dense_load(const ZD* __restrict__ T, const ZD* __restrict__ E, int k,
                                                    DenseWork w) {
    const int idx = blockIdx.x * kDB + threadIdx.x;
    if (idx >= k * k) return;
    w.X[idx] = T[idx];
    w.Wk[idx] = T[idx];
    if (E) w.Y[idx] = E[idx];
}

void launch_dense_load(const ZD* T, const ZD* E, int k, const DenseWork& w, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_load, dim3(grid_for(k * k, kDB)), dim3(kDB), 0, st, T, E, k, w);
}

// ------------------------------------------------------------------ Gauss-Jordan
__global__ __launch_bounds__(kDB) void k_rowperm_init(SrcList L, DenseWork w0) {
    const int e = blockIdx.z;
    const DenseWork w = w0.at(L.slot[e]);
    const int i = blockIdx.x * kDB + threadIdx.x;
    if (i < L.k[e]) w.rowperm[i] = i;
}

template <int CTRL>
__device__ __forceinline__ void dpp_argmax_step(double& v, int& i) {
    const double ov = dpp_d<CTRL>(v);
    const int oi = __builtin_amdgcn_update_dpp(0, i, CTRL, 0xf, 0xf, false);
    if (ov > v || (ov == v && oi < i)) {
        v = ov;
        i = oi;
    }
}

// Largest v over the wavefront (smallest i among equal v), returned in every lane.
// Rows of 16 lanes combine through DPP (swap within pairs, within quads, mirror
// within halves of 8, mirror within 16); the four rows through lane reads.
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
    dpp_argmax_step<kDppSwap1>(v, i);
    dpp_argmax_step<kDppSwap2>(v, i);
    dpp_argmax_step<kDppHalfMirror>(v, i);
    dpp_argmax_step<kDppMirror>(v, i);
    double bv = readlane_d(v, 0);
    int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
    for (int r = 16; r < kWave; r += 16) {
        const double ov = readlane_d(v, r);
        const int oi = __builtin_amdgcn_readlane(i, r);
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    v = bv;
    i = bi;
}

// Pivot candidate key of the register panel: |P[i][q]|^2 (at most DBL_MAX) with its
// low 9 mantissa bits replaced by 511 - i.  Non-negative doubles order like their
// bit patterns, so the largest key is the largest value (to 2^-43 relative) and,
// among values equal to that precision, the smallest row index; rows that are not
// candidates take -1.  One v_max_f64 per reduction stage instead of a value and an
// index compared and selected.
__device__ __forceinline__ double gj_key(double m, int row) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(std::fmin(m, DBL_MAX));
    return __longlong_as_double((long long)((b & ~0x1FFull) | (unsigned long long)(511 - row)));
}
__device__ __forceinline__ int gj_key_row(double key) { return 511 - (int)(__double_as_longlong(key) & 0x1FF); }

// Largest v over the wavefront, in every lane (rows of 16 through DPP, then lane reads).
__device__ __forceinline__ double wave_max_d(double v) {
    v = std::fmax(v, dpp_d<kDppSwap1>(v));
    v = std::fmax(v, dpp_d<kDppSwap2>(v));
    v = std::fmax(v, dpp_d<kDppHalfMirror>(v));
    v = std::fmax(v, dpp_d<kDppMirror>(v));
    return std::fmax(std::fmax(readlane_d(v, 0), readlane_d(v, 16)), std::fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// Panel K: columns [c0, c0 + nbK) of Wk, all k rows, held in LDS and factored by
// one block of four wavefronts; thread t owns rows t, t + 256, ...  For each pivot
// p = c0 + q: the largest |P[i][q]| over rows i >= p (smallest index on ties) is
// the pivot row imax; with inv = 1/P[imax][q] and prow = P[imax] * inv,
//   new row p    = prow with column q set to inv,
//   new row imax = old row p - f prow,  f = old P[p][q]   (the row swap),
//   new row i    = row i - f prow,       f = P[i][q]   (other rows),
// and in every eliminated row column q becomes -f inv (in-place Gauss-Jordan: the
// column then holds the transform's column).  All reads of a pivot step precede
// its writes, so two block barriers per pivot suffice; no global memory traffic
// happens inside the loop (a barrier would wait for it).
template <int NB>
__global__ __launch_bounds__(kDB) void k_gj_panel(DenseWork w0, SrcList L, int c0) {
    extern __shared__ ZD P[];   // k rows of stride NB + 1 (odd: spreads rows over the LDS banks)
    constexpr int LD = NB + 1;
    const int e = blockIdx.z, k = L.k[e];
    if (c0 >= k) return;
    const DenseWork w = w0.at(L.slot[e]);
    ZD* __restrict__ Wk = w.Wk;
    int* __restrict__ rowperm = w.rowperm;
    int* __restrict__ ipiv = w.rowperm + w.kcap;
    int* perm = reinterpret_cast<int*>(P + (size_t)k * LD);
    __shared__ int piv_s[NB];
    __shared__ double wbest[kDB / kWave];
    __shared__ int wi[kDB / kWave];
    const int tid = threadIdx.x;
    const int nbK = min(NB, k - c0);
    for (int i = tid; i < k; i += kDB) perm[i] = rowperm[i];
#pragma unroll 8
    for (int x = tid; x < k * NB; x += kDB) {
        const int i = x / NB, q = x % NB;
        P[i * LD + q] = Wk[(size_t)i * k + c0 + (q < nbK ? q : nbK - 1)];
    }
    __syncthreads();
    for (int q = 0; q < nbK; ++q) {
        const int p = c0 + q;
        double best = -1.0;
        int bi = k;
        for (int i = tid; i < k; i += kDB) {
            const double m = (i >= p) ? norm2(P[i * LD + q]) : -1.0;
            if (m > best) { best = m; bi = i; }
        }
        wave_argmax(best, bi);
        if (tid % kWave == 0) { wbest[tid / kWave] = best; wi[tid / kWave] = bi; }
        __syncthreads();
        double b = wbest[0];
        int imax = wi[0];
#pragma unroll
        for (int v = 1; v < kDB / kWave; ++v)
            if (wbest[v] > b || (wbest[v] == b && wi[v] < imax)) { b = wbest[v]; imax = wi[v]; }
        if (imax < p || imax >= k) imax = p;   // non-finite column: keep the order, the NaN propagates
        // reads: pivot row (all threads), old row p (owner of row imax), own rows' factors
        const ZD inv = zdiv(mk<double>(1.0, 0.0), P[imax * LD + q]);
        ZD prow[NB];
#pragma unroll
        for (int qq = 0; qq < NB; ++qq) prow[qq] = P[imax * LD + qq] * inv;
        ZD rowp[NB];
        ZD fp = mk<double>(0, 0);
        const bool own_imax = (imax != p) && (imax % kDB == tid);
        if (own_imax) {   // old row p is overwritten after the barrier: read it now
#pragma unroll
            for (int qq = 0; qq < NB; ++qq) rowp[qq] = P[p * LD + qq];
            fp = P[p * LD + q];
        }
        if (tid == 0) {
            piv_s[q] = imax;
            if (imax != p) {
                const int t = perm[p];
                perm[p] = perm[imax];
                perm[imax] = t;
            }
        }
        __syncthreads();
        for (int i = tid; i < k; i += kDB) {
            if (i == p) {
#pragma unroll
                for (int qq = 0; qq < NB; ++qq) P[i * LD + qq] = prow[qq];
                P[i * LD + q] = inv;
            } else {
                ZD row[NB];
                if (i == imax) {
#pragma unroll
                    for (int qq = 0; qq < NB; ++qq) row[qq] = rowp[qq];
                } else {
#pragma unroll
                    for (int qq = 0; qq < NB; ++qq) row[qq] = P[i * LD + qq];
                }
                const ZD f = (i == imax) ? fp : P[i * LD + q];
#pragma unroll
                for (int qq = 0; qq < NB; ++qq) P[i * LD + qq] = row[qq] - f * prow[qq];
                P[i * LD + q] = -(f * inv);
            }
        }
        __syncthreads();
    }
    if (tid < nbK) ipiv[c0 + tid] = piv_s[tid];
    for (int i = tid; i < k; i += kDB) rowperm[i] = perm[i];
#pragma unroll 8
    for (int x = tid; x < k * NB; x += kDB) {
        const int i = x / NB, q = x % NB;
        if (q < nbK) Wk[(size_t)i * k + c0 + q] = P[i * LD + q];
    }
}

// Register-resident panel for k <= BLK: the same elimination as k_gj_panel, each
// thread of a BLK-thread block holding one row of the panel in registers.  One
// block barrier per pivot: before it, each wavefront publishes its best candidate
// row (the largest candidate key of gj_key) in LDS slots that alternate
// between even and odd pivots; after it, every thread picks the block's pivot from
// the candidates and updates its own row as row - (f / P[imax][q]) P[imax].  The
// row exchange moves no data: threads carry the index of the row they hold, the
// pivot row's thread takes index p and the old row p's thread index imax (whose
// update, with its own f, is the exchanged row's).  Rows are written back under
// their final indices.  The pivot is the unique maximum under that order, so the
// result does not depend on BLK.  A column without a finite candidate makes every
// row NaN (the matrix has no usable inverse; the caller's finiteness check reports it).
constexpr int kGjRegMax = 512;   // largest k served by the register-resident panel

template <int NB, int BLK>
__global__ __launch_bounds__(BLK) void k_gj_panel_reg(DenseWork w0, SrcList L, int c0) {
    constexpr int kNW = BLK / kWave;
    static_assert(BLK <= 512, "candidate keys hold 9 bits of row index");
    __shared__ ZD cand[2][kNW][NB];
    __shared__ double cval[2][kNW];
    __shared__ int perm[BLK];
    __shared__ int piv_s[NB];
    const int e = blockIdx.z, k = L.k[e];
    if (c0 >= k) return;
    const DenseWork w = w0.at(L.slot[e]);
    ZD* __restrict__ Wk = w.Wk;
    int* __restrict__ rowperm = w.rowperm;
    int* __restrict__ ipiv = w.rowperm + w.kcap;
    const int i = threadIdx.x, wave = i / kWave, lane = i % kWave;
    const bool mine = i < k;   // this thread holds a row
    int lr = i;                // the index of the row it holds
    const int nbK = min(NB, k - c0);
    if (mine) perm[i] = rowperm[i];
    ZD row[NB];
#pragma unroll
    for (int qq = 0; qq < NB; ++qq) row[qq] = (mine && qq < nbK) ? Wk[(size_t)i * k + c0 + qq] : mk<double>(0, 0);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        if (q < nbK) {   // uniform; the loop unrolls fully so that row[q] stays in registers
            const int p = c0 + q, b = q & 1;
            const double m = norm2(row[q]);
            const double key = (mine && lr >= p && m >= 0.0) ? gj_key(m, lr) : -1.0;   // NaN: never a candidate
            const double wbest = wave_max_d(key);
            if (lane == 0) cval[b][wave] = wbest;
            if (wbest >= 0.0 && key == wbest)   // keys are unique: the wavefront's candidate
#pragma unroll
                for (int qq = 0; qq < NB; ++qq) cand[b][wave][qq] = row[qq];
            __syncthreads();
            // all candidates in one round of LDS reads, then a branch-free choice
            double cv[kNW];
#pragma unroll
            for (int v = 0; v < kNW; ++v) cv[v] = cval[b][v];
            double bv = cv[0];
            int wwin = 0;
#pragma unroll
            for (int v = 1; v < kNW; ++v) {
                const bool t = cv[v] > bv;
                bv = t ? cv[v] : bv;
                wwin = t ? v : wwin;
            }
            const int imax = bv >= 0.0 ? gj_key_row(bv) : k;
            const bool valid = imax >= p && imax < k;
            if (i == 0) piv_s[q] = valid ? imax : p;
            if (!valid) {   // uniform
#pragma unroll
                for (int qq = 0; qq < NB; ++qq) row[qq] = mk<double>(__builtin_nan(""), __builtin_nan(""));
                continue;
            }
            const ZD* __restrict__ src = &cand[b][wwin][0];
            const ZD inv = zdiv(mk<double>(1.0, 0.0), src[q]);
            if (mine && lr == imax) {   // the pivot row becomes row p
#pragma unroll
                for (int qq = 0; qq < NB; ++qq) row[qq] = row[qq] * inv;
                row[q] = inv;
                lr = p;
            } else if (mine) {
                if (lr == p) lr = imax;   // the old row p takes the pivot row's place
                ZD piv[NB];
#pragma unroll
                for (int qq = 0; qq < NB; ++qq) piv[qq] = src[qq];
                const ZD f = row[q] * inv;
#pragma unroll
                for (int qq = 0; qq < NB; ++qq) row[qq] = row[qq] - f * piv[qq];
                row[q] = -f;
            }
        }
    }
    __syncthreads();
    if (i == 0)
        for (int q = 0; q < nbK; ++q) {
            const int p = c0 + q, im = piv_s[q];
            ipiv[p] = im;
            if (im != p) {
                const int t = perm[p];
                perm[p] = perm[im];
                perm[im] = t;
            }
        }
    if (mine)
#pragma unroll
        for (int qq = 0; qq < NB; ++qq)
            if (qq < nbK) Wk[(size_t)lr * k + c0 + qq] = row[qq];
    __syncthreads();
    if (mine) rowperm[i] = perm[i];
}

// Apply panel K's row swaps and transform to TC columns outside the panel:
// x <- swaps(x);  x_new[i] = [i outside panel] x[i] + sum_q P[i][q] x[c0 + q].
// Thread t owns rows i = t, t + 256, ... of the block's TC columns.  Any k: the
// columns are staged in LDS and swapped there.
template <int NB>
__global__ __launch_bounds__(kDB) void k_gj_trailing_staged(DenseWork w0, SrcList L, int c0, int TC) {
    extern __shared__ ZD smem[];
    const int e = blockIdx.z, k = L.k[e];
    if (c0 >= k) return;
    const int nbK = min(NB, k - c0);
    const int nother = k - nbK;
    const int cid0 = blockIdx.x * TC;
    const int tcv = min(TC, nother - cid0);
    if (tcv <= 0) return;
    const DenseWork w = w0.at(L.slot[e]);
    ZD* __restrict__ Wk = w.Wk;
    const int* __restrict__ ipiv = w.rowperm + w.kcap;
    const int LT = TC + 1;      // odd row stride: rows spread over the LDS banks
    ZD* xs = smem;              // k rows of stride LT
    ZD* xp = smem + k * LT;     // nbK * TC
    const int tid = threadIdx.x;
    // flat, unrolled staging (TC is a power of two): columns past the last valid
    // one are clamped instead of branched around, so loads stay in flight
    const int sh = __builtin_ctz(TC);
#pragma unroll 8
    for (int x = tid; x < k * TC; x += kDB) {
        const int i = x >> sh, t = x & (TC - 1);
        const int cid = cid0 + (t < tcv ? t : tcv - 1);
        const int c = cid < c0 ? cid : cid + nbK;
        xs[i * LT + t] = Wk[(size_t)i * k + c];
    }
    __syncthreads();
    if (tid < tcv) {
        for (int q = 0; q < nbK; ++q) {
            const int p = c0 + q, im = ipiv[p];
            if (im != p) {
                const ZD t = xs[p * LT + tid];
                xs[p * LT + tid] = xs[im * LT + tid];
                xs[im * LT + tid] = t;
            }
        }
    }
    __syncthreads();
    if (tid < tcv)
        for (int q = 0; q < nbK; ++q) xp[q * TC + tid] = xs[(c0 + q) * LT + tid];
    __syncthreads();
    for (int i = tid; i < k; i += kDB) {
        const bool inblk = i >= c0 && i < c0 + nbK;
        const ZD* prow = Wk + (size_t)i * k + c0;
        ZD pr[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) pr[q] = (q < nbK) ? prow[q] : mk<double>(0, 0);
        for (int t = 0; t < tcv; ++t) {
            ZD acc = inblk ? mk<double>(0, 0) : xs[i * LT + t];
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (q < nbK) acc = acc + pr[q] * xp[q * TC + t];
            const int cid = cid0 + t;
            const int c = cid < c0 ? cid : cid + nbK;
            Wk[(size_t)i * k + c] = acc;
        }
    }
}

// The same for k <= BLK (thread i owns row i): the swaps are not carried out.  Row
// i of the swapped column is row src(i) of the stored one, found by undoing the
// panel's exchanges in reverse order; every global load (panel row, the row's
// column entries, the pivot rows' entries) is issued before the one block barrier,
// and every entry is read before any is written.  Same arithmetic, same order.
__device__ __forceinline__ int gj_swapped_row(int i, const int* __restrict__ ipiv, int c0, int nbK) {
    int src = i;
    for (int q = nbK - 1; q >= 0; --q) {
        const int p = c0 + q, im = ipiv[p];
        src = src == p ? im : (src == im ? p : src);
    }
    return src;
}

constexpr int kTrailTC = 16;   // largest TC of the register trailing kernel

template <int NB, int BLK>
__global__ __launch_bounds__(BLK) void k_gj_trailing(DenseWork w0, SrcList L, int c0, int TC) {
    __shared__ ZD xp[NB * kTrailTC];   // the pivot rows' entries of the swapped columns
    const int e = blockIdx.z, k = L.k[e];
    if (c0 >= k) return;
    const int nbK = min(NB, k - c0);
    const int nother = k - nbK;
    const int cid0 = blockIdx.x * TC;
    const int tcv = min(TC, nother - cid0);
    if (tcv <= 0) return;
    const DenseWork w = w0.at(L.slot[e]);
    ZD* __restrict__ Wk = w.Wk;
    const int* __restrict__ ipiv = w.rowperm + w.kcap;
    const int i = threadIdx.x;
    auto col = [&](int t) {
        const int cid = cid0 + t;
        return cid < c0 ? cid : cid + nbK;
    };
    if (i < nbK * tcv) {
        const int q = i / tcv, t = i % tcv;
        xp[q * kTrailTC + t] = Wk[(size_t)gj_swapped_row(c0 + q, ipiv, c0, nbK) * k + col(t)];
    }
    const bool mine = i < k;
    const bool inblk = i >= c0 && i < c0 + nbK;
    const int src = mine ? gj_swapped_row(i, ipiv, c0, nbK) : 0;
    const ZD* prow = Wk + (size_t)(mine ? i : 0) * k + c0;
    ZD pr[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) pr[q] = (q < nbK) ? prow[q] : mk<double>(0, 0);
    ZD xv[kTrailTC];
#pragma unroll
    for (int t = 0; t < kTrailTC; ++t)
        xv[t] = (mine && !inblk && t < tcv) ? Wk[(size_t)src * k + col(t)] : mk<double>(0, 0);
    __syncthreads();
    if (mine)
#pragma unroll
        for (int t = 0; t < kTrailTC; ++t)
            if (t < tcv) {
                ZD acc = xv[t];
#pragma unroll
                for (int q = 0; q < NB; ++q)
                    if (q < nbK) acc = acc + pr[q] * xp[q * kTrailTC + t];
                Wk[(size_t)i * k + col(t)] = acc;
            }
}

// X^{-1}[:, rowperm[i]] = Wk[:, i], with per-block partials of |X^{-1}|_F^2 and |X|_F^2.
__global__ __launch_bounds__(kDB) void k_dense_scatter(DenseWork w0, SrcList L) {
    const int e = blockIdx.z, k = L.k[e];
    const DenseWork w = w0.at(L.slot[e]);
    const int idx = blockIdx.x * kDB + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (idx < k * k) {
        const int r = idx / k, i = idx % k;
        const ZD x = w.Wk[idx];
        w.Xinv[(size_t)r * k + w.rowperm[i]] = x;
        v[0] = norm2(x);
        v[1] = norm2(w.X[idx]);
    }
    write_partials<2, kDB>(w.part + 2 * w.npart_max, v);
}

// Largest column sum of |x| (the 1-norm) of X^{-1} and of X, per block of 16
// columns: sixteen row groups sum a column, the group sums are added in group order,
// then the block takes the maximum over its columns.
__global__ __launch_bounds__(kDB) void k_dense_colnorm(DenseWork w0, SrcList L) {
    __shared__ double cs[2][16][17];
    const int e = blockIdx.z, k = L.k[e];
    const DenseWork w = w0.at(L.slot[e]);
    const int tx = threadIdx.x % 16, grp = threadIdx.x / 16;
    const int c = blockIdx.x * 16 + tx;
    double si = 0.0, sx = 0.0;
    if (c < k)
#pragma unroll 4
        for (int r = grp; r < k; r += 16) {
            si += std::sqrt(norm2(w.Xinv[(size_t)r * k + c]));
            sx += std::sqrt(norm2(w.X[(size_t)r * k + c]));
        }
    cs[0][grp][tx] = si;
    cs[1][grp][tx] = sx;
    __syncthreads();
    if (threadIdx.x < 16) {   // lanes 0-15 of wavefront 0: column sums, then their maximum
        double mi = 0.0, mx = 0.0;
#pragma unroll
        for (int g = 0; g < 16; ++g) {
            mi += cs[0][g][tx];
            mx += cs[1][g][tx];
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
            mi = std::fmax(mi, __shfl_xor(mi, o, 16));
            mx = std::fmax(mx, __shfl_xor(mx, o, 16));
        }
        if (tx == 0) {
            double* q = w.part + 5 * w.npart_max + 8 + 2 * blockIdx.x;
            q[0] = mi;
            q[1] = mx;
        }
    }
}

// Newton scaling while it is on (flag), else 1: mu = sqrt(mu_F mu_1), the geometric
// mean of the Frobenius-norm scaling mu_F = sqrt(|X^{-1}|_F / |X|_F) and the 1-norm
// scaling mu_1 = sqrt(|X^{-1}|_1 / |X|_1).  Either alone is a cheap stand-in for the
// spectral-norm scaling; their mean needs fewer inverse-based steps than either on the
// Krylov matrices of the lattice workloads.
__global__ __launch_bounds__(kDB) void k_dense_mu(DenseWork w0, SrcList L, int npart, int ncb) {
    const int e = blockIdx.z;
    const DenseWork w = w0.at(L.slot[e]);
    double red[2];
    reduce_partials<2, kDB>(w.part + 2 * w.npart_max, npart, red);
    if (threadIdx.x == 0) {
        const double* q = w.part + 5 * w.npart_max + 8;
        double n1i = 0.0, n1x = 0.0;
        for (int b = 0; b < ncb; ++b) {
            n1i = std::fmax(n1i, q[2 * b]);
            n1x = std::fmax(n1x, q[2 * b + 1]);
        }
        const double mf = std::sqrt(std::sqrt(red[0] / red[1])), m1 = std::sqrt(n1i / n1x);
        w.part[4 * w.npart_max] = L.flag[e] ? std::sqrt(mf * m1) : 1.0;
    }
}

// ------------------------------------------------------------------ complex GEMM
// Operands by index into the entry's matrices: 0 X, 1 Y, 2 Wk, 3 Xinv, 4 Zt, 5 Y2, 6 P2, 7 Y3.
__device__ __forceinline__ ZD* dmat(const DenseWork& w, int i) {
    switch (i) {
        case 0: return w.X;
        case 1: return w.Y;
        case 2: return w.Wk;
        case 3: return w.Xinv;
        case 4: return w.Zt;
        case 5: return w.Y2;
        case 6: return w.P2;
        default: return w.Y3;
    }
}
enum { kMX = 0, kMY = 1, kMWk = 2, kMXinv = 3, kMZt = 4, kMY2 = 5, kMP2 = 6, kMY3 = 7 };

// C = a (A B) + b D (D may be C; A, B must not be C).  mode 1 instead forms the
// Newton Frechet update C <- (mu C - (A B)/mu)/2 with mu read from the device.
// 16 x 16 output tiles, one output per thread, 16-deep LDS tiles of A and B.
__global__ __launch_bounds__(kDB) void k_zgemm(DenseWork w0, SrcList L, int ia, int ib, int ic, int id, double a,
                                               double b, int mode) {
    __shared__ ZD As[16][17];
    __shared__ ZD Bs[16][17];
    const int e = blockIdx.z, k = L.k[e];
    if ((int)blockIdx.x * 16 >= k || (int)blockIdx.y * 16 >= k) return;
    const DenseWork w = w0.at(L.slot[e]);
    const ZD* __restrict__ A = dmat(w, ia);
    const ZD* __restrict__ B = dmat(w, ib);
    ZD* C = dmat(w, ic);
    const ZD* D = dmat(w, id);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int r = blockIdx.y * 16 + ty, c = blockIdx.x * 16 + tx;
    ZD acc = mk<double>(0, 0);
    for (int kk = 0; kk < k; kk += 16) {
        As[ty][tx] = (r < k && kk + tx < k) ? A[(size_t)r * k + kk + tx] : mk<double>(0, 0);
        Bs[ty][tx] = (kk + ty < k && c < k) ? B[(size_t)(kk + ty) * k + c] : mk<double>(0, 0);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) acc = acc + As[ty][q] * Bs[q][tx];
        __syncthreads();
    }
    if (r < k && c < k) {
        const size_t o = (size_t)r * k + c;
        if (mode == 1) {
            const double mu = w.part[4 * w.npart_max];
            C[o] = 0.5 * (mu * C[o] - (1.0 / mu) * acc);
        } else {
            ZD v = a * acc;
            if (b != 0.0) v = v + b * D[o];
            C[o] = v;
        }
    }
}

// Several outputs of one inverse-free step in one launch: grid dimension z runs
// over (entry, output) pairs.  Output o forms C = a (A B) + b D, where B is the sum
// of two matrices, taken as its tiles load, when ibs >= 0 (A, B, Bs must not be C;
// D may be C).  Same tiles as k_zgemm.
struct GemmOut {
    int ia, ib, ibs, ic, id;
    double a, b;
};
struct GemmOuts {
    GemmOut o0, o1, o2;
    int n;
};

__global__ __launch_bounds__(kDB) void k_zgemm_outs(DenseWork w0, SrcList L, GemmOuts outs) {
    __shared__ ZD As[16][17], Bs[16][17];
    const int e = (int)blockIdx.z / outs.n, k = L.k[e];
    if ((int)blockIdx.x * 16 >= k || (int)blockIdx.y * 16 >= k) return;
    const int o = (int)blockIdx.z % outs.n;   // uniform: each field picked without indexing
    auto pick = [&](int f0, int f1, int f2) { return o == 0 ? f0 : (o == 1 ? f1 : f2); };
    auto pickd = [&](double f0, double f1, double f2) { return o == 0 ? f0 : (o == 1 ? f1 : f2); };
    const int ia = pick(outs.o0.ia, outs.o1.ia, outs.o2.ia), ib = pick(outs.o0.ib, outs.o1.ib, outs.o2.ib);
    const int ibs = pick(outs.o0.ibs, outs.o1.ibs, outs.o2.ibs);
    const int ic = pick(outs.o0.ic, outs.o1.ic, outs.o2.ic), id = pick(outs.o0.id, outs.o1.id, outs.o2.id);
    const double a = pickd(outs.o0.a, outs.o1.a, outs.o2.a), b = pickd(outs.o0.b, outs.o1.b, outs.o2.b);
    const DenseWork w = w0.at(L.slot[e]);
    const bool sum = ibs >= 0;
    const ZD* __restrict__ A = dmat(w, ia);
    const ZD* __restrict__ B = dmat(w, ib);
    const ZD* __restrict__ B2 = dmat(w, sum ? ibs : ib);
    ZD* C = dmat(w, ic);
    const ZD* D = dmat(w, id);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int r = blockIdx.y * 16 + ty, c = blockIdx.x * 16 + tx;
    ZD acc = mk<double>(0, 0);
    for (int kk = 0; kk < k; kk += 16) {
        const bool rb = kk + ty < k && c < k;
        As[ty][tx] = (r < k && kk + tx < k) ? A[(size_t)r * k + kk + tx] : mk<double>(0, 0);
        const size_t ob = (size_t)(kk + ty) * k + c;
        Bs[ty][tx] = rb ? (sum ? B[ob] + B2[ob] : B[ob]) : mk<double>(0, 0);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) acc = acc + As[ty][q] * Bs[q][tx];
        __syncthreads();
    }
    if (r < k && c < k) {
        const size_t oc = (size_t)r * k + c;
        ZD v = a * acc;
        if (b != 0.0) v = v + b * D[oc];
        C[oc] = v;
    }
}

// X <- (mu X + X^{-1}/mu)/2, copy into Wk for the next inversion, partials of
// |X_new - X|^2 and |X_new|^2.
__global__ __launch_bounds__(kDB) void k_dense_update(DenseWork w0, SrcList L) {
    const int e = blockIdx.z, k = L.k[e];
    const DenseWork w = w0.at(L.slot[e]);
    const int idx = blockIdx.x * kDB + threadIdx.x;
    const double mu = w.part[4 * w.npart_max];
    double v[2] = {0.0, 0.0};
    if (idx < k * k) {
        const ZD x = w.X[idx];
        const ZD xn = 0.5 * (mu * x + (1.0 / mu) * w.Xinv[idx]);
        v[0] = norm2(xn - x);
        v[1] = norm2(xn);
        w.X[idx] = xn;
        w.Wk[idx] = xn;
    }
    write_partials<2, kDB>(w.part, v);
}

__global__ __launch_bounds__(kDB) void k_dense_delta(DenseWork w0, SrcList L, int npart) {
    const int e = blockIdx.z;
    const DenseWork w = w0.at(L.slot[e]);
    double red[2];
    reduce_partials<2, kDB>(w.part, npart, red);
    if (threadIdx.x == 0) {
        w.delta[0] = red[0];
        w.delta[1] = red[1];
    }
}

// Panel launches for the active entries (sorted by decreasing k): entries with
// k > kGjRegMax use the LDS panel, the rest the register-resident one (whose result
// does not depend on how many rows each thread holds).
template <int NB>
void launch_panels(const SrcList& act, int c0, size_t panel_lds, const DenseWork& w, hipStream_t st) {
    int m = 0;
    while (m < act.n && act.k[m] > kGjRegMax) ++m;
    if (m > 0) {
        SrcList big = act;
        big.n = m;
        hipLaunchKernelGGL(k_gj_panel<NB>, dim3(1, 1, m), dim3(kDB), panel_lds, st, w, big, c0);
    }
    if (m < act.n) {
        SrcList small{};
        small.n = act.n - m;
        for (int e = 0; e < small.n; ++e) {
            small.slot[e] = act.slot[m + e];
            small.src[e] = act.src[m + e];
            small.k[e] = act.k[m + e];
            small.flag[e] = act.flag[m + e];
        }
        if (small.k[0] > kDB)
            hipLaunchKernelGGL((k_gj_panel_reg<NB, 2 * kDB>), dim3(1, 1, small.n), dim3(2 * kDB), 0, st, w, small, c0);
        else
            hipLaunchKernelGGL((k_gj_panel_reg<NB, kDB>), dim3(1, 1, small.n), dim3(kDB), 0, st, w, small, c0);
    }
}

template <int NB>
void gj_sweep(const SrcList& L, int TC, size_t panel_lds, const DenseWork& w, hipStream_t st) {
    const int kmax = L.k[0];
    SrcList act = L;
    for (int c0 = 0; c0 < kmax; c0 += NB) {
        while (act.n > 0 && act.k[act.n - 1] <= c0) --act.n;   // entries sorted by decreasing k
        launch_panels<NB>(act, c0, panel_lds, w, st);
        const int nbK = (kmax - c0) < NB ? (kmax - c0) : NB;
        const int nother = kmax - nbK;
        if (nother > 0) {
            if (kmax <= kDB && TC <= kTrailTC) {
                hipLaunchKernelGGL((k_gj_trailing<NB, kDB>), dim3(grid_for(nother, TC), 1, act.n), dim3(kDB), 0, st,
                                   w, act, c0, TC);
            } else if (kmax <= 2 * kDB && TC <= kTrailTC) {
                hipLaunchKernelGGL((k_gj_trailing<NB, 2 * kDB>), dim3(grid_for(nother, TC), 1, act.n), dim3(2 * kDB),
                                   0, st, w, act, c0, TC);
            } else {
                const size_t tl = (size_t)(kmax * (TC + 1) + NB * TC) * sizeof(ZD);
                hipLaunchKernelGGL(k_gj_trailing_staged<NB>, dim3(grid_for(nother, TC), 1, act.n), dim3(kDB), tl, st,
                                   w, act, c0, TC);
            }
        }
    }
}

// Inverse of a tridiagonal X (the first Newton step, X = T_k): Gaussian elimination
// with partial pivoting on the band (thread 0, O(k), operands staged in LDS; a row
// exchange puts a second superdiagonal into U), then one forward and back
// substitution per column of the identity (thread c, O(k)), written straight into
// Xinv; the back substitution reads its stored column in batches of kTriBatch so
// that the loads overlap.  Also the partials of |X^{-1}|_F^2 and |X|_F^2 for the
// scaling (slot 0 of the scatter partials).
// Dynamic LDS: k x (diagonal, sub- and superdiagonal of X, multiplier, 1/diagonal,
// first and second superdiagonal of U) + k flags.
constexpr int kTriBatch = 16;

__device__ __forceinline__ ZD zrcp(ZD d) { return (1.0 / norm2(d)) * cj(d); }

__global__ __launch_bounds__(kDB) void k_tridiag_inv(DenseWork w0, SrcList L) {
    extern __shared__ ZD tb[];
    const int e = blockIdx.z, k = L.k[e];
    if (k <= 0) return;   // empty entries never reach the dense step; keep the indexing safe anyway
    const DenseWork w = w0.at(L.slot[e]);
    ZD* dg = tb;             // X[i][i]
    ZD* lo = tb + k;         // X[i+1][i]
    ZD* hi = tb + 2 * k;     // X[i][i+1]
    ZD* mlt = tb + 3 * k;    // elimination multipliers
    ZD* idd = tb + 4 * k;    // 1 / diagonal of U
    ZD* du = tb + 5 * k;     // first superdiagonal of U
    ZD* u2 = tb + 6 * k;     // second superdiagonal of U (from row exchanges)
    int* swp = reinterpret_cast<int*>(tb + 7 * k);
    const ZD* X = w.X;
    const ZD zero = mk<double>(0, 0);
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < k; i += kDB) {
        dg[i] = X[(size_t)i * k + i];
        lo[i] = i + 1 < k ? X[(size_t)(i + 1) * k + i] : zero;
        hi[i] = i + 1 < k ? X[(size_t)i * k + i + 1] : zero;
        v[1] += norm2(dg[i]) + norm2(lo[i]) + norm2(hi[i]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ZD d = dg[0], up = hi[0];   // running row i: X-entries at columns i and i+1
        // step i's band values, each step reading the next one's before its own
        // stores (the band is never written here), so no LDS round trip sits on the chain
        ZD l = lo[0], dn = dg[k > 1 ? 1 : 0], un = hi[k > 1 ? 1 : 0];
        for (int i = 0; i + 1 < k; ++i) {
            const int in = i + 2 < k ? i + 1 : i;   // the last step reads in-range dummies
            const ZD l_n = lo[in], dn_n = dg[in + 1], un_n = hi[in + 1];
            if (norm2(l) > norm2(d)) {   // exchange rows i and i+1
                const ZD r = zrcp(l), m = d * r;
                mlt[i] = m;
                swp[i] = 1;
                idd[i] = r;
                du[i] = dn;
                u2[i] = un;
                d = up - m * dn;
                up = zero - m * un;
            } else {
                const ZD r = zrcp(d), m = l * r;
                mlt[i] = m;
                swp[i] = 0;
                idd[i] = r;
                du[i] = up;
                u2[i] = zero;
                d = dn - m * up;
                up = un;
            }
            l = l_n;
            dn = dn_n;
            un = un_n;
        }
        idd[k - 1] = zrcp(d);
        du[k - 1] = zero;
        u2[k - 1] = zero;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < k; c += kDB) {
        ZD* col = w.Xinv + c;   // column c, stride k (holds y, then x)
        // forward, every lane through every step in step with the others, so that each
        // store covers consecutive columns of one row: the right-hand side e_c is zero
        // above row c, and y stays exactly +0 until step c - 1 (the only earlier step
        // that can move the 1, via an exchange) brings the 1 in
        ZD cur = c == 0 ? mk<double>(1.0, 0.0) : zero;   // running y[i]
        for (int i = 0; i + 1 < k; ++i) {
            ZD nxt = (i + 1 == c) ? mk<double>(1.0, 0.0) : zero;   // untouched y[i+1]
            if (swp[i]) {
                const ZD t = cur;
                cur = nxt;
                nxt = t;
            }
            col[(size_t)i * k] = cur;
            cur = nxt - mlt[i] * cur;
        }
        // back substitution with the three diagonals of U; y[k-1] is still in cur
        ZD x1 = zero, x2 = zero;   // x[i+1], x[i+2]
        for (int top = k - 1; top >= 0; top -= kTriBatch) {
            ZD yb[kTriBatch];
#pragma unroll
            for (int t = 0; t < kTriBatch; ++t) {
                const int r = top - t;
                yb[t] = r == k - 1 ? cur : (r >= 0 ? col[(size_t)r * k] : zero);
            }
#pragma unroll
            for (int t = 0; t < kTriBatch; ++t) {
                const int r = top - t;
                if (r >= 0) {
                    const ZD x = (yb[t] - du[r] * x1 - u2[r] * x2) * idd[r];
                    col[(size_t)r * k] = x;
                    v[0] += norm2(x);
                    x2 = x1;
                    x1 = x;
                }
            }
        }
    }
    block_sum<2, kDB>(v);
    if (threadIdx.x == 0) {
        w.part[2 * w.npart_max] = v[0];
        w.part[2 * w.npart_max + 1] = v[1];
    }
}

void dense_newton_step(const SrcList& L, int grad, int nb, size_t lds_bytes, const DenseWork& w, hipStream_t st,
                       int tridiag) {
    const int kmax = L.k[0];
    const int nblk = grid_for(kmax * kmax, kDB);
    const int ncb = dense_colnorm_blocks(kmax);
    if (tridiag) {
        const size_t tl = (size_t)7 * kmax * sizeof(ZD) + (size_t)kmax * sizeof(int);
        hipLaunchKernelGGL(k_tridiag_inv, dim3(1, 1, L.n), dim3(kDB), tl, st, w, L);
        hipLaunchKernelGGL(k_dense_colnorm, dim3(ncb, 1, L.n), dim3(kDB), 0, st, w, L);
        hipLaunchKernelGGL(k_dense_mu, dim3(1, 1, L.n), dim3(kDB), 0, st, w, L, 1, ncb);
    } else {
        hipLaunchKernelGGL(k_rowperm_init, dim3(grid_for(kmax, kDB), 1, L.n), dim3(kDB), 0, st, L, w);
        const size_t panel_lds = (size_t)(kmax * (nb + 1)) * sizeof(ZD) + (size_t)kmax * sizeof(int);
        // trailing tile: TC columns per block; small enough to spread over many CUs,
        // large enough to amortise each row's panel load, and within the LDS budget
        const int tc_want = (kmax - nb) / 96;
        const int tc_lds = (int)((lds_bytes - 2048) / ((size_t)(kmax + nb) * sizeof(ZD))) - 1;
        int TC = 1;   // largest power of two <= min(tc_want, tc_lds, 16)
        while (TC * 2 <= tc_want && TC * 2 <= tc_lds && TC * 2 <= 16) TC *= 2;
        switch (nb) {
            case 16: gj_sweep<16>(L, TC, panel_lds, w, st); break;
            case 8: gj_sweep<8>(L, TC, panel_lds, w, st); break;
            case 4: gj_sweep<4>(L, TC, panel_lds, w, st); break;
            case 2: gj_sweep<2>(L, TC, panel_lds, w, st); break;
            default: gj_sweep<1>(L, TC, panel_lds, w, st); break;
        }
        hipLaunchKernelGGL(k_dense_scatter, dim3(nblk, 1, L.n), dim3(kDB), 0, st, w, L);
        hipLaunchKernelGGL(k_dense_colnorm, dim3(ncb, 1, L.n), dim3(kDB), 0, st, w, L);
        hipLaunchKernelGGL(k_dense_mu, dim3(1, 1, L.n), dim3(kDB), 0, st, w, L, nblk, ncb);
    }
    if (grad) {
        dim3 g2(grid_for(kmax, 16), grid_for(kmax, 16), L.n);
        hipLaunchKernelGGL(k_zgemm, g2, dim3(kDB), 0, st, w, L, kMXinv, kMY, kMZt, kMZt, 1.0, 0.0, 0);
        hipLaunchKernelGGL(k_zgemm, g2, dim3(kDB), 0, st, w, L, kMZt, kMXinv, kMY, kMY, 0.0, 0.0, 1);
    }
    hipLaunchKernelGGL(k_dense_update, dim3(nblk, 1, L.n), dim3(kDB), 0, st, w, L);
    hipLaunchKernelGGL(k_dense_delta, dim3(1, 1, L.n), dim3(kDB), 0, st, w, L, nblk);
}

void launch_tridiag_inverse(const SrcList& L, const DenseWork& w, hipStream_t st) {
    const int kmax = L.k[0];
    const size_t tl = (size_t)7 * kmax * sizeof(ZD) + (size_t)kmax * sizeof(int);
    hipLaunchKernelGGL(k_tridiag_inv, dim3(1, 1, L.n), dim3(kDB), tl, st, w, L);
}

void launch_dense_gemm(const SrcList& L, const DenseWork& w, int ia, int ib, int ic, hipStream_t st) {
    const int kmax = L.k[0];
    dim3 g2(grid_for(kmax, 16), grid_for(kmax, 16), L.n);
    hipLaunchKernelGGL(k_zgemm, g2, dim3(kDB), 0, st, w, L, ia, ib, ic, ic, 1.0, 0.0, 0);
}

// X <- Wk (the new iterate), Y <- Y2 if grad, partials of |X_new - X|^2 and |X_new|^2.
__global__ __launch_bounds__(kDB) void k_ns_commit(DenseWork w0, SrcList L, int grad) {
    const int e = blockIdx.z, k = L.k[e];
    const DenseWork w = w0.at(L.slot[e]);
    const int idx = blockIdx.x * kDB + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (idx < k * k) {
        const ZD x = w.X[idx], xn = w.Wk[idx];
        v[0] = norm2(xn - x);
        v[1] = norm2(xn);
        w.X[idx] = xn;
        if (grad) w.Y[idx] = w.Y2[idx] + w.Y3[idx];
    }
    write_partials<2, kDB>(w.part, v);
}

void dense_ns_step(const SrcList& L, int grad, const DenseWork& w, hipStream_t st) {
    const int kmax = L.k[0];
    const dim3 g2(grid_for(kmax, 16), grid_for(kmax, 16), L.n);
    auto gemm = [&](int ia, int ib, int ic, int id, double a, double b) {
        hipLaunchKernelGGL(k_zgemm, g2, dim3(kDB), 0, st, w, L, ia, ib, ic, id, a, b, 0);
    };
    if (grad) {
        // two launches of three single-product outputs: first the products of the
        // current X and Y, then the new iterates from them (Y in two parts, added by
        // the commit)
        const dim3 g3(g2.x, g2.y, 3 * L.n);
        GemmOuts p1{};
        p1.n = 3;
        p1.o0 = GemmOut{kMX, kMX, -1, kMZt, kMZt, 1.0, 0.0};       // Q = X^2
        p1.o1 = GemmOut{kMX, kMY, -1, kMXinv, kMXinv, 1.0, 0.0};   // P_a = X Y
        p1.o2 = GemmOut{kMY, kMX, -1, kMP2, kMP2, 1.0, 0.0};       // P_b = Y X
        hipLaunchKernelGGL(k_zgemm_outs, g3, dim3(kDB), 0, st, w, L, p1);
        GemmOuts p2{};
        p2.n = 3;
        p2.o0 = GemmOut{kMX, kMZt, -1, kMWk, kMX, -0.5, 1.5};      // X_new = 1.5 X - 0.5 X Q
        p2.o1 = GemmOut{kMY, kMZt, -1, kMY2, kMY, -0.5, 1.5};      // 1.5 Y - 0.5 Y Q
        p2.o2 = GemmOut{kMX, kMXinv, kMP2, kMY3, kMY3, -0.5, 0.0}; // -0.5 X (P_a + P_b)
        hipLaunchKernelGGL(k_zgemm_outs, g3, dim3(kDB), 0, st, w, L, p2);
    } else {
        gemm(kMX, kMX, kMZt, kMZt, 1.0, 0.0);   // Q = X^2
        gemm(kMX, kMZt, kMWk, kMX, -0.5, 1.5);  // X_new = 1.5 X - 0.5 X Q
    }
    const int nblk = grid_for(kmax * kmax, kDB);
    hipLaunchKernelGGL(k_ns_commit, dim3(nblk, 1, L.n), dim3(kDB), 0, st, w, L, grad);
    hipLaunchKernelGGL(k_dense_delta, dim3(1, 1, L.n), dim3(kDB), 0, st, w, L, nblk);
}

// Partials of |I - Q|_F^2 for Q = Zt (X^2 from the preceding GEMM), then their sum
// into delta[2]: once below 1, E = I - X^2 obeys E' = E^2 (3 + E)/4 under the
// inverse-free step (X commutes with E), so that step converges quadratically.
__global__ __launch_bounds__(kDB) void k_dense_resid(DenseWork w0, SrcList L) {
    const int e = blockIdx.z, k = L.k[e];
    const DenseWork w = w0.at(L.slot[e]);
    const int idx = blockIdx.x * kDB + threadIdx.x;
    double v[1] = {0.0};
    if (idx < k * k) {
        ZD q = w.Zt[idx];
        if (idx / k == idx % k) q.re -= 1.0;
        v[0] = norm2(q);
    }
    write_partials<1, kDB>(w.part + 4 * w.npart_max + 8, v);
}

__global__ __launch_bounds__(kDB) void k_dense_resid_sum(DenseWork w0, SrcList L, int npart) {
    const DenseWork w = w0.at(L.slot[blockIdx.z]);
    double red[1];
    reduce_partials<1, kDB>(w.part + 4 * w.npart_max + 8, npart, red);
    if (threadIdx.x == 0) w.delta[2] = red[0];
}

void dense_residual(const SrcList& L, const DenseWork& w, hipStream_t st) {
    const int kmax = L.k[0];
    const dim3 g2(grid_for(kmax, 16), grid_for(kmax, 16), L.n);
    hipLaunchKernelGGL(k_zgemm, g2, dim3(kDB), 0, st, w, L, kMX, kMX, kMZt, kMZt, 1.0, 0.0, 0);
    const int nblk = grid_for(kmax * kmax, kDB);
    hipLaunchKernelGGL(k_dense_resid, dim3(nblk, 1, L.n), dim3(kDB), 0, st, w, L);
    hipLaunchKernelGGL(k_dense_resid_sum, dim3(1, 1, L.n), dim3(kDB), 0, st, w, L, nblk);
}

// c_j = X[j][0]; adjoint seeds alphabar_j = conj(G_jj), betabar_{j+1} = Re G_{j,j+1},
// gammabar_{j+1} = conj(G_{j+1,j}) from G = Y (so that dS = Re tr(dT G));
// S = |x| Re sum_j c_j h_j.
__global__ __launch_bounds__(kDB) void k_dense_extract(Coef coef0, SrcList L, int grad, DenseWork w0) {
    const int e = blockIdx.z, slot = L.slot[e], k = L.k[e];
    const Coef coef = coef0.at(slot);
    const DenseWork w = w0.at(slot);
    double v[1] = {0.0};
    for (int j = threadIdx.x; j < k; j += kDB) {
        const ZD c = w.X[(size_t)j * k];
        coef.c[j + 1] = c;
        if (grad) {
            v[0] += (c * coef.h[j + 1]).re;
            coef.abar_T[j + 1] = cj(w.Y[(size_t)j * k + j]);
            if (j + 1 < k) {
                const double bb = w.Y[(size_t)j * k + j + 1].re;
                const ZD gb = cj(w.Y[(size_t)(j + 1) * k + j]);
                coef.bbar_T[j + 2] = bb;
                coef.gbar_T[j + 2] = gb;
                coef.bbar_tot[j + 2] = bb;
                coef.gbar_tot[j + 2] = gb;
            }
        }
    }
    block_sum<1, kDB>(v);
    if (threadIdx.x == 0 && grad) coef.misc[1] = coef.misc[0] * v[0];
}

void launch_dense_extract(Coef coef, const SrcList& L, int grad, const DenseWork& w, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_extract, dim3(1, 1, L.n), dim3(kDB), 0, st, coef, L, grad, w);
}

}  // namespace tslov
