// Projected-matrix step on the GPU: sgn(T_k) of the k x k Lanczos matrix by the
// scaled Newton iteration X <- (mu X + X^{-1}/mu)/2, and the Frechet derivative
// L_sgn(T_k, E) from Theorem 1 (the upper-right block of sgn([[T, E], [0, T]])):
// Newton on the block-triangular matrix keeps the form [[X, Y], [0, X]] and
// updates Y <- (mu Y - X^{-1} Y X^{-1} / mu)/2.  The inverse comes from an
// in-place, blocked Gauss-Jordan elimination with partial pivoting: one block
// factors a panel of nb columns in LDS, then all blocks apply the panel's
// transform to the remaining columns; the row permutation is undone by a
// column scatter.  All arithmetic is float64 complex.
#include "kernels.h"

#include <cmath>

namespace tslov {

constexpr int kDB = 256;   // threads per block of the dense kernels

__global__ __launch_bounds__(kDB) void k_dense_build(Coef coef, int k, int grad, ZD* __restrict__ X,
                                                     ZD* __restrict__ Wk, ZD* __restrict__ Y) {
    const int idx = blockIdx.x * kDB + threadIdx.x;
    if (idx >= k * k) return;
    const int i = idx / k, c = idx % k;   // 0-based; Lanczos index j = i + 1
    ZD v = mk<double>(0, 0);
    if (i == c) v = coef.alpha[i + 1];
    else if (i == c + 1) v = mk<double>(coef.beta[i + 1], 0.0);   // T_{j+1,j} = beta_{j+1}
    else if (c == i + 1) v = coef.gamma[c + 1];                   // T_{j,j+1} = gamma_{j+1}
    X[idx] = v;
    Wk[idx] = v;
    if (grad) Y[idx] = (i == 0) ? coef.misc[0] * coef.h[c + 1] : mk<double>(0, 0);  // E = e_1 cbar^H
}

void launch_dense_build(Coef coef, int k, int grad, DenseWork w, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_build, dim3(grid_for(k * k, kDB)), dim3(kDB), 0, st, coef, k, grad, w.X, w.Wk, w.Y);
}

__global__ __launch_bounds__(kDB) void k_dense_load(const ZD* __restrict__ T, const ZD* __restrict__ E, int k,
                                                    ZD* __restrict__ X, ZD* __restrict__ Wk, ZD* __restrict__ Y) {
    const int idx = blockIdx.x * kDB + threadIdx.x;
    if (idx >= k * k) return;
    X[idx] = T[idx];
    Wk[idx] = T[idx];
    if (E) Y[idx] = E[idx];
}

void launch_dense_load(const ZD* T, const ZD* E, int k, DenseWork w, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_load, dim3(grid_for(k * k, kDB)), dim3(kDB), 0, st, T, E, k, w.X, w.Wk, w.Y);
}

// ------------------------------------------------------------------ Gauss-Jordan
__global__ __launch_bounds__(kDB) void k_rowperm_init(int* rowperm, int k) {
    const int i = blockIdx.x * kDB + threadIdx.x;
    if (i < k) rowperm[i] = i;
}

// Panel K: columns [c0, c0 + nbK) of Wk, all k rows, held in LDS.  For each
// pivot p = c0 + q: choose the largest |P[i][q]| over rows i >= p (smallest
// index on ties), swap rows, scale the pivot row, eliminate the column from
// every other row; column q then holds the transform's column (in-place GJ).
__global__ __launch_bounds__(kDB) void k_gj_panel(ZD* __restrict__ Wk, int k, int c0, int nb, int* __restrict__ rowperm,
                                                  int* __restrict__ ipiv, double* __restrict__ logpiv) {
    extern __shared__ ZD smem[];
    ZD* P = smem;               // k * nb
    ZD* fcol = smem + k * nb;   // k
    __shared__ double wbest[kDB / kWave];
    __shared__ int wi[kDB / kWave];
    __shared__ int s_imax;
    const int tid = threadIdx.x;
    const int nbK = min(nb, k - c0);
    for (int e = tid; e < k * nbK; e += kDB) {
        const int i = e / nbK, q = e % nbK;
        P[i * nb + q] = Wk[(size_t)i * k + c0 + q];
    }
    __syncthreads();
    for (int q = 0; q < nbK; ++q) {
        const int p = c0 + q;
        double best = -1.0;
        int bi = k;
        for (int i = p + tid; i < k; i += kDB) {
            const double m = norm2(P[i * nb + q]);
            if (m > best) { best = m; bi = i; }
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double ob = __shfl_down(best, off, kWave);
            const int oi = __shfl_down(bi, off, kWave);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (tid % kWave == 0) { wbest[tid / kWave] = best; wi[tid / kWave] = bi; }
        __syncthreads();
        if (tid == 0) {
            double b = wbest[0];
            int ii = wi[0];
            for (int w = 1; w < kDB / kWave; ++w)
                if (wbest[w] > b || (wbest[w] == b && wi[w] < ii)) { b = wbest[w]; ii = wi[w]; }
            if (ii < p || ii >= k) ii = p;   // non-finite column: keep the row order, the NaN propagates
            s_imax = ii;
            ipiv[p] = ii;
            if (ii != p) {
                const int t = rowperm[p];
                rowperm[p] = rowperm[ii];
                rowperm[ii] = t;
            }
        }
        __syncthreads();
        const int imax = s_imax;
        if (imax != p) {
            for (int qq = tid; qq < nbK; qq += kDB) {
                const ZD t = P[p * nb + qq];
                P[p * nb + qq] = P[imax * nb + qq];
                P[imax * nb + qq] = t;
            }
        }
        __syncthreads();
        const ZD piv = P[p * nb + q];
        const ZD inv = zdiv(mk<double>(1.0, 0.0), piv);
        if (tid == 0) logpiv[p] = 0.5 * std::log(norm2(piv));
        __syncthreads();
        for (int qq = tid; qq < nbK; qq += kDB) {
            const ZD val = (qq == q) ? mk<double>(1.0, 0.0) : P[p * nb + qq];
            P[p * nb + qq] = val * inv;
        }
        for (int i = tid; i < k; i += kDB) fcol[i] = (i == p) ? mk<double>(0, 0) : P[i * nb + q];
        __syncthreads();
        for (int e = tid; e < k * nbK; e += kDB) {
            const int i = e / nbK, qq = e % nbK;
            if (i == p) continue;
            const ZD base = (qq == q) ? mk<double>(0, 0) : P[i * nb + qq];
            P[i * nb + qq] = base - fcol[i] * P[p * nb + qq];
        }
        __syncthreads();
    }
    for (int e = tid; e < k * nbK; e += kDB) {
        const int i = e / nbK, q = e % nbK;
        Wk[(size_t)i * k + c0 + q] = P[i * nb + q];
    }
}

// Apply panel K's row swaps and transform to TC columns outside the panel:
// x <- swaps(x);  x_new[i] = [i outside panel] x[i] + sum_q P[i][q] x[c0 + q].
__global__ __launch_bounds__(kDB) void k_gj_trailing(ZD* __restrict__ Wk, int k, int c0, int nb, int TC,
                                                     const int* __restrict__ ipiv) {
    extern __shared__ ZD smem[];
    const int nbK = min(nb, k - c0);
    ZD* xs = smem;              // k * TC
    ZD* xp = smem + k * TC;     // nbK * TC
    const int tid = threadIdx.x;
    const int nother = k - nbK;
    const int cid0 = blockIdx.x * TC;
    const int tcv = min(TC, nother - cid0);
    if (tcv <= 0) return;
    for (int e = tid; e < k * tcv; e += kDB) {
        const int i = e / tcv, t = e % tcv;
        const int cid = cid0 + t;
        const int c = cid < c0 ? cid : cid + nbK;
        xs[i * TC + t] = Wk[(size_t)i * k + c];
    }
    __syncthreads();
    if (tid < tcv) {
        for (int q = 0; q < nbK; ++q) {
            const int p = c0 + q, im = ipiv[p];
            if (im != p) {
                const ZD t = xs[p * TC + tid];
                xs[p * TC + tid] = xs[im * TC + tid];
                xs[im * TC + tid] = t;
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < nbK * tcv; e += kDB) {
        const int q = e / tcv, t = e % tcv;
        xp[q * TC + t] = xs[(c0 + q) * TC + t];
    }
    __syncthreads();
    for (int e = tid; e < k * tcv; e += kDB) {
        const int i = e / tcv, t = e % tcv;
        const int cid = cid0 + t;
        const int c = cid < c0 ? cid : cid + nbK;
        const bool inblk = i >= c0 && i < c0 + nbK;
        ZD acc = inblk ? mk<double>(0, 0) : xs[i * TC + t];
        const ZD* prow = Wk + (size_t)i * k + c0;
        for (int q = 0; q < nbK; ++q) acc = acc + prow[q] * xp[q * TC + t];
        Wk[(size_t)i * k + c] = acc;
    }
}

// X^{-1}[:, rowperm[i]] = Wk[:, i]; block 0 also forms the scaling mu = |det X|^{-1/k}.
__global__ __launch_bounds__(kDB) void k_dense_scatter(const ZD* __restrict__ Wk, const int* __restrict__ rowperm,
                                                       int k, ZD* __restrict__ Xinv, const double* __restrict__ logpiv,
                                                       int scaling, double* __restrict__ mu_out) {
    const int idx = blockIdx.x * kDB + threadIdx.x;
    if (blockIdx.x == 0) {
        double v[1] = {0.0};
        for (int i = threadIdx.x; i < k; i += kDB) v[0] += logpiv[i];
        block_sum<1, kDB>(v);
        if (threadIdx.x == 0) *mu_out = scaling ? std::exp(-v[0] / k) : 1.0;
    }
    if (idx >= k * k) return;
    const int r = idx / k, i = idx % k;
    Xinv[(size_t)r * k + rowperm[i]] = Wk[idx];
}

// ------------------------------------------------------------------ complex GEMM
// mode 0: C = A B;  mode 1: C <- (mu C - (A B)/mu)/2  (mu read from device).
__global__ __launch_bounds__(kDB) void k_zgemm(const ZD* __restrict__ A, const ZD* __restrict__ B, ZD* __restrict__ C,
                                               int k, int mode, const double* __restrict__ mu_p) {
    __shared__ ZD As[32][17];
    __shared__ ZD Bs[16][33];
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    const int row0 = blockIdx.y * 32, col0 = blockIdx.x * 32;
    ZD acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = mk<double>(0, 0);
    for (int kk = 0; kk < k; kk += 16) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = tid + kDB * u;
            const int r = e / 16, cc = e % 16;
            const int gr = row0 + r, gc = kk + cc;
            As[r][cc] = (gr < k && gc < k) ? A[(size_t)gr * k + gc] : mk<double>(0, 0);
            const int r2 = e / 32, c2 = e % 32;
            const int br = kk + r2, bc = col0 + c2;
            Bs[r2][c2] = (br < k && bc < k) ? B[(size_t)br * k + bc] : mk<double>(0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const ZD a0 = As[ty * 2][q], a1 = As[ty * 2 + 1][q];
            const ZD b0 = Bs[q][tx * 2], b1 = Bs[q][tx * 2 + 1];
            acc[0][0] = acc[0][0] + a0 * b0;
            acc[0][1] = acc[0][1] + a0 * b1;
            acc[1][0] = acc[1][0] + a1 * b0;
            acc[1][1] = acc[1][1] + a1 * b1;
        }
        __syncthreads();
    }
    const double mu = mode ? *mu_p : 1.0;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int r = row0 + ty * 2 + u, c = col0 + tx * 2 + v;
            if (r < k && c < k) {
                const size_t o = (size_t)r * k + c;
                if (mode == 0) C[o] = acc[u][v];
                else C[o] = 0.5 * (mu * C[o] - (1.0 / mu) * acc[u][v]);
            }
        }
}

// X <- (mu X + X^{-1}/mu)/2, copy into Wk for the next inversion, partials of
// |X_new - X|^2 and |X_new|^2.
__global__ __launch_bounds__(kDB) void k_dense_update(ZD* __restrict__ X, ZD* __restrict__ Wk,
                                                      const ZD* __restrict__ Xinv, int k, const double* __restrict__ mu_p,
                                                      double* __restrict__ part) {
    const int idx = blockIdx.x * kDB + threadIdx.x;
    const double mu = *mu_p;
    double v[2] = {0.0, 0.0};
    if (idx < k * k) {
        const ZD x = X[idx];
        const ZD xn = 0.5 * (mu * x + (1.0 / mu) * Xinv[idx]);
        v[0] = norm2(xn - x);
        v[1] = norm2(xn);
        X[idx] = xn;
        Wk[idx] = xn;
    }
    write_partials<2, kDB>(part, v);
}

int dense_newton_step(int k, int grad, int scaling, int nb, size_t lds_bytes, DenseWork w, hipStream_t st) {
    hipLaunchKernelGGL(k_rowperm_init, dim3(grid_for(k, kDB)), dim3(kDB), 0, st, w.rowperm, k);
    int* ipiv = w.rowperm + k;
    const size_t panel_lds = (size_t)(k * nb + k) * sizeof(ZD);
    // trailing tile: TC columns of k + nb complex values each, within the LDS budget
    int TC = (int)((lds_bytes - 2048) / ((size_t)(k + nb) * sizeof(ZD)));
    if (TC < 1) TC = 1;
    if (TC > 16) TC = 16;
    for (int c0 = 0; c0 < k; c0 += nb) {
        hipLaunchKernelGGL(k_gj_panel, dim3(1), dim3(kDB), panel_lds, st, w.Wk, k, c0, nb, w.rowperm, ipiv, w.logpiv);
        const int nbK = (k - c0) < nb ? (k - c0) : nb;
        const int nother = k - nbK;
        if (nother > 0) {
            const size_t tl = (size_t)(k * TC + nbK * TC) * sizeof(ZD);
            hipLaunchKernelGGL(k_gj_trailing, dim3(grid_for(nother, TC)), dim3(kDB), tl, st, w.Wk, k, c0, nb, TC, ipiv);
        }
    }
    double* mu = w.part + 2 * w.npart_max;   // device scalar after the partials
    hipLaunchKernelGGL(k_dense_scatter, dim3(grid_for(k * k, kDB)), dim3(kDB), 0, st, w.Wk, w.rowperm, k, w.Xinv,
                       w.logpiv, scaling, mu);
    if (grad) {
        dim3 g2(grid_for(k, 32), grid_for(k, 32));
        hipLaunchKernelGGL(k_zgemm, g2, dim3(kDB), 0, st, w.Xinv, w.Y, w.Zt, k, 0, mu);
        hipLaunchKernelGGL(k_zgemm, g2, dim3(kDB), 0, st, w.Zt, w.Xinv, w.Y, k, 1, mu);
    }
    const int nblk = grid_for(k * k, kDB);
    hipLaunchKernelGGL(k_dense_update, dim3(nblk), dim3(kDB), 0, st, w.X, w.Wk, w.Xinv, k, mu, w.part);
    return nblk;
}

// c_j = X[j][0]; adjoint seeds alphabar_j = conj(G_jj), betabar_{j+1} = Re G_{j,j+1},
// gammabar_{j+1} = conj(G_{j+1,j}) from G = Y (so that dS = Re tr(dT G));
// S = |x| Re sum_j c_j h_j.
__global__ __launch_bounds__(kDB) void k_dense_extract(Coef coef, int k, int grad, const ZD* __restrict__ X,
                                                       const ZD* __restrict__ Y) {
    double v[1] = {0.0};
    for (int j = threadIdx.x; j < k; j += kDB) {
        const ZD c = X[(size_t)j * k];
        coef.c[j + 1] = c;
        if (grad) {
            v[0] += (c * coef.h[j + 1]).re;
            coef.abar_T[j + 1] = cj(Y[(size_t)j * k + j]);
            if (j + 1 < k) {
                const double bb = Y[(size_t)j * k + j + 1].re;
                const ZD gb = cj(Y[(size_t)(j + 1) * k + j]);
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

void launch_dense_extract(Coef coef, int k, int grad, DenseWork w, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_extract, dim3(1), dim3(kDB), 0, st, coef, k, grad, w.X, w.Y);
}

}  // namespace tslov
