// Nested projected-matrix step (one level of nesting, Sec. 4.1): with T = T_k the
// outer Lanczos matrix,
//   sgn(T) e_1 = T W^{1/2} e_1,   W = (T^2)^{-1}   (principal square root),
// and W^{1/2} e_1 ~ V' (T')^{1/2} e_1 from an inner two-sided Lanczos process of
// size m on the dense W, both inner Krylov spaces started from e_1.  The inner
// square root is the (1, 2) block of sgn([[0, T'], [I, 0]]), formed by the dense
// Newton step of dense.hip.  Kernels here: the transposed copy of W (so that both
// W v and W^H w read W with unit stride across a wavefront), the two products of
// an inner step, the inner recurrence (one workgroup: k <= 1024 elements, one per
// thread), the block matrix, and the final c = T V' q.
#include "kernels.h"

namespace tslov {

namespace {
constexpr int kNT = 256;    // threads of the product and elementwise kernels
constexpr int kNR = 1024;   // threads of the inner-recurrence kernel (one element each)
}  // namespace

// WT = W^T for W = Zt of slot 0.
__global__ __launch_bounds__(kNT) void k_nest_transpose(DenseWork w, int k) {
    const int idx = blockIdx.x * kNT + threadIdx.x;
    if (idx >= k * k) return;
    const int i = idx / k, j = idx % k;
    w.Y2[(size_t)j * k + i] = w.Zt[idx];
}

// Inner step j: a = W v_j (blockIdx.y = 0, through the rows of WT) and
// b = W^H w_j (blockIdx.y = 1, through the columns of W); thread i forms element i,
// so every load of the matrix covers consecutive elements.
__global__ __launch_bounds__(kNT) void k_nest_products(DenseWork w, NestWork nw, int k) {
    if (*(volatile const int*)nw.status) return;   // the inner process has stopped
    const int i = blockIdx.x * kNT + threadIdx.x;
    if (i >= k) return;
    const bool left = blockIdx.y == 1;
    const ZD* M = left ? w.Zt : w.Y2;
    const ZD* x = nw.vec + (left ? 1 : 0) * (size_t)k;   // w_j or v_j
    ZD acc = mk<double>(0, 0);
    for (int l = 0; l < k; ++l) {
        const ZD m = M[(size_t)l * k + i];   // W^T[l][i] = W[i][l], or W[l][i]
        acc = acc + (left ? cj(m) : m) * x[l];
    }
    nw.vec[(size_t)(left ? 3 : 2) * k + i] = acc;   // a or b
}

// The inner recurrence of step j (0-based; the same plain recursion as the outer
// process): alpha_j = w_j^H a; unless j is the last step, r = a - alpha_j v_j -
// gamma_j v_{j-1}, s = b - conj(alpha_j) w_j - beta_j w_{j-1}, a lucky breakdown
// when |r| <= tau |a| (the inner space is invariant: stop with m_used = j + 1), a
// serious one when |s^H r| <= tau' |r||s|, else beta_{j+1} = |s^H r|^{1/2},
// gamma_{j+1} = s^H r / beta_{j+1}, v_{j+1} = r / beta, w_{j+1} = s / conj(gamma),
// stored as column j + 1 of V'.  Vectors: 0 v, 1 w, 2 a, 3 b, 4 v_prev, 5 w_prev.
__global__ __launch_bounds__(kNR) void k_nest_recur(NestWork nw, int k, int j, int m) {
    if (*(volatile const int*)nw.status) return;
    const int i = threadIdx.x;
    ZD* v = nw.vec;
    ZD* wv = nw.vec + k;
    const ZD* a = nw.vec + 2 * (size_t)k;
    const ZD* b = nw.vec + 3 * (size_t)k;
    ZD* vp = nw.vec + 4 * (size_t)k;
    ZD* wp = nw.vec + 5 * (size_t)k;
    ZD vi = mk<double>(0, 0), wi = vi, ai = vi, bi = vi, vpi = vi, wpi = vi;
    if (i < k) {
        vi = v[i];
        wi = wv[i];
        ai = a[i];
        bi = b[i];
        vpi = vp[i];
        wpi = wp[i];
    }
    double s1[3] = {0.0, 0.0, 0.0};   // w^H a (re, im), |a|^2
    {
        const ZD t = cjmul(wi, ai);
        s1[0] = t.re;
        s1[1] = t.im;
        s1[2] = norm2(ai);
    }
    block_sum<3, kNR>(s1);
    const ZD al = mk<double>(s1[0], s1[1]);
    if (j == m - 1) {   // the last step only records alpha
        if (i == 0) {
            nw.alpha[j] = al;
            nw.status[0] = 1;
            nw.status[1] = j + 1;
        }
        return;
    }
    const ZD gj = j > 0 ? nw.gamma[j] : mk<double>(0, 0);
    const double bj = j > 0 ? nw.beta[j] : 0.0;
    const ZD r = ai - al * vi - gj * vpi;
    const ZD s = bi - cj(al) * wi - bj * wpi;
    double s2[4];
    {
        const ZD t = cjmul(s, r);
        s2[0] = t.re;
        s2[1] = t.im;
        s2[2] = norm2(r);
        s2[3] = norm2(s);
    }
    block_sum<4, kNR>(s2);
    const ZD om = mk<double>(s2[0], s2[1]);
    const double aom = sqrt(norm2(om));
    if (i == 0) nw.alpha[j] = al;
    if (s2[2] <= kTauLucky * kTauLucky * s1[2]) {   // invariant inner space
        if (i == 0) {
            nw.status[0] = 1;
            nw.status[1] = j + 1;
        }
        return;
    }
    if (!(aom > kTauSerious * sqrt(s2[2] * s2[3]))) {   // serious breakdown (or non-finite)
        if (i == 0) {
            nw.status[0] = 1;
            nw.status[1] = j + 1;
            nw.status[2] = 1;
        }
        return;
    }
    const double be = sqrt(aom);
    const ZD ga = (1.0 / be) * om;
    if (i == 0) {
        nw.beta[j + 1] = be;
        nw.gamma[j + 1] = ga;
    }
    if (i < k) {
        const ZD vn = (1.0 / be) * r;
        const ZD wn = zdiv(s, cj(ga));
        vp[i] = vi;
        wp[i] = wi;
        v[i] = vn;
        wv[i] = wn;
        nw.Vb[(size_t)(j + 1) * k + i] = vn;
    }
}

// Start: v = w = e_1 (column 0 of V'), previous vectors zero, status cleared.
__global__ __launch_bounds__(kNR) void k_nest_init(NestWork nw, int k) {
    const int i = threadIdx.x;
    if (i < k) {
        const ZD e = mk<double>(i == 0 ? 1.0 : 0.0, 0.0);
        const ZD z = mk<double>(0, 0);
        nw.vec[i] = e;
        nw.vec[(size_t)k + i] = e;
        nw.vec[4 * (size_t)k + i] = z;
        nw.vec[5 * (size_t)k + i] = z;
        nw.Vb[i] = e;
    }
    if (i < 4) nw.status[i] = 0;
}

// X = Wk = [[0, T'], [I, 0]] (n = 2m) from the inner coefficients.
__global__ __launch_bounds__(kNT) void k_nest_block(NestWork nw, DenseWork w2, int m) {
    const int n = 2 * m;
    const int idx = blockIdx.x * kNT + threadIdx.x;
    if (idx >= n * n) return;
    const int i = idx / n, c = idx % n;
    ZD v = mk<double>(0, 0);
    if (i < m && c >= m) {
        const int jj = c - m;
        if (jj == i) v = nw.alpha[i];
        else if (i == jj + 1) v = mk<double>(nw.beta[i], 0.0);   // T'_{j+1,j}
        else if (jj == i + 1) v = nw.gamma[jj];                  // T'_{j,j+1}
    } else if (i >= m && c == i - m) {
        v = mk<double>(1.0, 0.0);
    }
    w2.X[idx] = v;
    w2.Wk[idx] = v;
}

// q = (T')^{1/2} e_1 = column m of sgn(M) (rows 0..m-1), u = V' q, c = T u with T
// the outer tridiagonal (T_rr = alpha_{r+1}, T_{r+1,r} = beta_{r+2}, T_{r,r+1} =
// gamma_{r+2}); c_r goes to coef.c[r + 1].  One workgroup, thread r < k.
__global__ __launch_bounds__(kNR) void k_nest_finish(NestWork nw, DenseWork w2, Coef coef, int k, int m) {
    __shared__ ZD u[kNR];
    const int r = threadIdx.x;
    const int n = 2 * m;
    if (r < k) {
        ZD acc = mk<double>(0, 0);
        for (int i = 0; i < m; ++i) acc = acc + nw.Vb[(size_t)i * k + r] * w2.X[(size_t)i * n + m];
        u[r] = acc;
    }
    __syncthreads();
    if (r < k) {
        ZD c = coef.alpha[r + 1] * u[r];
        if (r + 1 < k) c = c + coef.gamma[r + 2] * u[r + 1];
        if (r > 0) c = c + coef.beta[r + 1] * u[r - 1];
        coef.c[r + 1] = c;
    }
}

void nest_prepare(const DenseWork& w, int k, hipStream_t st) {
    hipLaunchKernelGGL(k_nest_transpose, dim3(grid_for(k * k, kNT)), dim3(kNT), 0, st, w, k);
}

void nest_init(const NestWork& nw, int k, hipStream_t st) {
    hipLaunchKernelGGL(k_nest_init, dim3(1), dim3(kNR), 0, st, nw, k);
}

void nest_step(const DenseWork& w, const NestWork& nw, int k, int j, int m, hipStream_t st) {
    hipLaunchKernelGGL(k_nest_products, dim3(grid_for(k, kNT), 2), dim3(kNT), 0, st, w, nw, k);
    hipLaunchKernelGGL(k_nest_recur, dim3(1), dim3(kNR), 0, st, nw, k, j, m);
}

void nest_block(const NestWork& nw, const DenseWork& w2, int m, hipStream_t st) {
    hipLaunchKernelGGL(k_nest_block, dim3(grid_for(4 * m * m, kNT)), dim3(kNT), 0, st, nw, w2, m);
}

void nest_finish(const NestWork& nw, const DenseWork& w2, Coef coef, int k, int m, hipStream_t st) {
    hipLaunchKernelGGL(k_nest_finish, dim3(1), dim3(kNR), 0, st, nw, w2, coef, k, m);
}

}  // namespace tslov
