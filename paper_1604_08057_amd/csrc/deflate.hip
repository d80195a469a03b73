// Deflation by known eigenpairs (Sec. 3, eq. final_res; App. E) and the
// a-posteriori error estimate (Sec. 4.1, eq. error_est), on canonical
// [V][4][3] complex128 spinors.
//
//   c_i   = L_i^H psi                      (L^H R = 1, left/right eigenvectors of H)
//   psi_p = psi - sum_i c_i R_i            (the projection P-bar psi)
//   out   = TSL(psi_p) + sum_i s_i c_i R_i,   s_i = sgn(Re lambda_i)
#include "kernels.h"

#include <algorithm>

namespace tslov {

// The deflation kernels treat a canonical spinor as a flat array of n = 12 V complex
// values: block b covers elements [12 kBlock b, 12 kBlock (b + 1)) (the spinors of kBlock
// sites) and lane t takes the 12 elements t, t + kBlock, ..., so that every load of a
// wavefront reads 64 consecutive values.  Element j has spin (j mod 12) / 3.
__device__ __forceinline__ size_t flat_elem(int m) {
    return (size_t)blockIdx.x * 12 * kBlock + (size_t)m * kBlock + threadIdx.x;
}

// Per-block partial sums of L_i^H psi for i < l: part[b][2 i + {0, 1}].
__global__ __launch_bounds__(kBlock) void k_defl_dots(const ZD* __restrict__ L, const ZD* __restrict__ psi, int V,
                                                      int l, double* __restrict__ part) {
    const size_t n = (size_t)V * 12;
    ZD x[12];
#pragma unroll
    for (int m = 0; m < 12; ++m) x[m] = flat_elem(m) < n ? psi[flat_elem(m)] : mk<double>(0, 0);
    for (int i = 0; i < l; ++i) {
        double v[2] = {0.0, 0.0};
        const ZD* Li = L + (size_t)i * n;
#pragma unroll
        for (int m = 0; m < 12; ++m) {
            const size_t j = flat_elem(m);
            if (j < n) {
                const ZD t = cjmul(Li[j], x[m]);
                v[0] += t.re;
                v[1] += t.im;
            }
        }
        block_sum<2, kBlock>(v);
        if (threadIdx.x == 0) {
            part[(size_t)blockIdx.x * 2 * l + 2 * i] = v[0];
            part[(size_t)blockIdx.x * 2 * l + 2 * i + 1] = v[1];
        }
    }
}

// c_i = sum_b part[b][i] (fixed order), one block.
__global__ __launch_bounds__(kBlock) void k_defl_reduce(const double* __restrict__ part, int nb, int l,
                                                        ZD* __restrict__ c) {
    for (int i = 0; i < l; ++i) {
        double v[2] = {0.0, 0.0};
        for (int b = threadIdx.x; b < nb; b += kBlock) {
            v[0] += part[(size_t)b * 2 * l + 2 * i];
            v[1] += part[(size_t)b * 2 * l + 2 * i + 1];
        }
        block_sum<2, kBlock>(v);
        if (threadIdx.x == 0) c[i] = mk<double>(v[0], v[1]);
    }
}

// out = psi - sum_i c_i R_i
__global__ __launch_bounds__(kBlock) void k_defl_project(const ZD* __restrict__ R, const ZD* __restrict__ psi,
                                                         const ZD* __restrict__ c, int V, int l, ZD* __restrict__ out) {
    const size_t n = (size_t)V * 12;
    ZD x[12];
#pragma unroll
    for (int m = 0; m < 12; ++m) x[m] = flat_elem(m) < n ? psi[flat_elem(m)] : mk<double>(0, 0);
    for (int i = 0; i < l; ++i) {
        const ZD ci = c[i];
        const ZD* Ri = R + (size_t)i * n;
#pragma unroll
        for (int m = 0; m < 12; ++m)
            if (flat_elem(m) < n) x[m] = x[m] - ci * Ri[flat_elem(m)];
    }
#pragma unroll
    for (int m = 0; m < 12; ++m)
        if (flat_elem(m) < n) out[flat_elem(m)] = x[m];
}

// out = [psi +] g5^{overlap} (y_p + sum_i sgn_i c_i R_i)
__global__ __launch_bounds__(kBlock) void k_defl_finish(const ZD* __restrict__ R, const ZD* __restrict__ c,
                                                        const double* __restrict__ sgn, const ZD* __restrict__ yp,
                                                        const ZD* __restrict__ psi, int V, int l, int overlap,
                                                        ZD* __restrict__ out) {
    const size_t n = (size_t)V * 12;
    ZD y[12];
#pragma unroll
    for (int m = 0; m < 12; ++m) y[m] = (yp && flat_elem(m) < n) ? yp[flat_elem(m)] : mk<double>(0, 0);
    for (int i = 0; i < l; ++i) {
        const ZD ci = sgn[i] * c[i];
        const ZD* Ri = R + (size_t)i * n;
#pragma unroll
        for (int m = 0; m < 12; ++m)
            if (flat_elem(m) < n) y[m] = y[m] + ci * Ri[flat_elem(m)];
    }
#pragma unroll
    for (int m = 0; m < 12; ++m) {
        const size_t j = flat_elem(m);
        if (j >= n) continue;
        ZD o = y[m];
        if (overlap) o = ((j % 12 >= 6) ? -1.0 : 1.0) * o + psi[j];
        out[j] = o;
    }
}

void launch_defl_coeffs(const ZD* L, const ZD* psi, int V, int l, double* part, ZD* c, hipStream_t st) {
    const int nb = grid_for(V);
    hipLaunchKernelGGL(k_defl_dots, dim3(nb), dim3(kBlock), 0, st, L, psi, V, l, part);
    hipLaunchKernelGGL(k_defl_reduce, dim3(1), dim3(kBlock), 0, st, part, nb, l, c);
}

void launch_defl_project(const ZD* R, const ZD* psi, const ZD* c, int V, int l, ZD* out, hipStream_t st) {
    hipLaunchKernelGGL(k_defl_project, dim3(grid_for(V)), dim3(kBlock), 0, st, R, psi, c, V, l, out);
}

void launch_defl_finish(const ZD* R, const ZD* c, const double* sgn, const ZD* yp, const ZD* psi, int V, int l,
                        int overlap, ZD* out, hipStream_t st) {
    hipLaunchKernelGGL(k_defl_finish, dim3(grid_for(V)), dim3(kBlock), 0, st, R, c, sgn, yp, psi, V, l, overlap, out);
}

// out = [a +] g5^{g5} b on canonical spinors (a nullable); out may be a or b.
__global__ __launch_bounds__(kBlock) void k_combine(const ZD* a, const ZD* b, int g5, int V, ZD* out) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= V) return;
#pragma unroll
    for (int p = 0; p < 12; ++p) {
        const size_t i = (size_t)s * 12 + p;
        ZD o = ((g5 && p >= 6) ? -1.0 : 1.0) * b[i];
        if (a) o = o + a[i];
        out[i] = o;
    }
}

void launch_combine(const ZD* a, const ZD* b, int g5, int V, ZD* out, hipStream_t st) {
    hipLaunchKernelGGL(k_combine, dim3(grid_for(V)), dim3(kBlock), 0, st, a, b, g5, V, out);
}

// Pointwise vector operations of the overlap solve on canonical arrays of n complex values:
// y += a x (a real); y = x + b y (b real); out = f g5 in (f complex, per site and spin).
__global__ __launch_bounds__(kBlock) void k_caxpy(const ZD* __restrict__ x, double a, ZD* __restrict__ y, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        y[i] = y[i] + a * x[i];
}

__global__ __launch_bounds__(kBlock) void k_cxpby(const ZD* __restrict__ x, double b, ZD* __restrict__ y, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        y[i] = x[i] + b * y[i];
}

__global__ __launch_bounds__(kBlock) void k_g5_scale(const ZD* __restrict__ in, ZD f, int V, ZD* __restrict__ out) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= V) return;
#pragma unroll
    for (int p = 0; p < 12; ++p) {
        const size_t i = (size_t)s * 12 + p;
        const ZD o = f * in[i];
        out[i] = p >= 6 ? -1.0 * o : o;
    }
}

void launch_caxpy(const ZD* x, double a, ZD* y, size_t n, hipStream_t st) {
    const int nb = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_caxpy, dim3(nb), dim3(kBlock), 0, st, x, a, y, n);
}

void launch_cxpby(const ZD* x, double b, ZD* y, size_t n, hipStream_t st) {
    const int nb = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_cxpby, dim3(nb), dim3(kBlock), 0, st, x, b, y, n);
}

void launch_g5_scale(const ZD* in, ZD f, int V, ZD* out, hipStream_t st) {
    hipLaunchKernelGGL(k_g5_scale, dim3(grid_for(V)), dim3(kBlock), 0, st, in, f, V, out);
}

// Partials of |a - b|^2 and |b|^2 over n complex values (error estimate).
__global__ __launch_bounds__(kBlock) void k_diff_norm(const ZD* __restrict__ a, const ZD* __restrict__ b, size_t n,
                                                      double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        v[0] += norm2(a[i] - b[i]);
        v[1] += norm2(b[i]);
    }
    write_partials<2, kBlock>(part, v);
}

int launch_diff_norm(const ZD* a, const ZD* b, size_t n, double* part, hipStream_t st) {
    int nb = (int)((n + kBlock - 1) / kBlock);
    if (nb > 1024) nb = 1024;
    hipLaunchKernelGGL(k_diff_norm, dim3(nb), dim3(kBlock), 0, st, a, b, n, part);
    return nb;
}

}  // namespace tslov
