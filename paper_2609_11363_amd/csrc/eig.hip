// Basis kernels of the thick-restart Lanczos iteration that finds the
// dominant eigenpairs of E = A^-1 - X (Section 2.5, Algorithm 1). The basis
// V (n x (m + 1), column c at V + c n) lives in device memory; per expansion
// step the new vector w is orthogonalised against the basis by two passes of
// classical Gram-Schmidt (h = V^T w, w -= V h), and a restart or the final
// result forms V Y for a small host matrix Y. Every sum has a fixed order
// (lane-strided partials, a fixed shuffle tree, then blocks in index order),
// so the iteration repeats bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace asi {
namespace dev {

namespace {
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
constexpr int kCombineCols = 8;  // columns of Y per combine block
}  // namespace

// part[c * gridDim.x + b] = V(r, c) . w(r) over the rows r of block b's
// chunk; wave q of the block takes the columns c = q, q + 4, ...
__global__ __launch_bounds__(256) void k_gs_dots_part(int64_t n, int32_t ncols, int64_t chunk,
                                                      const double *__restrict__ V, const double *__restrict__ w,
                                                      double *__restrict__ part) {
    const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = std::min(n, r0 + chunk);
    for (int32_t c = q; c < ncols; c += 4) {
        const double *v = V + (int64_t)c * n;
        double s0 = 0.0, s1 = 0.0;
        int64_t r = r0 + lane;
        for (; r + 64 < r1; r += 128) {
            s0 = fma(v[r], w[r], s0);
            s1 = fma(v[r + 64], w[r + 64], s1);
        }
        if (r < r1) s0 = fma(v[r], w[r], s0);
        const double s = wave_sum(s0 + s1);
        if (lane == 0) part[(int64_t)c * gridDim.x + blockIdx.x] = s;
    }
}

// h[c] = sum over blocks b (in index order of the lanes' strides) of
// part[c * nb + b]; one wavefront per column
__global__ __launch_bounds__(256) void k_gs_dots_final(int32_t nb, int32_t ncols, const double *__restrict__ part,
                                                       double *__restrict__ h) {
    const int32_t c = (int32_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= ncols) return;  // uniform per wavefront
    double s = 0.0;
    for (int32_t b = lane; b < nb; b += 64) s += part[(int64_t)c * nb + b];
    s = wave_sum(s);
    if (lane == 0) h[c] = s;
}

// w -= V(:, 0:ncols) h
__global__ __launch_bounds__(256) void k_gs_update(int64_t n, int32_t ncols, const double *__restrict__ V,
                                                   const double *__restrict__ h, double *__restrict__ w) {
    __shared__ double sh[kEigMaxBasis + 1];
    for (int t = threadIdx.x; t < ncols; t += blockDim.x) sh[t] = h[t];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int32_t c = 0; c < ncols; ++c) s = fma(V[(int64_t)c * n + i], sh[c], s);
    w[i] -= s;
}

// out(:, t) = V(:, 0:m) Y(:, t) for the kCombineCols columns t of Y that
// block row blockIdx.y covers (Y: m x p row-major). Column-major output
// (out + t n) for a new basis, row-major (out[i p + t]) for the result.
__global__ __launch_bounds__(256) void k_basis_combine(int64_t n, int32_t m, int32_t p, const double *__restrict__ V,
                                                       const double *__restrict__ Y, double *__restrict__ out,
                                                       int rowmajor) {
    __shared__ double sY[kEigMaxBasis * kCombineCols];
    const int32_t t0 = (int32_t)blockIdx.y * kCombineCols;
    const int nt = std::min(kCombineCols, p - t0);
    for (int x = threadIdx.x; x < m * kCombineCols; x += blockDim.x) {
        const int c = x / kCombineCols, t = x % kCombineCols;
        sY[x] = t < nt ? Y[(int64_t)c * p + t0 + t] : 0.0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc[kCombineCols];
#pragma unroll
    for (int t = 0; t < kCombineCols; ++t) acc[t] = 0.0;
    for (int32_t c = 0; c < m; ++c) {
        const double v = V[(int64_t)c * n + i];
#pragma unroll
        for (int t = 0; t < kCombineCols; ++t) acc[t] = fma(v, sY[c * kCombineCols + t], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < kCombineCols; ++t) {
        if (t < nt) {
            if (rowmajor)
                out[i * p + t0 + t] = acc[t];
            else
                out[(int64_t)(t0 + t) * n + i] = acc[t];
        }
    }
}

__global__ __launch_bounds__(256) void k_scale(int64_t n, double s, double *__restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] *= s;
}

}  // namespace dev

int gs_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 1023) / 1024)); }

static dim3 row_grid(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_gs_dots(int64_t n, int32_t ncols, const double *V, const double *w, double *part, double *h,
                          hipStream_t st) {
    if (ncols < 1 || ncols > kEigMaxBasis + 1 || n < 1) return hipErrorInvalidValue;
    const int nb = gs_blocks(n);
    const int64_t chunk = (n + nb - 1) / nb;
    hipLaunchKernelGGL(dev::k_gs_dots_part, dim3(nb), dim3(256), 0, st, n, ncols, chunk, V, w, part);
    hipLaunchKernelGGL(dev::k_gs_dots_final, dim3((unsigned)((ncols + 3) / 4)), dim3(256), 0, st, nb, ncols, part, h);
    return hipGetLastError();
}

hipError_t launch_gs_update(int64_t n, int32_t ncols, const double *V, const double *h, double *w, hipStream_t st) {
    if (ncols < 1 || ncols > kEigMaxBasis + 1 || n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(dev::k_gs_update, row_grid(n), dim3(256), 0, st, n, ncols, V, h, w);
    return hipGetLastError();
}

hipError_t launch_basis_combine(int64_t n, int32_t m, int32_t p, const double *V, const double *Y, double *out,
                                bool rowmajor, hipStream_t st) {
    if (m < 1 || m > kEigMaxBasis || p < 1 || n < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)((p + 7) / 8));
    hipLaunchKernelGGL(dev::k_basis_combine, grid, dim3(256), 0, st, n, m, p, V, Y, out, rowmajor ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_scale(int64_t n, double s, double *x, hipStream_t st) {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(dev::k_scale, row_grid(n), dim3(256), 0, st, n, s, x);
    return hipGetLastError();
}

}  // namespace asi
