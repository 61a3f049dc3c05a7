// Operator applications for the eigen step of the spectral correction
// (Section 2.5, Algorithm 1: the eigenpairs of A^-1 - X need products with X
// and solves with A, preconditioned by the incomplete factor):
//   y = X x for X on S (both triangles),
//   y = Ah x for Ah = P^T A P (A in its own ordering, perm), the diagonal
//   of Z Ah (a diagnostic of an approximate inverse, 1 where Z is exact),
//   y = (L D L^T)^-1 x with the loaded factor, by the level schedule of the
//   SelInv sweep: the rows of a level depend only on rows of other levels,
//   forward substitution runs the levels last to first, backward first to
//   last, each row a pass over its part of S with its L values stored in
//   S's order (so the row reads them in sequence) and a gather of the vector;
// and the vector kernels of preconditioned CG and simplified QMR on Ah.
// Every sum has a fixed order (segment lanes, then a fixed shuffle tree, and
// fixed-order two-stage reductions), so the results repeat bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace asi {
namespace dev {

namespace {
constexpr int kSeg = 16;  // lanes per row

__device__ inline double seg_sum(double v) {
#pragma unroll
    for (int o = kSeg / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
}  // namespace

// y = X x on S, kSeg lanes per row
__global__ __launch_bounds__(256) void k_spmv_s(int32_t n, const int64_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ col, const double *__restrict__ X,
                                                const double *__restrict__ x, double *__restrict__ y) {
    const int32_t i = (int32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSeg);
    const int sub = threadIdx.x % kSeg;
    double s = 0.0;
    if (i < n)
        for (int64_t p = rowptr[i] + sub; p < rowptr[i + 1]; p += kSeg) s += X[p] * x[col[p]];
    s = seg_sum(s);
    if (i < n && sub == 0) y[i] = s;
}

// y = Ah x, Ah(i, j) = A(perm[i], perm[j]); iperm maps A's columns back
__global__ __launch_bounds__(256) void k_spmv_ahat(int32_t n, const int64_t *__restrict__ Ap,
                                                   const int32_t *__restrict__ Aj, const double *__restrict__ Av,
                                                   const int32_t *__restrict__ perm,
                                                   const int32_t *__restrict__ iperm, const double *__restrict__ x,
                                                   double *__restrict__ y) {
    const int32_t i = (int32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSeg);
    const int sub = threadIdx.x % kSeg;
    double s = 0.0;
    if (i < n) {
        const int32_t r = perm[i];
        for (int64_t p = Ap[r] + sub; p < Ap[r + 1]; p += kSeg) s += Av[p] * x[iperm[Aj[p]]];
    }
    s = seg_sum(s);
    if (i < n && sub == 0) y[i] = s;
}

// d_i = (Z Ah)_ii = sum_k Z_ik Ah_ki over k in row i of S and of Ah (Ah
// symmetric, so Ah_ki = Ah_ik): row perm[i] of A is walked, each column
// mapped to the factor ordering and searched in the sorted row i of S
__global__ __launch_bounds__(256) void k_za_diag(int32_t n, const int64_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col, const double *__restrict__ Z,
                                                 const int64_t *__restrict__ Ap, const int32_t *__restrict__ Aj,
                                                 const double *__restrict__ Av, const int32_t *__restrict__ perm,
                                                 const int32_t *__restrict__ iperm, double *__restrict__ d) {
    const int32_t i = (int32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSeg);
    const int sub = threadIdx.x % kSeg;
    double s = 0.0;
    if (i < n) {
        const int32_t r = perm[i];
        const int64_t b0 = rowptr[i], b1 = rowptr[i + 1];
        for (int64_t p = Ap[r] + sub; p < Ap[r + 1]; p += kSeg) {
            const int32_t k = iperm[Aj[p]];
            int64_t lo = b0, hi = b1;  // first position with col >= k
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col[mid] < k)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (lo < b1 && col[lo] == k) s += Z[lo] * Av[p];
        }
    }
    s = seg_sum(s);
    if (i < n && sub == 0) d[i] = s;
}

// v = D^-1 v (1x1 and 2x2 blocks, inverses from the D-block kernel)
__global__ void k_ldl_diag(int32_t n, const int8_t *__restrict__ piv, const double *__restrict__ dinv,
                           double *__restrict__ v) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n || piv[j] == 2) return;  // the second row of a 2x2 block is done with its first
    const double *iv = dinv + 3 * (int64_t)j;
    if (piv[j] == 1) {
        const double a = v[j], b = v[j + 1];
        v[j] = iv[0] * a + iv[1] * b;
        v[j + 1] = iv[1] * a + iv[2] * b;
    } else {
        v[j] = iv[0] * v[j];
    }
}

// fixed-order dot products: per block of 256 entries, then one block
__global__ __launch_bounds__(256) void k_dot_part(int64_t n, const double *__restrict__ a,
                                                  const double *__restrict__ b, double *__restrict__ part) {
    __shared__ double s[4];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) v += a[i] * b[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

__global__ __launch_bounds__(256) void k_dot_final(int nb, const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double s[4];
    double v = 0.0;
    for (int q = threadIdx.x; q < nb; q += 256) v += part[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) *out = (s[0] + s[1]) + (s[2] + s[3]);
}

// y += a x (a read from device memory: *a_num / *a_den, times sign)
__global__ void k_axpy_ratio(int64_t n, const double *__restrict__ num, const double *__restrict__ den, double sign,
                             const double *__restrict__ x, double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += sign * (*num / *den) * x[i];
}

// p = z + (num / den) p
__global__ void k_xpby_ratio(int64_t n, const double *__restrict__ z, const double *__restrict__ num,
                             const double *__restrict__ den, double *__restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = z[i] + (*num / *den) * p[i];
}

// d = a d + b q, x += d (scalars from the host)
__global__ void k_qmr_update(int64_t n, double a, double b, const double *__restrict__ q, double *__restrict__ d,
                             double *__restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double v = a * d[i] + b * q[i];
        d[i] = v;
        x[i] += v;
    }
}

// r = b - t
__global__ void k_sub(int64_t n, const double *__restrict__ b, const double *__restrict__ t, double *__restrict__ r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = b[i] - t[i];
}

__global__ void k_copy_f64(int64_t n, const double *__restrict__ a, double *__restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_fill_f64(int64_t n, double v, double *__restrict__ a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_iperm_only(int32_t n, const int32_t *__restrict__ perm, int32_t *__restrict__ iperm,
                             int32_t *status) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t p = perm[i];
    if (p < 0 || p >= n) {
        atomicCAS(status, 0, ST_LIMIT);
        return;
    }
    iperm[p] = i;
}

__global__ void k_build_ls(int64_t nnz, const int32_t *__restrict__ s2u, const double *__restrict__ Lu,
                           double *__restrict__ Ls) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const int32_t u = s2u[p];
    Ls[p] = u >= 0 ? Lu[u] : 0.0;
}

// ---- several right-hand sides at once ---------------------------------------
// The block solves keep their NV vectors interleaved (entry i of vector v at
// V[i NV + v]): one walk over a row's entries (column, L value) serves every
// vector, and the NV values a gather needs sit in one 8 NV-byte run. Each
// vector's arithmetic is that of the one-vector kernels above, in the same
// order. Lane v of a row's segment writes vector v.

template <int NV>
__device__ inline void load_run(const double *__restrict__ src, double (&x)[NV]) {
    if constexpr (NV % 2 == 0) {  // 16-byte aligned: the buffers are, and 8 NV bytes per entry
        const double2 *s2 = reinterpret_cast<const double2 *>(src);
#pragma unroll
        for (int v = 0; v < NV / 2; ++v) {
            const double2 t = s2[v];
            x[2 * v] = t.x;
            x[2 * v + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = src[v];
    }
}

// One level of the forward or backward substitution, in place on V: kSeg
// lanes per row record (the level's rows are consecutive records, so a
// segment starts from one 16-byte load). Row i subtracts L v over its range
// of S positions (forward: the lower part of row i, L(i, c) v_c; backward:
// the upper part, L(r, i) v_r), the 2x2 partner's position skipped. v_i is
// read beside the gathers: no other row of the level writes it, and the
// rows gathered were finished by earlier levels. NV = 1 is the one-vector
// solve.
template <int NV>
__global__ __launch_bounds__(256) void k_ldl_rows(const SolveRow *__restrict__ rows, int32_t nr,
                                                  const int32_t *__restrict__ col, const double *__restrict__ Ls,
                                                  double *__restrict__ V) {
    const int32_t b = (int32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSeg);
    const int sub = threadIdx.x % kSeg;
    if (b >= nr) return;  // the segment's lanes leave together
    const SolveRow R = rows[b];
    const int64_t vi = (int64_t)R.i * NV;
    const double own = sub < NV ? V[vi + sub] : 0.0;
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
    for (int32_t p = R.p0 + sub; p < R.p1; p += kSeg) {
        if (p == R.skip) continue;
        const double l = Ls[p];
        double x[NV];
        load_run<NV>(V + (int64_t)col[p] * NV, x);
#pragma unroll
        for (int v = 0; v < NV; ++v) s[v] += l * x[v];
    }
    double mine = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        s[v] = seg_sum(s[v]);
        if (sub == v) mine = s[v];
    }
    if (sub < NV) V[vi + sub] = own - mine;
}

__global__ void k_ldl_diag_m(int32_t n, int32_t nv, const int8_t *__restrict__ piv, const double *__restrict__ dinv,
                             double *__restrict__ V) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (int64_t)n * nv) return;
    const int32_t j = (int32_t)(x / nv), v = (int32_t)(x % nv);
    if (piv[j] == 2) return;
    const double *iv = dinv + 3 * (int64_t)j;
    if (piv[j] == 1) {
        const double a = V[x], c = V[x + nv];
        V[x] = iv[0] * a + iv[1] * c;
        V[x + nv] = iv[1] * a + iv[2] * c;
    } else {
        V[x] = iv[0] * V[x];
    }
    (void)v;
}

// y_v = X x_v on S for column-major x, y (vector v at x + v ld): the
// Lanczos basis's layout
template <int NV>
__global__ __launch_bounds__(256) void k_spmv_s_m(int32_t n, const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col, const double *__restrict__ X,
                                                  int64_t ld, const double *__restrict__ x, double *__restrict__ y) {
    const int32_t i = (int32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSeg);
    const int sub = threadIdx.x % kSeg;
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
    if (i < n)
        for (int64_t p = rowptr[i] + sub; p < rowptr[i + 1]; p += kSeg) {
            const double a = X[p];
            const int32_t c = col[p];
#pragma unroll
            for (int v = 0; v < NV; ++v) s[v] += a * x[v * ld + c];
        }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        s[v] = seg_sum(s[v]);
        if (i < n && sub == v) y[v * ld + i] = s[v];
    }
}

template <int NV>
__global__ __launch_bounds__(256) void k_spmv_ahat_m(int32_t n, const int64_t *__restrict__ Ap,
                                                     const int32_t *__restrict__ Aj, const double *__restrict__ Av,
                                                     const int32_t *__restrict__ perm,
                                                     const int32_t *__restrict__ iperm,
                                                     const double *__restrict__ x, double *__restrict__ y) {
    const int32_t i = (int32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSeg);
    const int sub = threadIdx.x % kSeg;
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
    if (i < n) {
        const int32_t r = perm[i];
        for (int64_t p = Ap[r] + sub; p < Ap[r + 1]; p += kSeg) {
            const double a = Av[p];
            double xv[NV];
            load_run<NV>(x + (int64_t)iperm[Aj[p]] * NV, xv);
#pragma unroll
            for (int v = 0; v < NV; ++v) s[v] += a * xv[v];
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        s[v] = seg_sum(s[v]);
        if (i < n && sub == v) y[(int64_t)i * NV + v] = s[v];
    }
}

// part[v nb + b] = partial of a_v . b_v over block b's grid stride, the same
// partition and order as k_dot_part; out[v] = the partials of v in index order
template <int NV>
__global__ __launch_bounds__(256) void k_dotm_part(int64_t n, const double *__restrict__ a,
                                                   const double *__restrict__ b, double *__restrict__ part) {
    __shared__ double sm[4][NV];
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double xa[NV], xb[NV];
        load_run<NV>(a + i * NV, xa);
        load_run<NV>(b + i * NV, xb);
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += xa[v] * xb[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double w = acc[v];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, 64);
        if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6][v] = w;
    }
    __syncthreads();
    if (threadIdx.x < NV)
        part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] =
            (sm[0][threadIdx.x] + sm[1][threadIdx.x]) + (sm[2][threadIdx.x] + sm[3][threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_dotm_final(int nb, const double *__restrict__ part,
                                                    double *__restrict__ out) {
    __shared__ double s[4];
    double v = 0.0;
    for (int q = threadIdx.x; q < nb; q += 256) v += part[(int64_t)blockIdx.x * nb + q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

// Y_v += sign (num_v / den_v) X_v for the vectors with act[v] != 0
__global__ void k_axpy_ratio_m(int64_t n, int32_t nv, const double *__restrict__ num, const double *__restrict__ den,
                               const int32_t *__restrict__ act, double sign, const double *__restrict__ X,
                               double *__restrict__ Y) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n * nv) return;
    const int32_t v = (int32_t)(x % nv);
    if (!act[v]) return;
    Y[x] += sign * (num[v] / den[v]) * X[x];
}

// P_v = Z_v + (num_v / den_v) P_v for the vectors with act[v] != 0
__global__ void k_xpby_ratio_m(int64_t n, int32_t nv, const double *__restrict__ Z, const double *__restrict__ num,
                               const double *__restrict__ den, const int32_t *__restrict__ act,
                               double *__restrict__ P) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n * nv) return;
    const int32_t v = (int32_t)(x % nv);
    if (!act[v]) return;
    P[x] = Z[x] + (num[v] / den[v]) * P[x];
}

// D_v = coef[2v] D_v + coef[2v + 1] Q_v, X_v += D_v for the vectors with act[v] != 0
__global__ void k_qmr_update_m(int64_t n, int32_t nv, const double *__restrict__ coef,
                               const int32_t *__restrict__ act, const double *__restrict__ Q, double *__restrict__ D,
                               double *__restrict__ X) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n * nv) return;
    const int32_t v = (int32_t)(x % nv);
    if (!act[v]) return;
    const double w = coef[2 * v] * D[x] + coef[2 * v + 1] * Q[x];
    D[x] = w;
    X[x] += w;
}

// for the vectors with sel[v] != 0: mode 0 dst = src, mode 1 dst = a - src,
// mode 2 dst = 0 (entries i v of n x nv interleaved arrays)
__global__ void k_select_m(int64_t n, int32_t nv, const int32_t *__restrict__ sel, int mode,
                           const double *__restrict__ a, const double *__restrict__ src, double *__restrict__ dst) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n * nv) return;
    if (!sel[x % nv]) return;
    dst[x] = mode == 0 ? src[x] : (mode == 1 ? a[x] - src[x] : 0.0);
}

// interleave (to != 0: dst[i nv + v] = src[v n + i]) or back (dst[v n + i] = src[i nv + v])
__global__ void k_interleave(int64_t n, int32_t nv, int to, const double *__restrict__ src, double *__restrict__ dst) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n * nv) return;
    const int64_t i = x / nv, v = x % nv;
    if (to)
        dst[x] = src[v * n + i];
    else
        dst[v * n + i] = src[x];
}

}  // namespace dev

static dim3 seg_grid(int64_t rows) { return dim3((unsigned)((rows * dev::kSeg + 255) / 256)); }
static dim3 elem_grid(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_spmv_s(int32_t n, const int64_t *rowptr, const int32_t *col, const double *X, const double *x,
                         double *y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_spmv_s, seg_grid(n), dim3(256), 0, st, n, rowptr, col, X, x, y);
    return hipGetLastError();
}

hipError_t launch_spmv_ahat(int32_t n, const int64_t *Ap, const int32_t *Aj, const double *Av, const int32_t *perm,
                            const int32_t *iperm, const double *x, double *y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_spmv_ahat, seg_grid(n), dim3(256), 0, st, n, Ap, Aj, Av, perm, iperm, x, y);
    return hipGetLastError();
}

hipError_t launch_za_diag(int32_t n, const int64_t *rowptr, const int32_t *col, const double *Z, const int64_t *Ap,
                          const int32_t *Aj, const double *Av, const int32_t *perm, const int32_t *iperm, double *d,
                          hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_za_diag, seg_grid(n), dim3(256), 0, st, n, rowptr, col, Z, Ap, Aj, Av, perm, iperm, d);
    return hipGetLastError();
}

hipError_t launch_iperm(int32_t n, const int32_t *perm, int32_t *iperm, int32_t *status, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_iperm_only, elem_grid(n), dim3(256), 0, st, n, perm, iperm, status);
    return hipGetLastError();
}

hipError_t launch_ldl_solve(const LdlSolveParams &P, const double *x, double *v, hipStream_t st) {
    const int32_t n = P.n;
    if (n <= 0) return hipSuccess;
    if (x != v) hipLaunchKernelGGL(dev::k_copy_f64, elem_grid(n), dim3(256), 0, st, (int64_t)n, x, v);
    // forward: levels last to first (a row's lower entries belong to blocks of higher levels)
    for (int32_t l = P.n_levels - 1; l >= 0; --l) {
        const int32_t nr = P.lvl_rows[l + 1] - P.lvl_rows[l];
        if (nr == 0) continue;
        hipLaunchKernelGGL(dev::k_ldl_rows<1>, seg_grid(nr), dim3(256), 0, st, P.rows_fwd + P.lvl_rows[l], nr, P.col,
                           P.Ls, v);
    }
    hipLaunchKernelGGL(dev::k_ldl_diag, elem_grid(n), dim3(256), 0, st, n, P.piv, P.dinv, v);
    for (int32_t l = 0; l < P.n_levels; ++l) {
        const int32_t nr = P.lvl_rows[l + 1] - P.lvl_rows[l];
        if (nr == 0) continue;
        hipLaunchKernelGGL(dev::k_ldl_rows<1>, seg_grid(nr), dim3(256), 0, st, P.rows_bwd + P.lvl_rows[l], nr, P.col,
                           P.Ls, v);
    }
    return hipGetLastError();
}

int dot_blocks(int64_t n) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256)); }

hipError_t launch_dot(int64_t n, const double *a, const double *b, double *part, double *out, hipStream_t st) {
    const int nb = dot_blocks(n);
    hipLaunchKernelGGL(dev::k_dot_part, dim3(nb), dim3(256), 0, st, n, a, b, part);
    hipLaunchKernelGGL(dev::k_dot_final, dim3(1), dim3(256), 0, st, nb, part, out);
    return hipGetLastError();
}

hipError_t launch_axpy_ratio(int64_t n, const double *num, const double *den, double sign, const double *x, double *y,
                             hipStream_t st) {
    hipLaunchKernelGGL(dev::k_axpy_ratio, elem_grid(n), dim3(256), 0, st, n, num, den, sign, x, y);
    return hipGetLastError();
}

hipError_t launch_xpby_ratio(int64_t n, const double *z, const double *num, const double *den, double *p,
                             hipStream_t st) {
    hipLaunchKernelGGL(dev::k_xpby_ratio, elem_grid(n), dim3(256), 0, st, n, z, num, den, p);
    return hipGetLastError();
}

hipError_t launch_qmr_update(int64_t n, double a, double b, const double *q, double *d, double *x, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_qmr_update, elem_grid(n), dim3(256), 0, st, n, a, b, q, d, x);
    return hipGetLastError();
}

hipError_t launch_sub(int64_t n, const double *b, const double *t, double *r, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_sub, elem_grid(n), dim3(256), 0, st, n, b, t, r);
    return hipGetLastError();
}

hipError_t launch_copy_f64(int64_t n, const double *a, double *b, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_copy_f64, elem_grid(n), dim3(256), 0, st, n, a, b);
    return hipGetLastError();
}

hipError_t launch_fill_f64(int64_t n, double v, double *a, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_fill_f64, elem_grid(n), dim3(256), 0, st, n, v, a);
    return hipGetLastError();
}


// ---- launchers of the several-right-hand-side kernels ------------------------

#define ASI_NV_SWITCH(nv, CALL)                                                                                       \
    switch (nv) {                                                                                                     \
        case 1: CALL(1); break;                                                                                       \
        case 2: CALL(2); break;                                                                                       \
        case 3: CALL(3); break;                                                                                       \
        case 4: CALL(4); break;                                                                                       \
        case 5: CALL(5); break;                                                                                       \
        case 6: CALL(6); break;                                                                                       \
        case 7: CALL(7); break;                                                                                       \
        case 8: CALL(8); break;                                                                                       \
        default: return hipErrorInvalidValue;                                                                         \
    }

hipError_t launch_ldl_solve_m(const LdlSolveParams &P, int32_t nv, const double *x, double *V, hipStream_t st) {
    const int32_t n = P.n;
    if (n <= 0) return hipSuccess;
    if (nv < 1 || nv > kMaxRhs) return hipErrorInvalidValue;
    if (x != V) hipLaunchKernelGGL(dev::k_copy_f64, elem_grid((int64_t)n * nv), dim3(256), 0, st, (int64_t)n * nv, x, V);
    for (int32_t l = P.n_levels - 1; l >= 0; --l) {
        const int32_t nr = P.lvl_rows[l + 1] - P.lvl_rows[l];
        if (nr == 0) continue;
#define ASI_FWD(K)                                                                                                    \
    hipLaunchKernelGGL((dev::k_ldl_rows<K>), seg_grid(nr), dim3(256), 0, st, P.rows_fwd + P.lvl_rows[l], nr, P.col,  \
                       P.Ls, V)
        ASI_NV_SWITCH(nv, ASI_FWD)
#undef ASI_FWD
    }
    hipLaunchKernelGGL(dev::k_ldl_diag_m, elem_grid((int64_t)n * nv), dim3(256), 0, st, n, nv, P.piv, P.dinv, V);
    for (int32_t l = 0; l < P.n_levels; ++l) {
        const int32_t nr = P.lvl_rows[l + 1] - P.lvl_rows[l];
        if (nr == 0) continue;
#define ASI_BWD(K)                                                                                                    \
    hipLaunchKernelGGL((dev::k_ldl_rows<K>), seg_grid(nr), dim3(256), 0, st, P.rows_bwd + P.lvl_rows[l], nr, P.col,  \
                       P.Ls, V)
        ASI_NV_SWITCH(nv, ASI_BWD)
#undef ASI_BWD
    }
    return hipGetLastError();
}

hipError_t launch_spmv_s_m(int32_t n, int32_t nv, const int64_t *rowptr, const int32_t *col, const double *X,
                           const double *x, double *y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
#define ASI_SPMV(K) \
    hipLaunchKernelGGL((dev::k_spmv_s_m<K>), seg_grid(n), dim3(256), 0, st, n, rowptr, col, X, (int64_t)n, x, y)
    ASI_NV_SWITCH(nv, ASI_SPMV)
#undef ASI_SPMV
    return hipGetLastError();
}

hipError_t launch_spmv_ahat_m(int32_t n, int32_t nv, const int64_t *Ap, const int32_t *Aj, const double *Av,
                              const int32_t *perm, const int32_t *iperm, const double *x, double *y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
#define ASI_SPMVA(K) \
    hipLaunchKernelGGL((dev::k_spmv_ahat_m<K>), seg_grid(n), dim3(256), 0, st, n, Ap, Aj, Av, perm, iperm, x, y)
    ASI_NV_SWITCH(nv, ASI_SPMVA)
#undef ASI_SPMVA
    return hipGetLastError();
}

hipError_t launch_dot_m(int64_t n, int32_t nv, const double *a, const double *b, double *part, double *out,
                        hipStream_t st) {
    const int nb = dot_blocks(n);
#define ASI_DOTM(K) hipLaunchKernelGGL((dev::k_dotm_part<K>), dim3(nb), dim3(256), 0, st, n, a, b, part)
    ASI_NV_SWITCH(nv, ASI_DOTM)
#undef ASI_DOTM
    hipLaunchKernelGGL(dev::k_dotm_final, dim3(nv), dim3(256), 0, st, nb, part, out);
    return hipGetLastError();
}

hipError_t launch_axpy_ratio_m(int64_t n, int32_t nv, const double *num, const double *den, const int32_t *act,
                               double sign, const double *X, double *Y, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_axpy_ratio_m, elem_grid(n * nv), dim3(256), 0, st, n, nv, num, den, act, sign, X, Y);
    return hipGetLastError();
}

hipError_t launch_xpby_ratio_m(int64_t n, int32_t nv, const double *Z, const double *num, const double *den,
                               const int32_t *act, double *P, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_xpby_ratio_m, elem_grid(n * nv), dim3(256), 0, st, n, nv, Z, num, den, act, P);
    return hipGetLastError();
}

hipError_t launch_qmr_update_m(int64_t n, int32_t nv, const double *coef, const int32_t *act, const double *Q,
                               double *D, double *X, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_qmr_update_m, elem_grid(n * nv), dim3(256), 0, st, n, nv, coef, act, Q, D, X);
    return hipGetLastError();
}

hipError_t launch_select_m(int64_t n, int32_t nv, const int32_t *sel, int mode, const double *a, const double *src,
                           double *dst, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_select_m, elem_grid(n * nv), dim3(256), 0, st, n, nv, sel, mode, a, src, dst);
    return hipGetLastError();
}

hipError_t launch_interleave(int64_t n, int32_t nv, bool to, const double *src, double *dst, hipStream_t st) {
    if (n * nv <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_interleave, elem_grid(n * nv), dim3(256), 0, st, n, nv, to ? 1 : 0, src, dst);
    return hipGetLastError();
}

hipError_t launch_build_ls(int64_t nnzS, const int32_t *s2u, const double *Lu, double *Ls, hipStream_t st) {
    if (nnzS <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_build_ls, elem_grid(nnzS), dim3(256), 0, st, nnzS, s2u, Lu, Ls);
    return hipGetLastError();
}

}  // namespace asi
