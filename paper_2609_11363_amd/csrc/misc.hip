// Elementwise and per-column kernels on S: diagonal extraction, Mix
// selection, the rank-k correction and SPAI refinement.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace asi {
namespace dev {

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ void k_zdiag(int32_t n, const int64_t *__restrict__ diagpos, const double *__restrict__ X,
                        double *__restrict__ d) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = X[diagpos[i]];
}

// Mix (Section 2.3): keep Z where |Z_ij| > eps sqrt(|Z_ii Z_jj|), else N.
// zdiag is a copy of Z's diagonal taken before this kernel so M may alias Z.
__global__ void k_mix(int64_t nnz, const int32_t *__restrict__ srow, const int32_t *__restrict__ col,
                      const double *__restrict__ zdiag, const double *Z, const double *N, double eps,
                      double *M) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    double z = Z[p];
    double thr = eps * sqrt(fabs(zdiag[srow[p]] * zdiag[col[p]]));
    M[p] = fabs(z) > thr ? z : N[p];
}

// Rank-k correction on S (Section 2.5): out_ij = in_ij + sum_m lam_m V_im V_jm.
// One wavefront per row i: V(i, :) is scaled by lambda once and kept in
// registers; each lane takes one entry (i, j) and reads row j of V.
template <int K>
__global__ __launch_bounds__(256) void k_lowrank(int32_t n, int32_t k, const int64_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col, const double *__restrict__ V,
                                                 const double *__restrict__ lam, const double *in, double *out) {
    const int lane = threadIdx.x & 63;
    const int32_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= n) return;
    double vi[K];
#pragma unroll
    for (int m = 0; m < K; ++m) vi[m] = m < k ? lam[m] * V[(int64_t)i * k + m] : 0.0;
    const int64_t p0 = rowptr[i], p1 = rowptr[i + 1];
    for (int64_t p = p0 + lane; p < p1; p += 64) {
        const double *vj = V + (int64_t)col[p] * k;
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < K; ++m)
            if (m < k) s += vi[m] * vj[m];
        out[p] = in[p] + s;
    }
}

// ---- SPAI -----------------------------------------------------------------

__global__ void k_iperm(int32_t n, const int32_t *__restrict__ perm, int32_t *__restrict__ iperm,
                        int32_t *status) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t p = perm[i];
    if (p < 0 || p >= n) {
        atomicCAS(status, 0, ST_LIMIT);
        return;
    }
    iperm[p] = i;
}

// ||Ah(:, i)||^2 = sum of squares of row perm[i] of A (symmetric A)
__global__ void k_colnorm2(int32_t n, const int32_t *__restrict__ perm, const int64_t *__restrict__ Ap,
                           const double *__restrict__ Ax, double *__restrict__ cn2) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t r = perm[i];
    double s = 0.0;
    for (int64_t q = Ap[r]; q < Ap[r + 1]; ++q) s += Ax[q] * Ax[q];
    cn2[i] = s;
}

constexpr int kSpaiH = 4096;
static_assert(kSpaiH == 1 << 12, "sslot assumes 2^12 slots");

// Fibonacci hashing on the top bits of the product (kSpaiH = 2^12)
__device__ inline uint32_t sslot(int32_t r) { return ((uint32_t)r * 2654435761u) >> (32 - 12); }

__device__ inline int sinsert(int32_t *keys, int32_t r) {
    uint32_t s = sslot(r);
    for (int probe = 0; probe < kSpaiH; ++probe) {
        int32_t k = keys[s];
        if (k == r) return (int)s;
        if (k == -1) {
            int32_t old = atomicCAS(&keys[s], -1, r);
            if (old == -1 || old == r) return (int)s;
        }
        s = (s + 1) & (uint32_t)(kSpaiH - 1);
    }
    return -1;
}

__device__ inline int sfind(const int32_t *keys, int32_t r) {
    uint32_t s = sslot(r);
    for (int probe = 0; probe < kSpaiH; ++probe) {
        int32_t k = keys[s];
        if (k == r) return (int)s;
        if (k == -1) return -1;
        s = (s + 1) & (uint32_t)(kSpaiH - 1);
    }
    return -1;
}

__device__ inline void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wavefront per column j of S (Section 2.4). G = Ah_J^T Ah_J is applied
// as Ah_J^T (Ah_J p): the first half scatters rows of Ah into an LDS hash
// keyed by row, the second half gathers them back per column of J.
__global__ __launch_bounds__(64) void k_spai(SpaiParams P) {
    constexpr int C = kSpaiMaxCols;
    __shared__ int32_t sJ[C];
    __shared__ double sx[C], sr[C], sz[C], sp[C], sg[C];
    __shared__ int32_t soff[C + 1];
    __shared__ int32_t hkey[kSpaiH];
    __shared__ double hval[kSpaiH];
    __shared__ int32_t sflag[1];
    const int lane = threadIdx.x;
    const int32_t j = blockIdx.x;
    if (j >= P.n) return;
    const int64_t s0 = P.rowptr[j];
    const int32_t c = (int32_t)(P.rowptr[j + 1] - s0);
    if (c > C) {
        if (lane == 0) atomicCAS(P.status, 0, ST_LIMIT);
        return;
    }
    for (int a = lane; a < c; a += 64) {
        int32_t i = P.col[s0 + a];
        sJ[a] = i;
        sx[a] = P.M[s0 + a];
        sr[a] = 0.0;  // b, filled below
        int32_t r = P.perm[i];
        soff[a + 1] = (int32_t)(P.A_rowptr[r + 1] - P.A_rowptr[r]);
    }
    if (lane == 0) sflag[0] = 0;
    wsync();
    {
        int32_t carry = 0;
        for (int base = 0; base < c; base += 64) {
            int t = base + lane;
            int32_t v = t < c ? soff[t + 1] : 0;
            int32_t s = v;
            for (int o = 1; o < 64; o <<= 1) {
                int32_t u = __shfl_up(s, o, 64);
                if (lane >= o) s += u;
            }
            s += carry;
            if (t < c) soff[t + 1] = s;
            carry = __shfl(s, 63, 64);
        }
        if (lane == 0) soff[0] = 0;
    }
    // b_a = Ah(j, J_a): row perm[j] of A, columns mapped to the factor order
    {
        const int32_t rj = P.perm[j];
        for (int64_t q = P.A_rowptr[rj] + lane; q < P.A_rowptr[rj + 1]; q += 64) {
            int32_t cc = P.iperm[P.A_col[q]];
            int lo = 0, hi = c - 1;
            while (lo <= hi) {
                int mid = (lo + hi) >> 1;
                if (sJ[mid] == cc) {
                    sr[mid] = P.A_val[q];
                    break;
                }
                if (sJ[mid] < cc)
                    lo = mid + 1;
                else
                    hi = mid - 1;
            }
        }
    }
    wsync();
    const int32_t total = soff[c];
    // g = G * v for v in {sx (initial residual), sp (iterations)}
    auto apply = [&](const double *v) {
        for (int s = lane; s < kSpaiH; s += 64) {
            hkey[s] = -1;
            hval[s] = 0.0;
        }
        wsync();
        for (int32_t t = lane; t < total; t += 64) {
            int lo = 0, hi = c - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (soff[mid] <= t)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            int64_t q = P.A_rowptr[P.perm[sJ[lo]]] + (t - soff[lo]);
            int s = sinsert(hkey, P.iperm[P.A_col[q]]);
            if (s < 0) {
                sflag[0] = 1;
                continue;
            }
            atomicAdd(&hval[s], P.A_val[q] * v[lo]);
        }
        for (int a = lane; a < c; a += 64) sg[a] = 0.0;
        wsync();
        for (int32_t t = lane; t < total; t += 64) {
            int lo = 0, hi = c - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (soff[mid] <= t)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            int64_t q = P.A_rowptr[P.perm[sJ[lo]]] + (t - soff[lo]);
            int s = sfind(hkey, P.iperm[P.A_col[q]]);
            if (s >= 0) atomicAdd(&sg[lo], P.A_val[q] * hval[s]);
        }
        wsync();
    };
    // r = b - G x, z = r / diag, p = z
    apply(sx);
    double rz = 0.0;
    for (int a = lane; a < c; a += 64) {
        double r = sr[a] - sg[a];
        double z = r / P.colnorm2[sJ[a]];
        sr[a] = r;
        sz[a] = z;
        sp[a] = z;
        rz += r * z;
    }
    rz = wsum(rz);
    wsync();
    for (int it = 0; it < P.iters; ++it) {
        if (rz == 0.0) break;
        apply(sp);
        double pgp = 0.0;
        for (int a = lane; a < c; a += 64) pgp += sp[a] * sg[a];
        pgp = wsum(pgp);
        if (pgp == 0.0) break;
        const double al = rz / pgp;
        double rzn = 0.0;
        for (int a = lane; a < c; a += 64) {
            sx[a] += al * sp[a];
            double r = sr[a] - al * sg[a];
            double z = r / P.colnorm2[sJ[a]];
            sr[a] = r;
            sz[a] = z;
            rzn += r * z;
        }
        rzn = wsum(rzn);
        const double be = rzn / rz;
        for (int a = lane; a < c; a += 64) sp[a] = sz[a] + be * sp[a];
        rz = rzn;
        wsync();
    }
    if (sflag[0] && lane == 0) atomicCAS(P.status, 0, ST_LIMIT);
    for (int a = lane; a < c; a += 64) P.X[s0 + a] = sx[a];
}

__global__ void k_symmetrize(int64_t nnz, const int64_t *__restrict__ mirror, const double *__restrict__ X,
                             double *__restrict__ R) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) R[p] = 0.5 * (X[p] + X[mirror[p]]);
}

}  // namespace dev

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

hipError_t launch_zdiag(int32_t n, const int64_t *diagpos, const double *X, double *d, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_zdiag, dim3((n + 255) / 256), dim3(256), 0, st, n, diagpos, X, d);
    return hipGetLastError();
}

hipError_t launch_mix(int64_t nnz, const int32_t *srow, const int32_t *col, const double *zdiag,
                      const double *Z, const double *N, double eps, double *M, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_mix, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, nnz, srow, col,
                       zdiag, Z, N, eps, M);
    return hipGetLastError();
}

hipError_t launch_lowrank(int32_t n, int32_t k, const int64_t *rowptr, const int32_t *col, const double *V,
                          const double *lam, const double *in, double *out, hipStream_t st) {
    dim3 g((n + 3) / 4), b(256);
    if (k <= 8)
        hipLaunchKernelGGL((dev::k_lowrank<8>), g, b, 0, st, n, k, rowptr, col, V, lam, in, out);
    else if (k <= 16)
        hipLaunchKernelGGL((dev::k_lowrank<16>), g, b, 0, st, n, k, rowptr, col, V, lam, in, out);
    else if (k <= 32)
        hipLaunchKernelGGL((dev::k_lowrank<32>), g, b, 0, st, n, k, rowptr, col, V, lam, in, out);
    else
        hipLaunchKernelGGL((dev::k_lowrank<64>), g, b, 0, st, n, k, rowptr, col, V, lam, in, out);
    return hipGetLastError();
}

hipError_t launch_spai(const SpaiParams &P, hipStream_t st) {
    dim3 g1((P.n + 255) / 256);
    hipLaunchKernelGGL(dev::k_iperm, g1, dim3(256), 0, st, P.n, P.perm, P.iperm, P.status);
    hipLaunchKernelGGL(dev::k_colnorm2, g1, dim3(256), 0, st, P.n, P.perm, P.A_rowptr, P.A_val, P.colnorm2);
    hipLaunchKernelGGL(dev::k_spai, dim3(P.n), dim3(64), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_symmetrize(int64_t nnz, const int64_t *mirror, const double *X, double *R, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_symmetrize, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, nnz, mirror,
                       X, R);
    return hipGetLastError();
}

}  // namespace asi
