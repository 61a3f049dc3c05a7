// HIP kernels of libasi for gfx950 (CDNA4, 64-wide wavefronts).
//
// Data layout in HBM (all indexed by positions of S's CSR, both triangles):
//   col[p], srow[p]     column / row of position p
//   diagpos[i]          position of (i, i)
//   mirror[p]           position of the transposed entry
//   lsrc[p]             for an upper position (j, r): index of L(r, j) in the
//                       caller's L arrays, -1 if not stored
// The upper part of row `last(J)` is R_J, so Z's lower triangle by columns is
// read straight from the output array: a gather of column l of Z is a
// contiguous, coalesced read of row l's upper segment.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace asi {
namespace dev {

__device__ inline void latch(int32_t *status, int32_t code) { atomicCAS(status, 0, code); }

// Orders this wavefront's LDS traffic (LDS operations of one wavefront
// complete in issue order) and stops the compiler from moving LDS accesses
// across the point.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int lane_id() { return threadIdx.x & 63; }

template <typename V>
__device__ inline V wave_sum(V v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline int32_t wave_incl_scan(int32_t v) {
    const int lane = lane_id();
    for (int o = 1; o < 64; o <<= 1) {
        int32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// largest b in [0, c) with off[b] <= t (off[0] = 0 <= t, off nondecreasing)
__device__ inline int seg_of(const int32_t *off, int c, int32_t t) {
    int lo = 0, hi = c - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// index of r in sorted R[lo..hi], or -1
__device__ inline int find_sorted(const int32_t *R, int lo, int hi, int32_t r) {
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int32_t v = R[mid];
        if (v == r) return mid;
        if (v < r)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// D-block inverses (1x1: 1/d; 2x2: scaled form [g, -1; -1, a] / (b (a g - 1)))
// dinv[3 j + {0,1,2}] = (inv00, inv10, inv11) at every block start j.
__global__ void k_dinv(int32_t n, const int8_t *__restrict__ piv, const double *__restrict__ dd,
                       const double *__restrict__ ds, double *__restrict__ dinv,
                       int32_t *__restrict__ status) {
    int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int8_t p = piv[j];
    if (p == 2) return;
    if (p == 0) {
        double d = dd[j];
        if (d == 0.0) latch(status, 3);
        if (!isfinite(d)) latch(status, 4);
        dinv[3 * j] = 1.0 / d;
        dinv[3 * j + 1] = 0.0;
        dinv[3 * j + 2] = 0.0;
    } else {
        double b = ds[j];
        if (!isfinite(b) || !isfinite(dd[j]) || !isfinite(dd[j + 1])) latch(status, 4);
        if (b == 0.0) {
            latch(status, 3);
            return;
        }
        double al = dd[j] / b, ga = dd[j + 1] / b;
        double den = b * (al * ga - 1.0);
        if (den == 0.0) latch(status, 3);
        dinv[3 * j] = ga / den;
        dinv[3 * j + 1] = -1.0 / den;
        dinv[3 * j + 2] = al / den;
    }
}

// ---------------------------------------------------------------------------
// SelInv block: Z(R_J, J) = -Zhat(R_J, R_J) L(R_J, J),
//               Z(J, J)   = D_J^-1 - L(R_J, J)^T Z(R_J, J).
// The pairs (r, l) in R_J x R_J with r > l and (r, l) in S are found by
// scanning row l's upper segment (contiguous) for every l in R_J and looking
// each column up in R_J (binary search in LDS). Each hit feeds two outputs:
// y_r += z L_lJ (scatter half, LDS atomic) and y_l += z L_rJ (LDS atomic).
// T is the working precision of the off-diagonal values and their
// accumulation; D^-1 and Z(J, J) stay in float64.
template <typename T>
struct SelinvLds {
    int32_t *R;
    T *l0, *l1, *y0, *y1;
    int32_t *off;  // c + 1
    int64_t *seg;  // c
};

template <typename T, int G>
__device__ inline void group_sync() {
    if constexpr (G == 64)
        wave_sync();
    else
        __syncthreads();
}

template <typename T, int G>
__device__ void selinv_block(const SelinvParams &P, int32_t j, const SelinvLds<T> &S, int tid,
                             double *red /* G == 256: 4 waves x 4 partial sums */) {
    const bool two = P.piv[j] == 1;
    const int32_t last = two ? j + 1 : j;
    const int64_t u0 = P.diagpos[last] + 1;
    const int32_t c = (int32_t)(P.rowptr[last + 1] - u0);
    const int64_t u0j = two ? P.diagpos[j] + 2 : u0;  // L(R_J, j) in row j
    T *Zw = reinterpret_cast<T *>(P.Zw);

    // stage R_J, L(R_J, J), the gather segments and the diagonal terms
    for (int t = tid; t < c; t += G) {
        int32_t r = P.col[u0 + t];
        S.R[t] = r;
        int64_t s0 = P.lsrc[u0j + t];
        T v0 = s0 >= 0 ? (T)P.Lval[s0] : T(0);
        S.l0[t] = v0;
        T v1 = T(0);
        if (two) {
            int64_t s1 = P.lsrc[u0 + t];
            v1 = s1 >= 0 ? (T)P.Lval[s1] : T(0);
            S.l1[t] = v1;
        }
        int64_t d = P.diagpos[r];
        S.seg[t] = d + 1;
        S.off[t + 1] = (int32_t)(P.rowptr[r + 1] - d - 1);
        T zll = (T)P.out[d];
        S.y0[t] = -zll * v0;
        if (two) S.y1[t] = -zll * v1;
    }
    group_sync<T, G>();
    // exclusive offsets of the segment lengths (one wavefront scans)
    if (tid < 64) {
        int32_t carry = 0;
        for (int base = 0; base < c; base += 64) {
            int t = base + tid;
            int32_t v = t < c ? S.off[t + 1] : 0;
            int32_t s = wave_incl_scan(v) + carry;
            if (t < c) S.off[t + 1] = s;
            carry = __shfl(s, 63, 64);
        }
        if (tid == 0) S.off[0] = 0;
    }
    group_sync<T, G>();
    const int32_t total = c > 0 ? S.off[c] : 0;
    for (int32_t t = tid; t < total; t += G) {
        int b = seg_of(S.off, c, t);
        int64_t p = S.seg[b] + (t - S.off[b]);
        int32_t r = P.col[p];
        int a = find_sorted(S.R, b + 1, c - 1, r);
        if (a >= 0) {
            T z = Zw[p];
            atomicAdd(&S.y0[a], -z * S.l0[b]);
            atomicAdd(&S.y0[b], -z * S.l0[a]);
            if (two) {
                atomicAdd(&S.y1[a], -z * S.l1[b]);
                atomicAdd(&S.y1[b], -z * S.l1[a]);
            }
        }
    }
    group_sync<T, G>();
    double d00 = 0.0, d11 = 0.0, d10 = 0.0, d01 = 0.0;
    for (int t = tid; t < c; t += G) {
        T y0 = S.y0[t];
        int64_t pu = u0j + t;
        if (!P.same) Zw[pu] = y0;
        P.out[pu] = (double)y0;
        P.out[P.mirror[pu]] = (double)y0;
        double l0 = (double)S.l0[t];
        d00 += l0 * (double)y0;
        if (two) {
            T y1 = S.y1[t];
            int64_t pu1 = u0 + t;
            if (!P.same) Zw[pu1] = y1;
            P.out[pu1] = (double)y1;
            P.out[P.mirror[pu1]] = (double)y1;
            double l1 = (double)S.l1[t];
            d11 += l1 * (double)y1;
            d10 += l1 * (double)y0;
            d01 += l0 * (double)y1;
        }
    }
    d00 = wave_sum(d00);
    d11 = wave_sum(d11);
    d10 = wave_sum(d10);
    d01 = wave_sum(d01);
    if constexpr (G > 64) {
        const int w = tid >> 6;
        if ((tid & 63) == 0) {
            red[4 * w + 0] = d00;
            red[4 * w + 1] = d11;
            red[4 * w + 2] = d10;
            red[4 * w + 3] = d01;
        }
        __syncthreads();
        d00 = d11 = d10 = d01 = 0.0;
        for (int q = 0; q < G / 64; ++q) {
            d00 += red[4 * q + 0];
            d11 += red[4 * q + 1];
            d10 += red[4 * q + 2];
            d01 += red[4 * q + 3];
        }
    }
    if (tid == 0) {
        const double *iv = P.dinv + 3 * (int64_t)j;
        double zjj = iv[0] - d00;
        P.out[P.diagpos[j]] = zjj;
        bool bad = !isfinite(zjj);
        if (two) {
            double z11 = iv[2] - d11;
            double off = iv[1] - 0.5 * (d10 + d01);
            P.out[P.diagpos[last]] = z11;
            int64_t pjl = P.diagpos[j] + 1;  // (j, j+1), an upper position read by gathers
            P.out[pjl] = off;
            P.out[P.diagpos[last] - 1] = off;
            if (!P.same) Zw[pjl] = (T)off;
            bad = bad || !isfinite(z11) || !isfinite(off);
        }
        if (bad) latch(P.status, 4);
    }
}

template <typename T, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_selinv_small(SelinvParams P) {
    __shared__ int32_t sR[WAVES][kSmallCols];
    __shared__ T sL0[WAVES][kSmallCols], sL1[WAVES][kSmallCols];
    __shared__ T sY0[WAVES][kSmallCols], sY1[WAVES][kSmallCols];
    __shared__ int32_t sOff[WAVES][kSmallCols + 1];
    __shared__ int64_t sSeg[WAVES][kSmallCols];
    const int w = threadIdx.x >> 6;
    const int32_t bi = blockIdx.x * WAVES + w;
    if (bi >= P.nblk) return;  // the whole wavefront leaves; no workgroup barrier follows
    SelinvLds<T> S{sR[w], sL0[w], sL1[w], sY0[w], sY1[w], sOff[w], sSeg[w]};
    selinv_block<T, 64>(P, P.blocks[bi], S, lane_id(), nullptr);
}

template <typename T>
__global__ __launch_bounds__(256) void k_selinv_big(SelinvParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    // layout: seg (int64, C) | l0, l1, y0, y1 (T, C each) | R (int32, C) | off (int32, C+1) | red
    const int C = kBigCols;
    int64_t *seg = reinterpret_cast<int64_t *>(smem);
    T *l0 = reinterpret_cast<T *>(seg + C);
    T *l1 = l0 + C;
    T *y0 = l1 + C;
    T *y1 = y0 + C;
    int32_t *R = reinterpret_cast<int32_t *>(y1 + C);
    int32_t *off = R + C;
    double *red = reinterpret_cast<double *>(off + C + 2);
    const int32_t bi = blockIdx.x;
    if (bi >= P.nblk) return;
    SelinvLds<T> S{R, l0, l1, y0, y1, off, seg};
    selinv_block<T, 256>(P, P.blocks[bi], S, threadIdx.x, red);
}

}  // namespace dev

size_t selinv_big_lds_bytes(bool fp64) {
    const size_t C = kBigCols, w = fp64 ? 8 : 4;
    return C * 8 + 4 * C * w + C * 4 + (C + 2) * 4 + 16 * 8 + 16;
}

hipError_t launch_dinv(int32_t n, const int8_t *piv, const double *dd, const double *ds, double *dinv,
                       int32_t *status, hipStream_t st) {
    dim3 g((n + 255) / 256);
    hipLaunchKernelGGL(dev::k_dinv, g, dim3(256), 0, st, n, piv, dd, ds, dinv, status);
    return hipGetLastError();
}

hipError_t launch_selinv_level(const SelinvParams &P, bool big, bool fp64, hipStream_t st) {
    if (P.nblk <= 0) return hipSuccess;
    if (!big) {
        constexpr int W = 4;
        dim3 g((P.nblk + W - 1) / W);
        if (fp64)
            hipLaunchKernelGGL((dev::k_selinv_small<double, W>), g, dim3(64 * W), 0, st, P);
        else
            hipLaunchKernelGGL((dev::k_selinv_small<float, W>), g, dim3(64 * W), 0, st, P);
    } else {
        size_t lds = selinv_big_lds_bytes(fp64);
        if (fp64)
            hipLaunchKernelGGL((dev::k_selinv_big<double>), dim3(P.nblk), dim3(256), lds, st, P);
        else
            hipLaunchKernelGGL((dev::k_selinv_big<float>), dim3(P.nblk), dim3(256), lds, st, P);
    }
    return hipGetLastError();
}

hipError_t set_big_lds_limits() {
    hipError_t e = hipFuncSetAttribute((const void *)dev::k_selinv_big<double>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)selinv_big_lds_bytes(true));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)dev::k_selinv_big<float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)selinv_big_lds_bytes(false));
}

}  // namespace asi
