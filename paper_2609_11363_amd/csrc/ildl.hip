// Numeric phase of the incomplete factorization P^T A P ~ L D L^T
// (Section 2.1) on the analysed pattern of L and its 1x1/2x2 pivot partition.
//
// The threshold factorization makes two kinds of decisions: which pivots
// (Bunch-Kaufman, 1x1 or 2x2) and which entries of L are kept. Given both,
// every kept entry follows from the Crout recurrence
//     w(i, B) = Ah(i, B) - sum_{C < B} L(i, C) D_C L(B, C)^T,
//     L(i, B) = w(i, B) D_B^-1,
//     D_B = Ah(B, B) - sum_{C < B} L(B, C) D_C L(B, C)^T,
// which only involves kept entries. Row i of L needs the finished rows of
// the blocks in its own pattern, so the blocks run level by level of the
// SelInv schedule taken last to first (the forward-substitution order).
//
// One wavefront per block. The row's columns c_0 < c_1 < ... and the running
// w(i, c) sit in LDS; note that L(i, C) D_C = w(i, C) for every column block,
// so the sum for column k is sum_j w(i, j) L(k, j) over row k of L: each
// lane takes entries of row k (read from global memory, written by earlier
// levels) and finds their column in the row's sorted list by binary search.
// Entries of the row at or beyond position a still hold Ah values, but row k
// only has columns below k = c_a, so the search never reaches them. The
// scalars of the next column block (its rows of L, D_C) are loaded one step
// ahead.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace asi {
namespace dev {
namespace {

__device__ inline void latch_ildl(int32_t *status, int32_t code) { atomicCAS(status, 0, code); }

// x of another lane of the same 16-lane row, moved by the DPP pattern CTRL
template <int CTRL>
__device__ inline double dpp_move(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double lane_value(double x, int lane) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)v, lane);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes, the same in every lane, in a fixed order: within
// each 16-lane row by DPP moves (swap neighbours, swap pairs, mirror the
// halves of 8, mirror the row: each lane then holds its row's sum), then the
// four row sums read out of lanes 0, 16, 32 and 48. The all-lane moves stay
// in the vector ALU instead of going through the LDS crossbar.
__device__ inline double wave_sum64(double x) {
    x += dpp_move<0xB1>(x);   // quad_perm [1, 0, 3, 2]
    x += dpp_move<0x4E>(x);   // quad_perm [2, 3, 0, 1]
    x += dpp_move<0x141>(x);  // row_half_mirror
    x += dpp_move<0x140>(x);  // row_mirror
    return (lane_value(x, 0) + lane_value(x, 16)) + (lane_value(x, 32) + lane_value(x, 48));
}

// Orders lane 0's LDS writes before the other lanes' next reads. A block is
// one wavefront and LDS accesses of a wavefront are performed in order, so
// wavefront-scope fences suffice; unlike a workgroup barrier they do not wait
// for the global loads still in flight (the next column block's prefetch).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// first position p in [0, hi) with c[p] >= key (hi if none)
__device__ inline int lower_pos(const int32_t *c, int hi, int32_t key) {
    int lo = 0;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (c[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// One column block C = {k} or {k, k+1} of the row being factored: where its
// rows of L live and its D block, plus this lane's first entry of each row.
struct ColBlock {
    int64_t s0, l0, s1, l1;  // S position and L_val offset of rows k and k+1
    int32_t m0, m1;          // entries of rows k and k+1 of L
    int32_t c0, c1;          // this lane's first column of each row (-1 past the end)
    double v0, v1;           // and its L value
    double d0, d1, sub;      // D(k, k), D(k+1, k+1), D(k+1, k)
    int32_t kind;            // piv[k]: 0 = 1x1, 1 = 2x2, 2 = second column of a 2x2 (invalid here)
};

__device__ inline ColBlock load_block(int32_t k, const IldlParams &P, int lane) {
    ColBlock C;
    C.kind = P.piv[k];
    C.s0 = P.rowptr[k];
    C.l0 = P.Lp[k];
    C.m0 = (int32_t)(P.Lp[k + 1] - C.l0);
    C.d0 = P.dd[k];
    C.c0 = lane < C.m0 ? P.col[C.s0 + lane] : -1;
    C.v0 = lane < C.m0 ? P.L[C.l0 + lane] : 0.0;
    C.s1 = C.l1 = 0;
    C.m1 = 0;
    C.c1 = -1;
    C.v1 = C.d1 = C.sub = 0.0;
    if (C.kind == 1) {
        C.s1 = P.rowptr[k + 1];
        C.l1 = P.Lp[k + 1];
        C.m1 = (int32_t)(P.Lp[k + 2] - C.l1);
        C.d1 = P.dd[k + 1];
        C.sub = P.ds[k];
        C.c1 = lane < C.m1 ? P.col[C.s1 + lane] : -1;
        C.v1 = lane < C.m1 ? P.L[C.l1 + lane] : 0.0;
    }
    return C;
}

// sum_j w(j) L(k, j) over row k of L (m entries from S position s and L_val
// offset l; the lane's first entry already loaded), for the row whose first a
// columns and their w are in c and w
__device__ inline double row_dot(const int32_t *c, const double *w, int a, int64_t s, int64_t l, int32_t m,
                                 int32_t cfirst, double vfirst, const IldlParams &P, int lane) {
    double acc = 0.0;
    if (lane < m) {
        const int p = lower_pos(c, a, cfirst);
        if (p < a && c[p] == cfirst) acc = w[p] * vfirst;
    }
    for (int e = lane + 64; e < m; e += 64) {
        const int32_t cc = P.col[s + e];
        const double v = P.L[l + e];
        const int p = lower_pos(c, a, cc);
        if (p < a && c[p] == cc) acc += w[p] * v;
    }
    return wave_sum64(acc);
}

__global__ __launch_bounds__(64) void k_ildl_level(const BlockMeta *__restrict__ ma, int32_t na,
                                                   const BlockMeta *__restrict__ mb, int32_t nb, IldlParams P) {
    extern __shared__ double lds[];
    __shared__ double s_adiag[2], s_asub;
    const int32_t blk = blockIdx.x;
    if (blk >= na + nb) return;
    const BlockMeta &M = blk < na ? ma[blk] : mb[blk - na];
    const int lane = threadIdx.x;
    const int rows = M.two ? 2 : 1;
    const int32_t j = M.j;
    int32_t m[2] = {0, 0};
    int64_t lp[2] = {0, 0}, sp[2] = {0, 0};
    for (int t = 0; t < rows; ++t) {
        lp[t] = P.Lp[j + t];
        m[t] = (int32_t)(P.Lp[j + t + 1] - lp[t]);
        sp[t] = P.rowptr[j + t];
    }
    const int R = m[0] + m[1];  // the host sized the launch's LDS for the level's largest R
    double *sw = lds;           // w of each column, Ah before it is reached
    double *sl = lds + R;       // L of each finished column
    int32_t *sc = reinterpret_cast<int32_t *>(lds + 2 * R);  // the columns
    for (int t = 0; t < rows; ++t) {
        const int off = t ? m[0] : 0;
        for (int e = lane; e < m[t]; e += 64) {
            sc[off + e] = P.col[sp[t] + e];
            sw[off + e] = 0.0;
        }
    }
    if (lane < 2) s_adiag[lane] = 0.0;
    if (lane == 0) s_asub = 0.0;
    __syncthreads();
    // Ah(r, :) = A(perm[r], perm[:]); entries outside the kept pattern are dropped
    for (int t = 0; t < rows; ++t) {
        const int32_t r = j + t, pr = P.perm[r];
        if (pr < 0 || pr >= P.n) continue;  // an invalid perm, already latched by the iperm kernel
        const int off = t ? m[0] : 0;
        for (int64_t e = P.Ap[pr] + lane; e < P.Ap[pr + 1]; e += 64) {
            const int32_t k = P.iperm[P.Aj[e]];
            const double v = P.Av[e];
            if (k == r) {
                s_adiag[t] = v;
            } else if (t == 1 && k == j) {
                s_asub = v;
            } else if (k < r) {
                const int p = lower_pos(sc + off, m[t], k);
                if (p < m[t] && sc[off + p] == k) sw[off + p] = v;
            }
        }
    }
    __syncthreads();
    for (int t = 0; t < rows; ++t) {
        const int off = t ? m[0] : 0;
        const int32_t *c = sc + off;
        double *w = sw + off;
        double *l = sl + off;
        const int mt = m[t];
        ColBlock cur;
        if (mt > 0) cur = load_block(c[0], P, lane);
        for (int a = 0; a < mt;) {
            // both columns of a 2x2 block must be adjacent in the row
            const bool bad = cur.kind == 2 || (cur.kind == 1 && (a + 1 >= mt || c[a + 1] != c[a] + 1));
            if (bad) {
                if (lane == 0) latch_ildl(P.status, 2);
                return;
            }
            const int step = cur.kind == 1 ? 2 : 1;
            ColBlock nxt = cur;
            if (a + step < mt) nxt = load_block(c[a + step], P, lane);
            const double w0 = w[a] - row_dot(c, w, a, cur.s0, cur.l0, cur.m0, cur.c0, cur.v0, P, lane);
            double w1 = 0.0, l0, l1 = 0.0;
            if (step == 2) {
                w1 = w[a + 1] - row_dot(c, w, a, cur.s1, cur.l1, cur.m1, cur.c1, cur.v1, P, lane);
                const double det = cur.d0 * cur.d1 - cur.sub * cur.sub;
                l0 = (w0 * cur.d1 - w1 * cur.sub) / det;
                l1 = (w1 * cur.d0 - w0 * cur.sub) / det;
            } else {
                l0 = w0 / cur.d0;
            }
            wave_sync();  // every lane has read w[a] (and w[a + 1])
            if (lane == 0) {
                w[a] = w0;
                l[a] = l0;
                P.L[lp[t] + a] = l0;
                if (step == 2) {
                    w[a + 1] = w1;
                    l[a + 1] = l1;
                    P.L[lp[t] + a + 1] = l1;
                }
                if (!isfinite(l0) || !isfinite(l1)) latch_ildl(P.status, 4);
            }
            wave_sync();
            a += step;
            cur = nxt;
        }
    }
    // D of the block: Ah(r, r) - sum_c w(r, c) L(r, c), and for a 2x2 block
    // D(j+1, j) = Ah(j+1, j) - sum_c w(j+1, c) L(j, c)
    double dv[2] = {0.0, 0.0};
    for (int t = 0; t < rows; ++t) {
        const int off = t ? m[0] : 0;
        double acc = 0.0;
        for (int e = lane; e < m[t]; e += 64) acc += sw[off + e] * sl[off + e];
        dv[t] = s_adiag[t] - wave_sum64(acc);
    }
    double sub = 0.0;
    if (rows == 2) {
        double acc = 0.0;
        for (int e = lane; e < m[1]; e += 64) {
            const int32_t cc = sc[m[0] + e];
            const int p = lower_pos(sc, m[0], cc);
            if (p < m[0] && sc[p] == cc) acc += sw[m[0] + e] * sl[p];
        }
        sub = s_asub - wave_sum64(acc);
    }
    if (lane == 0) {
        P.dd[j] = dv[0];
        P.ds[j] = sub;
        if (rows == 2) {
            P.dd[j + 1] = dv[1];
            P.ds[j + 1] = 0.0;
            const double det = dv[0] * dv[1] - sub * sub;
            if (!isfinite(det)) latch_ildl(P.status, 4);
            if (det == 0.0) latch_ildl(P.status, 3);
        } else {
            if (!isfinite(dv[0])) latch_ildl(P.status, 4);
            if (dv[0] == 0.0) latch_ildl(P.status, 3);
        }
    }
}

}  // namespace
}  // namespace dev

hipError_t launch_ildl_level(const BlockMeta *ma, int32_t na, const BlockMeta *mb, int32_t nb, int32_t max_entries,
                             const IldlParams &P, hipStream_t st) {
    if (na + nb <= 0) return hipSuccess;
    const size_t lds = (size_t)max_entries * 20 + 8;
    hipLaunchKernelGGL(dev::k_ildl_level, dim3(na + nb), dim3(64), lds, st, ma, na, mb, nb, P);
    return hipGetLastError();
}

}  // namespace asi
