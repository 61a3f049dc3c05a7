// HIP kernels of libasi for gfx950 (CDNA4, 64-wide wavefronts).
//
// Data layout in HBM. Results live on S's CSR (both triangles; positions p).
// The sweep works in "u-space", the upper triangle of S stored by rows, which
// is the lower triangle of Z stored by columns (the layout of L's columns):
//   ustart[j]           first u-index of row j (its entries are R_J, preceded
//                       by (j, j+1) when j starts a 2x2 block)
//   ucol[u]             column r of the upper entry u = (j, r)
//   useg[u]             start of row r's u-range (the gather segment of r)
//   hit_ptr, hits       per block, the pairs (r, l) in R_J x R_J found in S,
//                       precomputed as (a, b, offset in l's u-range)
//   mirror_u[u]         S position of the lower entry (r, j)
//   Lu[u], Zu[u]        L(r, j) and Z(r, j) in the working precision
// A gather of column l of Z is a contiguous, coalesced read of l's u-range.
#include <hip/hip_runtime.h>

#include <algorithm>
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

// Sum of v over the lanes of this wavefront that carry the same key k as the
// calling lane and sit at or after it; keys must be nondecreasing across
// lanes. The first lane of each key run receives the run's total.
template <typename V>
__device__ inline V seg_suffix_sum(V v, int32_t k) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        V vo = __shfl_down(v, o, 64);
        int32_t ko = __shfl_down(k, o, 64);
        if (lane + o < 64 && ko == k) v += vo;
    }
    return v;
}

__device__ inline bool run_head(int32_t k) {
    const int lane = lane_id();
    int32_t kp = __shfl_up(k, 1, 64);
    return lane == 0 || kp != k;
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
// Zhat(R_J, R_J) restricted to S is read through the block's precomputed hit
// list: each hit (a, b, off) is the entry Z(r, l) with r = R_J[a] > l = R_J[b],
// stored at u-index ustart[l] + off, and feeds two outputs,
// y_a += z L(l, J) (scatter half, LDS atomics on distinct targets) and
// y_b += z L(r, J) (dot half: hits are sorted by b, so a segmented wavefront
// sum leaves one atomic per run). Each lane keeps kUnroll hits in flight.
// T is the working precision of the off-diagonal values (storage, gathers
// and products); the sums y run in float64 LDS accumulators in both modes
// (float32 LDS atomic adds stall the sweep on gfx950); D^-1 and Z(J, J) stay
// in float64.
constexpr int kUnroll = 4;

template <typename T>
struct SelinvLds {
    T *l0, *l1;
    double *y0, *y1;
    int64_t *seg;  // c: u-range start of R_J[b]
};

// Accesses to the data that crosses blocks inside one launch (Z columns in
// u-space and the diagonal). In the dataflow sweep (CO = true) they are
// agent-coherent loads and stores, so a block's results are visible to other
// compute units once its stores have completed; no cache maintenance is needed.
template <bool CO, typename V>
__device__ inline V co_load(const V *p) {
    if constexpr (CO)
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *p;
}

template <bool CO, typename V>
__device__ inline void co_store(V *p, V v) {
    if constexpr (CO)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

template <int G>
__device__ inline void group_sync() {
    if constexpr (G == 64)
        wave_sync();
    else
        __syncthreads();
}

// Static part of a block's staging (data that no block of the sweep writes):
// L(R_J, J), the gather segments, the rows of R_J and the mirror positions.
template <typename T, int G, int NT>
__device__ inline void stage_static(const SelinvParams &P, const BlockMeta &M, const SelinvLds<T> &S, int tid,
                                    int32_t (&rr)[NT], int64_t (&mir0)[NT], int64_t (&mir1)[NT]) {
    const bool two = M.two != 0;
    const T *Lu = reinterpret_cast<const T *>(P.Lu);
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const int t = tid + k * G;
        rr[k] = -1;
        mir0[k] = mir1[k] = -1;
        if (t < M.c) {
            rr[k] = P.ucol[M.ub + t];
            S.seg[t] = P.useg[M.ub + t];
            S.l0[t] = Lu[M.ubj + t];
            if (two) S.l1[t] = Lu[M.ub + t];
            mir0[k] = P.mirror_u[M.ubj + t];
            if (two) mir1[k] = P.mirror_u[M.ub + t];
        }
    }
}

// The hit words of one pass (kUnroll per lane); words past the end are 0.
template <bool WIDE, int G>
__device__ inline void load_hit_words(const uint32_t *H, int32_t base, int32_t total, uint32_t (&w0)[kUnroll],
                                      uint32_t (&w1)[kUnroll]) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int32_t t = base + u * G;
        w0[u] = 0u;
        w1[u] = 0u;
        if (t < total) {
            if (WIDE) {
                w0[u] = H[2 * t];
                w1[u] = H[2 * t + 1];
            } else {
                w0[u] = H[t];
            }
        }
    }
}

// The dependent global loads of a block are kept to three rounds: the block
// record; then the staging, the first hit words and (once the rows are known)
// the diagonal entries Z(r, r), all in flight together; then the Z gathers of
// each pass, with the next pass's hit words loaded behind them. The diagonal
// term -Z(r, r) L(r, J) is added after the hits.
template <typename T, int G, int NT, bool WIDE, bool CO = false, bool PRE = false>
__device__ void selinv_block(const SelinvParams &P, const BlockMeta &M, const SelinvLds<T> &S, int tid,
                             double *red /* G > 64: (G / 64) waves x 4 partial sums */,
                             const int32_t *pre_r = nullptr, const int64_t *pre_m0 = nullptr,
                             const int64_t *pre_m1 = nullptr) {
    const bool two = M.two != 0;
    const int32_t j = M.j;
    const int32_t last = two ? j + 1 : j;
    const int32_t c = M.c;
    const int64_t ub = M.ub, ubj = M.ubj;
    const T *Lu = reinterpret_cast<const T *>(P.Lu);
    T *Zu = reinterpret_cast<T *>(P.Zu);
    const int32_t total = WIDE ? M.nwords / 2 : M.nwords;
    const uint32_t *H = P.hits + M.h0;
    constexpr int kStep = G * kUnroll;

    uint32_t w0[kUnroll], w1[kUnroll];
    load_hit_words<WIDE, G>(H, tid, total, w0, w1);
    // the block's D^-1 entries, needed last, are loaded first so that their
    // latency overlaps the staging instead of ending the block
    double iv0 = 0.0, iv1 = 0.0, iv2 = 0.0;
    if (tid == 0) {
        const double *iv = P.dinv + 3 * (int64_t)j;
        iv0 = iv[0];
        if (two) {
            iv1 = iv[1];
            iv2 = iv[2];
        }
    }
    // stage L(R_J, J) and the gather segments; rows, mirror positions and
    // the diagonal entries Z(r, r) stay in registers
    int32_t rr[NT];
    int64_t mir0[NT], mir1[NT];
    T zrr[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const int t = tid + k * G;
        if constexpr (PRE) {
            rr[k] = pre_r[k];
            mir0[k] = pre_m0[k];
            mir1[k] = pre_m1[k];
        } else {
            rr[k] = -1;
            mir0[k] = mir1[k] = -1;
            if (t < c) {
                rr[k] = P.ucol[ub + t];
                S.seg[t] = P.useg[ub + t];
                S.l0[t] = Lu[ubj + t];
                if (two) S.l1[t] = Lu[ub + t];
                mir0[k] = P.mirror_u[ubj + t];
                if (two) mir1[k] = P.mirror_u[ub + t];
            }
        }
        zrr[k] = T(0);
        if (t < c) {
            zrr[k] = (T)co_load<CO>(&P.zdiag[rr[k]]);
            S.y0[t] = 0.0;
            if (two) S.y1[t] = 0.0;
        }
    }
    group_sync<G>();
    // loop bound uniform across the group so every lane joins the shuffles
    for (int32_t base0 = 0; base0 < total; base0 += kStep) {
        int32_t a[kUnroll], b[kUnroll];
        T z[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int32_t t = base0 + tid + u * G;
            b[u] = -1;
            a[u] = 0;
            if (t < total) {
                int64_t off;
                if (WIDE) {
                    a[u] = (int32_t)(w0[u] & 0xffffu);
                    b[u] = (int32_t)(w0[u] >> 16);
                    off = (int64_t)w1[u];
                } else {
                    a[u] = (int32_t)(w0[u] & 0x7fu);
                    b[u] = (int32_t)((w0[u] >> 7) & 0x7fu);
                    off = (int64_t)(w0[u] >> 14);
                }
                z[u] = co_load<CO>(&Zu[S.seg[b[u]] + off]);
            }
        }
        if (base0 + kStep < total) load_hit_words<WIDE, G>(H, base0 + kStep + tid, total, w0, w1);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            // products in the working precision T, sums in float64 (LDS
            // accumulators: the float32 LDS atomic add stalls the sweep)
            double dot0 = 0.0, dot1 = 0.0;
            if (b[u] >= 0) {
                atomicAdd(&S.y0[a[u]], (double)(-z[u] * S.l0[b[u]]));
                dot0 = (double)(-z[u] * S.l0[a[u]]);
                if (two) {
                    atomicAdd(&S.y1[a[u]], (double)(-z[u] * S.l1[b[u]]));
                    dot1 = (double)(-z[u] * S.l1[a[u]]);
                }
            }
            dot0 = seg_suffix_sum(dot0, b[u]);
            if (two) dot1 = seg_suffix_sum(dot1, b[u]);
            if (b[u] >= 0 && run_head(b[u])) {
                atomicAdd(&S.y0[b[u]], dot0);
                if (two) atomicAdd(&S.y1[b[u]], dot1);
            }
        }
    }
    group_sync<G>();
    double d00 = 0.0, d11 = 0.0, d10 = 0.0, d01 = 0.0;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const int t = tid + k * G;
        if (t >= c) continue;
        const T l0t = S.l0[t];
        const T y0 = (T)(S.y0[t] - (double)(zrr[k] * l0t));
        co_store<CO>(&Zu[ubj + t], y0);
        P.out[M.pdj + t] = (double)y0;
        P.out[mir0[k]] = (double)y0;
        double l0 = (double)l0t;
        d00 += l0 * (double)y0;
        if (two) {
            const T l1t = S.l1[t];
            const T y1 = (T)(S.y1[t] - (double)(zrr[k] * l1t));
            co_store<CO>(&Zu[ub + t], y1);
            P.out[M.pdl + t] = (double)y1;
            P.out[mir1[k]] = (double)y1;
            double l1 = (double)l1t;
            d11 += l1 * (double)y1;
            d10 += l1 * (double)y0;
            d01 += l0 * (double)y1;
        }
    }
    d00 = wave_sum(d00);
    if (two) {
        d11 = wave_sum(d11);
        d10 = wave_sum(d10);
        d01 = wave_sum(d01);
    }
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
        for (int q2 = 0; q2 < G / 64; ++q2) {
            d00 += red[4 * q2 + 0];
            d11 += red[4 * q2 + 1];
            d10 += red[4 * q2 + 2];
            d01 += red[4 * q2 + 3];
        }
    }
    if (tid == 0) {
        const int64_t dj = two ? M.pdj - 2 : M.pdl - 1;  // diagpos[j]
        const int64_t dl = M.pdl - 1;                     // diagpos[last]
        double zjj = iv0 - d00;
        P.out[dj] = zjj;
        co_store<CO>(&P.zdiag[j], zjj);
        bool bad = !isfinite(zjj);
        if (two) {
            double z11 = iv2 - d11;
            double off = iv1 - 0.5 * (d10 + d01);
            P.out[dl] = z11;
            co_store<CO>(&P.zdiag[last], z11);
            P.out[dj + 1] = off;
            P.out[dl - 1] = off;
            co_store<CO>(&Zu[ubj - 1], (T)off);  // (j, j+1) at ustart[j], read by later gathers
            bad = bad || !isfinite(z11) || !isfinite(off);
        }
        if (bad) latch(P.status, 4);
    }
}

template <typename T, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_selinv_small(SelinvParams P) {
    __shared__ T sL0[WAVES][kSmallCols], sL1[WAVES][kSmallCols];
    __shared__ double sY0[WAVES][kSmallCols], sY1[WAVES][kSmallCols];
    __shared__ int64_t sSeg[WAVES][kSmallCols];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t bi = blockIdx.x * WAVES + w;
    if (bi >= P.nblk) return;  // the whole wavefront leaves; no workgroup barrier follows
    SelinvLds<T> S{sL0[w], sL1[w], sY0[w], sY1[w], sSeg[w]};
    const BlockMeta M = P.meta[bi];
    selinv_block<T, 64, kSmallCols / 64, false>(P, M, S, lane_id(), nullptr);
}

// A level of many blocks whose first P.nheavy blocks have many hits: each of
// those gets a 256-thread workgroup (a quarter of the passes over its hits),
// the others a wavefront each, four per workgroup; the level no longer waits
// on its longest hit lists walked by one wavefront.
template <typename T>
__global__ __launch_bounds__(256) void k_selinv_split(SelinvParams P) {
    constexpr int W = 4;
    __shared__ T sL0[W][kSmallCols], sL1[W][kSmallCols];
    __shared__ double sY0[W][kSmallCols], sY1[W][kSmallCols];
    __shared__ int64_t sSeg[W][kSmallCols];
    __shared__ double red[4 * W];
    const int32_t b = blockIdx.x;
    if (b < P.nheavy) {
        SelinvLds<T> S{sL0[0], sL1[0], sY0[0], sY1[0], sSeg[0]};
        const BlockMeta M = P.meta[b];
        selinv_block<T, 256, (kSmallCols + 255) / 256, false>(P, M, S, threadIdx.x, red);
        return;
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t bi = P.nheavy + (b - P.nheavy) * W + w;
    if (bi >= P.nblk) return;  // the whole wavefront leaves; no workgroup barrier follows
    SelinvLds<T> S{sL0[w], sL1[w], sY0[w], sY1[w], sSeg[w]};
    const BlockMeta M = P.meta[bi];
    selinv_block<T, 64, kSmallCols / 64, false>(P, M, S, lane_id(), nullptr);
}

// one workgroup of G threads per block (|R_J| <= kSmallCols), for levels with
// few blocks
template <typename T, int G>
__global__ __launch_bounds__(G) void k_selinv_group(SelinvParams P) {
    __shared__ T sL0[kSmallCols], sL1[kSmallCols];
    __shared__ double sY0[kSmallCols], sY1[kSmallCols];
    __shared__ int64_t sSeg[kSmallCols];
    __shared__ double red[4 * (G / 64)];
    const int32_t bi = blockIdx.x;
    if (bi >= P.nblk) return;
    SelinvLds<T> S{sL0, sL1, sY0, sY1, sSeg};
    const BlockMeta M = P.meta[bi];
    selinv_block<T, G, (kSmallCols + G - 1) / G, false>(P, M, S, threadIdx.x, red);
}

// one workgroup of G threads per block with |R_J| > kSmallCols; the dynamic
// LDS holds C = the largest |R_J| of the launch (at most kBigCols):
// red (4 G/64 doubles) | seg (int64, C) | l0, l1, y0, y1 (T, C each)
template <typename T, int G>
__global__ __launch_bounds__(G) void k_selinv_big(SelinvParams P, int32_t C) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *red = reinterpret_cast<double *>(smem);
    int64_t *seg = reinterpret_cast<int64_t *>(red + 4 * (G / 64));
    double *y0 = reinterpret_cast<double *>(seg + C);
    double *y1 = y0 + C;
    T *l0 = reinterpret_cast<T *>(y1 + C);
    T *l1 = l0 + C;
    const int32_t bi = blockIdx.x;
    if (bi >= P.nblk) return;
    SelinvLds<T> S{l0, l1, y0, y1, seg};
    const BlockMeta M = P.meta[bi];
    selinv_block<T, G, kBigCols / G, true>(P, M, S, threadIdx.x, red);
}

// ---------------------------------------------------------------------------
// Dataflow sweep: one cooperative launch, one wavefront per block. Blocks are
// taken in a topological order (level-major), wavefront w handling positions
// w, w + W, w + 2W, ... Before a block starts, its wavefront waits until every
// block that holds a row of R_J has published its column (flag == epoch);
// after finishing it publishes its own. Z columns and the diagonal are read
// and written with agent-coherent accesses and the flag is stored only after
// the block's stores have completed, so no L2 writeback or invalidation is
// issued per block. All wavefronts are co-resident (cooperative launch), so
// the earliest unfinished block can always proceed.
// The wait is bounded: after spin_limit polls the status word is latched and
// the block runs anyway, so the launch always drains.
template <typename T, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_selinv_flow(SelinvParams P, int32_t nblocks, int32_t *done,
                                                            int32_t epoch, int32_t spin_limit) {
    __shared__ T sL0[WAVES][kSmallCols], sL1[WAVES][kSmallCols];
    __shared__ double sY0[WAVES][kSmallCols], sY1[WAVES][kSmallCols];
    __shared__ int64_t sSeg[WAVES][kSmallCols];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = lane_id();
    SelinvLds<T> S{sL0[w], sL1[w], sY0[w], sY1[w], sSeg[w]};
    const int32_t stride = gridDim.x * WAVES;
    for (int32_t i = blockIdx.x * WAVES + w; i < nblocks; i += stride) {
        const BlockMeta M = P.meta[i];
        const int32_t j = M.j;
        const int32_t last = M.two ? j + 1 : j;
        // stage what no block writes before waiting for the dependencies
        constexpr int NT = kSmallCols / 64;
        int32_t rr[NT];
        int64_t m0[NT], m1[NT];
        stage_static<T, 64, NT>(P, M, S, lane, rr, m0, m1);
        const int32_t r0 = rr[0], r1 = rr[1];
        for (int32_t poll = 0;; ++poll) {
            bool ok = true;
            if (r0 >= 0) ok = __hip_atomic_load(&done[r0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch;
            if (r1 >= 0 && ok)
                ok = __hip_atomic_load(&done[r1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch;
            if (__all(ok)) break;
            if (poll >= spin_limit) {
                if (lane == 0) latch(P.status, ST_TIMEOUT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        wave_sync();
        selinv_block<T, 64, NT, false, true, true>(P, M, S, lane, nullptr, rr, m0, m1);
        // the block's agent-coherent stores are complete before its flag is set
        __builtin_amdgcn_s_waitcnt(0);
        if (lane == 0) {
            __hip_atomic_store(&done[j], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (last != j) __hip_atomic_store(&done[last], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <typename T>
__global__ void k_scatter_lu(int64_t nnzL, const int32_t *__restrict__ q2u, const double *__restrict__ Lval,
                             T *__restrict__ Lu) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnzL) return;
    Lu[q2u[q]] = (T)Lval[q];
}

__global__ void k_lu_to_float(int64_t nnzU, const double *__restrict__ Lu, float *__restrict__ Lf) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < nnzU) Lf[u] = (float)Lu[u];
}

}  // namespace dev

hipError_t launch_lu_to_float(int64_t nnzU, const double *Lu, float *Lf, hipStream_t st) {
    if (nnzU <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_lu_to_float, dim3((unsigned)((nnzU + 255) / 256)), dim3(256), 0, st, nnzU, Lu, Lf);
    return hipGetLastError();
}

size_t selinv_big_lds_bytes(bool fp64, int G, int32_t C) {
    const size_t w = fp64 ? 8 : 4;
    return (size_t)4 * (G / 64) * 8 + (size_t)C * 8 + 2 * (size_t)C * 8 + 2 * (size_t)C * w;
}

hipError_t launch_dinv(int32_t n, const int8_t *piv, const double *dd, const double *ds, double *dinv,
                       int32_t *status, hipStream_t st) {
    dim3 g((n + 255) / 256);
    hipLaunchKernelGGL(dev::k_dinv, g, dim3(256), 0, st, n, piv, dd, ds, dinv, status);
    return hipGetLastError();
}

template <typename T>
static void launch_variant(const SelinvParams &P, int variant, int32_t maxc, hipStream_t st) {
    constexpr int W = 4;
    switch (variant) {
        case SV_SPLIT:
            hipLaunchKernelGGL((dev::k_selinv_split<T>), dim3(P.nheavy + (P.nblk - P.nheavy + W - 1) / W),
                               dim3(64 * W), 0, st, P);
            break;
        case SV_GROUP128:
            hipLaunchKernelGGL((dev::k_selinv_group<T, 128>), dim3(P.nblk), dim3(128), 0, st, P);
            break;
        case SV_GROUP256:
            hipLaunchKernelGGL((dev::k_selinv_group<T, 256>), dim3(P.nblk), dim3(256), 0, st, P);
            break;
        case SV_GROUP512:
            hipLaunchKernelGGL((dev::k_selinv_group<T, 512>), dim3(P.nblk), dim3(512), 0, st, P);
            break;
        case SV_BIG256:
        case SV_BIG1024: {
            const int32_t C = std::min<int32_t>(kBigCols, (maxc + 63) & ~63);
            const bool wide = variant == SV_BIG1024;
            const size_t lds = selinv_big_lds_bytes(sizeof(T) == 8, wide ? 1024 : 256, C);
            if (wide)
                hipLaunchKernelGGL((dev::k_selinv_big<T, 1024>), dim3(P.nblk), dim3(1024), lds, st, P, C);
            else
                hipLaunchKernelGGL((dev::k_selinv_big<T, 256>), dim3(P.nblk), dim3(256), lds, st, P, C);
            break;
        }
        default:
            hipLaunchKernelGGL((dev::k_selinv_small<T, W>), dim3((P.nblk + W - 1) / W), dim3(64 * W), 0, st, P);
            break;
    }
}

hipError_t launch_selinv_level(const SelinvParams &P, int variant, bool fp64, hipStream_t st, int32_t maxc) {
    if (P.nblk <= 0) return hipSuccess;
    if (variant < 0 || variant >= SV_COUNT) return hipErrorInvalidValue;
    if (fp64)
        launch_variant<double>(P, variant, maxc, st);
    else
        launch_variant<float>(P, variant, maxc, st);
    return hipGetLastError();
}

hipError_t launch_scatter_lu(int64_t nnzL, const int32_t *q2u, const double *Lval, void *Lu, bool fp64,
                             hipStream_t st) {
    if (nnzL <= 0) return hipSuccess;
    dim3 g((unsigned)((nnzL + 255) / 256));
    if (fp64)
        hipLaunchKernelGGL(dev::k_scatter_lu<double>, g, dim3(256), 0, st, nnzL, q2u, Lval,
                           reinterpret_cast<double *>(Lu));
    else
        hipLaunchKernelGGL(dev::k_scatter_lu<float>, g, dim3(256), 0, st, nnzL, q2u, Lval,
                           reinterpret_cast<float *>(Lu));
    return hipGetLastError();
}

// Largest co-resident grid of the dataflow kernel (0 if unavailable).
int flow_grid(bool fp64) {
    constexpr int W = 4;
    int dev = 0, cus = 0, per = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = fp64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, dev::k_selinv_flow<double, W>, 64 * W, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, dev::k_selinv_flow<float, W>, 64 * W, 0);
    if (e != hipSuccess) return 0;
    return per * cus;
}

hipError_t launch_selinv_flow(const SelinvParams &P, int32_t nblocks, int32_t *done, int32_t epoch,
                              int32_t spin_limit, bool fp64, int grid, hipStream_t st) {
    constexpr int W = 4;
    SelinvParams p = P;
    void *args[] = {&p, &nblocks, &done, &epoch, &spin_limit};
    const void *fn = fp64 ? (const void *)dev::k_selinv_flow<double, W> : (const void *)dev::k_selinv_flow<float, W>;
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(64 * W), args, 0, st);
}

hipError_t set_big_lds_limits() {
    const void *fns[] = {(const void *)dev::k_selinv_big<double, 256>, (const void *)dev::k_selinv_big<double, 1024>,
                         (const void *)dev::k_selinv_big<float, 256>, (const void *)dev::k_selinv_big<float, 1024>};
    const size_t bytes[] = {selinv_big_lds_bytes(true, 256, kBigCols), selinv_big_lds_bytes(true, 1024, kBigCols),
                            selinv_big_lds_bytes(false, 256, kBigCols), selinv_big_lds_bytes(false, 1024, kBigCols)};
    for (int i = 0; i < 4; ++i) {
        hipError_t e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes[i]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace asi
