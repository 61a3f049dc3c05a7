// NInv kernels (truncated Neumann series of L^-1 and the product on S).
//
// Column j of L^inv: t^0 = e_j, t^m = drop_delta(E t^{m-1}) with E = I - L,
// L^inv(:, j) = sum_m t^m (Section 2.2). One wavefront builds one column in an
// LDS hash table keyed by row; E t^{m-1} scatters the columns of L of the
// current term's rows (their u-ranges of the column layout). Columns that
// outgrow the wavefront table are redone by a 256-thread workgroup with a
// larger table. The series is computed in float64 in both precisions, from
// the float64 copy of L: its drop tests are discontinuous in the values, so a
// float32 series would keep or drop different entries near delta than the
// float64 method; the mixed-precision form stores the finished columns (and
// w = D^-1 L^inv) in float32 for the product.
//
// N = (L^inv)^T D^-1 L^inv on S: for every (i, j) in S (i >= j by symmetry),
// N_ij = sum_k L^inv(k, i) w_j(k), w_j = D^-1 L^inv(:, j). The series columns
// are stored sorted by row with w beside L^inv; the product goes through the
// transposed pattern of L^inv (below), with an entry-by-entry merge of the two
// columns as the fallback. Products are in the pool's precision, their sums in
// float64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace asi {
namespace dev {

__device__ inline void latch2(int32_t *status, int32_t code) { atomicCAS(status, 0, code); }

template <int G>
__device__ inline void gsync() {
    if constexpr (G == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Fibonacci hashing: the top log2(H) bits of r * 2^32/phi (the low bits of the
// product only depend on the low bits of r, which cluster for grid orderings)
__device__ inline uint32_t hslot(int32_t r, int H) {
    return ((uint32_t)r * 2654435761u) >> (32 - (31 - __builtin_clz((unsigned)H)));
}

// insert-or-find r in an LDS open-addressing table; -1 when full
__device__ inline int hinsert(int32_t *keys, int H, int32_t r) {
    uint32_t s = hslot(r, H);
    for (int probe = 0; probe < H; ++probe) {
        int32_t k = keys[s];
        if (k == r) return (int)s;
        if (k == -1) {
            int32_t old = atomicCAS(&keys[s], -1, r);
            if (old == -1 || old == r) return (int)s;
        }
        s = (s + 1) & (uint32_t)(H - 1);
    }
    return -1;
}

__device__ inline int hfind(const int32_t *keys, int H, int32_t r) {
    uint32_t s = hslot(r, H);
    for (int probe = 0; probe < H; ++probe) {
        int32_t k = keys[s];
        if (k == r) return (int)s;
        if (k == -1) return -1;
        s = (s + 1) & (uint32_t)(H - 1);
    }
    return -1;
}

// largest b in [0, c) with off[b] <= t
__device__ inline int seg_of_n(const int32_t *off, int c, int32_t t) {
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

// group-wide exclusive prefix of per-thread counts; returns this thread's
// offset and writes the total to *tot (LDS scratch of G/64 + 1 ints)
template <int G>
__device__ inline int32_t group_excl_scan(int32_t v, int32_t *scratch, int32_t *tot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t s = v;
    for (int o = 1; o < 64; o <<= 1) {
        int32_t t = __shfl_up(s, o, 64);
        if (lane >= o) s += t;
    }
    if constexpr (G == 64) {
        *tot = __shfl(s, 63, 64);
        return s - v;
    } else {
        if (lane == 63) scratch[w] = s;
        __syncthreads();
        int32_t base = 0, all = 0;
        for (int q = 0; q < G / 64; ++q) {
            if (q < w) base += scratch[q];
            all += scratch[q];
        }
        __syncthreads();
        *tot = all;
        return base + s - v;
    }
}

// group-wide maximum (LDS scratch of G/64 ints)
template <int G>
__device__ inline int32_t group_max_i(int32_t v, int32_t *scratch) {
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t t = __shfl_xor(v, o, 64);
        v = t > v ? t : v;
    }
    if constexpr (G == 64) {
        return v;
    } else {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        __syncthreads();
        if (lane == 0) scratch[w] = v;
        __syncthreads();
        int32_t m = scratch[0];
        for (int q = 1; q < G / 64; ++q) m = scratch[q] > m ? scratch[q] : m;
        __syncthreads();
        return m;
    }
}

template <typename T>
struct LinvLds {
    int32_t *key;  // H
    double *nxt, *ser;  // H: the term being accumulated, the series (float64 sums in both precisions)
    int32_t *tl;   // H: slots touched by the current column
    int32_t *lk;   // H: rows of the current term (compact)
    T *lv;         // H: values of the current term
    int32_t *off;  // H + 1: flattened offsets of the L columns to scatter
    int64_t *seg;  // H: u-range starts of those columns
    int32_t *scr;  // scan scratch
    int32_t *flag; // [0] overflow, [1] current term size, [2] column fits the pool, [3] touched count
    int64_t *base; // [0] pool offset of the column, [1] next free entry of this group's
                   // pool chunk, [2] end of the chunk
};

// Pool entries are handed out in chunks per group so the global counter is
// touched once per chunk rather than once per column.
constexpr int64_t kPoolChunk = 512;

// insert-or-find r; a newly claimed slot is appended to the touched list
__device__ inline int hinsert_t(int32_t *keys, int H, int32_t r, int32_t *tl, int32_t *ntouched) {
    uint32_t s = hslot(r, H);
    for (int probe = 0; probe < H; ++probe) {
        int32_t k = keys[s];
        if (k == r) return (int)s;
        if (k == -1) {
            int32_t old = atomicCAS(&keys[s], -1, r);
            if (old == -1) {
                tl[atomicAdd(ntouched, 1)] = (int32_t)s;
                return (int)s;
            }
            if (old == r) return (int)s;
        }
        s = (s + 1) & (uint32_t)(H - 1);
    }
    return -1;
}

template <typename T, int G, int H>
__device__ void linv_init(const LinvLds<T> &S, int tid) {
    for (int s = tid; s < H; s += G) {
        S.key[s] = -1;
        S.nxt[s] = T(0);
        S.ser[s] = T(0);
    }
    if (tid == 0) {
        S.flag[3] = 0;
        S.base[1] = 0;  // empty chunk
        S.base[2] = 0;
    }
    gsync<G>();
}

// resets the slots the last column touched
template <typename T, int G, int H>
__device__ void linv_reset(const LinvLds<T> &S, int tid) {
    const int32_t nt = S.flag[3];
    for (int i = tid; i < nt; i += G) {
        int s = S.tl[i];
        S.key[s] = -1;
        S.nxt[s] = T(0);
        S.ser[s] = T(0);
    }
    gsync<G>();
    if (tid == 0) S.flag[3] = 0;
    gsync<G>();
}

// builds column j of L^inv; returns false if the table (H slots) or the
// current-term arrays (TC entries) overflowed
template <typename T, int G, int H, int TC>
__device__ bool linv_column(const NinvParams &P, int32_t j, const LinvLds<T> &S, int tid) {
    const T *Lu = reinterpret_cast<const T *>(P.Lu);
    if (tid == 0) {
        S.flag[0] = 0;
        int s = hinsert_t(S.key, H, j, S.tl, &S.flag[3]);
        S.ser[s] = T(1);
        S.lk[0] = j;
        S.lv[0] = T(1);
        S.flag[1] = 1;
    }
    gsync<G>();
    const double delta = P.delta;
    int m0 = 1;
    if (P.p >= 1) {
        // t^1 = drop_delta(E e_j) = drop_delta(-L(:, j)): the rows of column j
        // are distinct, so the first term is a filter of the column (the
        // values -(1 * l) and the test of the general step below, without its
        // accumulation table)
        const int64_t u0 = P.ustart[j], u1 = P.ustart[j + 1];
        int32_t nn = 0;
        for (int64_t b0 = u0; b0 < u1; b0 += G) {
            const int64_t q = b0 + tid;
            int32_t key = -1;
            T v = T(0);
            if (q < u1) {
                const T l = Lu[q];
                v = -(T(1) * l);
                if (l != T(0) && !(fabs((double)v) < delta)) key = P.ucol[q];
            }
            int32_t cnt;
            const int32_t p0 = group_excl_scan<G>(key >= 0 ? 1 : 0, S.scr, &cnt);
            if (key >= 0) {
                const int s = hinsert_t(S.key, H, key, S.tl, &S.flag[3]);
                if (s < 0)
                    S.flag[0] = 1;
                else
                    S.ser[s] += v;
                if (nn + p0 < TC) {
                    S.lk[nn + p0] = key;
                    S.lv[nn + p0] = v;
                }
            }
            nn += cnt;
        }
        gsync<G>();
        if (tid == 0) {
            S.flag[1] = nn;
            if (nn > TC) S.flag[0] = 1;
        }
        gsync<G>();
        if (S.flag[0]) return false;
        m0 = 2;
    }
    for (int m = m0; m <= P.p; ++m) {
        const int32_t nl = S.flag[1];
        if (nl == 0) break;
        // columns of L (u-ranges) to scatter: E t = -sum_k t_k L(:, k)
        for (int b = tid; b < nl; b += G) {
            int32_t k = S.lk[b];
            int64_t u0 = P.ustart[k];
            S.seg[b] = u0;
            S.off[b + 1] = (int32_t)(P.ustart[k + 1] - u0);
        }
        gsync<G>();
        if (tid < 64) {
            int32_t carry = 0;
            for (int base = 0; base < nl; base += 64) {
                int t = base + tid;
                int32_t v = t < nl ? S.off[t + 1] : 0;
                int32_t s = v;
                for (int o = 1; o < 64; o <<= 1) {
                    int32_t u = __shfl_up(s, o, 64);
                    if (tid >= o) s += u;
                }
                s += carry;
                if (t < nl) S.off[t + 1] = s;
                carry = __shfl(s, 63, 64);
            }
            if (tid == 0) S.off[0] = 0;
        }
        gsync<G>();
        const int32_t total = S.off[nl];
        for (int32_t t0 = tid; t0 < total; t0 += 2 * G) {
            int64_t q[2];
            int b[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                int32_t t = t0 + u * G;
                b[u] = -1;
                if (t < total) {
                    b[u] = seg_of_n(S.off, nl, t);
                    q[u] = S.seg[b[u]] + (t - S.off[b[u]]);
                }
            }
            int32_t r[2];
            T l[2];
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (b[u] >= 0) {
                    r[u] = P.ucol[q[u]];
                    l[u] = Lu[q[u]];
                }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (b[u] < 0 || l[u] == T(0)) continue;  // padding of a 2x2 union or (k, k+1)
                int s = hinsert_t(S.key, H, r[u], S.tl, &S.flag[3]);
                if (s < 0) {
                    S.flag[0] = 1;
                    continue;
                }
                atomicAdd(&S.nxt[s], (double)(-S.lv[b[u]] * l[u]));
            }
        }
        gsync<G>();
        if (S.flag[0]) return false;
        // drop |t| < delta from the new term, add it to the series and make
        // it the current term (only touched slots can hold a value)
        const int32_t nt = S.flag[3];
        int32_t nn = 0, pos = 0;
        for (int i0 = 0; i0 < nt; i0 += G) {
            const int i = i0 + tid;
            int32_t key = -1;
            double v = 0.0;
            if (i < nt) {
                int s = S.tl[i];
                v = S.nxt[s];
                S.nxt[s] = 0.0;
                key = S.key[s];
                bool keep = v != 0.0 && !(fabs(v) < delta);
                if (keep)
                    S.ser[s] += v;
                else
                    key = -1;
            }
            int32_t cnt;
            int32_t p0 = group_excl_scan<G>(key >= 0 ? 1 : 0, S.scr, &cnt);
            if (key >= 0 && nn + p0 < TC) {
                S.lk[nn + p0] = key;
                S.lv[nn + p0] = (T)v;
            }
            nn += cnt;
        }
        (void)pos;
        if (tid == 0) {
            S.flag[1] = nn;
            if (nn > TC) S.flag[0] = 1;
        }
        gsync<G>();
        if (S.flag[0]) return false;
    }
    // block partners of 2x2 rows must be present for w = D^-1 L^inv
    {
        const int32_t nt = S.flag[3];
        gsync<G>();
        for (int i = tid; i < nt; i += G) {
            int s = S.tl[i];
            int32_t r = S.key[s];
            if (S.ser[s] != T(0)) {
                int8_t pv = P.piv[r];
                if (pv != 0) {
                    int32_t partner = pv == 1 ? r + 1 : r - 1;
                    if (hinsert_t(S.key, H, partner, S.tl, &S.flag[3]) < 0) S.flag[0] = 1;
                }
            }
        }
    }
    gsync<G>();
    return S.flag[0] == 0;
}

// writes the finished column to the pool
template <typename TP, int G, int H, int TC>
__device__ void linv_emit(const NinvParams &P, int32_t j, const LinvLds<double> &S, int tid) {
    auto wanted = [&](int s) -> bool {
        int32_t r = S.key[s];
        if (S.ser[s] != 0.0) return true;
        int8_t pv = P.piv[r];
        if (pv == 0) return false;
        int ps = hfind(S.key, H, pv == 1 ? r + 1 : r - 1);
        return ps >= 0 && S.ser[ps] != 0.0;
    };
    // which touched slots the column keeps, once per slot (held in nxt, which
    // is zero between terms and reset with the column); the kept rows are
    // also listed compactly in lk (free once the series is built) when they
    // fit, so that each entry's rank in the row order is counted over the
    // kept rows only
    const int32_t nt = S.flag[3];
    int32_t mine = 0;
    for (int i = tid; i < nt; i += G) {
        const int s = S.tl[i];
        const bool keep = wanted(s);
        S.nxt[s] = keep ? 1.0 : 0.0;
        mine += keep;
    }
    int32_t cnt;
    int32_t pos = group_excl_scan<G>(mine, S.scr, &cnt);
    const bool compact = cnt <= TC;
    if (compact)
        for (int i = tid; i < nt; i += G) {
            const int s = S.tl[i];
            if (S.nxt[s] != 0.0) S.lk[pos++] = S.key[s];
        }
    if (tid == 0) {
        int64_t base = S.base[1];
        if (base + cnt > S.base[2]) {
            // chunk size: at most kPoolChunk and at most half the pool split
            // over all groups, so small pools are not exhausted by reservations
            const int64_t groups = (int64_t)gridDim.x * (blockDim.x / G);
            int64_t want = P.pool_cap / (2 * groups);
            want = want < kPoolChunk ? want : kPoolChunk;
            want = want > cnt ? want : (int64_t)cnt;
            base = (int64_t)atomicAdd(P.pool_top, (unsigned long long)want);
            S.base[2] = base + want;
        }
        S.base[1] = base + cnt;
        bool fits = base + cnt <= P.pool_cap;
        if (!fits) latch2(P.status, ST_POOL);
        S.flag[2] = fits ? 1 : 0;
        S.base[0] = base;
    }
    gsync<G>();
    const bool fits = S.flag[2] != 0;
    const int64_t base = S.base[0];
    int32_t last = -1;  // the column's largest row (quick test of the product)
    if (fits) {
        TP *plinv = reinterpret_cast<TP *>(P.plinv);
        TP *pw = reinterpret_cast<TP *>(P.pw);
        for (int i = tid; i < nt; i += G) {
            const int s = S.tl[i];
            if (S.nxt[s] == 0.0) continue;
            int32_t r = S.key[s];
            // the column is stored sorted by row: the entry's rank among the
            // column's kept rows (rows are distinct)
            int32_t rank = 0;
            if (compact) {
                for (int i2 = 0; i2 < cnt; ++i2) rank += S.lk[i2] < r ? 1 : 0;
            } else {
                for (int i2 = 0; i2 < nt; ++i2) {
                    const int s2 = S.tl[i2];
                    rank += (S.key[s2] < r && S.nxt[s2] != 0.0) ? 1 : 0;
                }
            }
            last = r > last ? r : last;
            // the series is float64 in both precisions; the pool stores it
            // (and w = D^-1 L^inv) in the call's precision
            const double lv = S.ser[s];
            int8_t pv = P.piv[r];
            double w;
            if (pv == 0) {
                w = P.dinv[3 * (int64_t)r] * lv;
            } else {
                int32_t K = pv == 1 ? r : r - 1;
                int ps = hfind(S.key, H, pv == 1 ? r + 1 : r - 1);
                const double other = ps >= 0 ? S.ser[ps] : 0.0;
                const double *iv = P.dinv + 3 * (int64_t)K;
                if (pv == 1)
                    w = iv[0] * lv + iv[1] * other;
                else
                    w = iv[1] * other + iv[2] * lv;
            }
            const int64_t d = base + rank;
            P.prow[d] = r;
            plinv[d] = (TP)lv;
            pw[d] = (TP)w;
        }
    }
    last = group_max_i<G>(last, S.scr);
    if (tid == 0) {
        P.cstart[j] = base;
        P.clen[j] = fits ? cnt : 0;
        P.clast[j] = fits ? last : -1;
    }
    gsync<G>();
}

// ---- N on S through the transposed series pattern ---------------------------
// Row k of L^inv lists the columns whose series reaches row k. N_ij can be
// nonzero only where columns i and j share a row, so: count the columns of
// every row, scan, list them with their row (in the pool's free tail), then,
// one thread per listed (k, i), go over the columns j <= i of row k with
// (i, j) in S and evaluate N_ij by the merge of the two columns (the value of
// the entry-by-entry kernel, bit for bit), writing it at (i, j) and (j, i);
// every other entry of S is zero. A pair is evaluated by the first row the two
// columns share: the merge runs in increasing row order and gives up at a
// first shared row other than k, so each N_ij is summed once.
// This path applies when the lists fit the pool's free tail and every row
// holds at most kPairMax columns (a thread walks its row's list); otherwise
// the entry-by-entry kernel runs (each kernel reads the flag and returns
// early when it does not apply).
constexpr int32_t kPairMax = 4096;

__global__ void k_tr_init(NinvParams P) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= P.n) P.tr_ptr[i] = 0ull;
    if (i == 0) *P.tr_flag = 1;
}

__global__ void k_tr_count(NinvParams P) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P.n) return;
    const int64_t b = P.cstart[j];
    const int32_t len = P.clen[j];
    for (int32_t a = 0; a < len; ++a) atomicAdd(&P.tr_ptr[P.prow[b + a] + 1], 1ull);
}

// the lists go to the pool's rows array after its last reserved entry
__global__ void k_tr_start(NinvParams P) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long top = *P.pool_top, total = P.tr_ptr[P.n];
    if (k == 0 && top + 2 * total > (unsigned long long)P.pool_cap) *P.tr_flag = 0;
    if (k < P.n) P.tr_cur[k] = P.tr_ptr[k];
}

__global__ void k_tr_fill(NinvParams P) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P.n || *P.tr_flag == 0) return;
    int32_t *colT = P.prow + *P.pool_top;
    int32_t *rowT = colT + P.tr_ptr[P.n];
    const int64_t b = P.cstart[j];
    const int32_t len = P.clen[j];
    for (int32_t a = 0; a < len; ++a) {
        const int32_t k = P.prow[b + a];
        const unsigned long long pos = atomicAdd(&P.tr_cur[k], 1ull);
        colT[pos] = j;
        rowT[pos] = k;
        if (pos - P.tr_ptr[k] >= (unsigned long long)kPairMax) *P.tr_flag = 0;
    }
}

// zeros of N on S: 16-byte stores (out is 16-byte aligned when its first
// entry is; otherwise one entry at a time)
__global__ void k_nzero(NinvParams P, int64_t nnz) {
    if (*P.tr_flag == 0) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if ((reinterpret_cast<uintptr_t>(P.out) & 15) == 0) {
        double2 *o2 = reinterpret_cast<double2 *>(P.out);
        for (int64_t q = t; q < nnz / 2; q += stride) o2[q] = make_double2(0.0, 0.0);
        if (t == 0 && (nnz & 1)) P.out[nnz - 1] = 0.0;
    } else {
        for (int64_t q = t; q < nnz; q += stride) P.out[q] = 0.0;
    }
}

// position of column j in the sorted row i of S, or -1
__device__ inline int64_t s_pos(const NinvParams &P, int32_t i, int32_t j) {
    int64_t lo = P.rowptr[i], hi = P.rowptr[i + 1] - 1;
    while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t c = P.col[mid];
        if (c == j) return mid;
        if (c < j)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

// N_ij (i >= j) by the merge of the stored columns i and j of the series
template <typename T>
__device__ inline double n_entry(const NinvParams &P, int32_t i, int32_t j) {
    const T *plinv = reinterpret_cast<const T *>(P.plinv);
    const T *pw = reinterpret_cast<const T *>(P.pw);
    const int64_t ci = P.cstart[i], cj = P.cstart[j];
    const int32_t li = P.clen[i], lj = P.clen[j];
    double sum = 0.0;  // float64 sums also in mixed precision (float32 products)
    int32_t a = 0, b = 0;
    int32_t ra = a < li ? P.prow[ci] : INT32_MAX, rb = b < lj ? P.prow[cj] : INT32_MAX;
    while (a < li && b < lj) {
        if (ra == rb) {
            sum += (double)(plinv[ci + a] * pw[cj + b]);
            ++a;
            ++b;
            ra = a < li ? P.prow[ci + a] : INT32_MAX;
            rb = b < lj ? P.prow[cj + b] : INT32_MAX;
        } else if (ra < rb) {
            ++a;
            ra = a < li ? P.prow[ci + a] : INT32_MAX;
        } else {
            ++b;
            rb = b < lj ? P.prow[cj + b] : INT32_MAX;
        }
    }
    return sum;
}

// N_ij (i >= j) as n_entry, for the pair met through row k (which both
// columns hold): false, without the sum, when the first row the two columns
// share is not k (that row evaluates the pair)
template <typename T>
__device__ inline bool n_entry_at(const NinvParams &P, int32_t i, int32_t j, int32_t k, double &v) {
    const T *plinv = reinterpret_cast<const T *>(P.plinv);
    const T *pw = reinterpret_cast<const T *>(P.pw);
    const int64_t ci = P.cstart[i], cj = P.cstart[j];
    const int32_t li = P.clen[i], lj = P.clen[j];
    double sum = 0.0;  // float64 sums also in mixed precision (float32 products)
    bool first = true;
    int32_t a = 0, b = 0;
    int32_t ra = a < li ? P.prow[ci] : INT32_MAX, rb = b < lj ? P.prow[cj] : INT32_MAX;
    while (a < li && b < lj) {
        if (ra == rb) {
            if (first) {
                if (ra != k) return false;
                first = false;
            }
            sum += (double)(plinv[ci + a] * pw[cj + b]);
            ++a;
            ++b;
            ra = a < li ? P.prow[ci + a] : INT32_MAX;
            rb = b < lj ? P.prow[cj + b] : INT32_MAX;
        } else if (ra < rb) {
            ++a;
            ra = a < li ? P.prow[ci + a] : INT32_MAX;
        } else {
            ++b;
            rb = b < lj ? P.prow[cj + b] : INT32_MAX;
        }
    }
    v = sum;
    return true;
}

template <typename T>
__global__ __launch_bounds__(256) void k_npairs(NinvParams P) {
    if (*P.tr_flag == 0) return;
    const int64_t total = (int64_t)P.tr_ptr[P.n];
    const int32_t *colT = P.prow + *P.pool_top;
    const int32_t *rowT = colT + total;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const int32_t k = rowT[t], i = colT[t];
        const int64_t c0 = (int64_t)P.tr_ptr[k], c1 = (int64_t)P.tr_ptr[k + 1];
        for (int64_t b = c0; b < c1; ++b) {
            const int32_t j = colT[b];
            if (j > i) continue;
            const int64_t p = s_pos(P, i, j);
            if (p < 0) continue;
            double v;
            if (!n_entry_at<T>(P, i, j, k, v)) continue;
            P.out[p] = v;
            if (i != j) P.out[P.mirror[p]] = v;
        }
    }
}

constexpr int kLinvH = 256;
constexpr int kLinvTerm = 64;    // kept entries of one term (the series columns are short)
constexpr int kLinvHBig = 2048;
constexpr int kLinvGrid = 2048;  // workgroups of the persistent column kernel

// TP: the storage type of the pool (the series itself is float64)
template <typename TP, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_linv_small(NinvParams P) {
    __shared__ int32_t key[WAVES][kLinvH];
    __shared__ double nxt[WAVES][kLinvH], ser[WAVES][kLinvH];
    __shared__ int32_t tl[WAVES][kLinvH];
    __shared__ int32_t lk[WAVES][kLinvTerm];
    __shared__ double lv[WAVES][kLinvTerm];
    __shared__ int32_t off[WAVES][kLinvTerm + 1];
    __shared__ int64_t seg[WAVES][kLinvTerm];
    __shared__ int32_t scr[WAVES][8];
    __shared__ int32_t flag[WAVES][8];
    __shared__ int64_t basev[WAVES][3];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    LinvLds<double> S{key[w], nxt[w], ser[w], tl[w], lk[w], lv[w], off[w], seg[w], scr[w], flag[w], basev[w]};
    linv_init<double, 64, kLinvH>(S, lane);
    const int32_t stride = gridDim.x * WAVES;
    for (int32_t j = blockIdx.x * WAVES + w; j < P.n; j += stride) {
        if (linv_column<double, 64, kLinvH, kLinvTerm>(P, j, S, lane)) {
            linv_emit<TP, 64, kLinvH, kLinvTerm>(P, j, S, lane);
        } else if (lane == 0) {
            P.clen[j] = -1;
            int32_t slot = atomicAdd(P.ovf_count, 1);
            P.ovf_list[slot] = j;
        }
        linv_reset<double, 64, kLinvH>(S, lane);
    }
}

template <typename TP>
__global__ __launch_bounds__(256) void k_linv_big(NinvParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int H = kLinvHBig;
    int64_t *basev = reinterpret_cast<int64_t *>(smem);
    int64_t *seg = basev + 4;
    double *nxt = reinterpret_cast<double *>(seg + H);
    double *ser = nxt + H;
    double *lv = ser + H;
    int32_t *key = reinterpret_cast<int32_t *>(lv + H);
    int32_t *tl = key + H;
    int32_t *lk = tl + H;
    int32_t *off = lk + H;
    int32_t *scr = off + H + 1;
    int32_t *flag = scr + 8;
    LinvLds<double> S{key, nxt, ser, tl, lk, lv, off, seg, scr, flag, basev};
    const int32_t cnt = *P.ovf_count;
    if (cnt == 0) return;
    linv_init<double, 256, H>(S, threadIdx.x);
    for (int32_t idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
        int32_t j = P.ovf_list[idx];
        if (linv_column<double, 256, H, H>(P, j, S, threadIdx.x)) {
            linv_emit<TP, 256, H, H>(P, j, S, threadIdx.x);
        } else if (threadIdx.x == 0) {
            P.clen[j] = 0;
            latch2(P.status, ST_LIMIT);
        }
        linv_reset<double, 256, H>(S, threadIdx.x);
    }
}

// ---- product N on S --------------------------------------------------------

// N on S entry by entry: for (r, c) in S with i = max(r, c), j = min(r, c),
// N_ij = sum_k L^inv(k, i) w_j(k) over the rows k the two stored columns
// share (both sorted by row: a two-pointer merge), in increasing k; a row of
// column i absent from column j has w_j(k) = 0 and adds nothing. Both
// triangles are written directly.
template <typename T>
__device__ inline void nprod_one(const NinvParams &P, int64_t p, const int32_t *__restrict__ srow) {
    const int32_t r = srow[p], c = P.col[p];
    const int32_t i = r > c ? r : c, j = r > c ? c : r;
    // the rows of column i are >= i: without a row >= i in column j the two
    // columns share none and N_ij = 0
    P.out[p] = P.clast[j] < i ? 0.0 : n_entry<T>(P, i, j);
}

template <typename T>
__global__ __launch_bounds__(256) void k_nprod_entry(NinvParams P, int64_t nnz, const int32_t *__restrict__ srow) {
    if (*P.tr_flag != 0) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride)
        nprod_one<T>(P, p, srow);
}

__global__ void k_ninv_reset(NinvParams P) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *P.pool_top = 0ull;
        *P.ovf_count = 0;
    }
}

template <typename T>
size_t linv_big_lds() {
    return 32 + 8 * (size_t)kLinvHBig + 3 * (size_t)kLinvHBig * 8 +
           (4 * (size_t)kLinvHBig + 1 + 8 + 8) * 4 + 64;
}
// Workgroups of the persistent column kernel: as many as can be resident at
// once (so the grid-stride loop ends evenly), at most kLinvGrid.
template <typename T, int W>
int linv_grid(int64_t n, int cap) {
    static int resident = 0;  // per element type; the same value on every device of one type
    if (resident == 0) {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_linv_small<T, W>, 64 * W, 0) != hipSuccess ||
            per <= 0)
            per = 2;
        resident = cus * per;
    }
    int64_t g = std::min<int64_t>(std::min<int64_t>((n + W - 1) / W, kLinvGrid), resident);
    if (cap < 0) g = std::max<int64_t>(1, g / (-cap));
    if (cap > 0) g = std::min<int64_t>(g, cap);
    return (int)g;
}

template <typename T>
hipError_t run_ninv(const NinvParams &P, hipStream_t st, int cap) {
    hipLaunchKernelGGL(k_ninv_reset, dim3(1), dim3(64), 0, st, P);
    constexpr int W = 4;
    const int grid = linv_grid<T, W>(P.n, cap);
    hipLaunchKernelGGL((k_linv_small<T, W>), dim3(grid), dim3(64 * W), 0, st, P);
    size_t l1 = linv_big_lds<T>();
    hipLaunchKernelGGL((k_linv_big<T>), dim3(256), dim3(256), l1, st, P);
    const int64_t nnz = P.rowptr_n;
    if (nnz > 0) {
        // the grids of the two alternatives are bounded (grid-stride loops):
        // the one that does not apply exits at once
        const dim3 gn((unsigned)((P.n + 256) / 256)), b(256);
        const dim3 gs((unsigned)std::min<int64_t>((nnz + 255) / 256, 16384));
        hipLaunchKernelGGL(k_tr_init, gn, b, 0, st, P);
        hipLaunchKernelGGL(k_tr_count, gn, b, 0, st, P);
        hipError_t e = launch_scan_counts(P.n, P.tr_ptr, P.tr_bsum, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_tr_start, gn, b, 0, st, P);
        hipLaunchKernelGGL(k_tr_fill, gn, b, 0, st, P);
        hipLaunchKernelGGL(k_nzero, gs, b, 0, st, P, nnz);
        hipLaunchKernelGGL((k_npairs<T>), gs, b, 0, st, P);
        hipLaunchKernelGGL((k_nprod_entry<T>), gs, b, 0, st, P, nnz, P.srow);
    }
    return hipGetLastError();
}

}  // namespace dev

hipError_t set_ninv_lds_limits() {
    const void *fns[] = {(const void *)dev::k_linv_big<double>, (const void *)dev::k_linv_big<float>};
    const size_t bytes[] = {dev::linv_big_lds<double>(), dev::linv_big_lds<float>()};
    for (int i = 0; i < 2; ++i) {
        hipError_t e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes[i]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_linv(const NinvParams &P, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_ninv_reset, dim3(1), dim3(64), 0, st, P);
    constexpr int W = 4;
    const int grid = dev::linv_grid<double, W>(P.n, 0);
    hipLaunchKernelGGL((dev::k_linv_small<double, W>), dim3(grid), dim3(64 * W), 0, st, P);
    hipLaunchKernelGGL((dev::k_linv_big<double>), dim3(256), dim3(256), dev::linv_big_lds<double>(), st, P);
    return hipGetLastError();
}

hipError_t launch_ninv(const NinvParams &P, bool fp64, hipStream_t st, int linv_grid) {
    return fp64 ? dev::run_ninv<double>(P, st, linv_grid) : dev::run_ninv<float>(P, st, linv_grid);
}

}  // namespace asi
