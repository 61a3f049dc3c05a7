// NInv kernels (truncated Neumann series of L^-1 and the product on S).
//
// Column j of L^inv: t^0 = e_j, t^m = drop_delta(E t^{m-1}) with E = I - L,
// L^inv(:, j) = sum_m t^m (Section 2.2). One wavefront builds one column in an
// LDS hash table keyed by row; the column of L that E t^{m-1} needs for a
// row k is the upper segment of row k of S (contiguous), with its values
// gathered through lsrc. Columns that outgrow the wavefront table are
// redone by a 256-thread workgroup with a larger table.
//
// N = (L^inv)^T D^-1 L^inv on S: for every (i, j) with i >= j in S,
// N_ij = sum_k L^inv(k, i) w_j(k), w_j = D^-1 L^inv(:, j). One wavefront per
// column j holds w_j in an LDS hash and streams the columns i of its row.
#include <hip/hip_runtime.h>

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

__device__ inline uint32_t hslot(int32_t r, int H) { return ((uint32_t)r * 2654435761u) & (uint32_t)(H - 1); }

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

template <typename T>
struct LinvLds {
    int32_t *key;
    T *cur, *nxt, *ser;
    int32_t *lk;   // compact list of the current term: rows
    T *lv;         //   and values
    int32_t *off;  // segment offsets (H + 1)
    int32_t *scr;  // scan scratch
    int32_t *flag; // [0] overflow, [2] column fits the pool
    int64_t *base; // pool offset of the column
};

// builds column j of L^inv; returns false if the table overflowed
template <typename T, int G>
__device__ bool linv_column(const NinvParams &P, int32_t j, const LinvLds<T> &S, int H, int tid) {
    for (int s = tid; s < H; s += G) {
        S.key[s] = -1;
        S.cur[s] = T(0);
        S.nxt[s] = T(0);
        S.ser[s] = T(0);
    }
    if (tid == 0) {
        S.flag[0] = 0;
        S.flag[1] = 0;
    }
    gsync<G>();
    if (tid == 0) {
        int s = hinsert(S.key, H, j);
        S.cur[s] = T(1);
        S.ser[s] = T(1);
    }
    gsync<G>();
    const T delta = (T)P.delta;
    for (int m = 1; m <= P.p; ++m) {
        // compact the support of t^{m-1}
        int32_t mine = 0;
        for (int s = tid; s < H; s += G) mine += (S.key[s] >= 0 && S.cur[s] != T(0));
        int32_t nl;
        int32_t pos = group_excl_scan<G>(mine, S.scr, &nl);
        for (int s = tid; s < H; s += G)
            if (S.key[s] >= 0 && S.cur[s] != T(0)) {
                S.lk[pos] = S.key[s];
                S.lv[pos] = S.cur[s];
                ++pos;
            }
        gsync<G>();
        if (nl == 0) break;
        // segment lengths of the L columns to scatter
        for (int b = tid; b < nl; b += G) {
            int32_t k = S.lk[b];
            S.off[b + 1] = (int32_t)(P.rowptr[k + 1] - P.diagpos[k] - 1);
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
        for (int32_t t = tid; t < total; t += G) {
            int lo = 0, hi = nl - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (S.off[mid] <= t)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            int32_t k = S.lk[lo];
            int64_t q = P.diagpos[k] + 1 + (t - S.off[lo]);
            int64_t src = P.lsrc[q];
            if (src < 0) continue;  // structural zero of a 2x2 union or the (k, k+1) slot
            T val = -S.lv[lo] * (T)P.Lval[src];
            int s = hinsert(S.key, H, P.col[q]);
            if (s < 0) {
                S.flag[0] = 1;
                continue;
            }
            atomicAdd(&S.nxt[s], val);
        }
        gsync<G>();
        if (S.flag[0]) return false;
        // drop |t| < delta from the new term and add it to the series
        for (int s = tid; s < H; s += G) {
            T v = S.nxt[s];
            S.nxt[s] = T(0);
            bool keep = S.key[s] >= 0 && v != T(0) && !(fabs(v) < delta);
            S.cur[s] = keep ? v : T(0);
            if (keep) S.ser[s] += v;
        }
        gsync<G>();
    }
    // block partners of 2x2 rows must be present for w = D^-1 L^inv
    for (int s = tid; s < H; s += G) {
        int32_t r = S.key[s];
        if (r >= 0 && S.ser[s] != T(0)) {
            int8_t pv = P.piv[r];
            if (pv != 0) {
                int32_t partner = pv == 1 ? r + 1 : r - 1;
                if (hinsert(S.key, H, partner) < 0) S.flag[0] = 1;
            }
        }
    }
    gsync<G>();
    return S.flag[0] == 0;
}

// writes the finished column to the pool
template <typename T, int G>
__device__ void linv_emit(const NinvParams &P, int32_t j, const LinvLds<T> &S, int H, int tid) {
    auto wanted = [&](int s) -> bool {
        int32_t r = S.key[s];
        if (r < 0) return false;
        if (S.ser[s] != T(0)) return true;
        int8_t pv = P.piv[r];
        if (pv == 0) return false;
        int ps = hfind(S.key, H, pv == 1 ? r + 1 : r - 1);
        return ps >= 0 && S.ser[ps] != T(0);
    };
    int32_t mine = 0;
    for (int s = tid; s < H; s += G) mine += wanted(s);
    int32_t cnt;
    int32_t pos = group_excl_scan<G>(mine, S.scr, &cnt);
    if (tid == 0) {
        unsigned long long base = atomicAdd(P.pool_top, (unsigned long long)cnt);
        bool fits = (int64_t)(base + cnt) <= P.pool_cap;
        if (!fits) latch2(P.status, ST_POOL);
        S.flag[2] = fits ? 1 : 0;
        S.base[0] = (int64_t)base;
    }
    gsync<G>();
    const bool fits = S.flag[2] != 0;
    const int64_t base = S.base[0];
    if (fits) {
        T *plinv = reinterpret_cast<T *>(P.plinv);
        T *pw = reinterpret_cast<T *>(P.pw);
        for (int s = tid; s < H; s += G) {
            if (!wanted(s)) continue;
            int32_t r = S.key[s];
            T lv = S.ser[s];
            int8_t pv = P.piv[r];
            T w;
            if (pv == 0) {
                w = (T)P.dinv[3 * (int64_t)r] * lv;
            } else {
                int32_t K = pv == 1 ? r : r - 1;
                int ps = hfind(S.key, H, pv == 1 ? r + 1 : r - 1);
                T other = ps >= 0 ? S.ser[ps] : T(0);
                const double *iv = P.dinv + 3 * (int64_t)K;
                if (pv == 1)
                    w = (T)iv[0] * lv + (T)iv[1] * other;
                else
                    w = (T)iv[1] * other + (T)iv[2] * lv;
            }
            int64_t d = base + pos++;
            P.prow[d] = r;
            plinv[d] = lv;
            pw[d] = w;
        }
    }
    if (tid == 0) {
        P.cstart[j] = base;
        P.clen[j] = fits ? cnt : 0;
    }
}

constexpr int kLinvH = 512;
constexpr int kLinvHBig = 2048;

template <typename T, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_linv_small(NinvParams P) {
    __shared__ int32_t key[WAVES][kLinvH];
    __shared__ T cur[WAVES][kLinvH], nxt[WAVES][kLinvH], ser[WAVES][kLinvH];
    __shared__ int32_t lk[WAVES][kLinvH];
    __shared__ T lv[WAVES][kLinvH];
    __shared__ int32_t off[WAVES][kLinvH + 1];
    __shared__ int32_t scr[WAVES][8];
    __shared__ int32_t flag[WAVES][8];
    __shared__ int64_t basev[WAVES];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t j = blockIdx.x * WAVES + w;
    if (j >= P.n) return;
    LinvLds<T> S{key[w], cur[w], nxt[w], ser[w], lk[w], lv[w], off[w], scr[w], flag[w], &basev[w]};
    if (linv_column<T, 64>(P, j, S, kLinvH, lane)) {
        linv_emit<T, 64>(P, j, S, kLinvH, lane);
    } else if (lane == 0) {
        P.clen[j] = -1;
        int32_t slot = atomicAdd(P.ovf_count, 1);
        P.ovf_list[slot] = j;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_linv_big(NinvParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int H = kLinvHBig;
    int64_t *basev = reinterpret_cast<int64_t *>(smem);
    T *cur = reinterpret_cast<T *>(smem + 16);
    T *nxt = cur + H;
    T *ser = nxt + H;
    T *lv = ser + H;
    int32_t *key = reinterpret_cast<int32_t *>(lv + H);
    int32_t *lk = key + H;
    int32_t *off = lk + H;
    int32_t *scr = off + H + 1;
    int32_t *flag = scr + 8;
    LinvLds<T> S{key, cur, nxt, ser, lk, lv, off, scr, flag, basev};
    const int32_t cnt = *P.ovf_count;
    for (int32_t idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
        int32_t j = P.ovf_list[idx];
        if (linv_column<T, 256>(P, j, S, H, threadIdx.x)) {
            linv_emit<T, 256>(P, j, S, H, threadIdx.x);
        } else if (threadIdx.x == 0) {
            P.clen[j] = 0;
            latch2(P.status, ST_LIMIT);
        }
        __syncthreads();
    }
}

// ---- product N on S --------------------------------------------------------

template <typename T>
struct ProdLds {
    int32_t *key;
    T *w;
    T *acc;
    int32_t *off;
    int64_t *start;
};

template <typename T, int G>
__device__ void nprod_column(const NinvParams &P, int32_t j, const ProdLds<T> &S, int H, int tid) {
    const T *plinv = reinterpret_cast<const T *>(P.plinv);
    const T *pw = reinterpret_cast<const T *>(P.pw);
    const int64_t p0 = P.diagpos[j];
    const int32_t ct = (int32_t)(P.rowptr[j + 1] - p0);  // targets i = col[p0 + t], i >= j
    for (int s = tid; s < H; s += G) S.key[s] = -1;
    gsync<G>();
    const int64_t cs = P.cstart[j];
    const int32_t cl = P.clen[j];
    for (int t = tid; t < cl; t += G) {
        int s = hinsert(S.key, H, P.prow[cs + t]);
        S.w[s] = pw[cs + t];
    }
    for (int t = tid; t < ct; t += G) {
        int32_t i = P.col[p0 + t];
        S.acc[t] = T(0);
        S.start[t] = P.cstart[i];
        S.off[t + 1] = P.clen[i];
    }
    gsync<G>();
    if (tid < 64) {
        int32_t carry = 0;
        for (int base = 0; base < ct; base += 64) {
            int t = base + tid;
            int32_t v = t < ct ? S.off[t + 1] : 0;
            int32_t s = v;
            for (int o = 1; o < 64; o <<= 1) {
                int32_t u = __shfl_up(s, o, 64);
                if (tid >= o) s += u;
            }
            s += carry;
            if (t < ct) S.off[t + 1] = s;
            carry = __shfl(s, 63, 64);
        }
        if (tid == 0) S.off[0] = 0;
    }
    gsync<G>();
    const int32_t total = S.off[ct];
    for (int32_t t = tid; t < total; t += G) {
        int lo = 0, hi = ct - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (S.off[mid] <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        int64_t q = S.start[lo] + (t - S.off[lo]);
        int s = hfind(S.key, H, P.prow[q]);
        if (s >= 0) atomicAdd(&S.acc[lo], plinv[q] * S.w[s]);
    }
    gsync<G>();
    for (int t = tid; t < ct; t += G) {
        double v = (double)S.acc[t];
        P.out[p0 + t] = v;
        if (t > 0) P.out[P.mirror[p0 + t]] = v;
    }
}

constexpr int kProdH = 512;
constexpr int kProdCt = 160;
constexpr int kProdHBig = 4096;
constexpr int kProdCtBig = kBigCols + 2;

template <typename T, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_nprod_small(NinvParams P) {
    __shared__ int32_t key[WAVES][kProdH];
    __shared__ T wv[WAVES][kProdH];
    __shared__ T acc[WAVES][kProdCt];
    __shared__ int32_t off[WAVES][kProdCt + 1];
    __shared__ int64_t start[WAVES][kProdCt];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t j = blockIdx.x * WAVES + w;
    if (j >= P.n) return;
    const int32_t ct = (int32_t)(P.rowptr[j + 1] - P.diagpos[j]);
    if (P.clen[j] > kProdH / 2 || ct > kProdCt) {
        if (lane == 0) {
            int32_t slot = atomicAdd(P.ovf2_count, 1);
            P.ovf2_list[slot] = j;
        }
        return;
    }
    ProdLds<T> S{key[w], wv[w], acc[w], off[w], start[w]};
    nprod_column<T, 64>(P, j, S, kProdH, lane);
}

template <typename T>
__global__ __launch_bounds__(256) void k_nprod_big(NinvParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int H = kProdHBig;
    int64_t *start = reinterpret_cast<int64_t *>(smem);
    T *wv = reinterpret_cast<T *>(start + kProdCtBig);
    T *acc = wv + H;
    int32_t *key = reinterpret_cast<int32_t *>(acc + kProdCtBig);
    int32_t *off = key + H;
    ProdLds<T> S{key, wv, acc, off, start};
    const int32_t cnt = *P.ovf2_count;
    for (int32_t idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
        int32_t j = P.ovf2_list[idx];
        if (P.clen[j] > H / 2) {
            if (threadIdx.x == 0) latch2(P.status, ST_LIMIT);
        } else {
            nprod_column<T, 256>(P, j, S, H, threadIdx.x);
        }
        __syncthreads();
    }
}

__global__ void k_ninv_reset(NinvParams P) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *P.pool_top = 0ull;
        *P.ovf_count = 0;
        *P.ovf2_count = 0;
    }
}

template <typename T>
size_t linv_big_lds() {
    return 16 + 4 * (size_t)kLinvHBig * sizeof(T) + (3 * (size_t)kLinvHBig + 1 + 8 + 8) * 4 + 64;
}
template <typename T>
size_t nprod_big_lds() {
    return (size_t)kProdCtBig * 8 + (size_t)kProdHBig * sizeof(T) + (size_t)kProdCtBig * sizeof(T) +
           (size_t)kProdHBig * 4 + ((size_t)kProdCtBig + 1) * 4 + 64;
}

template <typename T>
hipError_t run_ninv(const NinvParams &P, hipStream_t st) {
    hipLaunchKernelGGL(k_ninv_reset, dim3(1), dim3(64), 0, st, P);
    constexpr int W = 2;
    hipLaunchKernelGGL((k_linv_small<T, W>), dim3((P.n + W - 1) / W), dim3(64 * W), 0, st, P);
    size_t l1 = linv_big_lds<T>();
    hipFuncSetAttribute((const void *)k_linv_big<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l1);
    hipLaunchKernelGGL((k_linv_big<T>), dim3(256), dim3(256), l1, st, P);
    constexpr int W2 = 4;
    hipLaunchKernelGGL((k_nprod_small<T, W2>), dim3((P.n + W2 - 1) / W2), dim3(64 * W2), 0, st, P);
    size_t l2 = nprod_big_lds<T>();
    hipFuncSetAttribute((const void *)k_nprod_big<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l2);
    hipLaunchKernelGGL((k_nprod_big<T>), dim3(256), dim3(256), l2, st, P);
    return hipGetLastError();
}

}  // namespace dev

hipError_t launch_ninv(const NinvParams &P, bool fp64, hipStream_t st) {
    return fp64 ? dev::run_ninv<double>(P, st) : dev::run_ninv<float>(P, st);
}

}  // namespace asi
