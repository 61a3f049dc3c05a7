// NInv and Mix on their own pattern (an addition beside the S-restricted
// calls): the product N = (L^inv)^T D^-1 L^inv over every pair of columns of
// L^inv that meet a common D block, with the off-diagonal entries
// |N_ij| < drop sqrt(|N_ii N_jj|) removed (the product drop, Section 2.2), and
// Mix on that pattern joined with S_eps (Section 2.3). Both results are the
// lower triangle (diagonal included) in CSR with sorted columns.
//
// The columns of L^inv (rows, L^inv values and w = D^-1 L^inv) come from the
// series kernels into the NInv pool. Row i of N is sum_k L^inv(k, i) w(k, :),
// so the rows of w are needed: the pool's w is transposed (count, scan,
// fill, per-row sort). Every sum of this file runs in a fixed order (pool
// columns sorted by row, rows of w sorted by column, k ascending), so a call
// is repeatable bit for bit whenever the series columns are (they are not
// when a column needed the workgroup series kernel, whose LDS sums add in
// run-dependent order). One wavefront builds a row of N in an LDS hash keyed by
// column; rows with more distinct columns than its table holds are redone by
// a workgroup with a larger table. A count pass sizes the rows; the fill pass
// recomputes them and writes each row's kept entries in column order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace asi {
namespace dev {

namespace {

__device__ inline void latch3(int32_t *status, int32_t code) { atomicCAS(status, 0, code); }

// Fibonacci hashing as in the series kernels: top bits of j * 2^32 / phi
__device__ inline uint32_t fslot(int32_t j, int H) {
    return ((uint32_t)j * 2654435761u) >> (32 - (31 - __builtin_clz((unsigned)H)));
}

// insert-or-find j; counts claimed slots in *used; -1 once more than H / 2
// slots are in use (the caller then hands the row to the larger table)
__device__ inline int fins(int32_t *keys, int H, int32_t j, int32_t *used) {
    uint32_t s = fslot(j, H);
    for (int probe = 0; probe < H; ++probe) {
        int32_t k = keys[s];
        if (k == j) return (int)s;
        if (k == -1) {
            int32_t old = atomicCAS(&keys[s], -1, j);
            if (old == -1) {
                if (atomicAdd(used, 1) >= H / 2) return -1;
                return (int)s;
            }
            if (old == j) return (int)s;
        }
        s = (s + 1) & (uint32_t)(H - 1);
    }
    return -1;
}

template <int G>
__device__ inline void grp_sync() {
    if constexpr (G == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

}  // namespace

// pool column j sorted by row (insertion sort of (row, linv, w) in place)
__global__ void k_pool_sort(int32_t n, const int64_t *__restrict__ cstart, const int32_t *__restrict__ clen,
                            int32_t *__restrict__ prow, double *__restrict__ plinv, double *__restrict__ pw) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t b = cstart[j];
    const int32_t c = clen[j];
    for (int32_t a = 1; a < c; ++a) {
        const int32_t r = prow[b + a];
        const double l = plinv[b + a], w = pw[b + a];
        int32_t q = a - 1;
        while (q >= 0 && prow[b + q] > r) {
            prow[b + q + 1] = prow[b + q];
            plinv[b + q + 1] = plinv[b + q];
            pw[b + q + 1] = pw[b + q];
            --q;
        }
        prow[b + q + 1] = r;
        plinv[b + q + 1] = l;
        pw[b + q + 1] = w;
    }
}

// entries per row of w (cnt[k + 1] += 1 per entry; cnt[0] = 0 set by the caller)
__global__ void k_wt_count(int32_t n, const int64_t *__restrict__ cstart, const int32_t *__restrict__ clen,
                           const int32_t *__restrict__ prow, unsigned long long *__restrict__ cnt) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t b = cstart[j];
    for (int32_t a = 0; a < clen[j]; ++a) atomicAdd(&cnt[prow[b + a] + 1], 1ull);
}

// scatter of the pool's w into the rows of w (positions from the cursors)
__global__ void k_wt_fill(int32_t n, const int64_t *__restrict__ cstart, const int32_t *__restrict__ clen,
                          const int32_t *__restrict__ prow, const double *__restrict__ pw,
                          unsigned long long *__restrict__ cur, int32_t *__restrict__ colT, double *__restrict__ valT) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t b = cstart[j];
    for (int32_t a = 0; a < clen[j]; ++a) {
        const int64_t d = (int64_t)atomicAdd(&cur[prow[b + a]], 1ull);
        colT[d] = j;
        valT[d] = pw[b + a];
    }
}

// row k of w sorted by column
__global__ void k_wt_sort(int32_t n, const int64_t *__restrict__ rpT, int32_t *__restrict__ colT,
                          double *__restrict__ valT) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t b = rpT[k], e = rpT[k + 1];
    for (int64_t a = b + 1; a < e; ++a) {
        const int32_t c = colT[a];
        const double v = valT[a];
        int64_t q = a - 1;
        while (q >= b && colT[q] > c) {
            colT[q + 1] = colT[q];
            valT[q + 1] = valT[q];
            --q;
        }
        colT[q + 1] = c;
        valT[q + 1] = v;
    }
}

// N_jj = sum_k L^inv(k, j) w(k, j), k ascending
__global__ void k_ndiag(int32_t n, const int64_t *__restrict__ cstart, const int32_t *__restrict__ clen,
                        const double *__restrict__ plinv, const double *__restrict__ pw, double *__restrict__ dN) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t b = cstart[j];
    double s = 0.0;
    for (int32_t a = 0; a < clen[j]; ++a) s += plinv[b + a] * pw[b + a];
    dN[j] = s;
}

// One row i of N (lower part) in a hash of H slots held by a group of G
// threads. FILL = false: count the kept entries into cnt[i + 1]; FILL = true:
// write them in column order at rowptr[i]. Returns false if the row needs a
// larger table.
template <int G, bool FILL>
__device__ bool nfull_row(const NfullParams &P, int32_t i, int32_t *keys, double *acc, int32_t *list,
                          double *lval, int32_t *used, int H, int tid) {
    for (int s = tid; s < H; s += G) {
        keys[s] = -1;
        acc[s] = 0.0;
    }
    if (tid == 0) {
        used[0] = 0;
        used[1] = 0;
    }
    grp_sync<G>();
    const int64_t cb = P.cstart[i];
    const int32_t cl = P.clen[i];
    bool ok = true;
    for (int32_t a = 0; a < cl; ++a) {
        const int32_t k = P.prow[cb + a];
        const double lv = P.plinv[cb + a];
        const int64_t rb = P.rpT[k], re = P.rpT[k + 1];
        for (int64_t q = rb + tid; q < re; q += G) {
            const int32_t j = P.colT[q];
            if (j > i) continue;
            const int s = fins(keys, H, j, &used[0]);
            if (s < 0) {
                ok = false;
                continue;
            }
            acc[s] += lv * P.valT[q];  // the columns of one row of w are distinct
        }
        grp_sync<G>();
    }
    // the table overflowed in some thread: the whole group gives the row up
    if (!ok) used[1] = 1;
    grp_sync<G>();
    if (used[1]) return false;
    // kept entries: the diagonal, and |N_ij| >= drop sqrt(|N_ii N_jj|)
    const double di = P.dN[i];
    if (tid == 0) used[0] = 0;
    grp_sync<G>();
    for (int s = tid; s < H; s += G) {
        const int32_t j = keys[s];
        if (j < 0) continue;
        const double v = acc[s];
        if (j == i || fabs(v) >= P.drop * sqrt(fabs(di * P.dN[j]))) {
            const int32_t t = atomicAdd(&used[0], 1);
            list[t] = j;
            lval[t] = v;
        }
    }
    grp_sync<G>();
    const int32_t m = used[0];
    if constexpr (!FILL) {
        if (tid == 0) P.cnt[i + 1] = (unsigned long long)m;
    } else {
        const int64_t base = P.rowptr[i];
        const int64_t room = P.rowptr[i + 1] - base;  // the count pass's size of this row
        for (int t = tid; t < m; t += G) {
            const int32_t j = list[t];
            int32_t rank = 0;
            for (int32_t u = 0; u < m; ++u) rank += list[u] < j;
            if (rank < room) {
                P.col[base + rank] = j;
                P.val[base + rank] = lval[t];
            }
        }
        if (tid == 0 && m != room) latch3(P.status, ST_LIMIT);
    }
    grp_sync<G>();
    return true;
}

constexpr int kNfH = 512;       // wavefront table
constexpr int kNfHBig = 4096;   // workgroup table

template <bool FILL>
__global__ __launch_bounds__(256) void k_nfull_small(NfullParams P) {
    constexpr int W = 4;
    __shared__ int32_t keys[W][kNfH];
    __shared__ double acc[W][kNfH];
    __shared__ int32_t list[W][kNfH / 2];
    __shared__ double lval[W][kNfH / 2];
    __shared__ int32_t used[W][2];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t i = blockIdx.x * W + w;
    if (i >= P.n) return;  // the whole wavefront leaves; no workgroup barrier follows
    if (!nfull_row<64, FILL>(P, i, keys[w], acc[w], list[w], lval[w], used[w], kNfH, lane) && lane == 0) {
        const int32_t slot = atomicAdd(P.ovf_count, 1);
        P.ovf_list[slot] = i;
    }
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_nfull_big(NfullParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *acc = reinterpret_cast<double *>(smem);
    double *lval = acc + kNfHBig;
    int32_t *keys = reinterpret_cast<int32_t *>(lval + kNfHBig / 2);
    int32_t *list = keys + kNfHBig;
    int32_t *used = list + kNfHBig / 2;
    const int32_t cnt = *P.ovf_count;
    for (int32_t idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
        const int32_t i = P.ovf_list[idx];
        if (!nfull_row<256, FILL>(P, i, keys, acc, list, lval, used, kNfHBig, threadIdx.x)) {
            if (threadIdx.x == 0) latch3(P.status, ST_LIMIT);
            if constexpr (!FILL) {
                if (threadIdx.x == 0) P.cnt[i + 1] = 0ull;
            }
        }
        __syncthreads();
    }
}

size_t nfull_big_lds() { return (size_t)kNfHBig * 8 + (size_t)kNfHBig / 2 * 8 + (size_t)kNfHBig * 4 + (size_t)kNfHBig / 2 * 4 + 16; }

// ---- inclusive scan of a[1..n] (int64 counts, a[0] = 0) -------------------
constexpr int kScanB = 1024;

__global__ __launch_bounds__(kScanB) void k_scan_block(int64_t n, unsigned long long *__restrict__ a,
                                                       unsigned long long *__restrict__ bsum) {
    __shared__ unsigned long long s[kScanB];
    const int64_t i = (int64_t)blockIdx.x * kScanB + threadIdx.x + 1;
    s[threadIdx.x] = i <= n ? a[i] : 0ull;
    __syncthreads();
    for (int off = 1; off < kScanB; off <<= 1) {
        unsigned long long v = threadIdx.x >= off ? s[threadIdx.x - off] : 0ull;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    if (i <= n) a[i] = s[threadIdx.x];
    if (threadIdx.x == kScanB - 1) bsum[blockIdx.x] = s[kScanB - 1];
}

// exclusive scan of the block sums, one workgroup walking them in chunks
__global__ __launch_bounds__(kScanB) void k_scan_sums(int64_t nb, unsigned long long *__restrict__ bsum) {
    __shared__ unsigned long long s[kScanB];
    __shared__ unsigned long long carry;
    if (threadIdx.x == 0) carry = 0ull;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += kScanB) {
        const int64_t i = c0 + threadIdx.x;
        const unsigned long long x = i < nb ? bsum[i] : 0ull;
        s[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < kScanB; off <<= 1) {
            unsigned long long v = threadIdx.x >= off ? s[threadIdx.x - off] : 0ull;
            __syncthreads();
            s[threadIdx.x] += v;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + s[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == kScanB - 1) carry += s[kScanB - 1];
        __syncthreads();
    }
}

__global__ void k_scan_add(int64_t n, unsigned long long *__restrict__ a, const unsigned long long *__restrict__ bsum) {
    const int64_t i = (int64_t)blockIdx.x * kScanB + threadIdx.x + 1;
    if (i <= n) a[i] += bsum[blockIdx.x];
}

__global__ void k_copy_u64(int64_t n, const unsigned long long *__restrict__ a, unsigned long long *__restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_zero_u64(int64_t n, unsigned long long *__restrict__ a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0ull;
}

// ---- Mix on N's pattern joined with S_eps -----------------------------------
// Row i: merge of N's row (lower, sorted) with the lower entries of S's row i
// that pass the Mix test; Z where the test holds, N elsewhere.
template <bool FILL>
__global__ void k_mixfull(MixFullParams P) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    int64_t a = P.Nrp[i];
    const int64_t ae = P.Nrp[i + 1];
    int64_t b = P.srp[i];
    const int64_t be = P.diagpos[i] + 1;  // lower part of row i of S, diagonal included
    const double zi = P.zdiag[i];
    int64_t out = FILL ? P.rowptr[i] : 0;
    int64_t m = 0;
    auto sel = [&](int64_t q) {
        const int32_t j = P.scol[q];
        return fabs(P.Z[q]) > P.eps * sqrt(fabs(zi * P.zdiag[j]));
    };
    while (b < be && !sel(b)) ++b;
    while (a < ae || b < be) {
        const int32_t ja = a < ae ? P.Ncol[a] : INT32_MAX;
        const int32_t jb = b < be ? P.scol[b] : INT32_MAX;
        int32_t j;
        double v;
        if (jb <= ja) {
            j = jb;
            v = P.Z[b];
            if (ja == jb) ++a;
            ++b;
            while (b < be && !sel(b)) ++b;
        } else {
            j = ja;
            v = P.Nval[a];
            ++a;
        }
        if constexpr (FILL) {
            if (out + m < P.rowptr[i + 1]) {
                P.col[out + m] = j;
                P.val[out + m] = v;
            }
        }
        ++m;
    }
    if constexpr (!FILL) P.cnt[i + 1] = (unsigned long long)m;
}

}  // namespace dev

hipError_t set_nfull_lds_limits() {
    hipError_t e = hipFuncSetAttribute((const void *)dev::k_nfull_big<false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)dev::nfull_big_lds());
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)dev::k_nfull_big<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)dev::nfull_big_lds());
    return e;
}

hipError_t launch_scan_counts(int64_t n, unsigned long long *a, unsigned long long *bsum, hipStream_t st) {
    const int64_t nb = (n + dev::kScanB - 1) / dev::kScanB;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_scan_block, dim3((unsigned)nb), dim3(dev::kScanB), 0, st, n, a, bsum);
    hipLaunchKernelGGL(dev::k_scan_sums, dim3(1), dim3(dev::kScanB), 0, st, nb, bsum);
    hipLaunchKernelGGL(dev::k_scan_add, dim3((unsigned)nb), dim3(dev::kScanB), 0, st, n, a, bsum);
    return hipGetLastError();
}

hipError_t launch_nfull_count_w(const NfullParams &P, hipStream_t st) {
    const int32_t n = P.n;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    const dim3 g1((unsigned)((n + 1 + 255) / 256));
    hipLaunchKernelGGL(dev::k_pool_sort, g, b, 0, st, n, P.cstart, P.clen, P.prow, P.plinv, P.pw);
    // rows of w: counts and row pointers (rpT[n] = entries of the series)
    hipLaunchKernelGGL(dev::k_zero_u64, g1, b, 0, st, (int64_t)n + 1, reinterpret_cast<unsigned long long *>(P.rpT));
    hipLaunchKernelGGL(dev::k_wt_count, g, b, 0, st, n, P.cstart, P.clen, P.prow,
                       reinterpret_cast<unsigned long long *>(P.rpT));
    hipError_t e = launch_scan_counts(n, reinterpret_cast<unsigned long long *>(P.rpT), P.bsum, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_nfull_fill_w(const NfullParams &P, hipStream_t st) {
    const int32_t n = P.n;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    const dim3 g1((unsigned)((n + 1 + 255) / 256));
    hipLaunchKernelGGL(dev::k_copy_u64, g1, b, 0, st, (int64_t)n + 1,
                       reinterpret_cast<const unsigned long long *>(P.rpT), P.cur);
    hipLaunchKernelGGL(dev::k_wt_fill, g, b, 0, st, n, P.cstart, P.clen, P.prow, P.pw, P.cur, P.colT, P.valT);
    hipLaunchKernelGGL(dev::k_wt_sort, g, b, 0, st, n, P.rpT, P.colT, P.valT);
    hipLaunchKernelGGL(dev::k_ndiag, g, b, 0, st, n, P.cstart, P.clen, P.plinv, P.pw, P.dN);
    return hipGetLastError();
}

hipError_t launch_nfull_rows(const NfullParams &P, bool fill, hipStream_t st) {
    const int32_t n = P.n;
    if (!fill)
        hipLaunchKernelGGL(dev::k_zero_u64, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, st, (int64_t)n + 1,
                           P.cnt);
    hipError_t e0 = launch_fill_i32(P.ovf_count, 1, 0, st);
    if (e0 != hipSuccess) return e0;
    const dim3 g((unsigned)((n + 3) / 4)), b(256);
    const size_t lds = dev::nfull_big_lds();
    if (fill) {
        hipLaunchKernelGGL(dev::k_nfull_small<true>, g, b, 0, st, P);
        hipLaunchKernelGGL(dev::k_nfull_big<true>, dim3(256), b, lds, st, P);
    } else {
        hipLaunchKernelGGL(dev::k_nfull_small<false>, g, b, 0, st, P);
        hipLaunchKernelGGL(dev::k_nfull_big<false>, dim3(256), b, lds, st, P);
        hipError_t e = launch_scan_counts(n, P.cnt, P.bsum, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_mixfull(const MixFullParams &P, bool fill, hipStream_t st) {
    const int32_t n = P.n;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    if (fill) {
        hipLaunchKernelGGL(dev::k_mixfull<true>, g, b, 0, st, P);
    } else {
        hipLaunchKernelGGL(dev::k_zero_u64, dim3((unsigned)((n + 1 + 255) / 256)), b, 0, st, (int64_t)n + 1, P.cnt);
        hipLaunchKernelGGL(dev::k_mixfull<false>, g, b, 0, st, P);
        hipError_t e = launch_scan_counts(n, P.cnt, P.bsum, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace asi
