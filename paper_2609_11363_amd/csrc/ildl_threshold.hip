// Threshold incomplete LDL^T factorization on the device: the pivot and drop
// decisions as well as the values (the factor the method starts from,
// Section 2.1; the paper's factorization is a separate sequential package and
// a parallel one is its stated future work).
//
// What is computed is the right-looking threshold factorization of the
// symmetrically scaled matrix Ah = S A(q, q) S, s_i = 1/sqrt(max_j |a_ij|),
// with 1x1 pivots taken in the given order: column p of the Schur
// complement is w(i) = Ah(p, i) - sum_m (l_pm d_m) l_im over the eliminated
// columns m that kept both p and i, in increasing m; d_p is the Schur
// diagonal (a pivot below 1e-14 max|Ah| is replaced by +-1e-8 max|Ah|), and
// l_ip = w(i) / d_p is kept when |l_ip| >= tau. L <- S^-1 L S and
// D <- S^-1 D S^-1 at the end. Every sum is formed in the same order and
// with the same roundings (no fused multiply-adds) as the sequential
// definition, so the result is that factorization bit for bit.
//
// Parallel schedule. Column i can be eliminated as soon as no remaining
// (uneliminated) column k < i is adjacent to it in the current Schur graph:
// then no remaining column can ever update it, its Schur column is final and
// equals the one the sequential order sees. Rounds eliminate every such
// column at once. A column that is still blocked records one blocker (the
// largest) and is examined again only after that blocker is gone.
//   - adjacency of i: its entries in A, and for every eliminated m that kept
//     i, the other rows m kept (the Schur fill between them);
//   - per round: (1) columns whose blocker is gone (or never set) are listed;
//     (2) one wavefront per listed column looks for a remaining smaller
//     neighbour; (3) one wavefront per ready column forms its Schur column in
//     an LDS hash table (keys distinct within a step, so the m-steps keep
//     each entry's sum in increasing m), decides its pivot and drops, writes
//     its kept rows sorted into a column pool and appends (p, l_ip) to the
//     row list of every kept row i; (4) columns too large for a wavefront
//     table run on a workgroup with a larger one.
// Effects of a round are not visible inside it: a column counts as
// eliminated only for rounds after its own.
//
// Bunch-Kaufman: with pivoting on, a column whose Schur diagonal fails the
// 1x1 test |d| >= alpha max_i |w(i)| would need a swap or a 2x2 pivot, which
// this factorization does not make: the call then fails (ST_PIVOT) and the
// caller uses the host factorization. Diagonally dominant inputs always pass.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "kernels.h"

// The sums are those of the sequential definition, one rounding per
// operation: no multiply-add contraction anywhere in this file.
#pragma clang fp contract(off)

namespace asi {
namespace dev {
namespace {

constexpr int32_t kRemaining = INT32_MAX;  // elim[] of a column not eliminated yet

__device__ inline void latch_t(int32_t *status, int32_t code) { atomicCAS(status, 0, code); }

__device__ inline void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename V>
__device__ inline V wmax(V v) {
    for (int o = 32; o > 0; o >>= 1) {
        V t = __shfl_xor(v, o, 64);
        v = t > v ? t : v;
    }
    return v;
}

__device__ inline int32_t wsum_i(int32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Fibonacci hash: the top bits of r * 2^32 / phi
__device__ inline uint32_t hslot(int32_t r, int lg) { return ((uint32_t)r * 2654435769u) >> (32 - lg); }

// Adds t to the entry of key r (inserted with value t when absent); one
// rounding, no contraction with the product that formed t. Keys are
// distinct among the lanes calling together. Returns false when the table
// is full (no free slot met within cap probes).
__device__ inline bool hadd(int32_t *keys, double *vals, int lg, int32_t r, double t, int32_t *count) {
    const uint32_t mask = (1u << lg) - 1u;
    uint32_t s = hslot(r, lg);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const int32_t old = atomicCAS(&keys[s], -1, r);
        if (old == -1) {
            vals[s] = t;
            atomicAdd(count, 1);
            return true;
        }
        if (old == r) {
            vals[s] = (vals[s] + t);
            return true;
        }
        s = (s + 1) & mask;
    }
    return false;
}

}  // namespace

// ---- set-up: inverse ordering, scaling, max |Ah| ----------------------------
__global__ void k_ildlt_init(IldlTParams P) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    P.iq[i] = -1;
    P.elim[i] = kRemaining;
    P.watch[i] = -1;
    P.rowcnt[i] = 0;
    P.collen[i] = 0;
    P.colptr[i] = 0;
}

__global__ void k_ildlt_scale(IldlTParams P) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const int32_t r = P.q[i];
    if (r < 0 || r >= P.n) {
        latch_t(P.status, ST_PERM);
        P.scale[i] = 1.0;
        return;
    }
    P.iq[r] = i;
    double m = 0.0;
    for (int64_t e = P.Ap[r]; e < P.Ap[r + 1]; ++e) m = fmax(m, fabs(P.Av[e]));
    P.scale[i] = m > 0.0 ? 1.0 / sqrt(m) : 1.0;
}

// Validates the inputs (q a permutation, columns in range: a failure is
// latched before any round runs) and takes max |Ah|.
__global__ void k_ildlt_amax(IldlTParams P) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    if (P.iq[i] < 0) latch_t(P.status, ST_PERM);
    const int32_t r = P.q[i];
    if (r < 0 || r >= P.n) return;
    const double si = P.scale[i];
    double m = 0.0;
    for (int64_t e = P.Ap[r]; e < P.Ap[r + 1]; ++e) {
        const int32_t c = P.Aj[e];
        if (c < 0 || c >= P.n) {
            latch_t(P.status, ST_PERM);
            continue;
        }
        const int32_t k = P.iq[c];
        if (k < 0 || k >= P.n) continue;
        m = fmax(m, fabs(((si * P.Av[e]) * P.scale[k])));
    }
    // non-negative doubles order like their bit patterns
    atomicMax(P.amax_bits, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_ildlt_reset(int32_t *counts) {
    if (threadIdx.x < 3) counts[threadIdx.x] = 0;
}

// ---- (1) columns to examine this round --------------------------------------
__global__ void k_ildlt_filter(IldlTParams P) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    if (P.elim[i] != kRemaining) return;
    const int32_t w = P.watch[i];
    if (w >= 0 && P.elim[w] >= P.round) return;  // its blocker is still there
    P.list_check[atomicAdd(&P.counts[0], 1)] = i;
}

// ---- (2) look for a remaining smaller neighbour -----------------------------
__global__ __launch_bounds__(256) void k_ildlt_check(IldlTParams P) {
    const int lane = threadIdx.x & 63;
    const int32_t nw = gridDim.x * 4;
    const int32_t total = P.counts[0];
    for (int32_t item = blockIdx.x * 4 + (threadIdx.x >> 6); item < total; item += nw) {
        const int32_t i = P.list_check[item];
        int32_t blocker = -1;
        // entries of A
        const int32_t r = P.q[i];
        for (int64_t e = P.Ap[r] + lane; e < P.Ap[r + 1]; e += 64) {
            const int32_t k = P.iq[P.Aj[e]];
            if (k < i && P.elim[k] == kRemaining) blocker = max(blocker, k);
        }
        // fill through the eliminated columns that kept i: their other rows
        // below i (the column's rows are sorted)
        const int32_t cnt = min(P.rowcnt[i], P.row_cap);
        const int64_t rb = (int64_t)i * P.row_cap;
        for (int32_t e = lane; e < cnt; e += 64) {
            const int32_t m = P.rk[rb + e];
            const int64_t c0 = P.colptr[m];
            const int32_t len = P.collen[m];
            for (int32_t t = 0; t < len; ++t) {
                const int32_t k = P.pr[c0 + t];
                if (k >= i) break;
                if (P.elim[k] == kRemaining) blocker = max(blocker, k);
            }
        }
        blocker = wmax(blocker);
        if (lane == 0) {
            if (blocker < 0)
                P.list_ready[atomicAdd(&P.counts[1], 1)] = i;
            else
                P.watch[i] = blocker;
        }
    }
}

// ---- (3), (4) form, decide and store a ready column --------------------------
// G threads per column; LG: log2 of the hash slots; KCAP: entries of K_p held
// (rows of L before p); OCAP: kept entries held. A column that does not fit
// is handed on (small variant) or refused (large variant).
template <int G, int LG, int KCAP, int OCAP>
struct ColumnLds {
    int32_t keys[1 << LG];
    double vals[1 << LG];
    int32_t km[KCAP];
    double kl[KCAP];
    int32_t orow[OCAP];
    double oval[OCAP];
    int32_t count, kept, flag;
    double dsum;
};

template <int G>
__device__ inline void gsync() {
    if constexpr (G == 64)
        wsync();
    else
        __syncthreads();
}

template <int G>
__device__ inline double group_max(double v, double *red) {
    v = wmax(v);
    if constexpr (G > 64) {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[w] = v;
        __syncthreads();
        double m = red[0];
        for (int q = 1; q < G / 64; ++q) m = fmax(m, red[q]);
        __syncthreads();
        return m;
    } else {
        return v;
    }
}

// Returns false when the column did not fit (the caller hands it on).
template <int G, int LG, int KCAP, int OCAP>
__device__ bool factor_column(const IldlTParams &P, int32_t p, ColumnLds<G, LG, KCAP, OCAP> &L, int tid,
                              double *red) {
    constexpr int HS = 1 << LG;
    const int32_t cnt = P.rowcnt[p];
    if (cnt > KCAP || cnt > P.row_cap) return false;
    const int64_t rb = (int64_t)p * P.row_cap;
    // K_p sorted by column: ranks among distinct columns
    for (int32_t e = tid; e < cnt; e += G) {
        L.km[e] = P.rk[rb + e];
        L.kl[e] = P.rv[rb + e];
    }
    for (int s = tid; s < HS; s += G) L.keys[s] = -1;
    if (tid == 0) {
        L.count = 0;
        L.kept = 0;
        L.flag = 0;
        L.dsum = 0.0;
    }
    gsync<G>();
    constexpr int PER = (KCAP + G - 1) / G;
    int32_t mm[PER], rk[PER];
    double ll[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int32_t e = tid + u * G;
        rk[u] = -1;
        if (e < cnt) {
            mm[u] = L.km[e];
            ll[u] = L.kl[e];
            int32_t rank = 0;
            for (int32_t f = 0; f < cnt; ++f) rank += L.km[f] < mm[u];
            rk[u] = rank;
        }
    }
    gsync<G>();
#pragma unroll
    for (int u = 0; u < PER; ++u)
        if (rk[u] >= 0) {
            L.km[rk[u]] = mm[u];
            L.kl[rk[u]] = ll[u];
        }
    // Ah(p, :) first: the entries before p were eliminated, the diagonal
    // starts the pivot's sum (one entry at most; 0 if A has none)
    const double sp = P.scale[p];
    const int32_t r = P.q[p];
    bool ok = true;
    for (int64_t e = P.Ap[r] + tid; e < P.Ap[r + 1]; e += G) {
        const int32_t k = P.iq[P.Aj[e]];
        const double a = ((sp * P.Av[e]) * P.scale[k]);
        if (k == p)
            L.dsum = a;
        else if (k > p)
            ok = ok && hadd(L.keys, L.vals, LG, k, a, &L.count);
    }
    if (!ok) L.flag = 1;
    gsync<G>();
    double diag = L.dsum;
    const int32_t limit = HS * 3 / 4;
    for (int32_t t = 0; t < cnt; ++t) {
        if (L.flag || L.count > limit) break;
        const int32_t m = L.km[t];
        const double lpm = L.kl[t];
        const double lm = (lpm * P.dpiv[m]);
        diag = (diag - (lm * lpm));
        const int64_t c0 = P.colptr[m];
        const int32_t len = P.collen[m];
        bool okm = true;
        for (int32_t u = tid; u < len; u += G) {
            const int32_t i = P.pr[c0 + u];
            if (i > p) okm = okm && hadd(L.keys, L.vals, LG, i, -(lm * P.pv[c0 + u]), &L.count);
        }
        if (!okm) L.flag = 1;
        gsync<G>();
    }
    if (L.flag || L.count > limit) return false;
    // pivot: Bunch-Kaufman 1x1 test, tiny pivot replacement
    double lam = 0.0;
    for (int s = tid; s < HS; s += G)
        if (L.keys[s] >= 0) lam = fmax(lam, fabs(L.vals[s]));
    lam = group_max<G>(lam, red);
    if (P.pivoting && lam > 0.0 && fabs(diag) < (P.alpha * lam)) {
        if (tid == 0) latch_t(P.status, ST_PIVOT);
    }
    double d = diag;
    const bool perturbed = fabs(d) < P.tiny;
    if (perturbed) d = (d >= 0.0 ? 1.0 : -1.0) * P.repl;
    // kept entries, then sorted by row
    for (int s = tid; s < HS; s += G) {
        const int32_t key = L.keys[s];
        if (key < 0) continue;
        const double l = (L.vals[s] / d);
        if (fabs(l) < P.tau) continue;
        const int32_t o = atomicAdd(&L.kept, 1);
        if (o < OCAP) {
            L.orow[o] = key;
            L.oval[o] = l;
        }
    }
    gsync<G>();
    const int32_t kept = L.kept;
    if (kept > OCAP) return false;
    constexpr int OPER = (OCAP + G - 1) / G;
    int32_t orow[OPER], ork[OPER];
    double oval[OPER];
#pragma unroll
    for (int u = 0; u < OPER; ++u) {
        const int32_t e = tid + u * G;
        ork[u] = -1;
        if (e < kept) {
            orow[u] = L.orow[e];
            oval[u] = L.oval[e];
            int32_t rank = 0;
            for (int32_t f = 0; f < kept; ++f) rank += L.orow[f] < orow[u];
            ork[u] = rank;
        }
    }
    // pool space for the column (thread 0 allocates; the others read it back)
    __shared__ unsigned long long base_sh[G > 64 ? 1 : 4];
    unsigned long long *bs = &base_sh[G > 64 ? 0 : (threadIdx.x >> 6)];
    if (tid == 0) *bs = atomicAdd(P.pool_top, (unsigned long long)kept);
    gsync<G>();
    const unsigned long long base = *bs;
    const bool fits = base + (unsigned long long)kept <= (unsigned long long)P.pool_cap;
#pragma unroll
    for (int u = 0; u < OPER; ++u) {
        if (ork[u] < 0) continue;
        if (fits) {
            P.pr[base + ork[u]] = orow[u];
            P.pv[base + ork[u]] = oval[u];
        }
        const int32_t i = orow[u];
        const int32_t pos = atomicAdd(&P.rowcnt[i], 1);
        if (pos < P.row_cap) {
            P.rk[(int64_t)i * P.row_cap + pos] = p;
            P.rv[(int64_t)i * P.row_cap + pos] = oval[u];
        } else {
            latch_t(P.status, ST_POOL);
        }
    }
    if (tid == 0) {
        if (!fits) latch_t(P.status, ST_POOL);
        P.colptr[p] = fits ? (int64_t)base : 0;
        P.collen[p] = fits ? kept : 0;
        P.dpiv[p] = d;
        P.elim[p] = P.round;
        atomicAdd(&P.counts[3], 1);
        if (perturbed) atomicAdd(&P.counts[4], 1);
    }
    return true;
}

constexpr int kSmallLg = 10;   // 1024 slots: up to 768 distinct rows
constexpr int kSmallK = 256;   // rows of L before p held by a wavefront
constexpr int kSmallOut = 768;
constexpr int kBigLg = 12;     // 4096 slots: up to 3072 distinct rows
constexpr int kBigK = 2048;
constexpr int kBigOut = 3072;

// one wavefront per ready column (2 per workgroup); columns that do not fit
// go to the large-column list
__global__ __launch_bounds__(128) void k_ildlt_factor(IldlTParams P) {
    __shared__ ColumnLds<64, kSmallLg, kSmallK, kSmallOut> lds[2];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int32_t nw = gridDim.x * 2;
    const int32_t total = P.counts[1];
    for (int32_t item = blockIdx.x * 2 + w; item < total; item += nw) {
        const int32_t p = P.list_ready[item];
        if (!factor_column<64, kSmallLg, kSmallK, kSmallOut>(P, p, lds[w], lane, nullptr)) {
            if (lane == 0) P.list_big[atomicAdd(&P.counts[2], 1)] = p;
        }
        wsync();
    }
}

// one 256-thread workgroup per large column (dynamic LDS: ColumnLds of the
// large variant)
__global__ __launch_bounds__(256) void k_ildlt_factor_big(IldlTParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    auto &L = *reinterpret_cast<ColumnLds<256, kBigLg, kBigK, kBigOut> *>(smem);
    __shared__ double red[4];
    const int32_t total = P.counts[2];
    for (int32_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int32_t p = P.list_big[item];
        if (!factor_column<256, kBigLg, kBigK, kBigOut>(P, p, L, threadIdx.x, red)) {
            if (threadIdx.x == 0) latch_t(P.status, ST_LIMIT);
        }
        __syncthreads();
    }
}

// ---- extraction: L in CSR (rows sorted, unscaled) and D ---------------------
__global__ void k_ildlt_rowcounts(IldlTParams P, int64_t *Lp) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) Lp[0] = 0;
    if (i >= P.n) return;
    Lp[i + 1] = min(P.rowcnt[i], P.row_cap);
}

__global__ __launch_bounds__(256) void k_ildlt_rows(IldlTParams P, const int64_t *Lp, int32_t *Lc, double *Lv,
                                                    double *dd, double *ds, int8_t *piv) {
    const int lane = threadIdx.x & 63;
    const int32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= P.n) return;
    const int32_t cnt = (int32_t)(Lp[i + 1] - Lp[i]);
    const int64_t rb = (int64_t)i * P.row_cap, o0 = Lp[i];
    const double si = P.scale[i];
    for (int32_t e = lane; e < cnt; e += 64) {
        const int32_t m = P.rk[rb + e];
        int32_t rank = 0;
        for (int32_t f = 0; f < cnt; ++f) rank += P.rk[rb + f] < m;
        Lc[o0 + rank] = m;
        Lv[o0 + rank] = (P.rv[rb + e] * P.scale[m]) / si;
    }
    if (lane == 0) {
        dd[i] = (P.dpiv[i] / (si * si));
        ds[i] = 0.0;
        piv[i] = 0;
    }
}

}  // namespace dev

size_t ildlt_big_lds_bytes() { return sizeof(dev::ColumnLds<256, dev::kBigLg, dev::kBigK, dev::kBigOut>); }

hipError_t ildlt_setup(const IldlTParams &P, hipStream_t st) {
    const dim3 g((unsigned)((P.n + 255) / 256)), b(256);
    hipLaunchKernelGGL(dev::k_ildlt_init, g, b, 0, st, P);
    hipLaunchKernelGGL(dev::k_ildlt_scale, g, b, 0, st, P);
    hipLaunchKernelGGL(dev::k_ildlt_amax, g, b, 0, st, P);
    return hipGetLastError();
}

hipError_t ildlt_round(const IldlTParams &P, int check_groups, int factor_groups, int big_groups, hipStream_t st) {
    const dim3 g((unsigned)((P.n + 255) / 256)), b(256);
    hipLaunchKernelGGL(dev::k_ildlt_reset, dim3(1), dim3(64), 0, st, P.counts);
    hipLaunchKernelGGL(dev::k_ildlt_filter, g, b, 0, st, P);
    hipLaunchKernelGGL(dev::k_ildlt_check, dim3((unsigned)check_groups), dim3(256), 0, st, P);
    hipLaunchKernelGGL(dev::k_ildlt_factor, dim3((unsigned)factor_groups), dim3(128), 0, st, P);
    hipLaunchKernelGGL(dev::k_ildlt_factor_big, dim3((unsigned)big_groups), dim3(256), ildlt_big_lds_bytes(), st, P);
    return hipGetLastError();
}

hipError_t ildlt_extract(const IldlTParams &P, int64_t *Lp, int32_t *Lc, double *Lv, double *dd, double *ds,
                         int8_t *piv, unsigned long long *bsum, hipStream_t st) {
    const dim3 g((unsigned)((P.n + 255) / 256)), b(256);
    hipLaunchKernelGGL(dev::k_ildlt_rowcounts, g, b, 0, st, P, Lp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_scan_counts(P.n, reinterpret_cast<unsigned long long *>(Lp), bsum, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dev::k_ildlt_rows, dim3((unsigned)((P.n + 3) / 4)), dim3(256), 0, st, P, Lp, Lc, Lv, dd, ds,
                       piv);
    return hipGetLastError();
}

hipError_t ildlt_set_limits() {
    return hipFuncSetAttribute((const void *)dev::k_ildlt_factor_big, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)ildlt_big_lds_bytes());
}

}  // namespace asi
