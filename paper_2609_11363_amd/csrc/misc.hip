// Elementwise and per-column kernels on S: diagonal extraction, Mix
// selection, the rank-k correction and SPAI refinement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace asi {
namespace dev {

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

__global__ void k_zdiag(int32_t n, const int64_t *__restrict__ diagpos, const double *__restrict__ X,
                        double *__restrict__ d) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = X[diagpos[i]];
}

// Mix (Section 2.3): keep Z where |Z_ij| > eps sqrt(|Z_ii Z_jj|), else N.
// zdiag is a copy of Z's diagonal taken before this kernel so M may alias Z.
__device__ inline double mix_pick(double z, double n, double zi, double zj, double eps) {
    return fabs(z) > eps * sqrt(fabs(zi * zj)) ? z : n;
}

__global__ __launch_bounds__(256) void k_mix1(int64_t nnz, const int32_t *__restrict__ srow,
                                              const int32_t *__restrict__ col, const double *__restrict__ zdiag,
                                              const double *Z, const double *N, double eps, double *M) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) M[p] = mix_pick(Z[p], N[p], zdiag[srow[p]], zdiag[col[p]], eps);
}

// two entries per thread with 8- and 16-byte accesses when Z, N and M are
// 16-byte aligned (the index arrays are workspace regions); an odd tail
// entry is done alone
__global__ __launch_bounds__(256) void k_mix(int64_t nnz, const int32_t *__restrict__ srow,
                                             const int32_t *__restrict__ col, const double *__restrict__ zdiag,
                                             const double *Z, const double *N, double eps, double *M) {
    const int64_t p = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (p + 1 < nnz) {
        const int2 r = *reinterpret_cast<const int2 *>(srow + p);
        const int2 c = *reinterpret_cast<const int2 *>(col + p);
        const double2 z = *reinterpret_cast<const double2 *>(Z + p);
        const double2 n = *reinterpret_cast<const double2 *>(N + p);
        double2 m;
        m.x = mix_pick(z.x, n.x, zdiag[r.x], zdiag[c.x], eps);
        m.y = mix_pick(z.y, n.y, zdiag[r.y], zdiag[c.y], eps);
        *reinterpret_cast<double2 *>(M + p) = m;
    } else if (p < nnz) {
        M[p] = mix_pick(Z[p], N[p], zdiag[srow[p]], zdiag[col[p]], eps);
    }
}

// Rank-k correction on S (Section 2.5): out_ij = in_ij + sum_m lam_m V_im V_jm.
// One thread per entry of S (all lanes busy whatever the row lengths): the
// row index comes from the stored row of each entry, rows i and j of V are
// read as 16-byte vectors when V is 16-byte aligned (consecutive entries share
// row i, so its reads hit the cache); lambda is uniform across the wavefront.
template <int K>
__global__ __launch_bounds__(256) void k_lowrank(int64_t nnz, int32_t k, const int32_t *__restrict__ srow,
                                                 const int32_t *__restrict__ col, const double *__restrict__ V,
                                                 const double *__restrict__ lam, const double *in, double *out) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= nnz) return;
    const double *vi = V + (int64_t)srow[p] * k;
    const double *vj = V + (int64_t)col[p] * k;
    double s = 0.0;
    if (K > 1 && k == K) {
        const double2 *a = reinterpret_cast<const double2 *>(vi);
        const double2 *b = reinterpret_cast<const double2 *>(vj);
#pragma unroll
        for (int m = 0; m < K / 2; ++m) {
            const double2 x = a[m], y = b[m];
            s += lam[2 * m] * x.x * y.x;
            s += lam[2 * m + 1] * x.y * y.y;
        }
    } else {
        for (int m = 0; m < k; ++m) s += lam[m] * vi[m] * vj[m];
    }
    out[p] = in[p] + s;
}

// ---- SPAI -----------------------------------------------------------------

__global__ void k_iperm(int32_t n, const int32_t *__restrict__ perm, int32_t *__restrict__ iperm,
                        int32_t *status, int32_t *list_count) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2) list_count[i] = 0;
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

struct SpaiGeneralLds {
    int32_t sJ[kSpaiMaxCols];
    double sx[kSpaiMaxCols], sr[kSpaiMaxCols], sz[kSpaiMaxCols], sp[kSpaiMaxCols], sg[kSpaiMaxCols];
    int32_t soff[kSpaiMaxCols + 1];
    int32_t hkey[kSpaiH];
    double hval[kSpaiH];
    int32_t sflag[1];
};

// General SPAI column (Section 2.4) for columns the staged kernel cannot hold:
// one wavefront, up to 512 entries in the column of S and 2048 distinct rows
// of Ah(:, J). G = Ah_J^T Ah_J is applied as Ah_J^T (Ah_J p): the first half
// scatters rows of Ah into an LDS hash keyed by row, the second half gathers
// them back per column of J, both reading A from global memory.
__device__ void spai_general_column(const SpaiParams &P, int32_t j, SpaiGeneralLds &Lg) {
    constexpr int C = kSpaiMaxCols;
    int32_t *sJ = Lg.sJ;
    double *sx = Lg.sx, *sr = Lg.sr, *sz = Lg.sz, *sp = Lg.sp, *sg = Lg.sg;
    int32_t *soff = Lg.soff;
    int32_t *hkey = Lg.hkey;
    double *hval = Lg.hval;
    int32_t *sflag = Lg.sflag;
    const int lane = threadIdx.x & 63;
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

// Columns listed by the staged kernel, one wavefront per block.
__global__ __launch_bounds__(64) void k_spai_general(SpaiParams P, const int32_t *__restrict__ list,
                                                     const int32_t *__restrict__ count) {
    __shared__ SpaiGeneralLds Lg;
    const int32_t cnt = *count;
    for (int32_t q = blockIdx.x; q < cnt; q += gridDim.x) {
        wsync();
        spai_general_column(P, list[q], Lg);
    }
}

// ---- SPAI, staged variant --------------------------------------------------
// One wavefront per column j of S. The column's entries J_a are spread over
// the lanes with lpc lanes per entry, lpc the largest power of two with
// c lpc <= 64 (c = |J|; lpc = 1 from c > 32 on, and then lane l owns the
// entries a = l + 64 k, k < E): lane l serves entry a = l mod (64 / lpc) as
// its sub-lane h = l div (64 / lpc). Every lane of an entry keeps that
// entry's CG scalars (the same arithmetic in each); sub-lane h stages and
// walks the entries h, h + lpc, ... of column J_a of Ah (its rows as slots of
// a per-wavefront LDS hash, its values), so each application of
// G = Ah_J^T Ah_J is an LDS scatter of Ah_J p into the slots and a strided
// gather back, whose lpc partial sums are added across the sub-lanes, with
// no global traffic. The E = 1 kernel runs over every column and lists those
// it cannot hold (more than 64 entries, or more than 384 entries in
// Ah(:, J)); the E = 2 kernel takes that list and passes what it cannot hold
// on to the general kernel.
template <int E>
struct SpaiStaged {
    static constexpr int C = 64 * E;    // entries of the column of S
    static constexpr int T = 384 * E;   // entries of Ah(:, J)
    static constexpr int HB = 8 + E;    // log2 of the hash slots (2^HB > T)
    static constexpr int H = 1 << HB;
    static_assert(H > T, "every row of Ah(:, J) must find a slot");
    union {
        int32_t key[H];  // setup: row of each slot
        double y[H];     // CG: (Ah_J p) per slot
    };
    double val[T];
    uint16_t slot[T];
    int32_t flag;
};

// slot of row r in a table of 2^hb slots (linear probing; -1 if full)
__device__ inline int sp_insert(int32_t *key, int32_t r, int hb) {
    const int H = 1 << hb;
    uint32_t s = ((uint32_t)r * 2654435761u) >> (32 - hb);
    for (int probe = 0; probe < H; ++probe) {
        int32_t k = key[s];
        if (k == r) return (int)s;
        if (k == -1) {
            int32_t old = atomicCAS(&key[s], -1, r);
            if (old == -1 || old == r) return (int)s;
        }
        s = (s + 1) & (uint32_t)(H - 1);
    }
    return -1;
}

// v summed over the lanes l, l + cw, l + 2 cw, ... (cw a power of two <= 64)
__device__ inline double sublane_sum(double v, int cw) {
    for (int o = cw; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int E, int W>
__global__ __launch_bounds__(64 * W) void k_spai_staged(SpaiParams P, const int32_t *__restrict__ in_list,
                                                        const int32_t *__restrict__ in_count,
                                                        int32_t *__restrict__ out_list,
                                                        int32_t *__restrict__ out_count) {
    using Lds = SpaiStaged<E>;
    __shared__ Lds lds[W];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Lds &L = lds[w];
    const int32_t total = in_list ? *in_count : P.n;
    for (int32_t q = blockIdx.x * W + w; q < total; q += gridDim.x * W) {
        const int32_t j = in_list ? in_list[q] : q;
        const int64_t s0 = P.rowptr[j];
        const int32_t c = (int32_t)(P.rowptr[j + 1] - s0);
        if (c > Lds::C) {
            if (lane == 0) out_list[atomicAdd(out_count, 1)] = j;
            continue;
        }
        int lpc = 1;
        while (lpc < 64 && 2 * lpc * c <= 64) lpc <<= 1;
        const int cw = 64 / lpc;          // entries per pass of the wavefront (k = 0)
        const int h = lane / cw;          // sub-lane of the lane's entry
        double xa[E], cna[E];
        int64_t qa[E];
        int32_t dega[E], e0[E];
        bool own[E];                      // the lane answers for entry a (sub-lane 0 of a valid entry)
        int32_t carry = 0;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const int a = k == 0 ? lane % cw : lane + 64 * k;
            const bool valid = a < c && (k == 0 || lpc == 1);
            own[k] = valid && h == 0;
            xa[k] = 0.0;
            cna[k] = 1.0;
            qa[k] = 0;
            dega[k] = 0;
            if (valid) {
                const int32_t ja = P.col[s0 + a];
                xa[k] = P.M[s0 + a];
                cna[k] = P.colnorm2[ja];
                const int32_t ra = P.perm[ja];
                qa[k] = P.A_rowptr[ra];
                dega[k] = (int32_t)(P.A_rowptr[ra + 1] - qa[k]);
            }
            // offsets of the entries' Ah columns: a scan over the owning lanes
            // (lanes 0..cw-1 for k = 0), then each sub-lane takes its entry's
            const int32_t d = own[k] ? dega[k] : 0;
            int32_t incl = d;
            for (int o = 1; o < 64; o <<= 1) {
                int32_t u = __shfl_up(incl, o, 64);
                if (lane >= o) incl += u;
            }
            incl += carry;
            e0[k] = incl - d;
            if (k == 0) e0[k] = __shfl(e0[k], lane % cw, 64);
            carry = __shfl(incl, 63, 64);
        }
        if (carry > Lds::T) {
            if (lane == 0) out_list[atomicAdd(out_count, 1)] = j;
            continue;
        }
        // hash slots in use: at least twice the column's rows of Ah (fewer
        // slots to clear per application), at most the table
        int hb = 6;
        while (hb < Lds::HB && (1 << hb) < 2 * carry) ++hb;
        const int hs = 1 << hb;
        wsync();  // the previous column's readers of L are done
        for (int s = lane; s < hs; s += 64) L.key[s] = -1;
        if (lane == 0) L.flag = 0;
        wsync();
        // b_a = Ah(j, J_a) = entry of column J_a of Ah in row j (Ah symmetric)
        const int32_t rj = P.perm[j];
        double ba[E];
#pragma unroll
        for (int k = 0; k < E; ++k) {
            ba[k] = 0.0;
            for (int32_t e = h; e < dega[k]; e += lpc) {
                const int32_t r = P.A_col[qa[k] + e];
                const double v = P.A_val[qa[k] + e];
                const int sl = sp_insert(L.key, r, hb);
                if (sl < 0) L.flag = 1;
                L.slot[e0[k] + e] = (uint16_t)(sl < 0 ? 0 : sl);
                L.val[e0[k] + e] = v;
                if (r == rj) ba[k] = v;
            }
        }
        ba[0] = sublane_sum(ba[0], cw);  // one sub-lane found it (or none): exact
        wsync();
        if (L.flag) {
            if (lane == 0) out_list[atomicAdd(out_count, 1)] = j;
            continue;
        }
        // g = G v for the lane's vector entries v
        auto apply = [&](const double(&va)[E], double(&ga)[E]) {
            wsync();
            for (int s = lane; s < hs; s += 64) L.y[s] = 0.0;
            wsync();
#pragma unroll
            for (int k = 0; k < E; ++k)
                for (int32_t e = e0[k] + h; e < e0[k] + dega[k]; e += lpc)
                    atomicAdd(&L.y[L.slot[e]], L.val[e] * va[k]);
            wsync();
#pragma unroll
            for (int k = 0; k < E; ++k) {
                double g = 0.0;
                for (int32_t e = e0[k] + h; e < e0[k] + dega[k]; e += lpc) g += L.val[e] * L.y[L.slot[e]];
                ga[k] = g;
            }
            ga[0] = sublane_sum(ga[0], cw);
        };
        // r = b - G x, z = r / diag, p = z (every lane of an entry alike; the
        // dot products count each entry once, from its sub-lane 0)
        double ga[E], ra[E], za[E], pa[E];
        apply(xa, ga);
        double rz = 0.0;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const bool valid = own[k] || (k == 0 && (lane % cw) < c);
            ra[k] = valid ? ba[k] - ga[k] : 0.0;
            za[k] = valid ? ra[k] / cna[k] : 0.0;
            pa[k] = za[k];
            if (own[k]) rz += ra[k] * za[k];
        }
        rz = wsum(rz);
        for (int it = 0; it < P.iters; ++it) {
            if (rz == 0.0) break;
            apply(pa, ga);
            double pgp = 0.0;
#pragma unroll
            for (int k = 0; k < E; ++k)
                if (own[k]) pgp += pa[k] * ga[k];
            pgp = wsum(pgp);
            if (pgp == 0.0) break;
            const double al = rz / pgp;
            double rzn = 0.0;
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const bool valid = own[k] || (k == 0 && (lane % cw) < c);
                xa[k] += al * pa[k];
                ra[k] -= al * ga[k];
                za[k] = valid ? ra[k] / cna[k] : 0.0;
                if (own[k]) rzn += ra[k] * za[k];
            }
            rzn = wsum(rzn);
            const double be = rzn / rz;
#pragma unroll
            for (int k = 0; k < E; ++k) pa[k] = za[k] + be * pa[k];
            rz = rzn;
        }
#pragma unroll
        for (int k = 0; k < E; ++k)
            if (own[k]) P.X[s0 + (k == 0 ? lane : lane + 64 * k)] = xa[k];
    }
}

__global__ void k_symmetrize(int64_t nnz, const int64_t *__restrict__ mirror, const double *__restrict__ X,
                             double *__restrict__ R) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) R[p] = 0.5 * (X[p] + X[mirror[p]]);
}

// First stage of the diagonal error: block b sums |d_ref - d_hat - sum_m
// lambda_m V_im^2| and |d_ref| over a grid-stride range of rows into part[2b],
// part[2b + 1].
__global__ __launch_bounds__(256) void k_err1_part(int32_t n, const double *__restrict__ d_ref,
                                                   const double *__restrict__ d_hat, int32_t k,
                                                   const double *__restrict__ V, const double *__restrict__ lam,
                                                   double *__restrict__ part) {
    __shared__ double s0[4], s1[4];
    double a = 0.0, b = 0.0;
    for (int32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        double c = d_hat[i];
        const double *v = V + (int64_t)i * k;
        for (int m = 0; m < k; ++m) c += lam[m] * v[m] * v[m];
        a += fabs(d_ref[i] - c);
        b += fabs(d_ref[i]);
    }
    a = wsum(a);
    b = wsum(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s0[w] = a;
        s1[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = (s0[0] + s0[1]) + (s0[2] + s0[3]);
        part[2 * blockIdx.x + 1] = (s1[0] + s1[1]) + (s1[2] + s1[3]);
    }
}

// Trace of a matrix on S with an optional rank-k term, per block of 256
// unknowns (same two-stage pattern as the err_1 sums): part = (sum_i c_i,
// sum_i |c_i|) with c_i = X(i, i) + sum_{m<k} lam_m V[i][m]^2.
__global__ __launch_bounds__(256) void k_trace_part(int32_t n, const int64_t *__restrict__ diagpos,
                                                    const double *__restrict__ X, int32_t k,
                                                    const double *__restrict__ V, const double *__restrict__ lam,
                                                    double *__restrict__ part) {
    __shared__ double s0[4], s1[4];
    double a = 0.0, b = 0.0;
    for (int32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        double c = X[diagpos[i]];
        const double *v = V + (int64_t)i * k;
        for (int m = 0; m < k; ++m) c += lam[m] * v[m] * v[m];
        a += c;
        b += fabs(c);
    }
    a = wsum(a);
    b = wsum(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s0[w] = a;
        s1[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = (s0[0] + s0[1]) + (s0[2] + s0[3]);
        part[2 * blockIdx.x + 1] = (s1[0] + s1[1]) + (s1[2] + s1[3]);
    }
}

// Second stage: one block adds the partial sums in a fixed order.
__global__ __launch_bounds__(256) void k_err1_final(int nblk, const double *__restrict__ part,
                                                    double *__restrict__ sums) {
    __shared__ double s0[4], s1[4];
    double a = 0.0, b = 0.0;
    for (int q = threadIdx.x; q < nblk; q += 256) {
        a += part[2 * q];
        b += part[2 * q + 1];
    }
    a = wsum(a);
    b = wsum(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s0[w] = a;
        s1[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sums[0] = (s0[0] + s0[1]) + (s0[2] + s0[3]);
        sums[1] = (s1[0] + s1[1]) + (s1[2] + s1[3]);
    }
}

}  // namespace dev

hipError_t launch_diag_err1(int32_t n, const double *d_ref, const double *d_hat, int32_t k, const double *V,
                            const double *lam, double *part, double *sums, hipStream_t st) {
    int nblk = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, ((int64_t)n + 255) / 256));
    hipLaunchKernelGGL(dev::k_err1_part, dim3(nblk), dim3(256), 0, st, n, d_ref, d_hat, k, V, lam, part);
    hipLaunchKernelGGL(dev::k_err1_final, dim3(1), dim3(256), 0, st, nblk, part, sums);
    return hipGetLastError();
}

hipError_t launch_trace(int32_t n, const int64_t *diagpos, const double *X, int32_t k, const double *V,
                        const double *lam, double *part, double *sums, hipStream_t st) {
    int nblk = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, ((int64_t)n + 255) / 256));
    hipLaunchKernelGGL(dev::k_trace_part, dim3(nblk), dim3(256), 0, st, n, diagpos, X, k, V, lam, part);
    hipLaunchKernelGGL(dev::k_err1_final, dim3(1), dim3(256), 0, st, nblk, part, sums);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 65536);
    hipLaunchKernelGGL(dev::k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

hipError_t launch_zdiag(int32_t n, const int64_t *diagpos, const double *X, double *d, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_zdiag, dim3((n + 255) / 256), dim3(256), 0, st, n, diagpos, X, d);
    return hipGetLastError();
}

hipError_t launch_mix(int64_t nnz, const int32_t *srow, const int32_t *col, const double *zdiag,
                      const double *Z, const double *N, double eps, double *M, hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    const bool aligned = ((reinterpret_cast<uintptr_t>(Z) | reinterpret_cast<uintptr_t>(N) |
                           reinterpret_cast<uintptr_t>(M)) & 15) == 0;
    if (aligned)
        hipLaunchKernelGGL(dev::k_mix, dim3((unsigned)((nnz + 511) / 512)), dim3(256), 0, st, nnz, srow, col, zdiag,
                           Z, N, eps, M);
    else
        hipLaunchKernelGGL(dev::k_mix1, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, nnz, srow, col,
                           zdiag, Z, N, eps, M);
    return hipGetLastError();
}

hipError_t launch_lowrank(int64_t nnz, int32_t k, const int32_t *srow, const int32_t *col, const double *V,
                          const double *lam, const double *in, double *out, hipStream_t st) {
    dim3 g((unsigned)((nnz + 255) / 256)), b(256);
    if (nnz == 0) return hipSuccess;
    const bool vec = (reinterpret_cast<uintptr_t>(V) & 15) == 0;
    switch (vec ? k : 0) {
    case 8: hipLaunchKernelGGL((dev::k_lowrank<8>), g, b, 0, st, nnz, k, srow, col, V, lam, in, out); break;
    case 16: hipLaunchKernelGGL((dev::k_lowrank<16>), g, b, 0, st, nnz, k, srow, col, V, lam, in, out); break;
    case 32: hipLaunchKernelGGL((dev::k_lowrank<32>), g, b, 0, st, nnz, k, srow, col, V, lam, in, out); break;
    case 64: hipLaunchKernelGGL((dev::k_lowrank<64>), g, b, 0, st, nnz, k, srow, col, V, lam, in, out); break;
    default: hipLaunchKernelGGL((dev::k_lowrank<1>), g, b, 0, st, nnz, k, srow, col, V, lam, in, out); break;
    }
    return hipGetLastError();
}

hipError_t launch_spai(const SpaiParams &P, hipStream_t st) {
    dim3 g1((P.n + 255) / 256);
    hipLaunchKernelGGL(dev::k_iperm, g1, dim3(256), 0, st, P.n, P.perm, P.iperm, P.status, P.list_count);
    hipLaunchKernelGGL(dev::k_colnorm2, g1, dim3(256), 0, st, P.n, P.perm, P.A_rowptr, P.A_val, P.colnorm2);
    // every column -> list 1 (too long for E = 1) -> list 2 (too long for E = 2)
    int32_t *list1 = P.list, *list2 = P.list + P.n;
    int32_t *cnt1 = P.list_count, *cnt2 = P.list_count + 1;
    const int64_t nb = std::min<int64_t>(((int64_t)P.n + 3) / 4, 8192);
    hipLaunchKernelGGL((dev::k_spai_staged<1, 4>), dim3((unsigned)nb), dim3(256), 0, st, P, nullptr, nullptr,
                       list1, cnt1);
    const int64_t nm = std::min<int64_t>(((int64_t)P.n + 1) / 2, 2048);
    hipLaunchKernelGGL((dev::k_spai_staged<2, 2>), dim3((unsigned)nm), dim3(128), 0, st, P, list1, cnt1, list2,
                       cnt2);
    const int64_t ng = std::min<int64_t>(P.n, 2048);
    hipLaunchKernelGGL(dev::k_spai_general, dim3((unsigned)ng), dim3(64), 0, st, P, list2, cnt2);
    return hipGetLastError();
}

hipError_t launch_symmetrize(int64_t nnz, const int64_t *mirror, const double *X, double *R, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_symmetrize, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, nnz, mirror,
                       X, R);
    return hipGetLastError();
}

}  // namespace asi
