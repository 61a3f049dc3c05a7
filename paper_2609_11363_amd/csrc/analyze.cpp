// Symbolic analysis of the factor pattern (host side of libasi).
//
// S is the pattern of L + D + L^T (Section 1). Column J of L (both columns of
// a 2x2 block, union of their rows) gives R_J, the rows below the block; the
// upper part of row `last(J)` of S is exactly R_J, so S's CSR doubles as the
// column layout of the lower triangle of Z that the SelInv gathers read.
// Block J depends on every block that holds a row of R_J (its Z(R_J, R_J)
// entries, Section 2.1), which gives the level schedule.
#include <algorithm>
#include <climits>
#include <cstring>
#include <numeric>
#include <thread>

#include "asi_internal.h"

namespace asi {

namespace {
enum { OK = 0, E_ARG = 1, E_PATTERN = 2, E_UNSUPPORTED = 8 };

// Runs fn(begin, end, worker) over [0, count) split into contiguous chunks,
// one per worker thread (the analysis' independent per-row and per-block
// loops; each worker gets its own scratch through its index).
template <typename Fn>
void parallel_chunks(int64_t count, int workers, Fn fn) {
    if (workers <= 1 || count < 4096) {
        fn((int64_t)0, count, 0);
        return;
    }
    std::vector<std::thread> th;
    const int64_t step = (count + workers - 1) / workers;
    for (int w = 0; w < workers; ++w) {
        const int64_t b = w * step, e = std::min(count, b + step);
        if (b >= e) break;
        th.emplace_back(fn, b, e, w);
    }
    for (auto &t : th) t.join();
}

int analysis_workers() {
    const unsigned hc = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(16u, hc));
}
}

int analyze(int32_t n, const int64_t *Lp, const int32_t *Li, const int8_t *piv, Analysis &A,
            std::string &msg) {
    A = Analysis();
    if (n <= 0) {
        msg = "n must be positive";
        return E_ARG;
    }
    A.n = n;
    A.piv.assign(piv, piv + n);
    if (Lp[0] != 0) {
        msg = "L_rowptr[0] must be 0";
        return E_PATTERN;
    }
    for (int32_t i = 0; i < n; ++i) {
        int8_t p = piv[i];
        if (p < 0 || p > 2) {
            msg = "piv values must be 0, 1 or 2";
            return E_PATTERN;
        }
        if (p == 1 && (i + 1 >= n || piv[i + 1] != 2)) {
            msg = "piv: a 1 must be followed by a 2";
            return E_PATTERN;
        }
        if (p == 2 && (i == 0 || piv[i - 1] != 1)) {
            msg = "piv: a 2 must follow a 1";
            return E_PATTERN;
        }
        if (Lp[i + 1] < Lp[i]) {
            msg = "L_rowptr must be nondecreasing";
            return E_PATTERN;
        }
        for (int64_t q = Lp[i]; q < Lp[i + 1]; ++q) {
            int32_t c = Li[q];
            if (c < 0 || c >= i) {
                msg = "L must be strictly lower triangular with in-range columns";
                return E_PATTERN;
            }
            if (q > Lp[i] && c <= Li[q - 1]) {
                msg = "L columns must be sorted and unique within each row";
                return E_PATTERN;
            }
            if (p == 2 && c == i - 1) {
                msg = "L must not store the (j+1, j) entry of a 2x2 block";
                return E_PATTERN;
            }
        }
    }
    A.nnzL = Lp[n];
    A.L_rowptr.assign(Lp, Lp + n + 1);

    // column lists of L (CSC) with the source index of every entry
    std::vector<int64_t> cp(n + 1, 0);
    for (int64_t q = 0; q < A.nnzL; ++q) cp[Li[q] + 1]++;
    for (int32_t j = 0; j < n; ++j) cp[j + 1] += cp[j];
    std::vector<int32_t> crow(A.nnzL);
    std::vector<int64_t> csrc(A.nnzL);
    {
        std::vector<int64_t> f(cp.begin(), cp.end() - 1);
        for (int32_t r = 0; r < n; ++r)
            for (int64_t q = Lp[r]; q < Lp[r + 1]; ++q) {
                int64_t d = f[Li[q]]++;
                crow[d] = r;  // rows ascending since r ascends
                csrc[d] = q;
            }
    }

    // upper part of every row: row j holds {j+1 if j starts a 2x2} + R_J,
    // row j+1 of a 2x2 holds R_J; R_J = union of the block's column rows
    std::vector<int64_t> up(n + 1, 0);
    std::vector<int32_t> ucol;
    ucol.reserve(A.nnzL + n);
    std::vector<int32_t> RJ;
    for (int32_t j = 0; j < n;) {
        if (piv[j] == 1) {
            RJ.clear();
            std::set_union(crow.begin() + cp[j], crow.begin() + cp[j + 1], crow.begin() + cp[j + 1],
                           crow.begin() + cp[j + 2], std::back_inserter(RJ));
            // row j: (j, j+1) then R_J
            up[j + 1] = up[j] + 1 + (int64_t)RJ.size();
            ucol.push_back(j + 1);
            ucol.insert(ucol.end(), RJ.begin(), RJ.end());
            up[j + 2] = up[j + 1] + (int64_t)RJ.size();
            ucol.insert(ucol.end(), RJ.begin(), RJ.end());
            j += 2;
        } else {
            up[j + 1] = up[j] + (cp[j + 1] - cp[j]);
            ucol.insert(ucol.end(), crow.begin() + cp[j], crow.begin() + cp[j + 1]);
            j += 1;
        }
    }

    // lower part of row r = transpose of the upper parts; build row lengths
    std::vector<int64_t> lowcnt(n + 1, 0);
    for (int32_t j = 0; j < n; ++j)
        for (int64_t q = up[j]; q < up[j + 1]; ++q) lowcnt[ucol[q] + 1]++;
    A.rowptr.assign(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) A.rowptr[i + 1] = A.rowptr[i] + lowcnt[i + 1] + 1 + (up[i + 1] - up[i]);
    A.nnzS = A.rowptr[n];
    A.col.resize(A.nnzS);
    A.srow.resize(A.nnzS);
    A.diagpos.resize(n);
    A.mirror.assign(A.nnzS, -1);
    for (int32_t i = 0; i < n; ++i) {
        A.diagpos[i] = A.rowptr[i] + lowcnt[i + 1];
        A.col[A.diagpos[i]] = i;
        A.mirror[A.diagpos[i]] = A.diagpos[i];
        int64_t q0 = A.diagpos[i] + 1;
        for (int64_t q = up[i]; q < up[i + 1]; ++q) A.col[q0 + (q - up[i])] = ucol[q];
        for (int64_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) A.srow[p] = i;
    }
    {
        // lower entries: (r, j) for every upper (j, r); rows j ascending keep them sorted
        std::vector<int64_t> f(n);
        for (int32_t i = 0; i < n; ++i) f[i] = A.rowptr[i];
        for (int32_t j = 0; j < n; ++j)
            for (int64_t p = A.diagpos[j] + 1; p < A.rowptr[j + 1]; ++p) {
                int32_t r = A.col[p];
                int64_t d = f[r]++;
                A.col[d] = j;
                A.mirror[d] = p;
                A.mirror[p] = d;
            }
    }
    // u-space: the upper part of each row, with the L source of every entry
    // (a merge of the sorted upper row j with the sorted column j of L)
    A.ustart.assign(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) A.ustart[i + 1] = A.ustart[i] + (A.rowptr[i + 1] - A.diagpos[i] - 1);
    A.nnzU = A.ustart[n];
    A.ucol.resize(A.nnzU);
    A.lsrc_u.assign(A.nnzU, -1);
    A.mirror_u.resize(A.nnzU);
    A.useg_u.resize(A.nnzU);
    const int workers = analysis_workers();
    parallel_chunks(n, workers, [&](int64_t jb, int64_t je, int) {
    for (int32_t j = (int32_t)jb; j < (int32_t)je; ++j) {
        const int64_t p0 = A.diagpos[j] + 1, u0 = A.ustart[j];
        for (int64_t u = u0; u < A.ustart[j + 1]; ++u) {
            int64_t p = p0 + (u - u0);
            A.ucol[u] = A.col[p];
            A.mirror_u[u] = A.mirror[p];
        }
        int64_t p = u0, pe = A.ustart[j + 1];
        int64_t q = cp[j], qe = cp[j + 1];
        while (p < pe && q < qe) {
            if (A.ucol[p] == crow[q]) {
                A.lsrc_u[p] = csrc[q];
                ++p;
                ++q;
            } else if (A.ucol[p] < crow[q]) {
                ++p;
            } else {
                ++q;
            }
        }
    }
    });
    parallel_chunks(A.nnzU, workers, [&](int64_t b, int64_t e, int) {
        for (int64_t u = b; u < e; ++u) A.useg_u[u] = A.ustart[A.ucol[u]];
    });
    // every L entry sits at exactly one u-index (the padding of 2x2 unions has none)
    if (A.nnzU > (int64_t)INT32_MAX) {
        msg = "more than 2^31 - 1 entries above the diagonal of S";
        return E_UNSUPPORTED;
    }
    A.q2u.assign(A.nnzL, -1);
    for (int64_t u = 0; u < A.nnzU; ++u)
        if (A.lsrc_u[u] >= 0) A.q2u[A.lsrc_u[u]] = (int32_t)u;
    // S position -> u-index of the entry's L value (int32; the learned
    // correction, which reads it, needs |S| < 2^31)
    A.s2u.assign(A.nnzS <= (int64_t)INT32_MAX ? A.nnzS : 0, -1);
    if (!A.s2u.empty())
        parallel_chunks(n, workers, [&](int64_t ib, int64_t ie, int) {
            for (int32_t i = (int32_t)ib; i < (int32_t)ie; ++i)
                for (int64_t p = A.diagpos[i] + 1; p < A.rowptr[i + 1]; ++p) {
                    const int32_t u = (int32_t)(A.ustart[i] + (p - A.diagpos[i] - 1));
                    A.s2u[p] = u;
                    A.s2u[A.mirror[p]] = u;
                }
        });

    // blocks, levels and work counts
    A.level.assign(n, 0);
    std::vector<int32_t> blocks;
    for (int32_t j = 0; j < n; j += (piv[j] == 1 ? 2 : 1)) blocks.push_back(j);
    A.n_blocks = (int32_t)blocks.size();
    std::vector<int32_t> bcols(n, 0);
    std::vector<int64_t> bhits(n, 0);
    int32_t maxlev = -1;
    for (auto it = blocks.rbegin(); it != blocks.rend(); ++it) {
        int32_t j = *it;
        int32_t last = piv[j] == 1 ? j + 1 : j;
        int64_t u0 = A.diagpos[last] + 1, u1 = A.rowptr[last + 1];
        int32_t lev = 0;
        for (int64_t p = u0; p < u1; ++p) lev = std::max(lev, A.level[A.col[p]] + 1);
        A.level[j] = lev;
        if (last != j) A.level[last] = lev;
        maxlev = std::max(maxlev, lev);
        int32_t c = (int32_t)(u1 - u0);
        bcols[j] = c;
        A.max_cols = std::max(A.max_cols, c);
    }
    A.n_levels = maxlev + 1;
    // hits of every block (independent per block: per-worker marks)
    {
        std::vector<int64_t> wpairs(workers, 0), whits(workers, 0);
        parallel_chunks((int64_t)blocks.size(), workers, [&](int64_t bb, int64_t be, int w) {
            std::vector<int32_t> mark(n, -1);
            int64_t pairs = 0, hits = 0;
            for (int64_t bi = bb; bi < be; ++bi) {
                const int32_t j = blocks[bi];
                const int32_t last = piv[j] == 1 ? j + 1 : j;
                const int64_t u0 = A.diagpos[last] + 1, u1 = A.rowptr[last + 1];
                for (int64_t p = u0; p < u1; ++p) mark[A.col[p]] = j;
                int64_t h = 0;
                for (int64_t p = u0; p < u1; ++p) {
                    const int32_t l = A.col[p];
                    const int64_t s0 = A.diagpos[l] + 1, s1 = A.rowptr[l + 1];
                    pairs += s1 - s0;
                    for (int64_t q = s0; q < s1; ++q) h += (mark[A.col[q]] == j);
                }
                bhits[j] = h;
                hits += h;
            }
            wpairs[w] = pairs;
            whits[w] = hits;
        });
        for (int w = 0; w < workers; ++w) {
            A.gather_pairs += wpairs[w];
            A.gather_hits += whits[w];
        }
    }
    if (A.max_cols > kBigCols) {
        msg = "a block has more than 2048 rows below it (|R_J| limit)";
        return E_UNSUPPORTED;
    }
    // hit lists, blocks in increasing start index
    {
        int64_t words = 0;
        for (int32_t j : blocks) words += bhits[j] * (bcols[j] <= kSmallCols ? 1 : 2);
        A.hits.resize(words);
        A.hit_ptr.assign(n + 1, 0);
        {
            int64_t w = 0;
            for (int32_t j : blocks) {
                const int32_t last = piv[j] == 1 ? j + 1 : j;
                A.hit_ptr[j] = w;
                w += bhits[j] * (bcols[j] <= kSmallCols ? 1 : 2);
                A.hit_ptr[j + 1] = w;
                if (last != j) A.hit_ptr[last + 1] = w;
            }
        }
        parallel_chunks((int64_t)blocks.size(), workers, [&](int64_t bb, int64_t be, int) {
        std::vector<int32_t> pos(n, -1);
        for (int64_t bi = bb; bi < be; ++bi) {
            const int32_t j = blocks[bi];
            const int32_t last = piv[j] == 1 ? j + 1 : j;
            const int64_t ub = A.ustart[last], ue = A.ustart[last + 1];
            const int32_t c = (int32_t)(ue - ub);
            const bool small = c <= kSmallCols;
            int64_t w = A.hit_ptr[j];
            for (int32_t t = 0; t < c; ++t) pos[A.ucol[ub + t]] = t;
            for (int32_t b = 0; b < c; ++b) {
                const int32_t l = A.ucol[ub + b];
                const int64_t s0 = A.ustart[l], s1 = A.ustart[l + 1];
                for (int64_t q = s0; q < s1; ++q) {
                    const int32_t a = pos[A.ucol[q]];
                    if (a < 0) continue;
                    const uint32_t off = (uint32_t)(q - s0);
                    if (small) {
                        A.hits[w++] = (uint32_t)a | ((uint32_t)b << 7) | (off << 14);
                    } else {
                        A.hits[w++] = (uint32_t)a | ((uint32_t)b << 16);
                        A.hits[w++] = off;
                    }
                }
            }
            for (int32_t t = 0; t < c; ++t) pos[A.ucol[ub + t]] = -1;
        }
        });
    }
    // level-major schedules (blocks in increasing start index within a level)
    std::vector<int32_t> cs(A.n_levels + 1, 0), cb(A.n_levels + 1, 0);
    for (int32_t j : blocks) (bcols[j] <= kSmallCols ? cs : cb)[A.level[j] + 1]++;
    for (int32_t l = 0; l < A.n_levels; ++l) {
        cs[l + 1] += cs[l];
        cb[l + 1] += cb[l];
    }
    A.lvl_small = cs;
    A.lvl_big = cb;
    A.sched_small.resize(cs[A.n_levels]);
    A.sched_big.resize(cb[A.n_levels]);
    for (int m = 0; m < 2; ++m) {
        A.lvl_bytes_small[m].assign(A.n_levels, 0.0);
        A.lvl_bytes_big[m].assign(A.n_levels, 0.0);
    }
    A.lvl_maxc_big.assign(A.n_levels, 0);
    A.lvl_heavy.assign(A.n_levels, 0);
    // small blocks with many hits first within their level
    for (int32_t j : blocks)
        if (bcols[j] <= kSmallCols && bhits[j] > kHeavyHits) {
            A.sched_small[cs[A.level[j]]++] = j;
            A.lvl_heavy[A.level[j]]++;
        }
    for (int32_t j : blocks) {
        const bool small = bcols[j] <= kSmallCols;
        if (small) {
            if (bhits[j] <= kHeavyHits) A.sched_small[cs[A.level[j]]++] = j;
        } else {
            A.sched_big[cb[A.level[j]]++] = j;
            A.lvl_maxc_big[A.level[j]] = std::max(A.lvl_maxc_big[A.level[j]], bcols[j]);
        }
        const int ncols = piv[j] == 1 ? 2 : 1;
        for (int m = 0; m < 2; ++m) {
            double b = selinv_block_bytes(bcols[j], ncols, bhits[j], m == 0);
            (small ? A.lvl_bytes_small[m] : A.lvl_bytes_big[m])[A.level[j]] += b;
        }
    }
    for (int k = 0; k < 2; ++k) {
        const std::vector<int32_t> &sched = k == 0 ? A.sched_small : A.sched_big;
        std::vector<BlockMeta> &meta = k == 0 ? A.meta_small : A.meta_big;
        meta.resize(sched.size());
        for (size_t s = 0; s < sched.size(); ++s) {
            const int32_t j = sched[s];
            const bool two = piv[j] == 1;
            const int32_t last = two ? j + 1 : j;
            BlockMeta m{};
            m.ub = A.ustart[last];
            m.ubj = two ? A.ustart[j] + 1 : m.ub;
            m.h0 = A.hit_ptr[j];
            m.pdl = A.diagpos[last] + 1;
            m.pdj = two ? A.diagpos[j] + 2 : m.pdl;
            m.j = j;
            m.c = (int32_t)(A.ustart[last + 1] - m.ub);
            m.nwords = (int32_t)(A.hit_ptr[last + 1] - m.h0);
            m.two = two ? 1 : 0;
            meta[s] = m;
        }
    }
    // the preconditioner solves' rows, level by level
    A.solve_fwd.clear();
    A.solve_bwd.clear();
    A.lvl_rows.assign(A.n_levels + 1, 0);
    if (!A.s2u.empty()) {
        A.solve_fwd.reserve(n);
        A.solve_bwd.reserve(n);
        for (int32_t l = 0; l < A.n_levels; ++l) {
            for (int k = 0; k < 2; ++k) {
                const std::vector<int32_t> &sched = k == 0 ? A.sched_small : A.sched_big;
                const std::vector<int32_t> &off = k == 0 ? A.lvl_small : A.lvl_big;
                for (int32_t s = off[l]; s < off[l + 1]; ++s) {
                    const int32_t j = sched[s];
                    const bool two = piv[j] == 1;
                    for (int t = 0; t < (two ? 2 : 1); ++t) {
                        const int32_t i = j + t;
                        const int64_t dp = A.diagpos[i];
                        // the partner (j + 1 - t) sits next to the diagonal: last of
                        // the lower part for the second row, first of the upper
                        // part for the first
                        int64_t skf = -1, skb = -1;
                        if (two && t == 1 && dp > A.rowptr[i] && A.col[dp - 1] == j) skf = dp - 1;
                        if (two && t == 0 && dp + 1 < A.rowptr[i + 1] && A.col[dp + 1] == j + 1) skb = dp + 1;
                        A.solve_fwd.push_back({i, (int32_t)A.rowptr[i], (int32_t)dp, (int32_t)skf});
                        A.solve_bwd.push_back({i, (int32_t)(dp + 1), (int32_t)A.rowptr[i + 1], (int32_t)skb});
                    }
                }
            }
            A.lvl_rows[l + 1] = (int32_t)A.solve_fwd.size();
        }
    }
    return OK;
}

}  // namespace asi
