/*
 * CPU oracle for approximate selected inversion from an incomplete LDL^T.
 *
 * TEST INFRASTRUCTURE ONLY. Plain, single-threaded, float64 code that states
 * what the method computes; it is used by the tests, the smoke check and the
 * CPU-baseline timing, and by nothing on the product path. It shares no code
 * with the GPU library.
 *
 * Inputs: n, L strictly lower CSR (unit diagonal implicit), D as d_diag /
 * d_sub / piv (piv 0: 1x1; 1/2: first/second index of a 2x2 block, with
 * d_sub[j] = D[j+1,j] at a block start). Outputs live on the pattern
 * S = {(i,j): (L + D + L^T)_ij != 0} (Section 1) as values over S's CSR
 * (both triangles, columns sorted within rows), built here by
 * orc_pattern.
 *
 * Readings where the paper is silent (listed with their reasons in the
 * design notes of the repository):
 *   - entries outside S are treated as zero, both when they are used and when
 *     they are produced (Section 2.1, "entries outside this pattern are
 *     discarded");
 *   - a 2x2 block J = {j, j+1} uses the union of the row sets of its two
 *     columns; its inverse is formed in the scaled form
 *     [gamma, -1; -1, alpha] / (b (alpha gamma - 1)) with b = B_21,
 *     alpha = B_11 / b, gamma = B_22 / b; the off-diagonal of Z_JJ is the mean
 *     of its two (mathematically equal) expressions;
 *   - NInv drops entries of each new Neumann term with |t| < delta
 *     (Section 2.2) and evaluates (L^inv)^T D^-1 L^inv only on S;
 *   - Mix keeps the SelInv value where |Z_ij| > eps sqrt(|Z_ii Z_jj|)
 *     (Section 2.3, relative reading of "above a target tolerance");
 *   - SPAI runs a fixed number of Jacobi-preconditioned CG steps on the
 *     normal equations of each column, starting from the Mix column, and
 *     stops early only on an exactly zero residual or curvature
 *     (Section 2.4).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_E_PATTERN = 1, ORC_E_SINGULAR = 2, ORC_E_ALLOC = 3 };

/* ---------- pattern S of L + D + L^T ------------------------------------ */

/* first index of the D block that contains i */
static int32_t block_start(const int8_t *piv, int32_t i) { return piv[i] == 2 ? i - 1 : i; }

/*
 * Builds S (both triangles) from the strict lower L and the block structure.
 * S_rowptr has n+1 entries; S_col must hold nnzS entries, where nnzS comes
 * from a first call with S_col == NULL.
 * The lower part of column j of S is: {j+1} if j starts a 2x2 block, plus
 * R_J = rows r > max J stored in any column of J's block.
 */
int orc_pattern(int32_t n, const int64_t *Lp, const int32_t *Li, const int8_t *piv, int64_t *S_rowptr,
                int32_t *S_col, int64_t *nnzS_out) {
    /* validate L and piv */
    for (int32_t i = 0; i < n; ++i) {
        if (piv[i] == 1 && (i + 1 >= n || piv[i + 1] != 2)) return ORC_E_PATTERN;
        if (piv[i] == 2 && (i == 0 || piv[i - 1] != 1)) return ORC_E_PATTERN;
        if (piv[i] < 0 || piv[i] > 2) return ORC_E_PATTERN;
        for (int64_t q = Lp[i]; q < Lp[i + 1]; ++q) {
            if (Li[q] < 0 || Li[q] >= i) return ORC_E_PATTERN;
            if (q > Lp[i] && Li[q] <= Li[q - 1]) return ORC_E_PATTERN;
            if (piv[i] == 2 && Li[q] == i - 1) return ORC_E_PATTERN; /* inside a 2x2 block */
        }
    }
    /* mark[(r, J)] via a dense marker per row: for row r, the set of block
       starts J with r in R_J is the set of block starts of the columns in row r */
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!mark || !cnt) {
        free(mark);
        free(cnt);
        return ORC_E_ALLOC;
    }
    for (int32_t i = 0; i < n; ++i) mark[i] = -1;
    /* pass 1: count per row. Row r of S holds: lower cols {block partners},
       each J with r in R_J (both columns of a 2x2 J), the diagonal, and the
       upper entries (mirrors). Count lower first, mirror by symmetry later. */
    for (int32_t r = 0; r < n; ++r) {
        for (int64_t q = Lp[r]; q < Lp[r + 1]; ++q) {
            int32_t J = block_start(piv, Li[q]);
            if (mark[J] == r) continue;
            mark[J] = r;
            int w = piv[J] == 1 ? 2 : 1;
            cnt[r] += w; /* lower entries of row r */
            cnt[J] += 1; /* upper mirrors in row J (and J+1) */
            if (w == 2) cnt[J + 1] += 1;
        }
        cnt[r] += 1; /* diagonal */
        if (piv[r] == 1) cnt[r] += 1; /* (r, r+1) */
        if (piv[r] == 2) cnt[r] += 1; /* (r, r-1) */
    }
    S_rowptr[0] = 0;
    for (int32_t i = 0; i < n; ++i) S_rowptr[i + 1] = S_rowptr[i] + cnt[i];
    *nnzS_out = S_rowptr[n];
    if (S_col) {
        /* pass 2: fill rows with lower entries in increasing column order,
           then the diagonal block, then uppers appended by increasing row */
        int64_t *fill = cnt;
        for (int32_t i = 0; i < n; ++i) fill[i] = S_rowptr[i];
        for (int32_t i = 0; i < n; ++i) mark[i] = -1;
        for (int32_t r = 0; r < n; ++r) {
            /* lower entries of row r (columns < block_start(r)) are emitted in
               column order because L's row r is sorted */
            for (int64_t q = Lp[r]; q < Lp[r + 1]; ++q) {
                int32_t J = block_start(piv, Li[q]);
                if (mark[J] == r) continue;
                mark[J] = r;
                S_col[fill[r]++] = J;
                if (piv[J] == 1) S_col[fill[r]++] = J + 1;
            }
            if (piv[r] == 2) S_col[fill[r]++] = r - 1;
            S_col[fill[r]++] = r;
            if (piv[r] == 1) S_col[fill[r]++] = r + 1;
            /* row r appears as an upper entry (column r) of rows J < r that it
               belongs to: emitted when row r is processed, rows J ascending */
        }
        /* upper entries: for every lower entry (r, c), add c's row entry r.
           Rows r are visited ascending, so each row's upper part is sorted. */
        for (int32_t r = 0; r < n; ++r) {
            for (int64_t q = S_rowptr[r]; q < S_rowptr[r + 1]; ++q) {
                int32_t c = S_col[q];
                if (c >= block_start(piv, r)) break;
                S_col[fill[c]++] = r;
            }
        }
        for (int32_t i = 0; i < n; ++i)
            if (fill[i] != S_rowptr[i + 1]) {
                free(mark);
                free(cnt);
                return ORC_E_PATTERN;
            }
    }
    free(mark);
    free(cnt);
    return ORC_OK;
}

/* position of column c in row r of S, or -1 */
static int64_t s_find(const int64_t *Sp, const int32_t *Sj, int32_t r, int32_t c) {
    int64_t lo = Sp[r], hi = Sp[r + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) >> 1;
        if (Sj[mid] == c) return mid;
        if (Sj[mid] < c)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

/* value of L(r, c) (strict lower, r > c), 0 if not stored */
static double l_get(const int64_t *Lp, const int32_t *Li, const double *Lx, int32_t r, int32_t c) {
    int64_t lo = Lp[r], hi = Lp[r + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) >> 1;
        if (Li[mid] == c) return Lx[mid];
        if (Li[mid] < c)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return 0.0;
}

/* inverse of the D block starting at j: 1x1 -> inv[0]; 2x2 -> inv[0..2] = (00, 10, 11) */
static int d_block_inverse(const double *dd, const double *ds, const int8_t *piv, int32_t j,
                           double inv[3]) {
    if (piv[j] == 0) {
        if (dd[j] == 0.0) return ORC_E_SINGULAR;
        inv[0] = 1.0 / dd[j];
        return ORC_OK;
    }
    double b = ds[j];
    if (b == 0.0) return ORC_E_SINGULAR;
    double al = dd[j] / b, ga = dd[j + 1] / b;
    double den = b * (al * ga - 1.0);
    if (den == 0.0 || !isfinite(den)) return ORC_E_SINGULAR;
    inv[0] = ga / den;
    inv[1] = -1.0 / den;
    inv[2] = al / den;
    return ORC_OK;
}

/*
 * SelInv on S (Section 2.1, recursion for G21 and G11).
 * Blocks J are processed from the last to the first. With R_J the rows below
 * the block that S holds in J's columns and Zhat the already computed part of
 * Z restricted to S (zero outside S):
 *     Z(R_J, J) = -Zhat(R_J, R_J) L(R_J, J)
 *     Z(J, J)   = D_J^-1 - L(R_J, J)^T Z(R_J, J).
 * Z_S receives all of Z on S in S's CSR layout.
 *
 * flags: ORC_SEL_SENTINEL starts from NaN instead of zero on S, so an entry
 * of Zhat read before its block has written it makes the result non-finite
 * (the recursion only ever reads entries of later blocks). ORC_SEL_FORWARD
 * visits the blocks from the first to the last: a deliberately wrong order,
 * used only by the tests to show that the sentinel detects such a mistake.
 */
#define ORC_SEL_SENTINEL 1
#define ORC_SEL_FORWARD 2
int orc_selinv(int32_t n, const int64_t *Lp, const int32_t *Li, const double *Lx, const double *dd,
               const double *ds, const int8_t *piv, const int64_t *Sp, const int32_t *Sj,
               double *Z_S, int32_t flags) {
    int rc = ORC_OK;
    int32_t *R = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    double *l0 = (double *)malloc(sizeof(double) * (n + 1));
    double *l1 = (double *)malloc(sizeof(double) * (n + 1));
    double *y0 = (double *)malloc(sizeof(double) * (n + 1));
    double *y1 = (double *)malloc(sizeof(double) * (n + 1));
    if (!R || !l0 || !l1 || !y0 || !y1) {
        rc = ORC_E_ALLOC;
        goto out;
    }
    const int forward = (flags & ORC_SEL_FORWARD) != 0;
    const double start = (flags & ORC_SEL_SENTINEL) ? NAN : 0.0;
    for (int64_t q = 0; q < Sp[n]; ++q) Z_S[q] = start;
    int32_t j = forward ? 0 : n - 1;
    while (forward ? j < n : j >= 0) {
        int32_t J = block_start(piv, j);
        int two = piv[J] == 1;
        int32_t last = two ? J + 1 : J;
        /* R_J: the upper part of row `last` of S (columns > last) */
        int32_t c = 0;
        for (int64_t q = Sp[last]; q < Sp[last + 1]; ++q)
            if (Sj[q] > last) R[c++] = Sj[q];
        for (int32_t a = 0; a < c; ++a) {
            l0[a] = l_get(Lp, Li, Lx, R[a], J);
            l1[a] = two ? l_get(Lp, Li, Lx, R[a], J + 1) : 0.0;
        }
        /* Y = -Zhat(R,R) L(R,J) */
        for (int32_t a = 0; a < c; ++a) {
            double s0 = 0.0, s1 = 0.0;
            for (int32_t b = 0; b < c; ++b) {
                int64_t q = s_find(Sp, Sj, R[a], R[b]);
                double z = q >= 0 ? Z_S[q] : 0.0;
                s0 += z * l0[b];
                s1 += z * l1[b];
            }
            y0[a] = -s0;
            y1[a] = -s1;
        }
        double inv[3];
        if ((rc = d_block_inverse(dd, ds, piv, J, inv)) != ORC_OK) goto out;
        for (int32_t a = 0; a < c; ++a) {
            Z_S[s_find(Sp, Sj, R[a], J)] = y0[a];
            Z_S[s_find(Sp, Sj, J, R[a])] = y0[a];
            if (two) {
                Z_S[s_find(Sp, Sj, R[a], J + 1)] = y1[a];
                Z_S[s_find(Sp, Sj, J + 1, R[a])] = y1[a];
            }
        }
        double d00 = 0.0, d10 = 0.0, d01 = 0.0, d11 = 0.0;
        for (int32_t a = 0; a < c; ++a) {
            d00 += l0[a] * y0[a];
            d11 += l1[a] * y1[a];
            d10 += l1[a] * y0[a];
            d01 += l0[a] * y1[a];
        }
        Z_S[s_find(Sp, Sj, J, J)] = inv[0] - d00;
        if (two) {
            double off = inv[1] - 0.5 * (d10 + d01);
            Z_S[s_find(Sp, Sj, J + 1, J + 1)] = inv[2] - d11;
            Z_S[s_find(Sp, Sj, J + 1, J)] = off;
            Z_S[s_find(Sp, Sj, J, J + 1)] = off;
        }
        j = forward ? last + 1 : J - 1;
    }
out:
    free(R);
    free(l0);
    free(l1);
    free(y0);
    free(y1);
    return rc;
}

/* ---------- NInv (Section 2.2) ------------------------------------------ */

/*
 * Truncated Neumann series L^inv = sum_{m=0}^{p} T_m with T_0 = I and
 * T_m = drop_delta(E T_{m-1}), E = I - L (the negated strict lower part), then
 * N = (L^inv)^T D^-1 L^inv on S.
 * Column j of L^inv is built from t^0 = e_j, t^m = drop(E t^{m-1}).
 * Linv_colptr (n+1) and the per-column rows/values are returned through
 * caller buffers of capacity cap (entries); *need receives the total count.
 * Rows within a column are sorted.
 */
int orc_linv(int32_t n, const int64_t *Lp, const int32_t *Li, const double *Lx, int32_t p,
             double delta, int64_t cap, int64_t *Vp, int32_t *Vi, double *Vx, int64_t *need) {
    /* column access to L */
    int64_t nnz = Lp[n];
    int64_t *Cp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *Ci = (int32_t *)malloc(sizeof(int32_t) * (nnz ? nnz : 1));
    double *Cx = (double *)malloc(sizeof(double) * (nnz ? nnz : 1));
    double *t = (double *)calloc(n, sizeof(double));
    double *tn = (double *)calloc(n, sizeof(double));
    double *acc = (double *)calloc(n, sizeof(double));
    int32_t *ts = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *tns = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *as = (int32_t *)malloc(sizeof(int32_t) * n);
    uint8_t *inT = (uint8_t *)calloc(n, 1);
    uint8_t *inA = (uint8_t *)calloc(n, 1);
    int rc = ORC_OK;
    if (!Cp || !Ci || !Cx || !t || !tn || !acc || !ts || !tns || !as || !inT || !inA) {
        rc = ORC_E_ALLOC;
        goto out;
    }
    for (int64_t q = 0; q < nnz; ++q) Cp[Li[q] + 1]++;
    for (int32_t i = 0; i < n; ++i) Cp[i + 1] += Cp[i];
    {
        int64_t *f = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
        if (!f) {
            rc = ORC_E_ALLOC;
            goto out;
        }
        memcpy(f, Cp, sizeof(int64_t) * ((size_t)n + 1));
        for (int32_t r = 0; r < n; ++r)
            for (int64_t q = Lp[r]; q < Lp[r + 1]; ++q) {
                int64_t d = f[Li[q]]++;
                Ci[d] = r;
                Cx[d] = Lx[q];
            }
        free(f);
    }
    int64_t tot = 0;
    if (Vp) Vp[0] = 0;
    for (int32_t j = 0; j < n; ++j) {
        /* t = e_j; acc = e_j */
        int32_t nt = 1, na = 1;
        ts[0] = j;
        t[j] = 1.0;
        as[0] = j;
        acc[j] = 1.0;
        inA[j] = 1;
        for (int32_t m = 1; m <= p && nt > 0; ++m) {
            /* tn = E t = -sum_k t_k L(:,k) */
            int32_t nn = 0;
            for (int32_t a = 0; a < nt; ++a) {
                int32_t k = ts[a];
                double tk = t[k];
                for (int64_t q = Cp[k]; q < Cp[k + 1]; ++q) {
                    int32_t r = Ci[q];
                    if (!inT[r]) {
                        inT[r] = 1;
                        tns[nn++] = r;
                        tn[r] = 0.0;
                    }
                    tn[r] -= tk * Cx[q];
                }
            }
            for (int32_t a = 0; a < nt; ++a) t[ts[a]] = 0.0;
            /* drop and accumulate */
            int32_t kept = 0;
            for (int32_t a = 0; a < nn; ++a) {
                int32_t r = tns[a];
                inT[r] = 0;
                double v = tn[r];
                tn[r] = 0.0;
                if (fabs(v) < delta) continue;
                ts[kept++] = r;
                t[r] = v;
                if (!inA[r]) {
                    inA[r] = 1;
                    as[na++] = r;
                    acc[r] = 0.0;
                }
                acc[r] += v;
            }
            nt = kept;
        }
        for (int32_t a = 0; a < nt; ++a) t[ts[a]] = 0.0;
        /* emit sorted (insertion sort on the small list) */
        for (int32_t a = 1; a < na; ++a) {
            int32_t v = as[a], b = a - 1;
            while (b >= 0 && as[b] > v) {
                as[b + 1] = as[b];
                --b;
            }
            as[b + 1] = v;
        }
        for (int32_t a = 0; a < na; ++a) {
            int32_t r = as[a];
            if (Vi && tot < cap) {
                Vi[tot] = r;
                Vx[tot] = acc[r];
            }
            ++tot;
            acc[r] = 0.0;
            inA[r] = 0;
        }
        if (Vp) Vp[j + 1] = tot;
    }
    *need = tot;
out:
    free(Cp);
    free(Ci);
    free(Cx);
    free(t);
    free(tn);
    free(acc);
    free(ts);
    free(tns);
    free(as);
    free(inT);
    free(inA);
    return rc;
}

/*
 * N on S from the columns of L^inv: N_ij = sum_k L^inv_ki (D^-1 L^inv)_kj,
 * computed for i >= j and mirrored.
 */
int orc_ninv_product(int32_t n, const int64_t *Vp, const int32_t *Vi, const double *Vx, const double *dd,
                     const double *ds, const int8_t *piv, const int64_t *Sp, const int32_t *Sj,
                     double *N_S) {
    double *w = (double *)calloc(n, sizeof(double));
    int rc = ORC_OK;
    if (!w) return ORC_E_ALLOC;
    for (int32_t j = 0; j < n; ++j) {
        /* w = D^-1 L^inv(:, j), scattered densely */
        for (int64_t q = Vp[j]; q < Vp[j + 1]; ++q) {
            int32_t k = Vi[q];
            int32_t K = block_start(piv, k);
            double inv[3];
            if ((rc = d_block_inverse(dd, ds, piv, K, inv)) != ORC_OK) goto out;
            if (piv[K] == 0) {
                w[k] += inv[0] * Vx[q];
            } else if (k == K) {
                w[K] += inv[0] * Vx[q];
                w[K + 1] += inv[1] * Vx[q];
            } else {
                w[K] += inv[1] * Vx[q];
                w[K + 1] += inv[2] * Vx[q];
            }
        }
        for (int64_t q = Sp[j]; q < Sp[j + 1]; ++q) {
            int32_t i = Sj[q];
            if (i < j) continue;
            double s = 0.0;
            for (int64_t t = Vp[i]; t < Vp[i + 1]; ++t) s += Vx[t] * w[Vi[t]];
            N_S[q] = s; /* position (j, i) */
            N_S[s_find(Sp, Sj, i, j)] = s;
        }
        /* clear w */
        for (int64_t q = Vp[j]; q < Vp[j + 1]; ++q) {
            int32_t K = block_start(piv, Vi[q]);
            w[K] = 0.0;
            if (piv[K] == 1) w[K + 1] = 0.0;
        }
    }
out:
    free(w);
    return rc;
}

/* ---------- Mix (Section 2.3) ------------------------------------------- */

void orc_mix(int32_t n, const int64_t *Sp, const int32_t *Sj, const double *Z_S, const double *N_S,
             double eps, double *M_S) {
    double *zd = (double *)malloc(sizeof(double) * (n ? n : 1));
    for (int32_t i = 0; i < n; ++i) zd[i] = Z_S[s_find(Sp, Sj, i, i)];
    for (int32_t i = 0; i < n; ++i)
        for (int64_t q = Sp[i]; q < Sp[i + 1]; ++q) {
            int32_t j = Sj[q];
            int keep = fabs(Z_S[q]) > eps * sqrt(fabs(zd[i] * zd[j]));
            M_S[q] = keep ? Z_S[q] : N_S[q];
        }
    free(zd);
}

/* ---------- SPAI refinement (Section 2.4) ------------------------------- */

/*
 * Column j of the refined inverse minimises ||Ah m - e_j||_2 over m supported
 * on J = {i : (i, j) in S}, Ah = P^T A P given as CSR (both triangles) in the
 * factor ordering. The normal equations (Ah_J^T Ah_J) m = Ah_J^T e_j are
 * solved by `iters` Jacobi-preconditioned CG steps from m = M(J, j). The
 * column is written transposed (into row j of X_S); R = (X + X^T)/2.
 */
int orc_spai(int32_t n, const int64_t *Ap, const int32_t *Aj, const double *Ax, const int64_t *Sp,
             const int32_t *Sj, const double *M_S, int32_t iters, double *R_S) {
    int rc = ORC_OK;
    int64_t nnzS = Sp[n];
    double *X = (double *)malloc(sizeof(double) * (nnzS ? nnzS : 1));
    double *colnorm2 = (double *)calloc(n, sizeof(double));
    int32_t maxc = 0;
    for (int32_t j = 0; j < n; ++j) maxc = (int32_t)fmax(maxc, (double)(Sp[j + 1] - Sp[j]));
    double *G = (double *)malloc(sizeof(double) * ((size_t)maxc * maxc + 1));
    double *x = (double *)malloc(sizeof(double) * (maxc + 1));
    double *b = (double *)malloc(sizeof(double) * (maxc + 1));
    double *r = (double *)malloc(sizeof(double) * (maxc + 1));
    double *z = (double *)malloc(sizeof(double) * (maxc + 1));
    double *pp = (double *)malloc(sizeof(double) * (maxc + 1));
    double *gp = (double *)malloc(sizeof(double) * (maxc + 1));
    double *dense = (double *)calloc(n, sizeof(double));
    if (!X || !colnorm2 || !G || !x || !b || !r || !z || !pp || !gp || !dense) {
        rc = ORC_E_ALLOC;
        goto out;
    }
    /* ||Ah(:, i)||^2 = ||Ah(i, :)||^2 by symmetry */
    for (int32_t i = 0; i < n; ++i)
        for (int64_t q = Ap[i]; q < Ap[i + 1]; ++q) colnorm2[i] += Ax[q] * Ax[q];
    for (int32_t j = 0; j < n; ++j) {
        int64_t s0 = Sp[j];
        int32_t c = (int32_t)(Sp[j + 1] - s0);
        const int32_t *J = Sj + s0;
        /* G = Ah_J^T Ah_J: G_ab = sum_r Ah(r, J_a) Ah(r, J_b) = <Ah(J_a,:), Ah(J_b,:)> */
        for (int32_t a = 0; a < c; ++a) {
            for (int64_t q = Ap[J[a]]; q < Ap[J[a] + 1]; ++q) dense[Aj[q]] = Ax[q];
            for (int32_t bb = 0; bb < c; ++bb) {
                double s = 0.0;
                for (int64_t q = Ap[J[bb]]; q < Ap[J[bb] + 1]; ++q) s += dense[Aj[q]] * Ax[q];
                G[(size_t)a * c + bb] = s;
            }
            for (int64_t q = Ap[J[a]]; q < Ap[J[a] + 1]; ++q) dense[Aj[q]] = 0.0;
            /* b_a = (Ah_J^T e_j)_a = Ah(j, J_a) */
            double v = 0.0;
            for (int64_t q = Ap[j]; q < Ap[j + 1]; ++q)
                if (Aj[q] == J[a]) v = Ax[q];
            b[a] = v;
            /* start: the Mix column, M(J_a, j) = M(j, J_a) (symmetric pattern) */
            x[a] = M_S[s0 + a];
        }
        /* r = b - G x, z = r / diag, p = z */
        double rz = 0.0;
        for (int32_t a = 0; a < c; ++a) {
            double s = 0.0;
            for (int32_t bb = 0; bb < c; ++bb) s += G[(size_t)a * c + bb] * x[bb];
            r[a] = b[a] - s;
            z[a] = r[a] / colnorm2[J[a]];
            pp[a] = z[a];
            rz += r[a] * z[a];
        }
        for (int32_t it = 0; it < iters; ++it) {
            if (rz == 0.0) break;
            double pgp = 0.0;
            for (int32_t a = 0; a < c; ++a) {
                double s = 0.0;
                for (int32_t bb = 0; bb < c; ++bb) s += G[(size_t)a * c + bb] * pp[bb];
                gp[a] = s;
                pgp += pp[a] * s;
            }
            if (pgp == 0.0) break;
            double al = rz / pgp, rzn = 0.0;
            for (int32_t a = 0; a < c; ++a) {
                x[a] += al * pp[a];
                r[a] -= al * gp[a];
                z[a] = r[a] / colnorm2[J[a]];
                rzn += r[a] * z[a];
            }
            double be = rzn / rz;
            for (int32_t a = 0; a < c; ++a) pp[a] = z[a] + be * pp[a];
            rz = rzn;
        }
        for (int32_t a = 0; a < c; ++a) X[s0 + a] = x[a]; /* X(j, J_a) = m_a = M'(J_a, j) */
    }
    for (int32_t i = 0; i < n; ++i)
        for (int64_t q = Sp[i]; q < Sp[i + 1]; ++q) {
            int32_t j = Sj[q];
            R_S[q] = 0.5 * (X[q] + X[s_find(Sp, Sj, j, i)]);
        }
out:
    free(X);
    free(colnorm2);
    free(G);
    free(x);
    free(b);
    free(r);
    free(z);
    free(pp);
    free(gp);
    free(dense);
    return rc;
}

/* ---------- rank-k correction on S (Section 2.5) ------------------------ */

/* out_ij = in_ij + sum_m lambda_m V_im V_jm for (i, j) in S; V is n x k row-major */
void orc_lowrank(int32_t n, int32_t k, const double *V, const double *lam, const int64_t *Sp,
                 const int32_t *Sj, const double *in_S, double *out_S) {
    for (int32_t i = 0; i < n; ++i)
        for (int64_t q = Sp[i]; q < Sp[i + 1]; ++q) {
            int32_t j = Sj[q];
            double s = 0.0;
            for (int32_t m = 0; m < k; ++m) s += lam[m] * V[(size_t)i * k + m] * V[(size_t)j * k + m];
            out_S[q] = in_S[q] + s;
        }
}
