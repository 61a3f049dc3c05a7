/*
 * Threshold incomplete LDL^T factorization with Bunch-Kaufman 1x1/2x2 pivots.
 *
 * This produces the inputs of approximate selected inversion: the paper takes
 * an incomplete block factorization P^T A P ~ L D L^T as given (Section 2.1,
 * block factorization equation; the factor comes from a separate block-ILDL
 * package whose algorithm is not described in the paper). The readings used
 * here for what the paper leaves open:
 *   - symmetric scaling s_i = 1/sqrt(max_j |a_ij|) before factoring, undone
 *     afterwards (L <- S^-1 L^ S, D <- S^-1 D^ S^-1);
 *   - right-looking elimination on the exact Schur complement of the dropped
 *     factor (equivalent to Crout ILDL), with Bunch-Kaufman pivot selection,
 *     alpha = (1 + sqrt(17))/8, on the current Schur column;
 *   - an L entry is dropped when |l_ik| < tau on the scaled factor; a row of a
 *     2x2 pivot is dropped only when both of its entries are below tau, and
 *     otherwise both entries are kept (explicit zeros included) so the two
 *     columns share one row set; D is never dropped; tau = 0 keeps every
 *     structural fill entry, numerical zeros included;
 *   - a pivot with |d| < 1e-14 max|A^| is replaced by sign(d) 1e-8 max|A^|
 *     (sign(0) = +) and counted.
 *
 * The Schur complement is held in full symmetric form as one open-addressing
 * hash table per unknown, keyed by unknown id; eliminated keys are skipped on
 * reads and pruned when a table grows. Unknown ids are the (already ordered)
 * input positions; pivoting only changes the final position of each id, so no
 * relabelling of stored data is ever needed.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t *key;
    double *val;
    int32_t cap;
    int32_t cnt;
} htab;

/* Fibonacci hashing: the top log2(cap) bits of k * 2^32/phi */
static inline uint32_t hslot(int32_t k, int32_t cap) {
    return ((uint32_t)k * 2654435761u) >> (32 - __builtin_ctz((unsigned)cap));
}

static int ht_init(htab *h, int32_t want) {
    int32_t cap = 8;
    while (cap < 2 * want) cap <<= 1;
    h->key = (int32_t *)malloc(sizeof(int32_t) * cap);
    h->val = (double *)malloc(sizeof(double) * cap);
    if (!h->key || !h->val) return -1;
    for (int32_t i = 0; i < cap; ++i) h->key[i] = -1;
    h->cap = cap;
    h->cnt = 0;
    return 0;
}

static void ht_free(htab *h) {
    free(h->key);
    free(h->val);
    h->key = NULL;
    h->val = NULL;
    h->cap = h->cnt = 0;
}

/* grow (and drop keys of eliminated unknowns) */
static int ht_grow(htab *h, const uint8_t *elim) {
    int32_t live = 0;
    for (int32_t i = 0; i < h->cap; ++i)
        if (h->key[i] >= 0 && !elim[h->key[i]]) ++live;
    int32_t cap = 8;
    while (cap < 4 * (live + 1)) cap <<= 1;
    int32_t *nk = (int32_t *)malloc(sizeof(int32_t) * cap);
    double *nv = (double *)malloc(sizeof(double) * cap);
    if (!nk || !nv) return -1;
    for (int32_t i = 0; i < cap; ++i) nk[i] = -1;
    for (int32_t i = 0; i < h->cap; ++i) {
        int32_t k = h->key[i];
        if (k < 0 || elim[k]) continue;
        uint32_t s = hslot(k, cap);
        while (nk[s] >= 0) s = (s + 1) & (uint32_t)(cap - 1);
        nk[s] = k;
        nv[s] = h->val[i];
    }
    free(h->key);
    free(h->val);
    h->key = nk;
    h->val = nv;
    h->cap = cap;
    h->cnt = live;
    return 0;
}

static inline int ht_add(htab *h, int32_t k, double d, const uint8_t *elim) {
    if (2 * (h->cnt + 1) > h->cap)
        if (ht_grow(h, elim)) return -1;
    uint32_t s = hslot(k, h->cap);
    for (;;) {
        int32_t kk = h->key[s];
        if (kk == k) {
            h->val[s] += d;
            return 0;
        }
        if (kk < 0) {
            h->key[s] = k;
            h->val[s] = d;
            h->cnt++;
            return 0;
        }
        s = (s + 1) & (uint32_t)(h->cap - 1);
    }
}

static inline int ht_get(const htab *h, int32_t k, double *out) {
    if (h->cap == 0) return 0;
    uint32_t s = hslot(k, h->cap);
    for (;;) {
        int32_t kk = h->key[s];
        if (kk == k) {
            *out = h->val[s];
            return 1;
        }
        if (kk < 0) return 0;
        s = (s + 1) & (uint32_t)(h->cap - 1);
    }
}

/* growable triplet list of L entries: (row id, column position, value) */
typedef struct {
    int32_t *rid;
    int32_t *cpos;
    double *v;
    int64_t n, cap;
} trip;

static int trip_push(trip *t, int32_t rid, int32_t cpos, double v) {
    if (t->n == t->cap) {
        int64_t nc = t->cap ? 2 * t->cap : 1024;
        int32_t *a = (int32_t *)realloc(t->rid, sizeof(int32_t) * nc);
        if (!a) return -1;
        t->rid = a;
        int32_t *b = (int32_t *)realloc(t->cpos, sizeof(int32_t) * nc);
        if (!b) return -1;
        t->cpos = b;
        double *c = (double *)realloc(t->v, sizeof(double) * nc);
        if (!c) return -1;
        t->v = c;
        t->cap = nc;
    }
    t->rid[t->n] = rid;
    t->cpos[t->n] = cpos;
    t->v[t->n] = v;
    t->n++;
    return 0;
}

typedef struct {
    int32_t n;
    int64_t nnzL;
    int64_t *L_rowptr; /* n+1 */
    int32_t *L_col;    /* nnzL */
    double *L_val;     /* nnzL */
    double *d_diag;    /* n */
    double *d_sub;     /* n */
    int8_t *piv;       /* n */
    int32_t *order;    /* n: position -> input id */
    int64_t n_perturbed;
    int64_t n_2x2;
    int64_t peak_schur;
} ildl_result;

/* column of the active Schur complement of unknown p: ids and values */
static int32_t gather_col(const htab *h, const uint8_t *elim, int32_t *ids, double *vals) {
    int32_t c = 0;
    for (int32_t s = 0; s < h->cap; ++s) {
        int32_t k = h->key[s];
        if (k >= 0 && !elim[k]) {
            ids[c] = k;
            vals[c] = h->val[s];
            ++c;
        }
    }
    return c;
}

/* largest magnitude entry; ties broken by the smallest current position */
static double col_max(const int32_t *ids, const double *vals, int32_t c, const int32_t *where,
                      int32_t *arg) {
    double best = 0.0;
    int32_t bi = -1;
    for (int32_t t = 0; t < c; ++t) {
        double a = fabs(vals[t]);
        if (a > best || (a == best && bi >= 0 && a > 0 && where[ids[t]] < where[bi])) {
            best = a;
            bi = ids[t];
        }
    }
    *arg = bi;
    return best;
}

static void swap_pos(int32_t *order, int32_t *where, int32_t a, int32_t b) {
    if (a == b) return;
    int32_t ia = order[a], ib = order[b];
    order[a] = ib;
    order[b] = ia;
    where[ib] = a;
    where[ia] = b;
}

void ildl_free(ildl_result *r) {
    if (!r) return;
    free(r->L_rowptr);
    free(r->L_col);
    free(r->L_val);
    free(r->d_diag);
    free(r->d_sub);
    free(r->piv);
    free(r->order);
    memset(r, 0, sizeof(*r));
}

/*
 * n, rowptr/col/val: the symmetric input (both triangles) in its ordered
 * numbering. tau: drop tolerance. pivoting: 0 = always 1x1 in the given order,
 * 1 = Bunch-Kaufman. Returns 0 on success, -1 on allocation failure,
 * -2 on a singular 2x2 block.
 */
/* Progress lines on stderr every `every` pivots (0: none), for long runs. */
static int32_t progress_every = 0;
void ildl_set_progress(int32_t every) { progress_every = every > 0 ? every : 0; }

int ildl_bk(int32_t n, const int64_t *rowptr, const int32_t *col, const double *val, double tau,
            int pivoting, ildl_result *res) {
    memset(res, 0, sizeof(*res));
    const double alpha = (1.0 + sqrt(17.0)) / 8.0;
    int rc = -1;
    double *scale = (double *)malloc(sizeof(double) * n);
    double *diag = (double *)calloc(n, sizeof(double));
    htab *tab = (htab *)calloc(n, sizeof(htab));
    uint8_t *elim = (uint8_t *)calloc(n, 1);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *where = (int32_t *)malloc(sizeof(int32_t) * n);
    double *dd = (double *)calloc(n, sizeof(double));
    double *ds = (double *)calloc(n, sizeof(double));
    int8_t *pv = (int8_t *)calloc(n, 1);
    int32_t *idp = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    double *vp = (double *)malloc(sizeof(double) * (n + 1));
    int32_t *idr = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    double *vr = (double *)malloc(sizeof(double) * (n + 1));
    int32_t *kid = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    double *k0 = (double *)malloc(sizeof(double) * (n + 1));
    double *k1 = (double *)malloc(sizeof(double) * (n + 1));
    double *w0 = (double *)malloc(sizeof(double) * (n + 1));
    double *w1 = (double *)malloc(sizeof(double) * (n + 1));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    trip L = {0};
    if (!scale || !diag || !tab || !elim || !order || !where || !dd || !ds || !pv || !idp || !vp ||
        !idr || !vr || !kid || !k0 || !k1 || !w0 || !w1 || !mark)
        goto done;

    /* scaling and the scaled input in the hash tables */
    double amax = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double m = 0.0;
        for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) m = fmax(m, fabs(val[q]));
        scale[i] = m > 0 ? 1.0 / sqrt(m) : 1.0;
    }
    for (int32_t i = 0; i < n; ++i) {
        if (ht_init(&tab[i], (int32_t)(rowptr[i + 1] - rowptr[i]))) goto done;
        for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            int32_t j = col[q];
            double a = scale[i] * val[q] * scale[j];
            amax = fmax(amax, fabs(a));
            if (j == i)
                diag[i] += a;
            else if (ht_add(&tab[i], j, a, elim))
                goto done;
        }
        order[i] = i;
        where[i] = i;
        mark[i] = -1;
    }
    const double tiny = 1e-14 * amax, repl = 1e-8 * amax;

    int32_t k = 0;
    int32_t next_report = progress_every;
    while (k < n) {
        if (progress_every > 0 && k >= next_report) {
            fprintf(stderr, "[ildl] %d of %d pivots, %lld entries of L so far\n", k, n, (long long)L.n);
            fflush(stderr);
            next_report += progress_every;
        }
        int32_t p = order[k];
        int32_t cp = gather_col(&tab[p], elim, idp, vp);
        int two = 0;
        int32_t r = -1;
        if (pivoting && cp > 0) {
            double lam = col_max(idp, vp, cp, where, &r);
            if (lam > 0 && fabs(diag[p]) < alpha * lam) {
                int32_t cr = gather_col(&tab[r], elim, idr, vr);
                int32_t dummy;
                double sig = col_max(idr, vr, cr, where, &dummy);
                if (fabs(diag[p]) * sig >= alpha * lam * lam) {
                    /* 1x1 with p */
                } else if (fabs(diag[r]) >= alpha * sig) {
                    swap_pos(order, where, k, where[r]);
                    p = r;
                    cp = cr;
                    memcpy(idp, idr, sizeof(int32_t) * cr);
                    memcpy(vp, vr, sizeof(double) * cr);
                } else {
                    two = 1;
                    swap_pos(order, where, k + 1, where[r]);
                }
            }
        }
        if (!two) {
            double d = diag[p];
            if (fabs(d) < tiny) {
                d = (d >= 0 ? 1.0 : -1.0) * repl;
                res->n_perturbed++;
            }
            int32_t c = 0;
            for (int32_t t = 0; t < cp; ++t) {
                double l = vp[t] / d;
                if (fabs(l) < tau) continue;
                kid[c] = idp[t];
                k0[c] = l;
                ++c;
            }
            dd[k] = d;
            pv[k] = 0;
            elim[p] = 1;
            for (int32_t a = 0; a < c; ++a) {
                if (trip_push(&L, kid[a], k, k0[a])) goto done;
                double la = k0[a] * d;
                diag[kid[a]] -= la * k0[a];
                htab *h = &tab[kid[a]];
                for (int32_t b = 0; b < c; ++b) {
                    if (b == a) continue;
                    if (ht_add(h, kid[b], -(la * k0[b]), elim)) goto done;
                }
            }
            ht_free(&tab[p]);
            k += 1;
        } else {
            /* 2x2 block on (p, r) at positions k, k+1 */
            double a11 = diag[p], a22 = diag[r], b = 0.0;
            ht_get(&tab[p], r, &b);
            if (b == 0.0) {
                rc = -2;
                goto done;
            }
            double al = a11 / b, ga = a22 / b, den = b * (al * ga - 1.0);
            if (den == 0.0 || !isfinite(den)) {
                rc = -2;
                goto done;
            }
            /* union of the active neighbours of p and r (without p, r) */
            int32_t cr = gather_col(&tab[r], elim, idr, vr);
            int32_t u = 0;
            for (int32_t t = 0; t < cp; ++t) {
                int32_t i = idp[t];
                if (i == r) continue;
                mark[i] = u;
                kid[u] = i;
                w0[u] = vp[t];
                w1[u] = 0.0;
                ++u;
            }
            for (int32_t t = 0; t < cr; ++t) {
                int32_t i = idr[t];
                if (i == p) continue;
                if (mark[i] >= 0) {
                    w1[mark[i]] = vr[t];
                } else {
                    mark[i] = u;
                    kid[u] = i;
                    w0[u] = 0.0;
                    w1[u] = vr[t];
                    ++u;
                }
            }
            int32_t c = 0;
            for (int32_t t = 0; t < u; ++t) {
                mark[kid[t]] = -1;
                double l0 = (w0[t] * ga - w1[t]) / den;
                double l1 = (-w0[t] + w1[t] * al) / den;
                if (fabs(l0) < tau && fabs(l1) < tau) continue;
                kid[c] = kid[t];
                k0[c] = l0;
                k1[c] = l1;
                w0[c] = w0[t];
                w1[c] = w1[t];
                ++c;
            }
            dd[k] = a11;
            dd[k + 1] = a22;
            ds[k] = b;
            pv[k] = 1;
            pv[k + 1] = 2;
            elim[p] = 1;
            elim[r] = 1;
            res->n_2x2++;
            for (int32_t a = 0; a < c; ++a) {
                if (trip_push(&L, kid[a], k, k0[a])) goto done;
                if (trip_push(&L, kid[a], k + 1, k1[a])) goto done;
                diag[kid[a]] -= k0[a] * w0[a] + k1[a] * w1[a];
                htab *h = &tab[kid[a]];
                for (int32_t bb = 0; bb < c; ++bb) {
                    if (bb == a) continue;
                    if (ht_add(h, kid[bb], -(k0[a] * w0[bb] + k1[a] * w1[bb]), elim)) goto done;
                }
            }
            ht_free(&tab[p]);
            ht_free(&tab[r]);
            k += 2;
        }
    }

    /* unscale and emit L as CSR over final positions */
    res->n = n;
    res->nnzL = L.n;
    res->L_rowptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    res->L_col = (int32_t *)malloc(sizeof(int32_t) * (L.n ? L.n : 1));
    res->L_val = (double *)malloc(sizeof(double) * (L.n ? L.n : 1));
    if (!res->L_rowptr || !res->L_col || !res->L_val) goto done;
    for (int64_t t = 0; t < L.n; ++t) res->L_rowptr[where[L.rid[t]] + 1]++;
    for (int32_t i = 0; i < n; ++i) res->L_rowptr[i + 1] += res->L_rowptr[i];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
        if (!fill) goto done;
        memcpy(fill, res->L_rowptr, sizeof(int64_t) * ((size_t)n + 1));
        /* triplets were pushed in increasing column position, so rows come out sorted */
        for (int64_t t = 0; t < L.n; ++t) {
            int32_t row = where[L.rid[t]];
            int32_t cpos = L.cpos[t];
            int64_t q = fill[row]++;
            res->L_col[q] = cpos;
            res->L_val[q] = L.v[t] * scale[order[cpos]] / scale[L.rid[t]];
        }
        free(fill);
    }
    res->d_diag = dd;
    res->d_sub = ds;
    res->piv = pv;
    res->order = order;
    for (int32_t q = 0; q < n; ++q) {
        double sq = scale[order[q]];
        dd[q] = dd[q] / (sq * sq);
        if (pv[q] == 1) ds[q] = ds[q] / (sq * scale[order[q + 1]]);
    }
    dd = NULL;
    ds = NULL;
    pv = NULL;
    order = NULL;
    rc = 0;

done:
    if (tab)
        for (int32_t i = 0; i < n; ++i) ht_free(&tab[i]);
    free(tab);
    free(scale);
    free(diag);
    free(elim);
    free(order);
    free(where);
    free(dd);
    free(ds);
    free(pv);
    free(idp);
    free(vp);
    free(idr);
    free(vr);
    free(kid);
    free(k0);
    free(k1);
    free(w0);
    free(w1);
    free(mark);
    free(L.rid);
    free(L.cpos);
    free(L.v);
    if (rc != 0) ildl_free(res);
    return rc;
}
