// Kernel launch interface of libasi (host <-> device code of the library).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "asi_internal.h"

namespace asi {

// Device-side status codes latched into the workspace status word.
enum : int32_t {
    ST_PERM = 1, ST_SINGULAR = 3, ST_NONFINITE = 4, ST_POOL = 6, ST_LIMIT = 8, ST_TIMEOUT = 9,
    ST_PIVOT = 10  // the device threshold factorization met a pivot that needs a swap or a 2x2 block
};

struct SelinvParams {
    const BlockMeta *meta;  // records of this launch's blocks
    int32_t nblk;
    int32_t nheavy;          // the first nheavy blocks have more than kHeavyHits hits
    const int64_t *ustart;   // n+1
    const int32_t *ucol;     // nnzU
    const int64_t *useg;     // nnzU
    const int64_t *hit_ptr;  // n+1
    const uint32_t *hits;    // hit records (see the analysis)
    const int64_t *mirror_u; // nnzU
    const int64_t *diagpos;  // n
    const int8_t *piv;       // n
    const void *Lu;          // nnzU, L values in u-space (double or float)
    const double *dinv;      // 3n
    void *Zu;                // nnzU, working off-diagonal Z in u-space (double or float)
    double *zdiag;           // n, float64 diagonal of Z
    double *out;             // |S|, float64 result
    int32_t *status;
};

hipError_t launch_dinv(int32_t n, const int8_t *piv, const double *dd, const double *ds, double *dinv,
                       int32_t *status, hipStream_t st);
// one level launch in the given SweepVariant; maxc = the level's largest
// |R_J| (the LDS size of the large-block variants)
hipError_t launch_selinv_level(const SelinvParams &P, int variant, bool fp64, hipStream_t st, int32_t maxc);
// Dataflow sweep over all blocks in one cooperative launch (|R_J| <= kSmallCols).
int flow_grid(bool fp64);
hipError_t launch_selinv_flow(const SelinvParams &P, int32_t nblocks, int32_t *done, int32_t epoch,
                              int32_t spin_limit, bool fp64, int grid, hipStream_t st);
hipError_t launch_lu_to_float(int64_t nnzU, const double *Lu, float *Lf, hipStream_t st);
// L's values from the input's row order into the column layout: Lu[q2u[q]] =
// Lval[q] (read in order, written scattered)
hipError_t launch_scatter_lu(int64_t nnzL, const int32_t *q2u, const double *Lval, void *Lu, bool fp64,
                             hipStream_t st);
hipError_t set_big_lds_limits();
size_t selinv_big_lds_bytes(bool fp64, int G, int32_t C);

// NInv: columns of L^inv into a pool, then (L^inv)^T D^-1 L^inv on S.
struct NinvParams {
    int32_t n;
    const int64_t *rowptr;
    const int32_t *col;
    const int32_t *srow;     // |S|: row of every entry of S
    int64_t rowptr_n;        // |S|
    const int64_t *diagpos;
    const int64_t *mirror;
    const int64_t *ustart;
    const int32_t *ucol;
    const int8_t *piv;
    const void *Lu;  // u-space L values (double or float)
    const double *dinv;
    int32_t p;
    double delta;
    // pool of L^inv columns: rows (int32), linv and w = D^-1 linv (float or double)
    int32_t *prow;
    void *plinv;
    void *pw;
    int64_t pool_cap;
    unsigned long long *pool_top;  // allocation counter
    int64_t *cstart;               // n
    int32_t *clen;                 // n (-1: pending in the large-column pass)
    int32_t *clast;                // n: largest row of the stored column (-1: empty)
    int32_t *ovf_list;             // n
    int32_t *ovf_count;            // 1
    double *out;                   // N on S (float64)
    int32_t *status;
    // product through the transposed series pattern (rows of L^inv): column
    // counts / row pointers (n + 1), fill cursors (n), scan sums, and a flag:
    // 1 while that path applies, 0 to use the entry-by-entry kernel
    unsigned long long *tr_ptr;
    unsigned long long *tr_cur;
    unsigned long long *tr_bsum;
    int32_t *tr_flag;
};

// linv_grid: 0 = as many workgroups of the series kernel as are resident,
// -k = 1/k of that, k > 0 = at most k
hipError_t launch_ninv(const NinvParams &P, bool fp64, hipStream_t st, int linv_grid = 0);
hipError_t set_ninv_lds_limits();

hipError_t launch_zdiag(int32_t n, const int64_t *diagpos, const double *X, double *d, hipStream_t st);
hipError_t launch_mix(int64_t nnz, const int32_t *srow, const int32_t *col, const double *zdiag,
                      const double *Z, const double *N, double eps, double *M, hipStream_t st);
hipError_t launch_diag_err1(int32_t n, const double *d_ref, const double *d_hat, int32_t k, const double *V,
                            const double *lam, double *part, double *sums, hipStream_t st);
hipError_t launch_trace(int32_t n, const int64_t *diagpos, const double *X, int32_t k, const double *V,
                        const double *lam, double *part, double *sums, hipStream_t st);
hipError_t launch_lowrank(int64_t nnz, int32_t k, const int32_t *srow, const int32_t *col, const double *V,
                          const double *lam, const double *in, double *out, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t st);

// Values on S in A's ordering (perm.hip): row perm[i] of the output holds row
// i of S with columns renamed by perm and sorted; iperm is work (n int32),
// bsum the scan's block sums (n / 1024 + 2 uint64). A perm that is not a
// permutation latches ST_PERM and leaves the rows without a preimage empty.
hipError_t launch_unpermute(int32_t n, const int64_t *rowptr, const int32_t *col, const int32_t *perm,
                            const double *X, int32_t *iperm, unsigned long long *bsum, int64_t *rowptr_out,
                            int32_t *col_out, double *val_out, int32_t *status, hipStream_t st);
// The same with the iperm and scan work in the library's static device
// scratch (no workspace, nothing allocated): n <= kUnpermStaticMaxN
// (hipErrorInvalidValue otherwise). unpermute_scratch_init resolves the
// scratch's address on `device` (current) once per process; later calls
// reuse it. Calls that overlap on one device race on the scratch.
constexpr int32_t kUnpermStaticMaxN = 1 << 21;
hipError_t unpermute_scratch_init(int device);
hipError_t launch_unpermute_static(int device, int32_t n, const int64_t *rowptr, const int32_t *col,
                                   const int32_t *perm, const double *X, int64_t *rowptr_out, int32_t *col_out,
                                   double *val_out, int32_t *status, hipStream_t st);
// inclusive scan of a[1..n] in place (a[0] untouched); bsum: n / 1024 + 2 entries
hipError_t launch_scan_counts(int64_t n, unsigned long long *a, unsigned long long *bsum, hipStream_t st);

struct SpaiParams {
    int32_t n;
    const int64_t *rowptr;  // S
    const int32_t *col;
    const int64_t *mirror;
    const int64_t *A_rowptr;  // A in original order
    const int32_t *A_col;
    const double *A_val;
    const int32_t *perm;
    int32_t *iperm;  // workspace, n
    double *colnorm2;  // workspace, n (||Ah(:, i)||^2 in factor order)
    const double *M;
    double *X;  // workspace, nnzS (column j of M' stored in row j)
    double *R;
    int32_t iters;
    int32_t *status;
    int32_t *list;        // workspace, 2n: columns passed on by the staged kernels
    int32_t *list_count;  // workspace, 2
};

hipError_t launch_spai(const SpaiParams &P, hipStream_t st);
hipError_t launch_symmetrize(int64_t nnz, const int64_t *mirror, const double *X, double *R, hipStream_t st);

struct MlpFeatParams {
    int32_t n;
    int64_t nnz;
    const int32_t *srow;
    const int32_t *col;
    const int64_t *diagpos;
    const int32_t *s2u;  // nnz: u-index of the entry's L value, -1 on the diagonal
    const int64_t *ustart;
    const int8_t *piv;
    const int32_t *level;
    int32_t maxlevel;
    const double *Lu;    // u-space L values (float64)
    const double *Lcsr;  // L values in the input's row order (null: take every L value from Lu)
    const int64_t *Lp;   // n + 1: the input L's row pointers
    const int64_t *rowptr;  // n + 1: S's row pointers
    const double *dinv;  // 3 per block start
    void *node;          // n per-node feature records of 32 bytes (workspace)
    const double *rn;    // 2n: ||L(i, :)||_2, then ||L(:, i)||_2
    const double *Z, *N, *M;
    double eps;
    uint16_t *F;  // nnz x 16 bfloat16
    float *scale; // nnz
    int fuse_mix;  // the correction forms M = Mix(Z, N) itself (M unused) and writes it to Mout if not null
    double *Mout;
};

// NInv and Mix on their own pattern (lower triangle, CSR)
struct NfullParams {
    int32_t n;
    const int64_t *cstart;  // pool columns of L^inv (rows, L^inv, w = D^-1 L^inv; float64)
    const int32_t *clen;
    int32_t *prow;
    double *plinv, *pw;
    int64_t *rpT;             // n + 1: row pointers of the rows of w
    unsigned long long *cur;  // n + 1: fill cursors
    int32_t *colT;            // rows of w: columns and values
    double *valT;
    double *dN;               // n: diagonal of N
    double drop;
    unsigned long long *bsum; // scan block sums
    unsigned long long *cnt;  // count pass: n + 1 (cnt[0] = 0), scanned into row pointers
    const int64_t *rowptr;    // fill pass: row pointers of the result
    int32_t *col;
    double *val;
    int32_t *ovf_list;        // n
    int32_t *ovf_count;       // 1
    int32_t *status;
};

struct MixFullParams {
    int32_t n;
    const int64_t *Nrp;  // N (lower, CSR)
    const int32_t *Ncol;
    const double *Nval;
    const int64_t *srp;  // S
    const int32_t *scol;
    const int64_t *diagpos;
    const double *Z;     // SelInv on S
    const double *zdiag;
    double eps;
    unsigned long long *bsum;
    unsigned long long *cnt;
    const int64_t *rowptr;
    int32_t *col;
    double *val;
};

hipError_t launch_linv(const NinvParams &P, hipStream_t st);  // float64 series columns into the pool
hipError_t launch_nfull_count_w(const NfullParams &P, hipStream_t st);  // pool sort, rows of w sized
hipError_t launch_nfull_fill_w(const NfullParams &P, hipStream_t st);   // rows of w filled, diagonal of N
hipError_t launch_nfull_rows(const NfullParams &P, bool fill, hipStream_t st);
hipError_t launch_mixfull(const MixFullParams &P, bool fill, hipStream_t st);
hipError_t set_nfull_lds_limits();

// Operator applications of the eigen step (y = X x on S, y = Ah x, LDL^T solves)
// Numeric phase of the incomplete factorization on the analysed pattern:
// L values at the offsets of the input L's CSR (Lp), columns read from S's
// CSR (the first Lp[i+1] - Lp[i] entries of row i of S are row i of L),
// Ah(i, j) = A(perm[i], perm[j]) from the caller's CSR of A.
struct IldlParams {
    int32_t n;
    const int64_t *rowptr;  // S
    const int32_t *col;
    const int64_t *Lp;      // input L's row pointers
    const int8_t *piv;
    const int64_t *Ap;
    const int32_t *Aj;
    const double *Av;
    const int32_t *perm, *iperm;
    double *L;               // out: L values (input L's CSR order)
    double *dd, *ds;         // out: D diagonal and D(j+1, j) at the first index of each 2x2 block
    int32_t *status;
};
// one level of blocks; max_entries = largest sum of the L row lengths of a block
hipError_t launch_ildl_level(const BlockMeta *ma, int32_t na, const BlockMeta *mb, int32_t nb, int32_t max_entries,
                             const IldlParams &P, hipStream_t st);
constexpr int kIldlMaxEntries = 3200;  // 20 B of LDS each: 64000 B per block

// Threshold factorization on the device (ildl_threshold.hip): inputs, the
// work arrays of the round schedule and the factor as it grows (scaled).
struct IldlTParams {
    int32_t n;
    const int64_t *Ap;       // A in its own ordering (symmetric pattern)
    const int32_t *Aj;
    const double *Av;
    const int32_t *q;        // Ah = A(q, q)
    int32_t *iq;             // n
    double *scale;           // n: s_i
    double *dpiv;            // n: scaled pivots (after a tiny-pivot replacement)
    int32_t *elim;           // n: round of elimination, INT32_MAX while remaining
    int32_t *watch;          // n: the blocker a column waits for (-1: none yet)
    int32_t *rowcnt;         // n: entries of row i's list
    int32_t *rk;             // n x row_cap: row lists (column m, scaled l_im)
    double *rv;
    int32_t row_cap;
    int64_t *colptr;         // n: kept rows of column m in the pool
    int32_t *collen;
    int32_t *pr;             // pool_cap: rows (sorted per column) and scaled values
    double *pv;
    int64_t pool_cap;
    unsigned long long *pool_top;
    unsigned long long *amax_bits;
    int32_t *list_check, *list_ready, *list_big;  // n each
    int32_t *counts;         // [0] listed, [1] ready, [2] large, [3] eliminated, [4] replaced pivots
    int32_t *status;         // counts + 5
    unsigned long long *bsum;  // n / 1024 + 2: scan sums of the extraction
    double tau, alpha, tiny, repl;
    int32_t pivoting;
    int32_t round;
};
hipError_t ildlt_setup(const IldlTParams &P, hipStream_t st);
hipError_t ildlt_round(const IldlTParams &P, int check_groups, int factor_groups, int big_groups, hipStream_t st);
hipError_t ildlt_extract(const IldlTParams &P, int64_t *Lp, int32_t *Lc, double *Lv, double *dd, double *ds,
                         int8_t *piv, unsigned long long *bsum, hipStream_t st);
hipError_t ildlt_set_limits();

struct LdlSolveParams {
    int32_t n, n_levels;
    const int32_t *lvl_rows;             // host: per-level offsets into the row records
    const SolveRow *rows_fwd, *rows_bwd;  // the rows of each level, forward and backward substitution
    const int32_t *col;
    const double *Ls;  // float64 L(max(i, j), min(i, j)) at every position of S
    const int8_t *piv;
    const double *dinv;
};
// Ls[p] = L(max(i, j), min(i, j)) for entry p = (i, j) of S (Lu[s2u[p]]),
// 0 on the diagonal
hipError_t launch_build_ls(int64_t nnzS, const int32_t *s2u, const double *Lu, double *Ls, hipStream_t st);
hipError_t launch_spmv_s(int32_t n, const int64_t *rowptr, const int32_t *col, const double *X, const double *x,
                         double *y, hipStream_t st);
hipError_t launch_spmv_ahat(int32_t n, const int64_t *Ap, const int32_t *Aj, const double *Av, const int32_t *perm,
                            const int32_t *iperm, const double *x, double *y, hipStream_t st);
hipError_t launch_iperm(int32_t n, const int32_t *perm, int32_t *iperm, int32_t *status, hipStream_t st);
hipError_t launch_za_diag(int32_t n, const int64_t *rowptr, const int32_t *col, const double *Z, const int64_t *Ap,
                          const int32_t *Aj, const double *Av, const int32_t *perm, const int32_t *iperm, double *d,
                          hipStream_t st);
hipError_t launch_ldl_solve(const LdlSolveParams &P, const double *x, double *v, hipStream_t st);
int dot_blocks(int64_t n);
hipError_t launch_dot(int64_t n, const double *a, const double *b, double *part, double *out, hipStream_t st);
hipError_t launch_axpy_ratio(int64_t n, const double *num, const double *den, double sign, const double *x, double *y,
                             hipStream_t st);
hipError_t launch_xpby_ratio(int64_t n, const double *z, const double *num, const double *den, double *p,
                             hipStream_t st);
hipError_t launch_copy_f64(int64_t n, const double *a, double *b, hipStream_t st);
hipError_t launch_qmr_update(int64_t n, double a, double b, const double *q, double *d, double *x, hipStream_t st);
hipError_t launch_sub(int64_t n, const double *b, const double *t, double *r, hipStream_t st);
hipError_t launch_fill_f64(int64_t n, double v, double *a, hipStream_t st);

// Several right-hand sides at once (solve.hip): nv <= kMaxRhs vectors of
// length n stored interleaved (entry i of vector v at x[i nv + v]), except
// launch_spmv_s_m, whose x and y are column-major (vector v at x + v n);
// dot products give nv results; the masked updates touch the vectors whose
// act[v] (sel[v]) is nonzero; coef holds (a_v, b_v) pairs of the QMR update.
constexpr int kMaxRhs = 8;
hipError_t launch_ldl_solve_m(const LdlSolveParams &P, int32_t nv, const double *x, double *V, hipStream_t st);
hipError_t launch_spmv_s_m(int32_t n, int32_t nv, const int64_t *rowptr, const int32_t *col, const double *X,
                           const double *x, double *y, hipStream_t st);
hipError_t launch_spmv_ahat_m(int32_t n, int32_t nv, const int64_t *Ap, const int32_t *Aj, const double *Av,
                              const int32_t *perm, const int32_t *iperm, const double *x, double *y, hipStream_t st);
hipError_t launch_dot_m(int64_t n, int32_t nv, const double *a, const double *b, double *part, double *out,
                        hipStream_t st);
hipError_t launch_axpy_ratio_m(int64_t n, int32_t nv, const double *num, const double *den, const int32_t *act,
                               double sign, const double *X, double *Y, hipStream_t st);
hipError_t launch_xpby_ratio_m(int64_t n, int32_t nv, const double *Z, const double *num, const double *den,
                               const int32_t *act, double *P, hipStream_t st);
hipError_t launch_qmr_update_m(int64_t n, int32_t nv, const double *coef, const int32_t *act, const double *Q,
                               double *D, double *X, hipStream_t st);
// masked per-vector copy (mode 0), difference a - src (1) or zero fill (2)
hipError_t launch_select_m(int64_t n, int32_t nv, const int32_t *sel, int mode, const double *a, const double *src,
                           double *dst, hipStream_t st);
// column-major <-> interleaved (to: column-major src to interleaved dst)
hipError_t launch_interleave(int64_t n, int32_t nv, bool to, const double *src, double *dst, hipStream_t st);

// Lanczos basis kernels (eig.hip): basis columns at V + c n, at most
// kEigMaxBasis columns per call (256 projected vectors and a residual block
// of up to 8)
constexpr int kEigMaxBasis = 264;
int gs_blocks(int64_t n);  // blocks (and partials per column) of launch_gs_dots
hipError_t launch_gs_dots(int64_t n, int32_t ncols, const double *V, const double *w, double *part, double *h,
                          hipStream_t st);
hipError_t launch_gs_update(int64_t n, int32_t ncols, const double *V, const double *h, double *w, hipStream_t st);
hipError_t launch_basis_combine(int64_t n, int32_t m, int32_t p, const double *V, const double *Y, double *out,
                                bool rowmajor, hipStream_t st);
hipError_t launch_scale(int64_t n, double s, double *x, hipStream_t st);

hipError_t launch_node_feats(const MlpFeatParams &P, hipStream_t st);
hipError_t launch_factor_norms(int32_t n, const int64_t *Lp, const double *Lval, const int64_t *ustart,
                              const double *Lu, double *rn, double *Lcopy, hipStream_t st);
hipError_t launch_mlp_features(const MlpFeatParams &P, hipStream_t st);
hipError_t launch_mlp_correct(const MlpFeatParams &P, const void *W, double *out, hipStream_t st);
hipError_t launch_mlp_pack(const float *theta, void *W, hipStream_t st);
hipError_t launch_mlp_forward(const void *W, const uint16_t *F, int64_t rows, float *y, hipStream_t st);
hipError_t launch_mlp_backward(const void *W, const uint16_t *F, const float *dy, int64_t rows, float *grad,
                               hipStream_t st);
hipError_t launch_mlp_loss(const float *y, const float *t, int64_t rows, float *dy, double *loss, hipStream_t st);
hipError_t launch_adam(float *theta, float *m, float *v, const float *g, int32_t np, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st);
hipError_t launch_mlp_apply(int64_t nnz, const double *M, const float *y, const float *s, double *out,
                            hipStream_t st);

}  // namespace asi
