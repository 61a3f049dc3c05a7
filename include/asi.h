/*
 * asi.h — approximate selected inversion from an incomplete LDL^T factor on
 * one AMD MI355X (gfx950). C ABI of libasi.so.
 *
 * Problem (Section 1 and Section 2.1 of the paper): given a symmetric
 * permutation P and factors with P^T A P ~ L D L^T, where L is unit lower
 * triangular with identity diagonal blocks and D is block diagonal with 1x1
 * and 2x2 blocks, compute entries of the inverse on the selected pattern
 *     S = {(i, j) : (L + D + L^T)_ij != 0}.
 * Everything is in the factor ordering (row/column k of the outputs is
 * unknown perm[k] of A).
 *
 * Conventions shared by all calls
 *  - Index types: row pointers int64, column indices int32, 0-based; columns
 *    sorted and unique within each row.
 *  - L is passed as its strictly lower part in CSR (the unit diagonal is
 *    implicit). A 2x2 block {j, j+1} must not store L(j+1, j). If the two
 *    columns of a 2x2 block hold different row sets, S uses their union and
 *    the missing L entries count as zero.
 *  - D is passed as d_diag[n] (D_jj), d_sub[n] (D_{j+1,j} where j starts a
 *    2x2 block, ignored elsewhere) and piv[n] (int8: 0 = 1x1 block, 1 = first
 *    and 2 = second index of a 2x2 block).
 *  - Values on S travel as one float64 array in S's CSR layout (both
 *    triangles, |S| entries) as returned by asi_get_pattern.
 *  - Host pointers are marked _h; every other pointer is device memory on the
 *    handle's device. The caller owns every buffer, including the workspace;
 *    the library never allocates device memory.
 *  - Numeric calls are enqueued asynchronously on the handle's stream and
 *    return after argument checks. Errors found on the device (a singular D
 *    block, a non-finite value, an exhausted pool) are latched in the
 *    workspace and returned by asi_sync.
 *  - A handle is not thread-safe; use one handle per host thread.
 */
#ifndef ASI_H
#define ASI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct asi_handle_s *asi_handle;

typedef enum {
    ASI_OK = 0,
    ASI_E_ARG = 1,         /* bad argument (null pointer, size, range) */
    ASI_E_PATTERN = 2,     /* L or piv violates the conventions above */
    ASI_E_SINGULAR_D = 3,  /* a D block is singular (device-detected) */
    ASI_E_NONFINITE = 4,   /* a non-finite value was produced (device-detected) */
    ASI_E_STATE = 5,       /* call order violated (e.g. numeric call before analyze) */
    ASI_E_WORKSPACE = 6,   /* workspace too small or a device pool exhausted */
    ASI_E_HIP = 7,         /* a HIP runtime call failed */
    ASI_E_UNSUPPORTED = 8, /* the pattern exceeds a documented kernel limit */
    ASI_E_TIMEOUT = 9      /* a dataflow wait exceeded its poll limit (results invalid) */
} asi_status;

typedef enum { ASI_FP64 = 0, ASI_MIXED = 1 } asi_precision;

/* Summary of the symbolic analysis (filled by asi_get_info). */
typedef struct {
    int32_t n;
    int32_t n_blocks;        /* D blocks */
    int32_t n_levels;        /* levels of the SelInv dependency DAG */
    int32_t max_cols;        /* max |R_J| over blocks */
    int64_t nnz_L;           /* stored L entries (input) */
    int64_t nnz_S;           /* |S|, both triangles */
    int64_t gather_pairs;    /* sum over J of the Z entries scanned by the sweep */
    int64_t gather_hits;     /* sum over J of the pairs (r, l) in R_J x R_J found in S */
    size_t workspace_min;    /* bytes without the NInv pool */
    size_t workspace_default;/* bytes with a default-sized NInv pool */
} asi_info;

/* Create a handle bound to HIP device `device` and stream `stream` (a
 * hipStream_t; NULL selects the null stream). device = -1 creates a
 * host-only handle that can run asi_analyze and asi_get_info but no device
 * call (those return ASI_E_STATE). */
asi_status asi_create(asi_handle *h, int device, void *stream);
asi_status asi_destroy(asi_handle h);
/* Rebind the stream used by subsequent numeric calls. */
asi_status asi_set_stream(asi_handle h, void *stream);
/* Message of the last failing call on this handle (valid until the next call). */
const char *asi_last_error(asi_handle h);

/*
 * Symbolic analysis of the pattern of L (Section 1: S is induced by the
 * pattern of L + D + L^T; Section 2.1: inverse information flows from the
 * last block to the first, so block J can run once every block holding a
 * row of R_J is done). Host pointers. Builds S, the dependency levels and
 * the index maps; reports |S| and the workspace size.
 * Errors: ASI_E_ARG, ASI_E_PATTERN, ASI_E_UNSUPPORTED (|R_J| above 2048).
 */
asi_status asi_analyze(asi_handle h, int32_t n, const int64_t *L_rowptr_h, const int32_t *L_col_h,
                       const int8_t *piv_h, int64_t *nnzS_out, size_t *workspace_bytes_out);

/* Hand the library a device workspace of `bytes` (at least workspace_min;
 * whatever exceeds it becomes the NInv pool) and upload the analysis into it
 * (synchronous). The workspace must stay alive while the handle uses it. */
asi_status asi_set_workspace(asi_handle h, void *dev_ws, size_t bytes);

asi_status asi_get_info(asi_handle h, asi_info *info);

/* Copy S's CSR pattern (device buffers of n+1 and |S| entries) and, if
 * level_d is not NULL, each unknown's DAG level (n entries). */
asi_status asi_get_pattern(asi_handle h, int64_t *S_rowptr_d, int32_t *S_col_d, int32_t *level_d);

/*
 * The factor values of one step (Section 1: L and D of P^T A P ~ L D L^T):
 * L_val in the order of the L_col array given to asi_analyze, d_diag (n),
 * d_sub (n, the (j+1, j) entry at the first column of each 2x2 block), all
 * device float64. The library inverts the D blocks and gathers L into its
 * column layout once (the first preconditioner solve after a load also
 * copies L's values into S's order); asi_selinv, asi_ninv,
 * asi_mlp_features and asi_mlp_correct then take NULL for all three factor
 * pointers to use it. A call that passes the pointers loads the factor it
 * is given the same way (replacing the loaded one), so later calls may pass
 * NULL for it. The caller may reuse its buffers after the stream has passed
 * this call (or that call).
 */
asi_status asi_load_factor(asi_handle h, const double *L_val, const double *d_diag, const double *d_sub);

/*
 * SelInv (Section 2.1, recursion for G21 and G11): for every block J from
 * the last to the first, Z(R_J, J) = -Zhat(R_J, R_J) L(R_J, J) and
 * Z(J, J) = D_J^-1 - L(R_J, J)^T Z(R_J, J), where Zhat is Z restricted to S
 * (entries outside S are discarded). L_val: values in the order of the
 * L_col array given to asi_analyze (or L_val, d_diag and d_sub all NULL:
 * the factor of asi_load_factor; ASI_E_STATE if none is loaded).
 * Z_S: |S| float64 outputs.
 * ASI_MIXED keeps the off-diagonal working values (their storage, the
 * gathers and the products) in float32 and sums the products of each block
 * in float64, with the D-block inverses and Z(J, J) in float64.
 */
asi_status asi_selinv(asi_handle h, const double *L_val, const double *d_diag, const double *d_sub,
                      asi_precision prec, double *Z_S);

/*
 * How asi_selinv schedules the blocks. ASI_SWEEP_LEVELS launches one kernel
 * per level of the dependency DAG. ASI_SWEEP_DATAFLOW runs the whole sweep as
 * one cooperative launch in which each block waits only for the blocks it
 * depends on (requires every |R_J| <= 128 and cooperative-launch support;
 * otherwise asi_selinv returns ASI_E_UNSUPPORTED). ASI_SWEEP_AUTO (default)
 * currently selects the level schedule, the faster of the two on MI355X for
 * the tested patterns.
 */
typedef enum { ASI_SWEEP_AUTO = 0, ASI_SWEEP_LEVELS = 1, ASI_SWEEP_DATAFLOW = 2 } asi_sweep;
asi_status asi_set_sweep(asi_handle h, asi_sweep mode);

/*
 * The level launches asi_selinv makes with ASI_SWEEP_LEVELS (Section 2.1:
 * one launch per level of the dependency DAG), by kernel variant. Each level
 * runs its blocks with |R_J| <= 128 in one launch of a wavefront-per-block
 * variant (levels of more than 3,072 blocks: ASI_SV_SMALL, or ASI_SV_SPLIT
 * when the level has blocks of more than 512 hits and at most 16,384 blocks)
 * or a workgroup-per-block variant (levels of 1,537-3,072 / 769-1,536 /
 * at most 768 blocks: 128 / 256 / 512 threads per block), and its blocks
 * with |R_J| > 128 in one launch of 1,024 threads per block (at most 1,024
 * such blocks) or 256. counts_h: host array of ASI_SV_COUNT int64, the
 * number of launches of each variant per sweep. Host-only; needs
 * asi_analyze. Errors: ASI_E_ARG, ASI_E_STATE.
 */
/*
 * Schedule check (debug): with on != 0, every SelInv sweep of the handle
 * first fills its working copy of Z (the column layout of the strictly lower
 * part, and the diagonal) with NaN. Section 2.1 computes block J from entries
 * of Zhat that earlier blocks have already written; an entry read before its
 * block writes it then turns the result non-finite instead of silently using
 * a stale value of an earlier call. Costs one extra pass over that working
 * copy per sweep (4 or 8 bytes per entry of L plus 8 per unknown); results
 * are otherwise unchanged. Default off. Errors: ASI_E_ARG (null handle).
 */
asi_status asi_set_sentinel(asi_handle h, int on);

typedef enum {
    ASI_SV_SMALL = 0, ASI_SV_SPLIT = 1, ASI_SV_GROUP128 = 2, ASI_SV_GROUP256 = 3,
    ASI_SV_GROUP512 = 4, ASI_SV_BIG256 = 5, ASI_SV_BIG1024 = 6, ASI_SV_COUNT = 7
} asi_sweep_variant;
asi_status asi_sweep_plan(asi_handle h, int64_t *counts_h);

/*
 * NInv (Section 2.2): L^inv = sum_{m=0}^{p} T_m with T_0 = I and
 * T_m = drop_delta(E T_{m-1}), E = I - L, dropping |t| < delta in each new
 * term; N = (L^inv)^T D^-1 L^inv evaluated on S. Columns of L^inv are kept in
 * the workspace pool (ASI_E_WORKSPACE at asi_sync if it runs out). Factor
 * pointers as for asi_selinv.
 */
asi_status asi_ninv(asi_handle h, const double *L_val, const double *d_diag, const double *d_sub,
                    int32_t p, double delta, asi_precision prec, double *N_S);

/*
 * NInv on its own pattern (Section 2.2): N = (L^inv)^T D^-1 L^inv, L^inv the
 * truncated series of asi_ninv (p terms, entry drop delta), evaluated at
 * every (i, j) whose columns of L^inv meet a common D block, with the
 * off-diagonal entries |N_ij| < drop sqrt(|N_ii N_jj|) removed (the drop of
 * the product, Section 2.2; read relative to the diagonal so that it does not
 * depend on the scaling of A). The result is the lower triangle (diagonal
 * included) in CSR with sorted columns: rowptr (n + 1 int64), col (int32)
 * and val (float64), device arrays of the caller; col and val hold cap
 * entries. The call is synchronous: it sizes the result (*nnz, host), and if
 * it exceeds cap writes only rowptr and returns ASI_E_WORKSPACE, so a caller
 * may call with cap = 0 first. The L^inv columns and, after them, the rows of
 * D^-1 L^inv use the workspace's NInv pool, which must hold the series'
 * entries twice over (ASI_E_WORKSPACE otherwise). Float64; repeatable bit for bit unless a
 * series column needed the workgroup kernel of asi_ninv (then to rounding).
 * Factor pointers as for asi_selinv (all NULL: the loaded factor).
 */
asi_status asi_ninv_full(asi_handle h, const double *L_val, const double *d_diag, const double *d_sub, int32_t p,
                         double delta, double drop, int64_t cap, int64_t *rowptr, int32_t *col, double *val,
                         int64_t *nnz);

/*
 * Mix on NInv's own pattern (Section 2.3: Mix keeps the structure of NInv
 * and takes SelInv's value on S_eps = {(i, j) in S : |Z_ij| > eps
 * sqrt(|Z_ii Z_jj|)}): the pattern of N joined with S_eps, Z_ij on S_eps and
 * N_ij elsewhere. Z_S: SelInv on S (|S| float64); N_rowptr, N_col, N_val: the
 * lower triangle of N as returned by asi_ninv_full. Output, cap and *nnz as
 * for asi_ninv_full (lower triangle, CSR, synchronous).
 */
asi_status asi_mix_full(asi_handle h, const double *Z_S, const int64_t *N_rowptr, const int32_t *N_col,
                        const double *N_val, double eps, int64_t cap, int64_t *rowptr, int32_t *col, double *val,
                        int64_t *nnz);

/*
 * SelInv and NInv of the same factor in one call (together they are the
 * inputs of Mix, Section 2.3): NInv runs on a second stream of the handle
 * (created on first use, default priority) concurrently with the SelInv
 * sweep on the handle's stream, and the handle's stream waits for it before
 * its next work, so later calls and asi_sync see both results. Given the
 * factor arrays, the call makes the column layouts the sweep reads on the
 * handle's stream and the row and column norms of L and its row-order copy
 * (read only by asi_mlp_features / asi_mlp_correct) on the second stream
 * after NInv. Arguments and results as for asi_selinv and asi_ninv. With
 * ASI_SWEEP_DATAFLOW the two run one after the other (that sweep needs every
 * workgroup resident).
 */
asi_status asi_selinv_ninv(asi_handle h, const double *L_val, const double *d_diag, const double *d_sub,
                           int32_t p, double delta, asi_precision prec, double *Z_S, double *N_S);

/*
 * Mix (Section 2.3): M_ij = Z_ij where |Z_ij| > eps sqrt(|Z_ii Z_jj|), else
 * N_ij. M_S may alias Z_S or N_S.
 */
asi_status asi_mix(asi_handle h, const double *Z_S, const double *N_S, double eps, double *M_S);

/*
 * SPAI refinement (Section 2.4): for each column j, cg_iters steps of
 * Jacobi-preconditioned CG on the normal equations of min ||Ah m - e_j||_2
 * with supp(m) in column j of S, starting from M(:, j); Ah = P^T A P from the
 * original-order CSR of A (both triangles) and perm; then R = (M' + M'^T)/2.
 * Column j of S may hold at most 512 entries.
 */
asi_status asi_spai(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                    const int32_t *perm, const double *M_S, int32_t cg_iters, double *R_S);

/*
 * Rank-k correction on S (Section 2.5, corrected inverse; Section 2.6,
 * corrected diagonal): out_ij = in_ij + sum_m lambda_m V_im V_jm with V an
 * n x k row-major float64 matrix in the factor ordering. 1 <= k <= 64.
 * out_S may alias in_S.
 */
asi_status asi_lowrank(asi_handle h, int32_t k, const double *V, const double *lambda,
                       const double *in_S, double *out_S);

/*
 * Learned per-entry correction of the Mix result (not part of the paper: a
 * 16 -> 64 -> 64 -> 1 ReLU network with bfloat16 weights and activations and
 * float32 accumulation, M'_ij = M_ij + y_ij s_ij, s_ij = sqrt(|M_ii M_jj|)).
 *
 * asi_mlp_features: the 16 features of every entry of S from Z (SelInv), N
 * (NInv), M (Mix with threshold eps), L and D: F is |S| x 16 bfloat16 (raw
 * 16-bit words, row-major), scale receives s_ij (float32, |S|).
 * Feature order: M/s, (Z-N)/s, [Mix took Z], [i == j], log(|D^-1_ii| + 1e-30),
 * log(|D^-1_jj| + 1e-30), log row norms of L at i and j, log column norms of L at i and
 * j, |L(max, min)|, log(1 + |N|/s), log(1 + |Z|/s), level(i)/max level,
 * level(j)/max level, log(1 + |R| of column min(i, j)).
 * The learned-correction calls that take an analysis need |S| < 2^31
 * (ASI_E_UNSUPPORTED otherwise).
 */
#define ASI_MLP_FEATURES 16
#define ASI_MLP_PARAMS 5313        /* float32 masters: W1[64][16], b1, W2[64][64], b2, w3, b3 */
#define ASI_MLP_PACKED_BYTES 12944 /* bfloat16 W1 (padded to [64][32]), W2, w3; float32 b1, b2, b3 */
asi_status asi_mlp_features(asi_handle h, const double *Z_S, const double *N_S, const double *M_S, double eps,
                            const double *L_val, const double *d_diag, const double *d_sub, uint16_t *F,
                            float *scale);
/* The following calls need a device handle but no analysis. */
/* Round the float32 masters (ASI_MLP_PARAMS) into the packed inference weights. */
asi_status asi_mlp_pack(asi_handle h, const float *theta, void *packed);
/* y[r] for rows feature rows (bfloat16 MFMA, float32 accumulation). */
asi_status asi_mlp_forward(asi_handle h, const void *packed, const uint16_t *F, int64_t rows, float *y);
/* grad += d(sum_r dy[r] y[r]) / d theta for the packed weights' network
 * (bfloat16 roundings treated as identity); float32, ASI_MLP_PARAMS entries.
 * The products run on bfloat16 MFMA with float32 sums: activations, features
 * and weights are bfloat16 already, and each float32 back-propagated value
 * enters as a bfloat16 head and tail (relative 2^-17). grad receives one
 * atomic addition per parameter and workgroup, so the summation order (and
 * the last bits) can vary between runs. */
asi_status asi_mlp_backward(asi_handle h, const void *packed, const uint16_t *F, const float *dy, int64_t rows,
                            float *grad);
/* Mean squared error: dy[r] = 2 (y[r] - t[r]) / rows and *loss += mean((y - t)^2)
 * (loss: one device float64). */
asi_status asi_mlp_loss(asi_handle h, const float *y, const float *t, int64_t rows, float *dy, double *loss);
/* One Adam step on the masters (step count t >= 1, bias-corrected). */
asi_status asi_mlp_adam(asi_handle h, float *theta, float *m, float *v, const float *grad, float lr, float beta1,
                        float beta2, float eps, int64_t t);
/* out = M + y * scale on S (out may alias M). */
asi_status asi_mlp_apply(asi_handle h, const double *M_S, const float *y, const float *scale, double *out_S);
/*
 * The whole correction in one pass: features of every entry of S (as
 * asi_mlp_features), the network (as asi_mlp_forward) and out = M + y s (as
 * asi_mlp_apply), with nothing but out written to memory; the result equals
 * that of the three calls bit for bit. W: packed weights (asi_mlp_pack).
 * Arguments as for asi_mlp_features; out_S: |S| float64, device, may alias
 * M_S. Needs an analysis.
 */
asi_status asi_mlp_correct(asi_handle h, const void *W, const double *Z_S, const double *N_S, const double *M_S,
                           double eps, const double *L_val, const double *d_diag, const double *d_sub,
                           double *out_S);
/*
 * asi_mlp_correct_mix: Mix (Section 2.3, as asi_mix with eps) and the
 * correction in one pass: M = Mix(Z, N) is formed entry by entry (its test
 * is the feature the network already reads) and written to M_S when M_S is
 * not NULL, out = M + y s as asi_mlp_correct; both equal asi_mix followed by
 * asi_mlp_correct bit for bit, without the separate pass over S. Arguments
 * as for asi_mlp_correct; M_S and out_S must be different arrays (either may
 * alias Z_S or N_S).
 */
asi_status asi_mlp_correct_mix(asi_handle h, const void *W, const double *Z_S, const double *N_S, double eps,
                               const double *L_val, const double *d_diag, const double *d_sub, double *M_S,
                               double *out_S);

/* Diagonal of a matrix on S: d[i] = X(i, i). */
asi_status asi_diag(asi_handle h, const double *X_S, double *d);

/*
 * Relative diagonal 1-norm error (Section 2.6) of a diagonal with an optional
 * rank-k term (Section 2.6, corrected diagonal), the quantity of the
 * acceptance test of Algorithm 1:
 *   sums[0] = sum_i |d_ref[i] - d_hat[i] - sum_{m<k} lambda_m V[i][m]^2|
 *   sums[1] = sum_i |d_ref[i]|
 * so err_1 = sums[0] / sums[1]. d_ref, d_hat: n float64 (factor ordering);
 * V: n x k row-major float64, lambda: k float64, both unused when k = 0;
 * 0 <= k <= 64. sums: 2 float64, device. Every pointer is a device pointer;
 * the call is asynchronous on the handle's stream. The summation order is
 * fixed (a per-block stage, then one block), so repeated calls give the same
 * bits. A mode can be left out by passing lambda_m = 0.
 */
asi_status asi_diag_err1(asi_handle h, const double *d_ref, const double *d_hat, int32_t k, const double *V,
                         const double *lambda, double *sums);

/*
 * Trace and diagonal 1-norm of an approximate inverse on S with an optional
 * rank-k term (Section 3.5, covariance and uncertainty quantification: the
 * trace of the covariance A^-1 is approximated by the sum of the diagonal of
 * the approximation, corrected by V_k Lambda_k V_k^T when a correction is
 * accepted):
 *   sums[0] = sum_i c_i,  sums[1] = sum_i |c_i|,
 *   c_i = X(i, i) + sum_{m<k} lambda_m V[i][m]^2.
 * X_S: |S| float64 on S; V: n x k row-major float64, lambda: k float64, both
 * unused when k = 0; 0 <= k <= 64. sums: 2 float64. Every pointer is a
 * device pointer; asynchronous on the handle's stream. The summation order is
 * fixed, so repeated calls give the same bits. Needs an analysis.
 */
asi_status asi_trace(asi_handle h, const double *X_S, int32_t k, const double *V, const double *lambda,
                     double *sums);

/*
 * Operator applications of the eigen step of the spectral correction
 * (Section 2.5: E x = A^-1 x - X x is applied matrix-free, A^-1 x by a Krylov
 * method preconditioned with the incomplete block factorization; conjugate
 * gradients in the positive definite case). All vectors are float64 device
 * arrays of length n in the factor ordering; asynchronous on the handle's
 * stream unless stated.
 *
 * asi_spmv: y = X x for X on S (|S| values, S's CSR order). x and y must
 * not alias.
 */
asi_status asi_spmv(asi_handle h, const double *X_S, const double *x, double *y);

/*
 * asi_ildl_numeric: the numeric phase of the incomplete factorization
 * Ah = P^T A P ~ L D L^T (Section 2.1) on the analysed pattern of L and its
 * pivot partition piv (asi_analyze), on the device. The threshold
 * factorization decides which pivots (1x1 or 2x2) and which entries of L are
 * kept; given those decisions, L and D follow from the Crout recurrence over
 * the kept entries, block B = {j} or {j, j+1} in order:
 *     w(i, B) = Ah(i, B) - sum_{C < B} L(i, C) D_C L(B, C)^T,
 *     D_B = w(B, B),   L(i, B) = w(i, B) D_B^-1 for every kept (i, B),
 * so that (L D L^T)_ij = Ah_ij on every kept entry and every D block. Run
 * again with new values of A on the same pattern, or with the pattern and
 * pivots of a host threshold factorization, it reproduces that factor up to
 * rounding (no pivot perturbation is applied: a zero D block is an error).
 * A: the caller's CSR in its own ordering (int64 row pointers, int32
 * columns, unique within a row, float64 values), perm: n int32 with
 * Ah(i, j) = A(perm[i], perm[j]); entries of Ah outside the kept pattern are
 * ignored. Outputs (device, caller-owned): L_val in the layout of the L_col
 * array given to asi_analyze, d_diag[n], d_sub[n] (D(j+1, j) at the first
 * index of each 2x2 block, 0 elsewhere), ready for asi_load_factor (this call
 * loads nothing). Blocks run level by level of the SelInv schedule, last
 * level first. Errors: ASI_E_ARG; ASI_E_UNSUPPORTED when a row of L holds
 * only one column of a 2x2 block or a block's rows of L hold more than 3200
 * entries together (checked on the first call after asi_analyze); at
 * asi_sync, ASI_E_SINGULAR_D (a zero 1x1 pivot or a singular 2x2 block),
 * ASI_E_NONFINITE, or ASI_E_ARG for an invalid perm. Asynchronous on the
 * handle's stream.
 */
asi_status asi_ildl_numeric(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                            const int32_t *perm, double *L_val, double *d_diag, double *d_sub);

/*
 * asi_ldl_solve: y = (L D L^T)^-1 x with the factor of asi_load_factor
 * (ASI_E_STATE if none is loaded): forward substitution with the unit lower
 * L, the D-block inverses, backward substitution with L^T, level by level of
 * the SelInv schedule. y may alias x. Needs |S| < 2^31.
 */
asi_status asi_ldl_solve(asi_handle h, const double *x, double *y);

/*
 * asi_pcg: x = Ah^-1 b by conjugate gradients on Ah = P^T A P (A: the
 * caller's CSR in its own ordering, int64 row pointers, int32 columns,
 * float64 values; perm: n int32 with Ah(i, j) = A(perm[i], perm[j]))
 * preconditioned with the loaded factor (L D L^T)^-1, from x = 0, until
 * ||b - Ah x||_2 <= tol ||b||_2 or maxit steps. For symmetric positive
 * definite A and a positive D. Synchronous (reads one residual norm per
 * step); *iters and *relres (host, nullable) receive the steps taken and the
 * final relative residual. ASI_E_NONFINITE on a breakdown. Uses the
 * workspace's CG vectors, so calls on one handle must not overlap.
 */
asi_status asi_pcg(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                   const int32_t *perm, const double *b, double *x, double tol, int32_t maxit, int32_t *iters,
                   double *relres);

/*
 * asi_sqmr: x = Ah^-1 b by the simplified QMR method with the symmetric
 * preconditioner (L D L^T)^-1 of the loaded factor (Section 2.5: the method
 * the paper uses for the indefinite case), from x = 0. Arguments, outputs,
 * synchrony and workspace use as for asi_pcg. The quasi-residual bound
 * sqrt(k + 1) tau_k decides when the true residual ||b - Ah x||_2 is
 * computed; the call stops when that is <= tol ||b||_2 or after maxit
 * steps (*relres is then the last true residual computed). When that true
 * residual is still above tol ||b||_2 (the recursion's residual has drifted
 * from it, as happens near the attainable accuracy of an ill-conditioned
 * Ah) the method restarts from the iterate on the true residual, and again
 * whenever the same happens, within the maxit steps. A near-breakdown (a
 * vanishing rho or sigma, or a quasi-residual that is no longer finite)
 * restarts it from the last iterate too; ASI_E_NONFINITE after 8 such
 * restarts.
 */
asi_status asi_sqmr(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                    const int32_t *perm, const double *b, double *x, double tol, int32_t maxit, int32_t *iters,
                    double *relres);

/*
 * Several right-hand sides at once (the block form of the solves above, for
 * the block eigen step): nrhs systems Ah x_v = b_v, 1 <= nrhs <= 8, B and X
 * n x nrhs column-major float64 device arrays (vector v at B + v n; X must
 * not overlap B or work), each vector with its own scalars, stopping test
 * (as for asi_pcg / asi_sqmr, per vector, including SQMR's restarts) and
 * outputs: iters[v], relres[v] (host, nrhs each). One preconditioner sweep
 * over the level schedule serves the whole block. work: device buffer of at
 * least asi_block_solve_work_bytes(n, nrhs) bytes, 256-byte aligned, owned
 * by the caller (the calls leave the handle's CG vectors alone).
 * Synchronous. Errors as for asi_pcg / asi_sqmr, and ASI_E_WORKSPACE.
 */
asi_status asi_block_solve_work_bytes(int32_t n, int32_t nrhs, size_t *bytes);
asi_status asi_pcg_block(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                         const int32_t *perm, int32_t nrhs, const double *B, double *X, double tol, int32_t maxit,
                         void *work, size_t work_bytes, int32_t *iters, double *relres);
asi_status asi_sqmr_block(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                          const int32_t *perm, int32_t nrhs, const double *B, double *X, double tol, int32_t maxit,
                          void *work, size_t work_bytes, int32_t *iters, double *relres);

/*
 * The eigen step itself (Section 2.5, Algorithm 1: the k eigenpairs of
 * largest |lambda| of the symmetric inverse-error operator E = A^-1 - X,
 * found matrix-free with A^-1 applied by a preconditioned Krylov solve).
 *
 * asi_eigs_error: thick-restart block Lanczos on E in the factor ordering,
 * block size b = block (b = 1: plain Lanczos). Each step applies E to b
 * basis vectors at once: a block Krylov solve on Ah = P^T A P with the
 * loaded factor as preconditioner (method 0: block PCG, positive definite
 * A; method 1: block SQMR, indefinite A; solve_tol and solve_maxit per
 * vector as for asi_pcg) minus X V on S; basis vector c + b is the image of
 * basis vector c, orthogonalised against every earlier basis vector by two
 * passes of classical Gram-Schmidt and normalised. With m + b basis
 * vectors the host diagonalises the m x m projection T = V^T E V
 * (asi_dense_symeig) and estimates the residual of each Ritz pair
 * (theta, y) as ||C y|| (C: the b x m coupling of the last b basis vectors
 * to the first m); the call stops when the k Ritz pairs of largest |theta|
 * all satisfy ||E u - theta u|| <= tol |theta| or after max_restarts
 * restarts, else it keeps min(k + (m - k) / 2, m - b) Ritz vectors plus the
 * last b basis vectors and expands again. For b = 1 a basis vector of norm
 * <= 1e-13 ||T||_max (an invariant subspace) ends the iteration with exact
 * Ritz pairs (ASI_E_NONFINITE if fewer than k); for b > 1 it is an error
 * (ASI_E_NONFINITE: the block became linearly dependent).
 *
 * A_rowptr, A_col, A_val, perm: as for asi_pcg (device). X_S: |S| float64
 * (device). v0: n x b column-major float64 starting block, linearly
 * independent columns (device; not modified). 1 <= k <= 64; 1 <= b <= 8;
 * k + b + 1 <= m <= 256, m + b <= n; tol > 0; max_restarts >= 0.
 * work: device buffer of at least asi_eigs_work_bytes(n, m, b) bytes,
 * 256-byte aligned, owned by the caller, contents undefined on return.
 * Outputs: lambda (host, k float64) in decreasing |lambda| (ties by index);
 * V (device, n x k row-major float64, orthonormal columns, must not overlap
 * work); resid (host, k float64, nullable): estimated relative residuals
 * ||E u - theta u|| / |theta|; stats (host, 5 float64, nullable): operator
 * applications (vectors), block Krylov iterations (each one preconditioner
 * sweep over a block), restarts, Ritz pairs converged among the k, largest
 * relative residual of a solve. Synchronous; the result is repeatable bit
 * for bit. Errors: ASI_E_ARG, ASI_E_STATE (no factor), ASI_E_WORKSPACE (work
 * too small), the errors of the Krylov solves.
 */
asi_status asi_eigs_work_bytes(int32_t n, int32_t m, int32_t block, size_t *bytes);
asi_status asi_eigs_error(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                          const int32_t *perm, const double *X_S, const double *v0, int32_t k, int32_t m,
                          int32_t block, double tol, int32_t max_restarts, int32_t method, double solve_tol,
                          int32_t solve_maxit, void *work, size_t work_bytes, double *lambda, double *V,
                          double *resid, double *stats);

/*
 * asi_dense_symeig: all eigenpairs of a small dense symmetric matrix on the
 * host (the projected problem of the Lanczos iteration above) by the cyclic
 * Jacobi method with Rutishauser's rotation formulas: rotations annihilate
 * the off-diagonal entries in row order until the off-diagonal Frobenius
 * norm is <= 1e-15 times the matrix's (or no rotation changes it).
 * T: m x m row-major float64 (host; symmetrised as (T + T^T) / 2; not
 * modified); theta: m float64 in ascending order (ties by index of the
 * diagonal position); Y: m x m row-major float64 whose column t is the unit
 * eigenvector of theta[t]. 1 <= m <= 4096. Needs no handle. Errors:
 * ASI_E_ARG, ASI_E_NONFINITE (non-finite entries, or no convergence in 100
 * sweeps).
 */
asi_status asi_dense_symeig(int32_t m, const double *T, double *theta, double *Y);

/*
 * Diagnostic (Section 2.1: where the pattern is closed SelInv equals A^-1 on
 * S, so Z Ah = I on the diagonal): d[i] = (Z Ah)_ii = sum_k Z_ik Ah_ki over
 * the k in row i of both S and Ah = P^T A P (A: the caller's CSR in its own
 * ordering, symmetric; perm as for asi_pcg). Z_S: |S| float64; d: n
 * float64 (factor ordering). Device pointers, asynchronous.
 */
asi_status asi_za_diag(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                       const int32_t *perm, const double *Z_S, double *d);

/*
 * asi_ildl_threshold: the whole threshold incomplete factorization on the
 * device, pivot and drop decisions included (Section 2.1 takes the factor
 * P^T A P ~ L D L^T as given; the paper's own factorization is sequential
 * and a parallel one is named as future work in its concluding remarks).
 * It computes, bit for bit, the right-looking threshold ILDL of the
 * scaled matrix Ah = S A(q, q) S (s_i = 1/sqrt(max_j |a_ij|)) with 1x1
 * pivots in the given order: the Schur column of pivot p is summed over the
 * earlier pivots in increasing order, a pivot below 1e-14 max|Ah| is replaced
 * by +-1e-8 max|Ah| and counted, l_ip = w(i)/d_p is kept when |l_ip| >= tau,
 * and L <- S^-1 L S, D <- S^-1 D S^-1 at the end. Pivots are taken as they
 * come: with pivoting != 0 the Bunch-Kaufman 1x1 test (alpha =
 * (1 + sqrt 17)/8) is applied to every pivot and a pivot that fails it (a
 * swap or a 2x2 block would be needed) ends the call with
 * ASI_E_UNSUPPORTED; with pivoting = 0 no test is made. Columns are
 * eliminated in rounds: every column with no uneliminated smaller neighbour
 * in the current Schur graph at once.
 * Inputs (device): A in its own ordering, CSR with int64 row pointers and
 * int32 columns, structurally symmetric (every stored (i, j) has a stored
 * (j, i)), unique columns per row; q: n int32, the ordering (Ah = A(q, q)),
 * a permutation. Work: a caller-owned device buffer of at least
 * asi_ildl_threshold_work_bytes(n, row_cap, pool_cap) bytes, 256-byte
 * aligned, that must stay alive until asi_ildl_threshold_extract has run:
 * row_cap bounds the entries of one row of L, pool_cap the entries of L.
 * Synchronous (one host read per round). Outputs (host): *nnzL_h = nnz(L);
 * stats_h (nullable, 2 int64): rounds, replaced pivots. Errors: ASI_E_ARG
 * (null pointer, q not a permutation, a column out of range),
 * ASI_E_WORKSPACE (work too small, or a row of L above row_cap or L above
 * pool_cap: retry with larger ones), ASI_E_UNSUPPORTED (a pivot that needs
 * Bunch-Kaufman pivoting, a Schur column above 3,072 entries, a row of L
 * above 2,048 entries).
 * asi_ildl_threshold_extract writes the factor of the last successful call
 * on this handle from its work buffer, in the layout asi_analyze and
 * asi_load_factor take: L_rowptr (n + 1 int64), L_col (nnzL int32, sorted
 * per row), L_val (nnzL float64), d_diag, d_sub (n float64; d_sub all 0) and
 * piv (n int8, all 0), device, caller-owned; the ordering is q.
 * Asynchronous.
 */
asi_status asi_ildl_threshold_work_bytes(int32_t n, int32_t row_cap, int64_t pool_cap, size_t *bytes);
asi_status asi_ildl_threshold(asi_handle h, int32_t n, const int64_t *A_rowptr, const int32_t *A_col,
                              const double *A_val, const int32_t *q, double tau, int32_t pivoting, int32_t row_cap,
                              int64_t pool_cap, void *work, size_t work_bytes, int64_t *nnzL_h, int64_t *stats_h);
asi_status asi_ildl_threshold_extract(asi_handle h, int64_t *L_rowptr, int32_t *L_col, double *L_val,
                                      double *d_diag, double *d_sub, int8_t *piv);

/*
 * Values on S in A's own ordering. Section 1 asks for entries of A^-1 and
 * Section 2.1 factors the permuted matrix P^T A P, so entry (i, j) of a
 * result in the factor ordering approximates (A^-1)(perm[i], perm[j]).
 * X_S: |S| float64 values in S's CSR layout (factor ordering); perm: n int32,
 * the factor ordering (P^T A P = A[perm][:, perm], as returned with the
 * factor). Outputs, the same |S| entries as a CSR matrix in A's ordering:
 * rowptr_out (n + 1 int64), col_out (|S| int32, sorted and unique within
 * each row), val_out (|S| float64); row perm[i] holds row i of S with every
 * column j renamed perm[j]. The values are copied, not recomputed. All
 * device pointers, owned by the caller; the outputs must not overlap X_S.
 * Asynchronous on the handle's stream (uses the workspace's inverse
 * permutation and scan areas, so calls on one handle must not overlap).
 * Errors: ASI_E_ARG (null pointer, overlap), ASI_E_STATE; at asi_sync,
 * ASI_E_ARG if perm is not a permutation of 0..n-1 (rows that no index maps
 * to are then left empty).
 */
asi_status asi_unpermute(asi_handle h, const int32_t *perm, const double *X_S, int64_t *rowptr_out,
                         int32_t *col_out, double *val_out);

/*
 * asi_unpermute for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments, outputs and errors, but its work arrays
 * (the inverse permutation and the row-pointer scan's block sums) live in a
 * static device array of the library (about 8 MB per device, held until the
 * process ends) instead of the handle's workspace, and the call allocates
 * nothing. n <= 2,097,152 (ASI_E_ARG with a message otherwise). Every call on
 * one device shares that array: calls that overlap on a device (two streams
 * or two handles) race and must not be issued. The array keeps the previous
 * call's contents; nothing in it needs to start at zero.
 */
asi_status asi_unpermute_noalloc(asi_handle h, const int32_t *perm, const double *X_S, int64_t *rowptr_out,
                                 int32_t *col_out, double *val_out);

/*
 * Input check of host arrays (Section 1: the method takes a symmetric A and
 * its permuted factorization), for debugging: perm (nullable) is a
 * permutation of 0..n-1; A is a valid CSR (A_rowptr[0] = 0, nondecreasing,
 * columns sorted, unique and in range, values finite) and symmetric in
 * pattern and values (|a_ij - a_ji| <= tol max(|a_ij|, |a_ji|); tol = 0 asks
 * for exact symmetry). ASI_E_PATTERN or ASI_E_NONFINITE with a message
 * (asi_last_error) otherwise. Host pointers; synchronous; needs only a
 * handle.
 */
asi_status asi_check_matrix(asi_handle h, int32_t n, const int64_t *A_rowptr_h, const int32_t *A_col_h,
                            const double *A_val_h, const int32_t *perm_h, double tol);

/* Wait for the handle's stream; return the first device-side error latched
 * since the previous asi_sync (and clear it). */
asi_status asi_sync(asi_handle h);

/*
 * Device-side tracing. asi_profile(h, 1) clears the counters and brackets
 * every subsequent kernel launch of the numeric calls with HIP events on the
 * handle's stream; asi_profile(h, 0) stops. asi_profile_read waits for the
 * stream and returns, for one kernel class, the number of launches, their
 * summed device time and their summed algorithmic bytes (0 where the class
 * has no byte model).
 */
typedef enum {
    ASI_K_DINV = 0,          /* D-block inverses */
    ASI_K_SELINV = 1,        /* SelInv level launches, wavefront-per-block kernel */
    ASI_K_SELINV_BIG = 2,    /* SelInv level launches, workgroup-per-block kernel */
    ASI_K_NINV = 3,          /* the NInv sequence (series columns and product on S) */
    ASI_K_MIX = 4,           /* Mix selection (with its diagonal copy) */
    ASI_K_SPAI = 5,          /* SPAI refinement and symmetrisation */
    ASI_K_LOWRANK = 6,       /* rank-k correction on S */
    ASI_K_GATHER = 7,        /* L values into the column layout (gather, or float32 copy of the loaded factor) */
    ASI_K_SELINV_FLOW = 8,   /* the dataflow SelInv sweep (one launch per call) */
    ASI_K_MLP_FEATURES = 9,  /* features of the learned correction */
    ASI_K_MLP_FORWARD = 10,  /* MLP inference */
    ASI_K_MLP_TRAIN = 11,    /* MLP backward, loss and Adam */
    ASI_K_DIAG = 12,         /* diagonal error reductions */
    ASI_K_ILDL = 13,         /* numeric phase of the incomplete factorization */
    ASI_K_COUNT = 14
} asi_kernel_class;
asi_status asi_profile(asi_handle h, int enable);
asi_status asi_profile_read(asi_handle h, int32_t kernel_class, int64_t *launches, double *total_ms,
                            double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* ASI_H */
