// C ABI of libasi: handle, workspace layout, argument checks and launch
// sequences. Declared in include/asi.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "asi.h"
#include "asi_internal.h"
#include "kernels.h"

struct asi_handle_s {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t aux = nullptr;      // second stream of asi_selinv_ninv (created on first use)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::string err;
    bool analyzed = false;
    bool ws_ready = false;
    asi::Analysis A;
    size_t ws_min = 0;
    size_t ws_default = 0;
    // device workspace
    unsigned char *ws = nullptr;
    size_t ws_bytes = 0;
    int64_t *rowptr = nullptr;
    int32_t *col = nullptr;
    int32_t *srow = nullptr;
    int64_t *diagpos = nullptr;
    int64_t *mirror = nullptr;
    int64_t *ustart = nullptr;
    int32_t *ucol = nullptr;
    int32_t *q2u = nullptr;        // u-index of each input L entry (the factor load's scatter)
    int64_t *mirror_u = nullptr;
    int64_t *useg = nullptr;
    int64_t *hit_ptr = nullptr;
    uint32_t *hits = nullptr;
    void *Lu = nullptr;
    void *Zu = nullptr;
    double *zd = nullptr;
    int32_t *done = nullptr;
    unsigned char *node = nullptr;
    int32_t *s2u = nullptr;       // S position -> u-index of its L value
    int64_t *nf_rpT = nullptr;    // NInv on its own pattern: rows of w, cursors, diagonal, scan sums
    unsigned long long *nf_cur = nullptr;
    double *nf_dN = nullptr;
    unsigned long long *nf_bsum = nullptr;
    double *cg = nullptr;  // Krylov work vectors (5 n), dot partials (1024), scalars (16)
    double *Ls = nullptr;         // L(max(i, j), min(i, j)) at every position of S (0 where L has none)
    double *Lcsr = nullptr;       // the loaded factor's L values in the input's row order
    asi::SolveRow *solve_fwd = nullptr, *solve_bwd = nullptr;  // preconditioner solve rows, level order
    bool rows_aligned = false;    // row i of L is the lower part of row i of S (the 2x2 (i, i-1) entry aside)
    bool ls_loaded = false;       // Ls holds the loaded factor's values
    double *rn = nullptr;         // ||L(i, :)||_2, then ||L(:, i)||_2, of the factor in Lu (set with it)
    int64_t *rowptr_L = nullptr;  // the input L's row pointers
    float *Lf = nullptr;          // float32 copy of the loaded factor's L (mixed precision)
    bool factor_loaded = false;   // Lu (float64), dinv, the norms and the row copy hold the last factor given
    bool lf_loaded = false;       // Lf holds the float32 copy of that factor's L
    int32_t epoch = 0;
    int sweep = ASI_SWEEP_AUTO;
    bool sentinel = false;        // SelInv sweeps start from a NaN-filled working Z (schedule check)
    int8_t *piv = nullptr;
    int32_t *level = nullptr;
    asi::BlockMeta *meta_small = nullptr;
    asi::BlockMeta *meta_big = nullptr;
    double *dinv = nullptr;
    double *zdiag = nullptr;
    int32_t *status = nullptr;
    int64_t *cstart = nullptr;
    int32_t *clen = nullptr;
    int32_t *ovf = nullptr;
    int32_t *clast = nullptr;      // NInv: largest row of each stored series column
    int32_t *counters = nullptr;  // [0] ovf count, [1] unused, [2], [3] SPAI list lengths
    unsigned long long *pool_top = nullptr;
    int32_t *iperm = nullptr;
    double *cn2 = nullptr;
    double *X = nullptr;
    double *red = nullptr;
    int32_t *spai_list = nullptr;
    int32_t *prow = nullptr;
    void *plinv = nullptr;
    void *pw = nullptr;
    int64_t pool_cap = 0;  // entries (sized for float64 values)
    // numeric factorization: per-level LDS entries and algorithmic bytes (set on its first call)
    bool ildl_ready = false;
    std::vector<int32_t> ildl_lvl_entries;
    double ildl_bytes = 0.0;
    // device threshold factorization: the last call's work buffer and sizes
    asi::IldlTParams ildlt{};
    bool ildlt_done = false;
    int64_t ildlt_nnz = 0;
    // tracing
    bool prof = false;
    struct Rec {
        hipEvent_t a, b;
        int kind;
        double bytes;
    };
    std::vector<hipEvent_t> ev_free;
    std::vector<Rec> pending;
    int64_t prof_n[ASI_K_COUNT] = {};
    double prof_ms[ASI_K_COUNT] = {};
    double prof_bytes[ASI_K_COUNT] = {};
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

asi_status fail(asi_handle h, asi_status s, const std::string &m) {
    if (h) h->err = m;
    return s;
}

asi_status hip_fail(asi_handle h, hipError_t e, const char *what) {
    return fail(h, ASI_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace layout: fixed regions followed by the NInv pool.
struct Layout {
    size_t off[48];
    int k = 0;
    size_t cur = 0;
    size_t add(size_t bytes) {
        size_t o = cur;
        cur = align256(cur + std::max<size_t>(bytes, 1));
        off[k++] = o;
        return o;
    }
};

Layout make_layout(const asi::Analysis &A) {
    const size_t n = (size_t)A.n, s = (size_t)A.nnzS, u = (size_t)A.nnzU;
    Layout L;
    L.add((n + 1) * 8);                 // 0 rowptr
    L.add(s * 4);                       // 1 col
    L.add(s * 4);                       // 2 srow
    L.add(n * 8);                       // 3 diagpos
    L.add(s * 8);                       // 4 mirror
    L.add((n + 1) * 8);                 // 5 ustart
    L.add(n);                           // 6 piv
    L.add(n * 4);                       // 7 level
    L.add(A.meta_small.size() * 64);    // 8 block records, wavefront-per-block schedule
    L.add(A.meta_big.size() * 64);      // 9 block records, workgroup-per-block schedule
    L.add(3 * n * 8);                   // 10 dinv
    L.add(u * 4);                       // 11 ucol
    L.add(n * 8);                       // 12 zdiag (Mix)
    L.add(256);                         // 13 status + counters + pool_top
    L.add(n * 8);                       // 14 cstart
    L.add(n * 4);                       // 15 clen
    L.add(n * 4);                       // 16 ovf
    L.add(n * 4);                       // 17 clast
    L.add(n * 4);                       // 18 iperm
    L.add(n * 8);                       // 19 cn2
    L.add(s * 8);                       // 20 X
    L.add(A.nnzL * 4);                  // 21 q2u: u-index of each input L entry
    L.add(u * 8);                       // 22 mirror_u
    L.add(u * 8);                       // 23 useg
    L.add((n + 1) * 8);                 // 24 hit_ptr
    L.add(u * 8);                       // 25 Lu
    L.add(u * 8);                       // 26 Zu
    L.add(n * 8);                       // 27 zd (SelInv diagonal)
    L.add(A.hits.size() * 4);           // 28 hits
    L.add(n * 4);                       // 29 done flags of the dataflow sweep
    L.add(n * 32);                      // 30 per-node feature records (learned correction)
    L.add(2 * asi::kRedBlocks * 8);     // 31 partial sums of the diagonal error
    L.add(2 * n * 4);                   // 32 column lists of the SPAI kernels
    L.add(u * 4);                       // 33 L in u-space, float32 (mixed precision)
    L.add(2 * n * 8);                   // 34 row and column norms of L (learned-correction features)
    L.add((n + 1) * 8);                 // 35 row pointers of the input L
    L.add(A.s2u.size() * 4);            // 36 u-index of each entry's L value (learned correction)
    L.add((n + 1) * 8);                 // 37 NInv on its own pattern: row pointers of the rows of w
    L.add((n + 1) * 8);                 // 38   their fill cursors
    L.add(n * 8);                       // 39   diagonal of N
    L.add((n / 1024 + 2) * 8);          // 40   scan block sums
    L.add((5 * n + 1024 + 16) * 8);     // 41 Krylov solves: 5 vectors, dot partials, scalars
    L.add(A.s2u.size() * 8);            // 42 L values in S's order (preconditioner solves)
    L.add(A.nnzL * 8);                  // 43 L values in the input's row order (copied with the factor)
    L.add(A.solve_fwd.size() * 16);     // 44 preconditioner solve rows, forward
    L.add(A.solve_bwd.size() * 16);     // 45   backward
    return L;
}

constexpr size_t kPoolEntryBytes = 4 + 8 + 8;

template <typename T>
T *at(unsigned char *base, size_t off) {
    return reinterpret_cast<T *>(base + off);
}

hipEvent_t take_event(asi_handle h) {
    if (!h->ev_free.empty()) {
        hipEvent_t e = h->ev_free.back();
        h->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets a launch sequence with events when tracing is on.
struct Trace {
    asi_handle h;
    int kind;
    double bytes;
    hipStream_t st;
    hipEvent_t a = nullptr;
    Trace(asi_handle hh, int k, double b, hipStream_t s = nullptr)
        : h(hh), kind(k), bytes(b), st(s ? s : hh->stream) {
        if (h->prof) {
            a = take_event(h);
            if (a) (void)hipEventRecord(a, st);
        }
    }
    ~Trace() {
        if (!a) return;
        hipEvent_t b = take_event(h);
        if (!b) {
            h->ev_free.push_back(a);
            return;
        }
        (void)hipEventRecord(b, st);
        h->pending.push_back({a, b, kind, bytes});
    }
};

asi_status need_ready(asi_handle h) {
    if (!h) return ASI_E_ARG;
    if (!h->analyzed) return fail(h, ASI_E_STATE, "asi_analyze has not run");
    if (!h->ws_ready) return fail(h, ASI_E_STATE, "asi_set_workspace has not run");
    return ASI_OK;
}

}  // namespace

extern "C" {

asi_status asi_create(asi_handle *h, int device, void *stream) {
    if (!h) return ASI_E_ARG;
    int count = 0;
    if (device != -1 && (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count))
        return ASI_E_ARG;
    auto *p = new asi_handle_s();
    p->device = device;
    p->stream = reinterpret_cast<hipStream_t>(stream);
    if (device >= 0) {
        // resolve the no-allocation scratch of asi_unpermute_noalloc on this
        // device once per process (its result is checked by that call)
        DeviceGuard g(device);
        (void)asi::unpermute_scratch_init(device);
    }
    *h = p;
    return ASI_OK;
}

asi_status asi_destroy(asi_handle h) {
    if (!h) return ASI_OK;
    if (h->device >= 0) {
        DeviceGuard g(h->device);
        (void)hipStreamSynchronize(h->stream);
        for (auto &r : h->pending) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : h->ev_free) (void)hipEventDestroy(e);
        if (h->aux) {
            (void)hipStreamSynchronize(h->aux);
            (void)hipStreamDestroy(h->aux);
        }
        if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
        if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    }
    delete h;
    return ASI_OK;
}

asi_status asi_set_stream(asi_handle h, void *stream) {
    if (!h) return ASI_E_ARG;
    h->stream = reinterpret_cast<hipStream_t>(stream);
    return ASI_OK;
}

const char *asi_last_error(asi_handle h) { return h ? h->err.c_str() : "null handle"; }

asi_status asi_analyze(asi_handle h, int32_t n, const int64_t *L_rowptr_h, const int32_t *L_col_h,
                       const int8_t *piv_h, int64_t *nnzS_out, size_t *workspace_bytes_out) {
    if (!h) return ASI_E_ARG;
    h->err.clear();
    h->analyzed = false;
    h->ws_ready = false;
    if (n <= 0 || !L_rowptr_h || !piv_h || (!L_col_h && n > 0 && L_rowptr_h[n] > 0))
        return fail(h, ASI_E_ARG, "null or empty analysis input");
    std::string msg;
    int rc = asi::analyze(n, L_rowptr_h, L_col_h, piv_h, h->A, msg);
    if (rc != 0) return fail(h, (asi_status)rc, msg);
    Layout L = make_layout(h->A);
    h->ws_min = L.cur;
    int64_t pool = 8 * (int64_t)n + 2 * h->A.nnzL + 4096;
    h->ws_default = L.cur + (size_t)pool * kPoolEntryBytes + 3 * 256;
    h->analyzed = true;
    h->ildl_ready = false;
    {
        // row i of L equals the lower part of row i of S (but for the (i, i-1)
        // entry of a 2x2 block, which L does not store): then the learned
        // correction reads L(i, j) for j < i in row order from the copy of L
        const asi::Analysis &A = h->A;
        bool al = true;
        for (int32_t i = 0; i < n && al; ++i)
            al = A.diagpos[i] - A.rowptr[i] - (A.piv[i] == 2 ? 1 : 0) == A.L_rowptr[i + 1] - A.L_rowptr[i];
        h->rows_aligned = al;
    }
    if (nnzS_out) *nnzS_out = h->A.nnzS;
    if (workspace_bytes_out) *workspace_bytes_out = h->ws_default;
    return ASI_OK;
}

asi_status asi_set_workspace(asi_handle h, void *dev_ws, size_t bytes) {
    if (!h) return ASI_E_ARG;
    if (h->device < 0) return fail(h, ASI_E_STATE, "host-only handle (device -1) has no workspace");
    if (!h->analyzed) return fail(h, ASI_E_STATE, "asi_analyze has not run");
    if (!dev_ws) return fail(h, ASI_E_ARG, "null workspace");
    if ((reinterpret_cast<uintptr_t>(dev_ws) & 255) != 0) return fail(h, ASI_E_ARG, "workspace must be 256-byte aligned");
    if (bytes < h->ws_min + 3 * 256 + 64 * kPoolEntryBytes)
        return fail(h, ASI_E_WORKSPACE, "workspace smaller than workspace_min");
    DeviceGuard g(h->device);
    const asi::Analysis &A = h->A;
    Layout L = make_layout(A);
    unsigned char *b = static_cast<unsigned char *>(dev_ws);
    h->ws = b;
    h->ws_bytes = bytes;
    h->rowptr = at<int64_t>(b, L.off[0]);
    h->col = at<int32_t>(b, L.off[1]);
    h->srow = at<int32_t>(b, L.off[2]);
    h->diagpos = at<int64_t>(b, L.off[3]);
    h->mirror = at<int64_t>(b, L.off[4]);
    h->ustart = at<int64_t>(b, L.off[5]);
    h->piv = at<int8_t>(b, L.off[6]);
    h->level = at<int32_t>(b, L.off[7]);
    h->meta_small = at<asi::BlockMeta>(b, L.off[8]);
    h->meta_big = at<asi::BlockMeta>(b, L.off[9]);
    h->dinv = at<double>(b, L.off[10]);
    h->ucol = at<int32_t>(b, L.off[11]);
    h->zdiag = at<double>(b, L.off[12]);
    h->status = at<int32_t>(b, L.off[13]);
    h->counters = h->status + 4;
    h->pool_top = reinterpret_cast<unsigned long long *>(h->status + 8);
    h->cstart = at<int64_t>(b, L.off[14]);
    h->clen = at<int32_t>(b, L.off[15]);
    h->ovf = at<int32_t>(b, L.off[16]);
    h->clast = at<int32_t>(b, L.off[17]);
    h->iperm = at<int32_t>(b, L.off[18]);
    h->cn2 = at<double>(b, L.off[19]);
    h->X = at<double>(b, L.off[20]);
    h->q2u = at<int32_t>(b, L.off[21]);
    h->mirror_u = at<int64_t>(b, L.off[22]);
    h->useg = at<int64_t>(b, L.off[23]);
    h->hit_ptr = at<int64_t>(b, L.off[24]);
    h->Lu = b + L.off[25];
    h->Zu = b + L.off[26];
    h->zd = at<double>(b, L.off[27]);
    h->hits = at<uint32_t>(b, L.off[28]);
    h->done = at<int32_t>(b, L.off[29]);
    h->node = b + L.off[30];
    h->red = at<double>(b, L.off[31]);
    h->spai_list = at<int32_t>(b, L.off[32]);
    h->Lf = at<float>(b, L.off[33]);
    h->rn = at<double>(b, L.off[34]);
    h->rowptr_L = at<int64_t>(b, L.off[35]);
    h->s2u = at<int32_t>(b, L.off[36]);
    h->nf_rpT = at<int64_t>(b, L.off[37]);
    h->nf_cur = at<unsigned long long>(b, L.off[38]);
    h->nf_dN = at<double>(b, L.off[39]);
    h->nf_bsum = at<unsigned long long>(b, L.off[40]);
    h->cg = at<double>(b, L.off[41]);
    h->Ls = at<double>(b, L.off[42]);
    h->ls_loaded = false;
    h->Lcsr = at<double>(b, L.off[43]);
    h->solve_fwd = at<asi::SolveRow>(b, L.off[44]);
    h->solve_bwd = at<asi::SolveRow>(b, L.off[45]);
    h->factor_loaded = false;
    h->lf_loaded = false;
    h->epoch = 0;
    // pool: rows | linv | w, each region 256-aligned
    size_t rest = bytes - L.cur - 3 * 256;
    int64_t cap = (int64_t)(rest / kPoolEntryBytes);
    size_t o = L.cur;
    h->prow = at<int32_t>(b, o);
    o = align256(o + (size_t)cap * 4);
    h->plinv = b + o;
    o = align256(o + (size_t)cap * 8);
    h->pw = b + o;
    h->pool_cap = cap;

    struct Up {
        void *dst;
        const void *src;
        size_t bytes;
    } ups[] = {
        {h->rowptr, A.rowptr.data(), A.rowptr.size() * 8},
        {h->col, A.col.data(), A.col.size() * 4},
        {h->srow, A.srow.data(), A.srow.size() * 4},
        {h->diagpos, A.diagpos.data(), A.diagpos.size() * 8},
        {h->mirror, A.mirror.data(), A.mirror.size() * 8},
        {h->ustart, A.ustart.data(), A.ustart.size() * 8},
        {h->ucol, A.ucol.data(), A.ucol.size() * 4},
        {h->q2u, A.q2u.data(), A.q2u.size() * 4},
        {h->mirror_u, A.mirror_u.data(), A.mirror_u.size() * 8},
        {h->useg, A.useg_u.data(), A.useg_u.size() * 8},
        {h->hit_ptr, A.hit_ptr.data(), A.hit_ptr.size() * 8},
        {h->hits, A.hits.data(), A.hits.size() * 4},
        {h->piv, A.piv.data(), A.piv.size()},
        {h->level, A.level.data(), A.level.size() * 4},
        {h->meta_small, A.meta_small.data(), A.meta_small.size() * 64},
        {h->meta_big, A.meta_big.data(), A.meta_big.size() * 64},
        {h->rowptr_L, A.L_rowptr.data(), A.L_rowptr.size() * 8},
        {h->s2u, A.s2u.data(), A.s2u.size() * 4},
        {h->solve_fwd, A.solve_fwd.data(), A.solve_fwd.size() * 16},
        {h->solve_bwd, A.solve_bwd.data(), A.solve_bwd.size() * 16},
    };
    for (auto &u : ups) {
        if (u.bytes == 0) continue;
        hipError_t e = hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "upload analysis");
    }
    hipError_t e = asi::launch_fill_i32(h->status, 64, 0, h->stream);
    if (e == hipSuccess) e = asi::launch_fill_i32(h->done, A.n, 0, h->stream);
    // the factor load scatters L's entries into the column layout; the
    // padding of 2x2 unions (no L entry) keeps these zeros
    if (e == hipSuccess && A.nnzU > 0) e = hipMemsetAsync(h->Lu, 0, A.nnzU * 8, h->stream);
    if (e == hipSuccess && A.nnzU > 0) e = hipMemsetAsync(h->Lf, 0, A.nnzU * 4, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "clear status");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "upload analysis");
    e = asi::set_big_lds_limits();
    if (e == hipSuccess) e = asi::set_ninv_lds_limits();
    if (e == hipSuccess) e = asi::set_nfull_lds_limits();
    if (e != hipSuccess) return hip_fail(h, e, "set LDS limits");
    h->ws_ready = true;
    return ASI_OK;
}

asi_status asi_get_info(asi_handle h, asi_info *info) {
    if (!h || !info) return ASI_E_ARG;
    if (!h->analyzed) return fail(h, ASI_E_STATE, "asi_analyze has not run");
    const asi::Analysis &A = h->A;
    info->n = A.n;
    info->n_blocks = A.n_blocks;
    info->n_levels = A.n_levels;
    info->max_cols = A.max_cols;
    info->nnz_L = A.nnzL;
    info->nnz_S = A.nnzS;
    info->gather_pairs = A.gather_pairs;
    info->gather_hits = A.gather_hits;
    info->workspace_min = h->ws_min + 3 * 256 + 64 * kPoolEntryBytes;
    info->workspace_default = h->ws_default;
    return ASI_OK;
}

asi_status asi_get_pattern(asi_handle h, int64_t *S_rowptr_d, int32_t *S_col_d, int32_t *level_d) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!S_rowptr_d || !S_col_d) return fail(h, ASI_E_ARG, "null output");
    DeviceGuard g(h->device);
    const asi::Analysis &A = h->A;
    hipError_t e = hipMemcpyAsync(S_rowptr_d, h->rowptr, (A.n + 1) * 8, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(S_col_d, h->col, A.nnzS * 4, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess && level_d)
        e = hipMemcpyAsync(level_d, h->level, A.n * 4, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "copy pattern");
    return ASI_OK;
}

// The factor of one call in the workspace: D-block inverses in dinv and L in
// u-space in the call's precision (Lu float64, Lf float32), from the given
// arrays, or (all three NULL) from the factor of asi_load_factor. Sets *Lu to
// the u-space values the call's kernels read.
// With side given the call also forks side off the calling stream: a new
// factor's column layouts (float64, and float32 for a mixed call) are made on
// the calling stream, and the norms and the row-order copy of L, which only
// the learned correction reads, are left to the caller (factor_norms_on, on
// side after NInv), which joins side back before anything else reads them.
static asi_status prepare_factor(asi_handle h, const double *L_val, const double *d_diag, const double *d_sub,
                                 bool fp64, const void **Lu, hipStream_t side = nullptr) {
    const asi::Analysis &A = h->A;
    hipError_t e;
    bool forked = false;
    auto fork = [&]() -> hipError_t {
        hipError_t e2 = hipEventRecord(h->ev_fork, h->stream);
        if (e2 == hipSuccess) e2 = hipStreamWaitEvent(side, h->ev_fork, 0);
        forked = true;
        return e2;
    };
    if (L_val || d_diag || d_sub) {
        if ((!L_val && A.nnzL > 0) || !d_diag || !d_sub)
            return fail(h, ASI_E_ARG, "null factor pointer (give L_val, d_diag and d_sub, or none of them)");
        h->factor_loaded = false;  // until dinv and Lu (and Lf for a mixed call) hold this call's factor
        h->lf_loaded = false;
        h->ls_loaded = false;
        {
            Trace t(h, ASI_K_DINV, 0.0);
            e = asi::launch_dinv(A.n, h->piv, d_diag, d_sub, h->dinv, h->status, h->stream);
        }
        if (e != hipSuccess) return hip_fail(h, e, "dinv");
        if (side) {
            {
                Trace t(h, ASI_K_GATHER, 20.0 * A.nnzL);
                e = asi::launch_scatter_lu(A.nnzL, h->q2u, L_val, h->Lu, true, h->stream);
            }
            if (e == hipSuccess && !fp64) {
                Trace t(h, ASI_K_GATHER, 12.0 * A.nnzU);
                e = asi::launch_lu_to_float(A.nnzU, reinterpret_cast<const double *>(h->Lu), h->Lf, h->stream);
                h->lf_loaded = true;
            }
            if (e == hipSuccess) e = fork();
            if (e != hipSuccess) return hip_fail(h, e, "gather L");
        } else {
            // the float64 copy in the column layout always (NInv's series
            // reads it in both precisions), with the row and column norms of
            // L (learned-correction features)
            Trace t(h, ASI_K_GATHER, 20.0 * A.nnzL);
            e = asi::launch_scatter_lu(A.nnzL, h->q2u, L_val, h->Lu, true, h->stream);
            if (e == hipSuccess)
                e = asi::launch_factor_norms(A.n, h->rowptr_L, L_val, h->ustart,
                                             reinterpret_cast<const double *>(h->Lu), h->rn, h->Lcsr, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "gather L");
        }
        h->factor_loaded = true;  // the call's factor stays loaded for later calls without factor pointers
    } else if (!h->factor_loaded) {
        return fail(h, ASI_E_STATE, "no factor given and none loaded (asi_load_factor)");
    }
    if (!fp64 && !h->lf_loaded) {
        Trace t(h, ASI_K_GATHER, 12.0 * A.nnzU);
        e = asi::launch_lu_to_float(A.nnzU, reinterpret_cast<const double *>(h->Lu), h->Lf, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "L to float32");
        h->lf_loaded = true;
    }
    if (side && !forked) {
        e = fork();
        if (e != hipSuccess) return hip_fail(h, e, "fork");
    }
    *Lu = fp64 ? h->Lu : (const void *)h->Lf;
    return ASI_OK;
}

// The row and column norms of L and its row-order copy (learned-correction
// features), from the caller's L_val and the float64 column layout, on st.
static asi_status factor_norms_on(asi_handle h, const double *L_val, hipStream_t st) {
    Trace t(h, ASI_K_GATHER, 0.0, st);
    hipError_t e = asi::launch_factor_norms(h->A.n, h->rowptr_L, L_val, h->ustart,
                                            reinterpret_cast<const double *>(h->Lu), h->rn, h->Lcsr, st);
    if (e != hipSuccess) return hip_fail(h, e, "factor norms");
    return ASI_OK;
}

// L's values in S's order (Ls) for the loaded float64 factor, gathered from
// the column layout on the first preconditioner solve after a load (a solve
// runs the whole level schedule twice; the copy lets each row read its L
// values in sequence instead of through the u-index).
static asi_status ensure_ls(asi_handle h) {
    if (h->ls_loaded) return ASI_OK;
    if (!h->factor_loaded) return fail(h, ASI_E_STATE, "no factor loaded (asi_load_factor)");
    if (h->A.s2u.empty() && h->A.nnzS > 0) return fail(h, ASI_E_UNSUPPORTED, "solves need |S| < 2^31");
    Trace t(h, ASI_K_GATHER, 20.0 * h->A.nnzS);
    hipError_t e = asi::launch_build_ls(h->A.nnzS, h->s2u, reinterpret_cast<const double *>(h->Lu), h->Ls,
                                        h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "L in S order");
    h->ls_loaded = true;
    return ASI_OK;
}

asi_status asi_load_factor(asi_handle h, const double *L_val, const double *d_diag, const double *d_sub) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if ((!L_val && h->A.nnzL > 0) || !d_diag || !d_sub) return fail(h, ASI_E_ARG, "null pointer");
    DeviceGuard g(h->device);
    const void *Lu = nullptr;
    s = prepare_factor(h, L_val, d_diag, d_sub, true, &Lu);
    if (s != ASI_OK) return s;
    h->factor_loaded = true;
    return ASI_OK;
}

// The SelInv sweep on stream st, reading L in u-space from Lu.
static asi_status selinv_launch(asi_handle h, const void *Lu, bool fp64, double *Z_S, hipStream_t st) {
    const asi::Analysis &A = h->A;
    const int m = fp64 ? 0 : 1;
    hipError_t e;
    asi::SelinvParams P{};
    P.ustart = h->ustart;
    P.ucol = h->ucol;
    P.useg = h->useg;
    P.hit_ptr = h->hit_ptr;
    P.hits = h->hits;
    P.mirror_u = h->mirror_u;
    P.diagpos = h->diagpos;
    P.piv = h->piv;
    P.Lu = Lu;
    P.dinv = h->dinv;
    P.Zu = h->Zu;
    P.zdiag = h->zd;
    P.out = Z_S;
    P.status = h->status;
    if (h->sentinel) {
        // every entry a block reads must have been written by an earlier
        // block of this sweep: NaN (all-ones words, in float32 and float64)
        // makes any other read visible in the result
        e = asi::launch_fill_i32(reinterpret_cast<int32_t *>(h->Zu), (int64_t)A.nnzU * (fp64 ? 2 : 1), -1, st);
        if (e == hipSuccess) e = asi::launch_fill_i32(reinterpret_cast<int32_t *>(h->zd), (int64_t)A.n * 2, -1, st);
        if (e != hipSuccess) return hip_fail(h, e, "sentinel fill");
    }
    const bool flow_ok = A.sched_big.empty() && A.n_blocks > 0;
    int grid = 0;
    // AUTO runs the level schedule: on MI355X it measured faster than the
    // dataflow sweep for the workloads here (per-block flag latency outweighs
    // the saved launch boundaries)
    if (h->sweep == ASI_SWEEP_DATAFLOW && flow_ok) grid = asi::flow_grid(fp64);
    if (h->sweep == ASI_SWEEP_DATAFLOW && grid <= 0)
        return fail(h, ASI_E_UNSUPPORTED, "dataflow sweep needs |R_J| <= 128 and cooperative launch");
    if (grid > 0) {
        double bytes = 0.0;
        for (int32_t l = 0; l < A.n_levels; ++l) bytes += A.lvl_bytes_small[m][l];
        h->epoch = h->epoch == INT32_MAX ? 1 : h->epoch + 1;
        Trace t(h, ASI_K_SELINV_FLOW, bytes, st);
        P.meta = h->meta_small;
        e = asi::launch_selinv_flow(P, A.n_blocks, h->done, h->epoch, 1 << 21, fp64, grid, st);
        if (e != hipSuccess) return hip_fail(h, e, "selinv dataflow launch");
        return ASI_OK;
    }
    for (int32_t l = 0; l < A.n_levels; ++l) {
        P.meta = h->meta_small + A.lvl_small[l];
        P.nblk = A.lvl_small[l + 1] - A.lvl_small[l];
        P.nheavy = A.lvl_heavy[l];
        if (P.nblk > 0) {
            Trace t(h, ASI_K_SELINV, A.lvl_bytes_small[m][l], st);
            e = asi::launch_selinv_level(P, asi::small_level_variant(P.nblk, P.nheavy), fp64, st, 0);
            if (e != hipSuccess) return hip_fail(h, e, "selinv level");
        }
        P.meta = h->meta_big + A.lvl_big[l];
        P.nblk = A.lvl_big[l + 1] - A.lvl_big[l];
        P.nheavy = 0;
        if (P.nblk > 0) {
            Trace t(h, ASI_K_SELINV_BIG, A.lvl_bytes_big[m][l], st);
            e = asi::launch_selinv_level(P, asi::big_level_variant(P.nblk), fp64, st, A.lvl_maxc_big[l]);
            if (e != hipSuccess) return hip_fail(h, e, "selinv level (large blocks)");
        }
    }
    return ASI_OK;
}

asi_status asi_selinv(asi_handle h, const double *L_val, const double *d_diag, const double *d_sub,
                      asi_precision prec, double *Z_S) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!Z_S) return fail(h, ASI_E_ARG, "null pointer");
    if (prec != ASI_FP64 && prec != ASI_MIXED) return fail(h, ASI_E_ARG, "unknown precision");
    DeviceGuard g(h->device);
    const bool fp64 = prec == ASI_FP64;
    const void *Lu = nullptr;
    s = prepare_factor(h, L_val, d_diag, d_sub, fp64, &Lu);
    if (s != ASI_OK) return s;
    return selinv_launch(h, Lu, fp64, Z_S, h->stream);
}

asi_status asi_set_sentinel(asi_handle h, int on) {
    if (!h) return ASI_E_ARG;
    h->sentinel = on != 0;
    return ASI_OK;
}

asi_status asi_set_sweep(asi_handle h, asi_sweep mode) {
    if (!h) return ASI_E_ARG;
    if (mode != ASI_SWEEP_AUTO && mode != ASI_SWEEP_LEVELS && mode != ASI_SWEEP_DATAFLOW)
        return fail(h, ASI_E_ARG, "unknown sweep mode");
    h->sweep = mode;
    return ASI_OK;
}

asi_status asi_sweep_plan(asi_handle h, int64_t *counts_h) {
    if (!h || !counts_h) return h ? fail(h, ASI_E_ARG, "null pointer") : ASI_E_ARG;
    if (!h->analyzed) return fail(h, ASI_E_STATE, "asi_analyze has not run");
    static_assert((int)asi::SV_COUNT == (int)ASI_SV_COUNT, "variant numbering");
    const asi::Analysis &A = h->A;
    for (int v = 0; v < asi::SV_COUNT; ++v) counts_h[v] = 0;
    for (int32_t l = 0; l < A.n_levels; ++l) {
        const int64_t ns = A.lvl_small[l + 1] - A.lvl_small[l];
        const int64_t nb = A.lvl_big[l + 1] - A.lvl_big[l];
        if (ns > 0) counts_h[asi::small_level_variant(ns, A.lvl_heavy[l])]++;
        if (nb > 0) counts_h[asi::big_level_variant(nb)]++;
    }
    return ASI_OK;
}

// NInv on stream st. The series reads the float64 copy of L (Lu) in both
// precisions; fp64 selects the storage of its columns and the precision of
// the product. linv_grid > 0 caps the workgroups of the persistent series
// kernel (0: as many as are resident; < 0: that fraction of them).
static asi_status ninv_launch(asi_handle h, bool fp64, int32_t p, double delta, double *N_S, hipStream_t st,
                              int linv_grid) {
    const asi::Analysis &A = h->A;
    asi::NinvParams P{};
    P.n = A.n;
    P.rowptr = h->rowptr;
    P.col = h->col;
    P.srow = h->srow;
    P.rowptr_n = A.nnzS;
    P.diagpos = h->diagpos;
    P.mirror = h->mirror;
    P.ustart = h->ustart;
    P.ucol = h->ucol;
    P.piv = h->piv;
    P.Lu = h->Lu;
    P.dinv = h->dinv;
    P.p = p;
    P.delta = delta;
    P.prow = h->prow;
    P.plinv = h->plinv;
    P.pw = h->pw;
    P.pool_cap = h->pool_cap;
    P.pool_top = h->pool_top;
    P.cstart = h->cstart;
    P.clen = h->clen;
    P.ovf_list = h->ovf;
    P.ovf_count = h->counters;
    P.clast = h->clast;
    P.out = N_S;
    P.status = h->status;
    P.tr_ptr = reinterpret_cast<unsigned long long *>(h->nf_rpT);
    P.tr_cur = h->nf_cur;
    P.tr_bsum = h->nf_bsum;
    P.tr_flag = h->status + 12;
    hipError_t e;
    {
        Trace t(h, ASI_K_NINV, 0.0, st);
        e = asi::launch_ninv(P, fp64, st, linv_grid);
    }
    if (e != hipSuccess) return hip_fail(h, e, "ninv");
    return ASI_OK;
}

asi_status asi_ninv(asi_handle h, const double *L_val, const double *d_diag, const double *d_sub, int32_t p,
                    double delta, asi_precision prec, double *N_S) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!N_S) return fail(h, ASI_E_ARG, "null pointer");
    if (p < 0 || p > 64) return fail(h, ASI_E_ARG, "p must be in [0, 64]");
    if (!(delta >= 0.0)) return fail(h, ASI_E_ARG, "delta must be >= 0");
    if (prec != ASI_FP64 && prec != ASI_MIXED) return fail(h, ASI_E_ARG, "unknown precision");
    DeviceGuard g(h->device);
    const bool fp64 = prec == ASI_FP64;
    const void *Lu = nullptr;
    s = prepare_factor(h, L_val, d_diag, d_sub, fp64, &Lu);
    if (s != ASI_OK) return s;
    return ninv_launch(h, fp64, p, delta, N_S, h->stream, 0);
}

// Result sizes of the full-pattern calls: the count pass leaves the row
// pointers in the caller's array; their last entry is the size.
static asi_status read_total(asi_handle h, const int64_t *rowptr, int64_t *nnz) {
    asi_status s = asi_sync(h);  // surfaces a latched device error
    if (s != ASI_OK) return s;
    hipError_t e = hipMemcpy(nnz, rowptr + h->A.n, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "read result size");
    return ASI_OK;
}

asi_status asi_ninv_full(asi_handle h, const double *L_val, const double *d_diag, const double *d_sub, int32_t p,
                         double delta, double drop, int64_t cap, int64_t *rowptr, int32_t *col, double *val,
                         int64_t *nnz) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!rowptr || !nnz || (cap > 0 && (!col || !val))) return fail(h, ASI_E_ARG, "null pointer");
    if (p < 0 || p > 64) return fail(h, ASI_E_ARG, "p must be in [0, 64]");
    if (!(delta >= 0.0) || !(drop >= 0.0)) return fail(h, ASI_E_ARG, "delta and drop must be >= 0");
    DeviceGuard g(h->device);
    const asi::Analysis &A = h->A;
    *nnz = 0;
    const void *Lu = nullptr;
    s = prepare_factor(h, L_val, d_diag, d_sub, true, &Lu);
    if (s != ASI_OK) return s;
    asi::NinvParams Q{};
    Q.n = A.n;
    Q.rowptr = h->rowptr;
    Q.col = h->col;
    Q.diagpos = h->diagpos;
    Q.mirror = h->mirror;
    Q.ustart = h->ustart;
    Q.ucol = h->ucol;
    Q.piv = h->piv;
    Q.Lu = Lu;
    Q.dinv = h->dinv;
    Q.p = p;
    Q.delta = delta;
    Q.prow = h->prow;
    Q.plinv = h->plinv;
    Q.pw = h->pw;
    Q.pool_cap = h->pool_cap;
    Q.pool_top = h->pool_top;
    Q.cstart = h->cstart;
    Q.clen = h->clen;
    Q.ovf_list = h->ovf;
    Q.ovf_count = h->counters;
    Q.clast = h->clast;
    Q.status = h->status;
    hipError_t e;
    {
        Trace t(h, ASI_K_NINV, 0.0);
        e = asi::launch_linv(Q, h->stream);
    }
    if (e != hipSuccess) return hip_fail(h, e, "ninv series");
    s = asi_sync(h);
    if (s != ASI_OK) return s;
    asi::NfullParams P{};
    P.n = A.n;
    P.cstart = h->cstart;
    P.clen = h->clen;
    P.prow = h->prow;
    P.plinv = reinterpret_cast<double *>(h->plinv);
    P.pw = reinterpret_cast<double *>(h->pw);
    P.rpT = h->nf_rpT;
    P.cur = h->nf_cur;
    P.dN = h->nf_dN;
    P.drop = drop;
    P.bsum = h->nf_bsum;
    P.cnt = reinterpret_cast<unsigned long long *>(rowptr);
    P.rowptr = rowptr;
    P.col = col;
    P.val = val;
    P.ovf_list = h->ovf;
    P.ovf_count = h->counters;
    P.status = h->status;
    {
        Trace t(h, ASI_K_NINV, 0.0);
        e = asi::launch_nfull_count_w(P, h->stream);
    }
    if (e != hipSuccess) return hip_fail(h, e, "ninv full pattern (rows of w)");
    s = asi_sync(h);
    if (s != ASI_OK) return s;
    // the rows of w go after the pool's reserved entries of the row and w regions
    unsigned long long used = 0;
    int64_t total = 0;
    e = hipMemcpy(&used, h->pool_top, 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&total, h->nf_rpT + A.n, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "read pool size");
    if ((int64_t)used + total > h->pool_cap)
        return fail(h, ASI_E_WORKSPACE, "NInv pool too small for the full pattern: enlarge the workspace");
    P.colT = h->prow + used;
    P.valT = reinterpret_cast<double *>(h->pw) + used;
    {
        Trace t(h, ASI_K_NINV, 0.0);
        e = asi::launch_nfull_fill_w(P, h->stream);
        if (e == hipSuccess) e = asi::launch_nfull_rows(P, false, h->stream);
    }
    if (e != hipSuccess) return hip_fail(h, e, "ninv full pattern (count)");
    s = read_total(h, rowptr, nnz);
    if (s != ASI_OK) return s;
    if (*nnz > cap) return fail(h, ASI_E_WORKSPACE, "result larger than cap (the size is in *nnz)");
    {
        Trace t(h, ASI_K_NINV, 0.0);
        e = asi::launch_nfull_rows(P, true, h->stream);
    }
    if (e != hipSuccess) return hip_fail(h, e, "ninv full pattern (fill)");
    return asi_sync(h);
}

asi_status asi_mix_full(asi_handle h, const double *Z_S, const int64_t *N_rowptr, const int32_t *N_col,
                        const double *N_val, double eps, int64_t cap, int64_t *rowptr, int32_t *col, double *val,
                        int64_t *nnz) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!Z_S || !N_rowptr || !rowptr || !nnz || (cap > 0 && (!col || !val))) return fail(h, ASI_E_ARG, "null pointer");
    if (!(eps >= 0.0)) return fail(h, ASI_E_ARG, "eps must be >= 0");
    DeviceGuard g(h->device);
    const asi::Analysis &A = h->A;
    *nnz = 0;
    hipError_t e = asi::launch_zdiag(A.n, h->diagpos, Z_S, h->zdiag, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "Z diagonal");
    asi::MixFullParams P{};
    P.n = A.n;
    P.Nrp = N_rowptr;
    P.Ncol = N_col;
    P.Nval = N_val;
    P.srp = h->rowptr;
    P.scol = h->col;
    P.diagpos = h->diagpos;
    P.Z = Z_S;
    P.zdiag = h->zdiag;
    P.eps = eps;
    P.bsum = h->nf_bsum;
    P.cnt = reinterpret_cast<unsigned long long *>(rowptr);
    P.rowptr = rowptr;
    P.col = col;
    P.val = val;
    {
        Trace t(h, ASI_K_MIX, 0.0);
        e = asi::launch_mixfull(P, false, h->stream);
    }
    if (e != hipSuccess) return hip_fail(h, e, "mix full pattern (count)");
    s = read_total(h, rowptr, nnz);
    if (s != ASI_OK) return s;
    if (*nnz > cap) return fail(h, ASI_E_WORKSPACE, "result larger than cap (the size is in *nnz)");
    {
        Trace t(h, ASI_K_MIX, 0.0);
        e = asi::launch_mixfull(P, true, h->stream);
    }
    if (e != hipSuccess) return hip_fail(h, e, "mix full pattern (fill)");
    return ASI_OK;
}

asi_status asi_selinv_ninv(asi_handle h, const double *L_val, const double *d_diag, const double *d_sub,
                           int32_t p, double delta, asi_precision prec, double *Z_S, double *N_S) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!Z_S || !N_S) return fail(h, ASI_E_ARG, "null pointer");
    if (p < 0 || p > 64) return fail(h, ASI_E_ARG, "p must be in [0, 64]");
    if (!(delta >= 0.0)) return fail(h, ASI_E_ARG, "delta must be >= 0");
    if (prec != ASI_FP64 && prec != ASI_MIXED) return fail(h, ASI_E_ARG, "unknown precision");
    DeviceGuard g(h->device);
    const bool fp64 = prec == ASI_FP64;
    const void *Lu = nullptr;
    // the dataflow sweep needs every workgroup resident: no concurrent work beside it
    if (h->sweep == ASI_SWEEP_DATAFLOW) {
        s = prepare_factor(h, L_val, d_diag, d_sub, fp64, &Lu);
        if (s != ASI_OK) return s;
        s = ninv_launch(h, fp64, p, delta, N_S, h->stream, 0);
        if (s != ASI_OK) return s;
        return selinv_launch(h, Lu, fp64, Z_S, h->stream);
    }
    hipError_t e = hipSuccess;
    if (!h->aux) {
        e = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(h, e, "second stream");
    }
    // forks the second stream: NInv, then the rest of a new factor's load
    // (only the learned correction reads it), run there, beside the sweep
    s = prepare_factor(h, L_val, d_diag, d_sub, fp64, &Lu, h->aux);
    if (s != ASI_OK) return s;
    // NInv's persistent kernel takes half the resident workgroups, leaving
    // compute units to the latency-bound SelInv levels running beside it
    s = ninv_launch(h, fp64, p, delta, N_S, h->aux, -2);
    if (s == ASI_OK && (L_val || d_diag || d_sub)) s = factor_norms_on(h, L_val, h->aux);
    if (s == ASI_OK) s = selinv_launch(h, Lu, fp64, Z_S, h->stream);
    e = hipEventRecord(h->ev_join, h->aux);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, h->ev_join, 0);
    if (e != hipSuccess) return hip_fail(h, e, "join");
    return s;
}

asi_status asi_mix(asi_handle h, const double *Z_S, const double *N_S, double eps, double *M_S) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!Z_S || !N_S || !M_S) return fail(h, ASI_E_ARG, "null pointer");
    if (!(eps >= 0.0)) return fail(h, ASI_E_ARG, "eps must be >= 0");
    DeviceGuard g(h->device);
    // bytes: Z, N and M values (24 B), row and column index (8 B) per entry; the
    // diagonal copy reads and writes 8 B per row twice
    Trace t(h, ASI_K_MIX, 32.0 * h->A.nnzS + 24.0 * h->A.n);
    hipError_t e = asi::launch_zdiag(h->A.n, h->diagpos, Z_S, h->zdiag, h->stream);
    if (e == hipSuccess)
        e = asi::launch_mix(h->A.nnzS, h->srow, h->col, h->zdiag, Z_S, N_S, eps, M_S, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "mix");
    return ASI_OK;
}

asi_status asi_spai(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                    const int32_t *perm, const double *M_S, int32_t cg_iters, double *R_S) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!A_rowptr || !A_col || !A_val || !perm || !M_S || !R_S) return fail(h, ASI_E_ARG, "null pointer");
    if (cg_iters < 0) return fail(h, ASI_E_ARG, "cg_iters must be >= 0");
    int64_t maxrow = 0;
    for (int32_t i = 0; i < h->A.n; ++i) maxrow = std::max(maxrow, h->A.rowptr[i + 1] - h->A.rowptr[i]);
    if (maxrow > asi::kSpaiMaxCols) return fail(h, ASI_E_UNSUPPORTED, "a column of S has more than 512 entries");
    DeviceGuard g(h->device);
    asi::SpaiParams P{};
    P.n = h->A.n;
    P.rowptr = h->rowptr;
    P.col = h->col;
    P.mirror = h->mirror;
    P.A_rowptr = A_rowptr;
    P.A_col = A_col;
    P.A_val = A_val;
    P.perm = perm;
    P.iperm = h->iperm;
    P.colnorm2 = h->cn2;
    P.M = M_S;
    P.X = h->X;
    P.R = R_S;
    P.iters = cg_iters;
    P.status = h->status;
    P.list = h->spai_list;
    P.list_count = h->counters + 2;
    Trace t(h, ASI_K_SPAI, 0.0);
    hipError_t e = asi::launch_spai(P, h->stream);
    if (e == hipSuccess) e = asi::launch_symmetrize(h->A.nnzS, h->mirror, h->X, R_S, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "spai");
    return ASI_OK;
}

asi_status asi_lowrank(asi_handle h, int32_t k, const double *V, const double *lambda, const double *in_S,
                       double *out_S) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (k < 1 || k > asi::kMaxRank) return fail(h, ASI_E_ARG, "k must be in [1, 64]");
    if (!V || !lambda || !in_S || !out_S) return fail(h, ASI_E_ARG, "null pointer");
    DeviceGuard g(h->device);
    // bytes per entry: column index, input and output values (20 B); V once
    Trace t(h, ASI_K_LOWRANK, 20.0 * h->A.nnzS + 8.0 * h->A.n * (k + 2));
    hipError_t e = asi::launch_lowrank(h->A.nnzS, k, h->srow, h->col, V, lambda, in_S, out_S, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "lowrank");
    return ASI_OK;
}

// Common set-up of the learned-correction calls: D-block inverses, L in its
// column layout, the per-node records; fills P.
static asi_status mlp_setup(asi_handle h, const double *Z_S, const double *N_S, const double *M_S, double eps,
                            const double *L_val, const double *d_diag, const double *d_sub, asi::MlpFeatParams &P,
                            bool fuse_mix = false, double *M_out = nullptr) {
    const asi::Analysis &A = h->A;
    if (A.nnzS > (int64_t)INT32_MAX) return fail(h, ASI_E_UNSUPPORTED, "the learned correction needs |S| < 2^31");
    const void *Lu = nullptr;
    asi_status s = prepare_factor(h, L_val, d_diag, d_sub, true, &Lu);
    if (s != ASI_OK) return s;
    hipError_t e;
    P = asi::MlpFeatParams{};
    P.n = A.n;
    P.nnz = A.nnzS;
    P.srow = h->srow;
    P.col = h->col;
    P.diagpos = h->diagpos;
    P.s2u = h->s2u;
    P.ustart = h->ustart;
    P.piv = h->piv;
    P.level = h->level;
    P.maxlevel = A.n_levels - 1;
    P.Lu = reinterpret_cast<const double *>(Lu);
    P.Lcsr = h->rows_aligned ? h->Lcsr : nullptr;
    P.Lp = h->rowptr_L;
    P.rowptr = h->rowptr;
    P.dinv = h->dinv;
    P.node = h->node;
    P.rn = h->rn;
    P.Z = Z_S;
    P.N = N_S;
    P.M = M_S;
    P.eps = eps;
    P.fuse_mix = fuse_mix ? 1 : 0;
    P.Mout = M_out;
    {
        Trace t(h, ASI_K_MLP_FEATURES, 0.0);
        e = asi::launch_node_feats(P, h->stream);
    }
    if (e != hipSuccess) return hip_fail(h, e, "node features");
    return ASI_OK;
}

asi_status asi_mlp_features(asi_handle h, const double *Z_S, const double *N_S, const double *M_S, double eps,
                            const double *L_val, const double *d_diag, const double *d_sub, uint16_t *F,
                            float *scale) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!Z_S || !N_S || !M_S || !F || !scale) return fail(h, ASI_E_ARG, "null pointer");
    DeviceGuard g(h->device);
    asi::MlpFeatParams P;
    s = mlp_setup(h, Z_S, N_S, M_S, eps, L_val, d_diag, d_sub, P);
    if (s != ASI_OK) return s;
    P.F = F;
    P.scale = scale;
    Trace t(h, ASI_K_MLP_FEATURES, 0.0);
    hipError_t e = asi::launch_mlp_features(P, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "features");
    return ASI_OK;
}

asi_status asi_mlp_correct(asi_handle h, const void *W, const double *Z_S, const double *N_S, const double *M_S,
                           double eps, const double *L_val, const double *d_diag, const double *d_sub,
                           double *out_S) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!W || !Z_S || !N_S || !M_S || !out_S) return fail(h, ASI_E_ARG, "null pointer");
    DeviceGuard g(h->device);
    asi::MlpFeatParams P;
    s = mlp_setup(h, Z_S, N_S, M_S, eps, L_val, d_diag, d_sub, P);
    if (s != ASI_OK) return s;
    // algorithmic bytes: row and column index, Z, N, M in and the result out
    // per entry; two node records of 32 B per entry come from the cache
    Trace t(h, ASI_K_MLP_FORWARD, 40.0 * h->A.nnzS + 32.0 * h->A.n);
    hipError_t e = asi::launch_mlp_correct(P, W, out_S, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "mlp correct");
    return ASI_OK;
}

asi_status asi_mlp_correct_mix(asi_handle h, const void *W, const double *Z_S, const double *N_S, double eps,
                               const double *L_val, const double *d_diag, const double *d_sub, double *M_S,
                               double *out_S) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!W || !Z_S || !N_S || !out_S) return fail(h, ASI_E_ARG, "null pointer");
    if (M_S && M_S == out_S) return fail(h, ASI_E_ARG, "M_S and out_S must be different arrays");
    DeviceGuard g(h->device);
    asi::MlpFeatParams P;
    s = mlp_setup(h, Z_S, N_S, nullptr, eps, L_val, d_diag, d_sub, P, true, M_S);
    if (s != ASI_OK) return s;
    // algorithmic bytes: row and column index, Z, N in and the result (and M) out per entry
    Trace t(h, ASI_K_MLP_FORWARD, (M_S ? 40.0 : 32.0) * h->A.nnzS + 32.0 * h->A.n);
    hipError_t e = asi::launch_mlp_correct(P, W, out_S, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "mlp correct (with Mix)");
    return ASI_OK;
}

static asi_status need_device(asi_handle h) {
    if (!h) return ASI_E_ARG;
    if (h->device < 0) return fail(h, ASI_E_STATE, "host-only handle");
    return ASI_OK;
}

asi_status asi_mlp_pack(asi_handle h, const float *theta, void *packed) {
    asi_status s = need_device(h);
    if (s != ASI_OK) return s;
    if (!theta || !packed) return fail(h, ASI_E_ARG, "null pointer");
    DeviceGuard g(h->device);
    hipError_t e = asi::launch_mlp_pack(theta, packed, h->stream);
    return e == hipSuccess ? ASI_OK : hip_fail(h, e, "mlp pack");
}

asi_status asi_mlp_forward(asi_handle h, const void *packed, const uint16_t *F, int64_t rows, float *y) {
    asi_status s = need_device(h);
    if (s != ASI_OK) return s;
    if (rows < 0 || (rows > 0 && (!packed || !F || !y))) return fail(h, ASI_E_ARG, "bad arguments");
    DeviceGuard g(h->device);
    // algorithmic bytes: 32 B of features in, 4 B out per row
    Trace t(h, ASI_K_MLP_FORWARD, 36.0 * rows);
    hipError_t e = asi::launch_mlp_forward(packed, F, rows, y, h->stream);
    return e == hipSuccess ? ASI_OK : hip_fail(h, e, "mlp forward");
}

asi_status asi_mlp_backward(asi_handle h, const void *packed, const uint16_t *F, const float *dy, int64_t rows,
                            float *grad) {
    asi_status s = need_device(h);
    if (s != ASI_OK) return s;
    if (rows < 0 || (rows > 0 && (!packed || !F || !dy || !grad))) return fail(h, ASI_E_ARG, "bad arguments");
    DeviceGuard g(h->device);
    Trace t(h, ASI_K_MLP_TRAIN, 0.0);
    hipError_t e = asi::launch_mlp_backward(packed, F, dy, rows, grad, h->stream);
    return e == hipSuccess ? ASI_OK : hip_fail(h, e, "mlp backward");
}

asi_status asi_mlp_loss(asi_handle h, const float *y, const float *t, int64_t rows, float *dy, double *loss) {
    asi_status s = need_device(h);
    if (s != ASI_OK) return s;
    if (rows < 0 || (rows > 0 && (!y || !t || !dy || !loss))) return fail(h, ASI_E_ARG, "bad arguments");
    DeviceGuard g(h->device);
    Trace tr(h, ASI_K_MLP_TRAIN, 0.0);
    hipError_t e = asi::launch_mlp_loss(y, t, rows, dy, loss, h->stream);
    return e == hipSuccess ? ASI_OK : hip_fail(h, e, "mlp loss");
}

asi_status asi_mlp_adam(asi_handle h, float *theta, float *m, float *v, const float *grad, float lr, float beta1,
                        float beta2, float eps, int64_t t) {
    asi_status s = need_device(h);
    if (s != ASI_OK) return s;
    if (!theta || !m || !v || !grad || t < 1) return fail(h, ASI_E_ARG, "bad arguments");
    DeviceGuard g(h->device);
    const float c1 = 1.0f - (float)std::pow((double)beta1, (double)t);
    const float c2 = 1.0f - (float)std::pow((double)beta2, (double)t);
    Trace tr(h, ASI_K_MLP_TRAIN, 0.0);
    hipError_t e = asi::launch_adam(theta, m, v, grad, asi::kMlpParams, lr, beta1, beta2, eps, c1, c2, h->stream);
    return e == hipSuccess ? ASI_OK : hip_fail(h, e, "adam");
}

asi_status asi_mlp_apply(asi_handle h, const double *M_S, const float *y, const float *scale, double *out_S) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!M_S || !y || !scale || !out_S) return fail(h, ASI_E_ARG, "null pointer");
    DeviceGuard g(h->device);
    Trace t(h, ASI_K_MLP_FORWARD, 28.0 * h->A.nnzS);
    hipError_t e = asi::launch_mlp_apply(h->A.nnzS, M_S, y, scale, out_S, h->stream);
    return e == hipSuccess ? ASI_OK : hip_fail(h, e, "mlp apply");
}

asi_status asi_diag(asi_handle h, const double *X_S, double *d) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!X_S || !d) return fail(h, ASI_E_ARG, "null pointer");
    DeviceGuard g(h->device);
    hipError_t e = asi::launch_zdiag(h->A.n, h->diagpos, X_S, d, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "diag");
    return ASI_OK;
}

asi_status asi_diag_err1(asi_handle h, const double *d_ref, const double *d_hat, int32_t k, const double *V,
                         const double *lambda, double *sums) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!d_ref || !d_hat || !sums) return fail(h, ASI_E_ARG, "null pointer");
    if (k < 0 || k > asi::kMaxRank) return fail(h, ASI_E_ARG, "k must be in [0, 64]");
    if (k > 0 && (!V || !lambda)) return fail(h, ASI_E_ARG, "null V or lambda with k > 0");
    DeviceGuard g(h->device);
    Trace t(h, ASI_K_DIAG, 16.0 * h->A.n + 8.0 * h->A.n * k);
    hipError_t e = asi::launch_diag_err1(h->A.n, d_ref, d_hat, k, V, lambda, h->red, sums, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "diag_err1");
    return ASI_OK;
}

asi_status asi_trace(asi_handle h, const double *X_S, int32_t k, const double *V, const double *lambda,
                     double *sums) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!X_S || !sums) return fail(h, ASI_E_ARG, "null pointer");
    if (k < 0 || k > asi::kMaxRank) return fail(h, ASI_E_ARG, "k must be in [0, 64]");
    if (k > 0 && (!V || !lambda)) return fail(h, ASI_E_ARG, "null V or lambda with k > 0");
    DeviceGuard g(h->device);
    Trace t(h, ASI_K_DIAG, 16.0 * h->A.n + 8.0 * h->A.n * k);
    hipError_t e = asi::launch_trace(h->A.n, h->diagpos, X_S, k, V, lambda, h->red, sums, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "trace");
    return ASI_OK;
}

// First call after an analysis: every row of L must hold both columns of
// each 2x2 block it touches (then the first Lp[i+1] - Lp[i] lower entries of
// row i of S are exactly row i of L), and the LDS of each level's launch is
// sized by its largest block (sum of its L row lengths). The algorithmic
// bytes count, per row i, row i of L written (8 B an entry) and, for each
// column k of row i, the index and value of row k of L read (12 B an entry);
// A's rows are not counted (their size is not known here).
static asi_status ildl_prepare(asi_handle h) {
    if (h->ildl_ready) return ASI_OK;
    const asi::Analysis &A = h->A;
    auto len = [&](int32_t i) { return A.L_rowptr[i + 1] - A.L_rowptr[i]; };
    double bytes = 0.0;
    for (int32_t i = 0; i < A.n; ++i) {
        const int64_t lower = A.diagpos[i] - A.rowptr[i] - (A.piv[i] == 2 ? 1 : 0);
        if (lower != len(i))
            return fail(h, ASI_E_UNSUPPORTED,
                        "the numeric factorization needs both columns of a 2x2 block in every row of L holding one");
        bytes += 8.0 * len(i);
        for (int64_t p = A.rowptr[i]; p < A.rowptr[i] + len(i); ++p) bytes += 12.0 * len(A.col[p]);
    }
    std::vector<int32_t> ent(A.n_levels, 0);
    for (int32_t l = 0; l < A.n_levels; ++l) {
        int64_t mx = 0;
        auto scan = [&](const std::vector<asi::BlockMeta> &meta, const std::vector<int32_t> &lvl) {
            for (int32_t s = lvl[l]; s < lvl[l + 1]; ++s) {
                const asi::BlockMeta &M = meta[s];
                mx = std::max<int64_t>(mx, len(M.j) + (M.two ? len(M.j + 1) : 0));
            }
        };
        scan(A.meta_small, A.lvl_small);
        scan(A.meta_big, A.lvl_big);
        if (mx > asi::kIldlMaxEntries)
            return fail(h, ASI_E_UNSUPPORTED, "a block's rows of L hold more than 3200 entries together");
        ent[l] = (int32_t)mx;
    }
    h->ildl_lvl_entries.swap(ent);
    h->ildl_bytes = bytes;
    h->ildl_ready = true;
    return ASI_OK;
}

asi_status asi_ildl_numeric(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                            const int32_t *perm, double *L_val, double *d_diag, double *d_sub) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!A_rowptr || !A_col || !A_val || !perm || (!L_val && h->A.nnzL > 0) || !d_diag || !d_sub)
        return fail(h, ASI_E_ARG, "null pointer");
    s = ildl_prepare(h);
    if (s != ASI_OK) return s;
    DeviceGuard g(h->device);
    const asi::Analysis &A = h->A;
    asi::IldlParams P{};
    P.n = A.n;
    P.rowptr = h->rowptr;
    P.col = h->col;
    P.Lp = h->rowptr_L;
    P.piv = h->piv;
    P.Ap = A_rowptr;
    P.Aj = A_col;
    P.Av = A_val;
    P.perm = perm;
    P.iperm = h->iperm;
    P.L = L_val;
    P.dd = d_diag;
    P.ds = d_sub;
    P.status = h->status;
    hipError_t e;
    {
        Trace t(h, ASI_K_ILDL, h->ildl_bytes);
        e = asi::launch_iperm(A.n, perm, h->iperm, h->status, h->stream);
        for (int32_t l = A.n_levels - 1; l >= 0 && e == hipSuccess; --l)
            e = asi::launch_ildl_level(h->meta_small + A.lvl_small[l], A.lvl_small[l + 1] - A.lvl_small[l],
                                       h->meta_big + A.lvl_big[l], A.lvl_big[l + 1] - A.lvl_big[l],
                                       h->ildl_lvl_entries[l], P, h->stream);
    }
    if (e != hipSuccess) return hip_fail(h, e, "numeric factorization");
    return ASI_OK;
}

// Work buffer of asi_ildl_threshold: offsets of its regions (256-byte
// aligned), filled into P when base is not null; returns the total size.
static size_t ildlt_layout(int32_t n, int32_t row_cap, int64_t pool_cap, unsigned char *base, asi::IldlTParams *P) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t nn = (size_t)n, rc = nn * (size_t)row_cap, pc = (size_t)pool_cap;
    const size_t o_scale = take(nn * 8), o_dpiv = take(nn * 8), o_elim = take(nn * 4), o_watch = take(nn * 4),
                 o_iq = take(nn * 4), o_rowcnt = take(nn * 4), o_colptr = take(nn * 8), o_collen = take(nn * 4),
                 o_lc = take(nn * 4), o_lr = take(nn * 4), o_lb = take(nn * 4), o_counts = take(8 * 4),
                 o_top = take(16), o_bsum = take((nn / 1024 + 2) * 8), o_rk = take(rc * 4), o_rv = take(rc * 8),
                 o_pr = take(pc * 4), o_pv = take(pc * 8);
    if (base && P) {
        P->scale = at<double>(base, o_scale);
        P->dpiv = at<double>(base, o_dpiv);
        P->elim = at<int32_t>(base, o_elim);
        P->watch = at<int32_t>(base, o_watch);
        P->iq = at<int32_t>(base, o_iq);
        P->rowcnt = at<int32_t>(base, o_rowcnt);
        P->colptr = at<int64_t>(base, o_colptr);
        P->collen = at<int32_t>(base, o_collen);
        P->list_check = at<int32_t>(base, o_lc);
        P->list_ready = at<int32_t>(base, o_lr);
        P->list_big = at<int32_t>(base, o_lb);
        P->counts = at<int32_t>(base, o_counts);
        P->status = P->counts + 5;
        P->pool_top = at<unsigned long long>(base, o_top);
        P->amax_bits = P->pool_top + 1;
        P->rk = at<int32_t>(base, o_rk);
        P->rv = at<double>(base, o_rv);
        P->pr = at<int32_t>(base, o_pr);
        P->pv = at<double>(base, o_pv);
        P->bsum = at<unsigned long long>(base, o_bsum);
    }
    return off;
}

asi_status asi_ildl_threshold_work_bytes(int32_t n, int32_t row_cap, int64_t pool_cap, size_t *bytes) {
    if (n <= 0 || row_cap <= 0 || pool_cap < 0 || !bytes) return ASI_E_ARG;
    *bytes = ildlt_layout(n, row_cap, pool_cap, nullptr, nullptr);
    return ASI_OK;
}

asi_status asi_ildl_threshold(asi_handle h, int32_t n, const int64_t *A_rowptr, const int32_t *A_col,
                              const double *A_val, const int32_t *q, double tau, int32_t pivoting, int32_t row_cap,
                              int64_t pool_cap, void *work, size_t work_bytes, int64_t *nnzL_h, int64_t *stats_h) {
    asi_status s = need_device(h);
    if (s != ASI_OK) return s;
    h->ildlt_done = false;
    if (n <= 0 || !A_rowptr || !A_col || !A_val || !q || !work || !nnzL_h) return fail(h, ASI_E_ARG, "null pointer");
    if (!(tau >= 0.0)) return fail(h, ASI_E_ARG, "tau must be >= 0");
    if (row_cap <= 0 || row_cap > (1 << 20) || pool_cap < 0) return fail(h, ASI_E_ARG, "bad row_cap or pool_cap");
    if ((reinterpret_cast<uintptr_t>(work) & 255) != 0) return fail(h, ASI_E_ARG, "work must be 256-byte aligned");
    const size_t need = ildlt_layout(n, row_cap, pool_cap, nullptr, nullptr);
    if (work_bytes < need) return fail(h, ASI_E_WORKSPACE, "work buffer smaller than asi_ildl_threshold_work_bytes");
    DeviceGuard g(h->device);
    static bool limits = false;
    hipError_t e = hipSuccess;
    if (!limits) {
        e = asi::ildlt_set_limits();
        if (e != hipSuccess) return hip_fail(h, e, "threshold factorization LDS limit");
        limits = true;
    }
    asi::IldlTParams P{};
    ildlt_layout(n, row_cap, pool_cap, static_cast<unsigned char *>(work), &P);
    P.n = n;
    P.Ap = A_rowptr;
    P.Aj = A_col;
    P.Av = A_val;
    P.q = q;
    P.row_cap = row_cap;
    P.pool_cap = pool_cap;
    P.tau = tau;
    P.alpha = (1.0 + std::sqrt(17.0)) / 8.0;
    P.pivoting = pivoting ? 1 : 0;
    hipStream_t st = h->stream;
    e = hipMemsetAsync(P.counts, 0, 8 * 4, st);
    if (e == hipSuccess) e = hipMemsetAsync(P.pool_top, 0, 16, st);
    if (e == hipSuccess) e = asi::ildlt_setup(P, st);
    unsigned long long amax_bits = 0;
    int32_t cnt[8] = {};
    if (e == hipSuccess) e = hipMemcpyAsync(&amax_bits, P.amax_bits, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(cnt, P.counts, 8 * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(h, e, "threshold factorization set-up");
    if (cnt[5] != 0) return fail(h, ASI_E_ARG, "q is not a permutation of 0..n-1 or A has a column out of range");
    double amax;
    std::memcpy(&amax, &amax_bits, 8);
    P.tiny = 1e-14 * amax;
    P.repl = 1e-8 * amax;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus <= 0)
        cus = 256;
    int32_t done = 0, round = 0;
    for (;; ++round) {
        P.round = round;
        e = asi::ildlt_round(P, 4 * cus, 3 * cus, cus, st);
        if (e == hipSuccess) e = hipMemcpyAsync(cnt, P.counts, 8 * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(h, e, "threshold factorization round");
        if (cnt[5] != 0) {
            const int32_t code = cnt[5];
            if (code == asi::ST_POOL)
                return fail(h, ASI_E_WORKSPACE, "a row of L exceeds row_cap or the columns exceed pool_cap");
            if (code == asi::ST_PIVOT)
                return fail(h, ASI_E_UNSUPPORTED,
                            "a pivot fails the Bunch-Kaufman 1x1 test (a swap or a 2x2 block would be needed); "
                            "the device factorization takes 1x1 pivots in order only");
            return fail(h, ASI_E_UNSUPPORTED, "a Schur column exceeds 3,072 entries or a row of L 2,048");
        }
        if (cnt[3] == n) break;
        if (cnt[3] <= done) return fail(h, ASI_E_HIP, "threshold factorization made no progress");
        done = cnt[3];
    }
    unsigned long long top = 0;
    e = hipMemcpy(&top, P.pool_top, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "threshold factorization size");
    *nnzL_h = (int64_t)top;
    if (stats_h) {
        stats_h[0] = round + 1;
        stats_h[1] = cnt[4];
    }
    h->ildlt = P;
    h->ildlt_done = true;
    h->ildlt_nnz = (int64_t)top;
    return ASI_OK;
}

asi_status asi_ildl_threshold_extract(asi_handle h, int64_t *L_rowptr, int32_t *L_col, double *L_val,
                                      double *d_diag, double *d_sub, int8_t *piv) {
    asi_status s = need_device(h);
    if (s != ASI_OK) return s;
    if (!h->ildlt_done) return fail(h, ASI_E_STATE, "asi_ildl_threshold has not completed on this handle");
    if (!L_rowptr || (h->ildlt_nnz > 0 && (!L_col || !L_val)) || !d_diag || !d_sub || !piv)
        return fail(h, ASI_E_ARG, "null pointer");
    DeviceGuard g(h->device);
    const asi::IldlTParams &P = h->ildlt;
    hipError_t e = asi::ildlt_extract(P, L_rowptr, L_col, L_val, d_diag, d_sub, piv, P.bsum, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "threshold factorization extract");
    return ASI_OK;
}

asi_status asi_za_diag(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                       const int32_t *perm, const double *Z_S, double *d) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!A_rowptr || !A_col || !A_val || !perm || !Z_S || !d) return fail(h, ASI_E_ARG, "null pointer");
    DeviceGuard g(h->device);
    Trace t(h, ASI_K_DIAG, 0.0);
    hipError_t e = asi::launch_iperm(h->A.n, perm, h->iperm, h->status, h->stream);
    if (e == hipSuccess)
        e = asi::launch_za_diag(h->A.n, h->rowptr, h->col, Z_S, A_rowptr, A_col, A_val, perm, h->iperm, d, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "za diag");
    return ASI_OK;
}

asi_status asi_unpermute(asi_handle h, const int32_t *perm, const double *X_S, int64_t *rowptr_out,
                         int32_t *col_out, double *val_out) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!perm || !X_S || !rowptr_out || !col_out || !val_out) return fail(h, ASI_E_ARG, "null pointer");
    const int64_t nnz = h->A.nnzS;
    const char *x0 = reinterpret_cast<const char *>(X_S), *x1 = x0 + nnz * 8;
    const char *v0 = reinterpret_cast<const char *>(val_out), *v1 = v0 + nnz * 8;
    const char *c0 = reinterpret_cast<const char *>(col_out), *c1 = c0 + nnz * 4;
    if ((v0 < x1 && x0 < v1) || (c0 < x1 && x0 < c1)) return fail(h, ASI_E_ARG, "the outputs overlap X_S");
    DeviceGuard g(h->device);
    Trace t(h, ASI_K_DIAG, 0.0);
    hipError_t e = asi::launch_unpermute(h->A.n, h->rowptr, h->col, perm, X_S, h->iperm, h->nf_bsum, rowptr_out,
                                         col_out, val_out, h->status, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "unpermute");
    return ASI_OK;
}

asi_status asi_unpermute_noalloc(asi_handle h, const int32_t *perm, const double *X_S, int64_t *rowptr_out,
                                 int32_t *col_out, double *val_out) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!perm || !X_S || !rowptr_out || !col_out || !val_out) return fail(h, ASI_E_ARG, "null pointer");
    if (h->A.n > asi::kUnpermStaticMaxN)
        return fail(h, ASI_E_ARG, "n exceeds the static scratch of asi_unpermute_noalloc (at most 2,097,152 "
                                  "unknowns); use asi_unpermute");
    const int64_t nnz = h->A.nnzS;
    const char *x0 = reinterpret_cast<const char *>(X_S), *x1 = x0 + nnz * 8;
    const char *v0 = reinterpret_cast<const char *>(val_out), *v1 = v0 + nnz * 8;
    const char *c0 = reinterpret_cast<const char *>(col_out), *c1 = c0 + nnz * 4;
    if ((v0 < x1 && x0 < v1) || (c0 < x1 && x0 < c1)) return fail(h, ASI_E_ARG, "the outputs overlap X_S");
    DeviceGuard g(h->device);
    hipError_t e = asi::launch_unpermute_static(h->device, h->A.n, h->rowptr, h->col, perm, X_S, rowptr_out,
                                                col_out, val_out, h->status, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "unpermute (static scratch)");
    return ASI_OK;
}

// Input checks of the host arrays (debug use): perm a permutation, A a
// valid CSR with sorted unique in-range columns, symmetric in pattern and
// values (exactly, or within tol relative to the larger entry).
asi_status asi_check_matrix(asi_handle h, int32_t n, const int64_t *A_rowptr_h, const int32_t *A_col_h,
                            const double *A_val_h, const int32_t *perm_h, double tol) {
    if (!h) return ASI_E_ARG;
    if (n < 0 || !A_rowptr_h || (n > 0 && (!A_col_h || !A_val_h))) return fail(h, ASI_E_ARG, "null pointer");
    if (perm_h) {
        std::vector<char> seen(n, 0);
        for (int32_t i = 0; i < n; ++i) {
            const int32_t p = perm_h[i];
            if (p < 0 || p >= n || seen[p]) return fail(h, ASI_E_PATTERN, "perm is not a permutation");
            seen[p] = 1;
        }
    }
    if (A_rowptr_h[0] != 0) return fail(h, ASI_E_PATTERN, "A_rowptr[0] must be 0");
    for (int32_t i = 0; i < n; ++i) {
        if (A_rowptr_h[i + 1] < A_rowptr_h[i]) return fail(h, ASI_E_PATTERN, "A_rowptr must be nondecreasing");
        for (int64_t q = A_rowptr_h[i]; q < A_rowptr_h[i + 1]; ++q) {
            const int32_t c = A_col_h[q];
            if (c < 0 || c >= n) return fail(h, ASI_E_PATTERN, "A column out of range");
            if (q > A_rowptr_h[i] && c <= A_col_h[q - 1])
                return fail(h, ASI_E_PATTERN, "A columns must be sorted and unique within each row");
            if (!std::isfinite(A_val_h[q])) return fail(h, ASI_E_NONFINITE, "A has a non-finite value");
        }
    }
    for (int32_t i = 0; i < n; ++i)
        for (int64_t q = A_rowptr_h[i]; q < A_rowptr_h[i + 1]; ++q) {
            const int32_t c = A_col_h[q];
            const int32_t *b = A_col_h + A_rowptr_h[c], *e = A_col_h + A_rowptr_h[c + 1];
            const int32_t *f = std::lower_bound(b, e, i);
            if (f == e || *f != i) return fail(h, ASI_E_PATTERN, "A is not structurally symmetric");
            const double a = A_val_h[q], at = A_val_h[f - A_col_h];
            if (std::fabs(a - at) > tol * std::max(std::fabs(a), std::fabs(at)))
                return fail(h, ASI_E_PATTERN, "A is not symmetric in its values");
        }
    return ASI_OK;
}

static asi::LdlSolveParams ldl_params(asi_handle h) {
    const asi::Analysis &A = h->A;
    asi::LdlSolveParams P{};
    P.n = A.n;
    P.n_levels = A.n_levels;
    P.lvl_rows = A.lvl_rows.data();
    P.rows_fwd = h->solve_fwd;
    P.rows_bwd = h->solve_bwd;
    P.col = h->col;
    P.Ls = h->Ls;
    P.piv = h->piv;
    P.dinv = h->dinv;
    return P;
}

asi_status asi_spmv(asi_handle h, const double *X_S, const double *x, double *y) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!X_S || !x || !y) return fail(h, ASI_E_ARG, "null pointer");
    if (x == y) return fail(h, ASI_E_ARG, "x and y must not alias");
    DeviceGuard g(h->device);
    Trace t(h, ASI_K_DIAG, 12.0 * h->A.nnzS + 16.0 * h->A.n);
    hipError_t e = asi::launch_spmv_s(h->A.n, h->rowptr, h->col, X_S, x, y, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "spmv");
    return ASI_OK;
}

asi_status asi_ldl_solve(asi_handle h, const double *x, double *y) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!x || !y) return fail(h, ASI_E_ARG, "null pointer");
    if (!h->factor_loaded) return fail(h, ASI_E_STATE, "no factor loaded (asi_load_factor)");
    if (h->A.s2u.empty() && h->A.nnzS > 0) return fail(h, ASI_E_UNSUPPORTED, "solves need |S| < 2^31");
    DeviceGuard g(h->device);
    s = ensure_ls(h);
    if (s != ASI_OK) return s;
    Trace t(h, ASI_K_DIAG, 24.0 * h->A.nnzS + 40.0 * h->A.n);
    hipError_t e = asi::launch_ldl_solve(ldl_params(h), x, y, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "ldl solve");
    return ASI_OK;
}

asi_status asi_pcg(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                   const int32_t *perm, const double *b, double *x, double tol, int32_t maxit, int32_t *iters,
                   double *relres) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!A_rowptr || !A_col || !A_val || !perm || !b || !x) return fail(h, ASI_E_ARG, "null pointer");
    if (!(tol > 0.0) || maxit < 0) return fail(h, ASI_E_ARG, "tol must be > 0 and maxit >= 0");
    if (!h->factor_loaded) return fail(h, ASI_E_STATE, "no factor loaded (asi_load_factor)");
    if (h->A.s2u.empty() && h->A.nnzS > 0) return fail(h, ASI_E_UNSUPPORTED, "solves need |S| < 2^31");
    DeviceGuard g(h->device);
    s = ensure_ls(h);
    if (s != ASI_OK) return s;
    const int32_t n = h->A.n;
    const int64_t nn = n;
    double *r = h->cg, *z = r + nn, *p = z + nn, *q = p + nn, *part = q + 2 * nn, *sc = part + 1024;
    double *rz = sc, *rzn = sc + 1, *pq = sc + 2, *rr = sc + 3, *bb = sc + 4;
    const asi::LdlSolveParams L = ldl_params(h);
    hipStream_t st = h->stream;
    int32_t it = 0;
    double res = 0.0;
    hipError_t e;
    {
        Trace t(h, ASI_K_DIAG, 0.0);
        e = asi::launch_iperm(n, perm, h->iperm, h->status, st);
        if (e == hipSuccess) e = asi::launch_fill_f64(nn, 0.0, x, st);
        if (e == hipSuccess) e = asi::launch_copy_f64(nn, b, r, st);
        if (e == hipSuccess) e = asi::launch_dot(nn, b, b, part, bb, st);
        if (e == hipSuccess) e = asi::launch_ldl_solve(L, r, z, st);
        if (e == hipSuccess) e = asi::launch_copy_f64(nn, z, p, st);
        if (e == hipSuccess) e = asi::launch_dot(nn, r, z, part, rz, st);
    }
    if (e != hipSuccess) return hip_fail(h, e, "pcg setup");
    double bnorm2 = 0.0;
    e = hipMemcpyAsync(&bnorm2, bb, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(h, e, "pcg norm");
    if (bnorm2 == 0.0) {
        if (iters) *iters = 0;
        if (relres) *relres = 0.0;
        return asi_sync(h);
    }
    for (it = 1; it <= maxit; ++it) {
        {
            Trace t(h, ASI_K_DIAG, 0.0);
            e = asi::launch_spmv_ahat(n, A_rowptr, A_col, A_val, perm, h->iperm, p, q, st);
            if (e == hipSuccess) e = asi::launch_dot(nn, p, q, part, pq, st);
            if (e == hipSuccess) e = asi::launch_axpy_ratio(nn, rz, pq, 1.0, p, x, st);
            if (e == hipSuccess) e = asi::launch_axpy_ratio(nn, rz, pq, -1.0, q, r, st);
            if (e == hipSuccess) e = asi::launch_dot(nn, r, r, part, rr, st);
        }
        if (e != hipSuccess) return hip_fail(h, e, "pcg step");
        double rnorm2 = 0.0;
        e = hipMemcpyAsync(&rnorm2, rr, 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(h, e, "pcg residual");
        res = std::sqrt(rnorm2 / bnorm2);
        if (!(res == res)) return fail(h, ASI_E_NONFINITE, "pcg breakdown (non-finite residual)");
        if (res <= tol) break;
        {
            Trace t(h, ASI_K_DIAG, 0.0);
            e = asi::launch_ldl_solve(L, r, z, st);
            if (e == hipSuccess) e = asi::launch_dot(nn, r, z, part, rzn, st);
            if (e == hipSuccess) e = asi::launch_xpby_ratio(nn, z, rzn, rz, p, st);
            if (e == hipSuccess) e = asi::launch_copy_f64(1, rzn, rz, st);
        }
        if (e != hipSuccess) return hip_fail(h, e, "pcg preconditioner");
    }
    if (iters) *iters = std::min(it, maxit);
    if (relres) *relres = res;
    return asi_sync(h);
}

asi_status asi_sqmr(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                    const int32_t *perm, const double *b, double *x, double tol, int32_t maxit, int32_t *iters,
                    double *relres) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!A_rowptr || !A_col || !A_val || !perm || !b || !x) return fail(h, ASI_E_ARG, "null pointer");
    if (!(tol > 0.0) || maxit < 0) return fail(h, ASI_E_ARG, "tol must be > 0 and maxit >= 0");
    if (!h->factor_loaded) return fail(h, ASI_E_STATE, "no factor loaded (asi_load_factor)");
    if (h->A.s2u.empty() && h->A.nnzS > 0) return fail(h, ASI_E_UNSUPPORTED, "solves need |S| < 2^31");
    DeviceGuard g(h->device);
    s = ensure_ls(h);
    if (s != ASI_OK) return s;
    const int32_t n = h->A.n;
    const int64_t nn = n;
    // vectors: r (residual), t (products), q (direction), u (preconditioned), d (step)
    double *r = h->cg, *t = r + nn, *q = t + nn, *u = q + nn, *d = u + nn, *part = d + nn, *sc = part + 1024;
    double *rho = sc, *rhon = sc + 1, *sig = sc + 2, *rr = sc + 3, *bb = sc + 4;
    const asi::LdlSolveParams L = ldl_params(h);
    hipStream_t st = h->stream;
    hipError_t e;
    auto read = [&](double *dst, const double *src, int cnt) {
        hipError_t e2 = hipMemcpyAsync(dst, src, 8 * (size_t)cnt, hipMemcpyDeviceToHost, st);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
        return e2;
    };
    {
        Trace tr(h, ASI_K_DIAG, 0.0);
        e = asi::launch_iperm(n, perm, h->iperm, h->status, st);
        if (e == hipSuccess) e = asi::launch_fill_f64(nn, 0.0, x, st);
        if (e == hipSuccess) e = asi::launch_dot(nn, b, b, part, bb, st);
    }
    if (e != hipSuccess) return hip_fail(h, e, "sqmr setup");
    double bnorm2 = 0.0;
    e = read(&bnorm2, bb, 1);
    if (e != hipSuccess) return hip_fail(h, e, "sqmr norm");
    if (bnorm2 == 0.0) {
        if (iters) *iters = 0;
        if (relres) *relres = 0.0;
        return asi_sync(h);
    }
    const double bnorm = std::sqrt(bnorm2);
    // (re)start from the current x: r = b - Ah x, q = M^-1 r, rho = r^T q,
    // tau = ||r||, theta = 0, d = 0; a near-breakdown (a vanishing sigma or
    // rho, or a quasi-residual that is no longer finite) restarts from the
    // last iterate, at most kRestarts times
    constexpr int kRestarts = 8;
    double tau = 0.0, theta = 0.0;
    auto restart = [&]() -> hipError_t {
        Trace tr(h, ASI_K_DIAG, 0.0);
        hipError_t e2 = asi::launch_spmv_ahat(n, A_rowptr, A_col, A_val, perm, h->iperm, x, t, st);
        if (e2 == hipSuccess) e2 = asi::launch_sub(nn, b, t, r, st);
        if (e2 == hipSuccess) e2 = asi::launch_fill_f64(nn, 0.0, d, st);
        if (e2 == hipSuccess) e2 = asi::launch_ldl_solve(L, r, q, st);
        if (e2 == hipSuccess) e2 = asi::launch_dot(nn, r, q, part, rho, st);
        if (e2 == hipSuccess) e2 = asi::launch_dot(nn, r, r, part, rr, st);
        double r2 = 0.0;
        if (e2 == hipSuccess) e2 = read(&r2, rr, 1);
        tau = std::sqrt(r2);
        theta = 0.0;
        return e2;
    };
    e = restart();
    if (e != hipSuccess) return hip_fail(h, e, "sqmr start");
    int32_t it = 0, restarts = 0;
    double res = tau / bnorm;
    int32_t since = 0;  // steps since the last (re)start
    for (it = 1; it <= maxit; ++it) {
        ++since;
        {
            Trace tr(h, ASI_K_DIAG, 0.0);
            e = asi::launch_spmv_ahat(n, A_rowptr, A_col, A_val, perm, h->iperm, q, t, st);
            if (e == hipSuccess) e = asi::launch_dot(nn, q, t, part, sig, st);
            if (e == hipSuccess) e = asi::launch_axpy_ratio(nn, rho, sig, -1.0, t, r, st);  // r -= (rho / sigma) t
            if (e == hipSuccess) e = asi::launch_dot(nn, r, r, part, rr, st);
        }
        if (e != hipSuccess) return hip_fail(h, e, "sqmr step");
        double v[4];
        e = read(v, sc, 4);  // rho, rhon (unused), sigma, ||r||^2
        if (e != hipSuccess) return hip_fail(h, e, "sqmr scalars");
        const double alpha = v[0] / v[2];
        const double theta_n = std::sqrt(v[3]) / tau;
        const double c = 1.0 / std::sqrt(1.0 + theta_n * theta_n);
        const double tau_n = tau * theta_n * c;
        const bool finite = std::isfinite(alpha) && std::isfinite(theta_n) && std::isfinite(tau_n) && c > 0.0;
        if (!finite || v[0] == 0.0 || v[2] == 0.0) {
            if (++restarts > kRestarts)
                return fail(h, ASI_E_NONFINITE, "sqmr breakdown at step " + std::to_string(it) + " after " +
                                                    std::to_string(kRestarts) + " restarts");
            e = restart();
            if (e != hipSuccess) return hip_fail(h, e, "sqmr restart");
            since = 0;
            continue;
        }
        tau = tau_n;
        e = asi::launch_qmr_update(nn, c * c * theta * theta, c * c * alpha, q, d, x, st);
        theta = theta_n;
        if (e != hipSuccess) return hip_fail(h, e, "sqmr update");
        // sqrt(k + 1) tau bounds the residual of the iterate; confirm with the true one
        if (std::sqrt((double)since + 1.0) * tau <= tol * bnorm || it == maxit) {
            {
                Trace tr(h, ASI_K_DIAG, 0.0);
                e = asi::launch_spmv_ahat(n, A_rowptr, A_col, A_val, perm, h->iperm, x, t, st);
                if (e == hipSuccess) e = asi::launch_sub(nn, b, t, u, st);
                if (e == hipSuccess) e = asi::launch_dot(nn, u, u, part, rr, st);
            }
            double tr2 = 0.0;
            if (e == hipSuccess) e = read(&tr2, rr, 1);
            if (e != hipSuccess) return hip_fail(h, e, "sqmr residual");
            res = std::sqrt(tr2) / bnorm;
            if (res <= tol) break;
            if (it < maxit) {
                // the recursion's residual has drifted from the true one (it
                // stalls near the attainable accuracy, eps times the condition
                // of Ah): start a fresh recursion from the iterate, on the true
                // residual; this is no breakdown and is not counted as one
                e = restart();
                if (e != hipSuccess) return hip_fail(h, e, "sqmr restart");
                since = 0;
                continue;
            }
        }
        {
            Trace tr(h, ASI_K_DIAG, 0.0);
            e = asi::launch_ldl_solve(L, r, u, st);
            if (e == hipSuccess) e = asi::launch_dot(nn, r, u, part, rhon, st);
            if (e == hipSuccess) e = asi::launch_xpby_ratio(nn, u, rhon, rho, q, st);  // q = u + (rhon / rho) q
            if (e == hipSuccess) e = asi::launch_copy_f64(1, rhon, rho, st);
        }
        if (e != hipSuccess) return hip_fail(h, e, "sqmr preconditioner");
    }
    if (iters) *iters = std::min(it, maxit);
    if (relres) *relres = res;
    return asi_sync(h);
}

// ---- several right-hand sides: block PCG and block SQMR --------------------

// Work of the block solves, in float64 slots, each region 256-byte aligned:
// seven interleaved blocks of nv vectors (r, t, q, u, d, and the right-hand
// sides and iterates), the dot partials, the scalars (rho, rhon, sigma, rr,
// bb, a second rr, per vector), the QMR update coefficients, the active
// flags and the restart flags.
struct BlockSolveLayout {
    size_t r, t, q, u, d, b, x, part, sc, coef, act, sel, total;
};

static size_t up32(size_t x) { return (x + 31) / 32 * 32; }

static BlockSolveLayout block_layout(int64_t n, int32_t nv) {
    BlockSolveLayout B{};
    const size_t blk = up32((size_t)nv * (size_t)n);
    size_t cur = 0;
    B.r = cur;
    cur += blk;
    B.t = cur;
    cur += blk;
    B.q = cur;
    cur += blk;
    B.u = cur;
    cur += blk;
    B.d = cur;
    cur += blk;
    B.b = cur;
    cur += blk;
    B.x = cur;
    cur += blk;
    B.part = cur;
    cur += up32((size_t)nv * asi::dot_blocks(n));
    B.sc = cur;
    cur += up32(6 * (size_t)nv);
    B.coef = cur;
    cur += up32(2 * (size_t)nv);
    B.act = cur;
    cur += up32((size_t)nv);
    B.sel = cur;
    cur += up32((size_t)nv);
    B.total = cur;
    return B;
}

asi_status asi_block_solve_work_bytes(int32_t n, int32_t nrhs, size_t *bytes) {
    if (n < 1 || nrhs < 1 || nrhs > asi::kMaxRhs || !bytes) return ASI_E_ARG;
    *bytes = block_layout(n, nrhs).total * 8;
    return ASI_OK;
}

static asi_status block_krylov_run(asi_handle h, int method, const int64_t *A_rowptr, const int32_t *A_col,
                                   const double *A_val, const int32_t *perm, int32_t nv, const double *B, double *X,
                                   double tol, int32_t maxit, double *work, int32_t *iters, double *relres,
                                   int32_t *sweeps);

// nv systems Ah x_v = b_v at once (B, X column-major, vector v at B + v n),
// method 0: PCG, 1: SQMR, each vector with its own scalars and its own
// stopping test; a stopped vector is left alone by the masked updates. The
// iteration works on interleaved copies. iters[v], relres[v]: host outputs;
// *sweeps (nullable): block iterations taken.
static asi_status block_krylov(asi_handle h, int method, const int64_t *A_rowptr, const int32_t *A_col,
                               const double *A_val, const int32_t *perm, int32_t nv, const double *B, double *X,
                               double tol, int32_t maxit, double *work, int32_t *iters, double *relres,
                               int32_t *sweeps) {
    const BlockSolveLayout W = block_layout(h->A.n, nv);
    double *bi = work + W.b, *xi = work + W.x;
    hipError_t e = asi::launch_interleave(h->A.n, nv, true, B, bi, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "block solve layout");
    asi_status s = block_krylov_run(h, method, A_rowptr, A_col, A_val, perm, nv, bi, xi, tol, maxit, work, iters,
                                    relres, sweeps);
    if (s != ASI_OK) return s;
    e = asi::launch_interleave(h->A.n, nv, false, xi, X, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "block solve layout");
    return asi_sync(h);
}

static asi_status block_krylov_run(asi_handle h, int method, const int64_t *A_rowptr, const int32_t *A_col,
                                   const double *A_val, const int32_t *perm, int32_t nv, const double *B, double *X,
                                   double tol, int32_t maxit, double *work, int32_t *iters, double *relres,
                                   int32_t *sweeps) {
    const int32_t n = h->A.n;
    const int64_t nn = n, nnv = nn * nv;
    const BlockSolveLayout W = block_layout(n, nv);
    double *r = work + W.r, *t = work + W.t, *q = work + W.q, *u = work + W.u, *d = work + W.d,
           *part = work + W.part, *sc = work + W.sc, *coef_d = work + W.coef;
    int32_t *act_d = reinterpret_cast<int32_t *>(work + W.act);
    int32_t *sel_d = reinterpret_cast<int32_t *>(work + W.sel);
    double *rho = sc, *rhon = sc + nv, *sig = sc + 2 * nv, *rr = sc + 3 * nv, *bb = sc + 4 * nv, *rr2 = sc + 5 * nv;
    const asi::LdlSolveParams L = ldl_params(h);
    hipStream_t st = h->stream;
    hipError_t e;
    auto read = [&](double *dst, const double *src, size_t cnt) {
        hipError_t e2 = hipMemcpyAsync(dst, src, 8 * cnt, hipMemcpyDeviceToHost, st);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
        return e2;
    };
    std::vector<int32_t> act(nv, 0);
    std::vector<double> coef(2 * (size_t)nv, 0.0), bn(nv, 0.0), bn2(nv, 0.0), hs(6 * (size_t)nv, 0.0);
    auto send_act = [&]() {
        hipError_t e2 = hipMemcpyAsync(act_d, act.data(), 4 * (size_t)nv, hipMemcpyHostToDevice, st);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
        return e2;
    };
    auto any_active = [&]() {
        for (int32_t v = 0; v < nv; ++v)
            if (act[v]) return true;
        return false;
    };
    for (int32_t v = 0; v < nv; ++v) {
        iters[v] = 0;
        relres[v] = 0.0;
    }
    if (sweeps) *sweeps = 0;
    {
        Trace tr(h, ASI_K_DIAG, 0.0);
        e = asi::launch_iperm(n, perm, h->iperm, h->status, st);
        if (e == hipSuccess) e = asi::launch_fill_f64(nnv, 0.0, X, st);
        if (e == hipSuccess) e = asi::launch_dot_m(nn, nv, B, B, part, bb, st);
    }
    if (e == hipSuccess) e = read(bn.data(), bb, nv);
    if (e != hipSuccess) return hip_fail(h, e, "block solve setup");
    for (int32_t v = 0; v < nv; ++v) {
        if (!std::isfinite(bn[v])) return fail(h, ASI_E_NONFINITE, "block solve: non-finite right-hand side");
        act[v] = bn[v] > 0.0;
        bn2[v] = bn[v];
        bn[v] = std::sqrt(bn[v]);
    }
    if (!any_active()) return asi_sync(h);
    e = send_act();
    if (e != hipSuccess) return hip_fail(h, e, "block solve flags");
    int32_t it = 0;
    if (method == 0) {
        // conjugate gradients: r = b, z = M^-1 r (in u), p = z (in q), rz = r.z (in rho)
        {
            Trace tr(h, ASI_K_DIAG, 0.0);
            e = asi::launch_copy_f64(nnv, B, r, st);
            if (e == hipSuccess) e = asi::launch_ldl_solve_m(L, nv, r, u, st);
            if (e == hipSuccess) e = asi::launch_copy_f64(nnv, u, q, st);
            if (e == hipSuccess) e = asi::launch_dot_m(nn, nv, r, u, part, rho, st);
        }
        if (e != hipSuccess) return hip_fail(h, e, "block pcg setup");
        for (it = 1; it <= maxit; ++it) {
            {
                Trace tr(h, ASI_K_DIAG, 0.0);
                e = asi::launch_spmv_ahat_m(n, nv, A_rowptr, A_col, A_val, perm, h->iperm, q, t, st);
                if (e == hipSuccess) e = asi::launch_dot_m(nn, nv, q, t, part, sig, st);
                if (e == hipSuccess) e = asi::launch_axpy_ratio_m(nn, nv, rho, sig, act_d, 1.0, q, X, st);
                if (e == hipSuccess) e = asi::launch_axpy_ratio_m(nn, nv, rho, sig, act_d, -1.0, t, r, st);
                if (e == hipSuccess) e = asi::launch_dot_m(nn, nv, r, r, part, rr, st);
            }
            if (e == hipSuccess) e = read(hs.data(), sc, 4 * (size_t)nv);
            if (e != hipSuccess) return hip_fail(h, e, "block pcg step");
            if (sweeps) *sweeps = it;
            for (int32_t v = 0; v < nv; ++v) {
                if (!act[v]) continue;
                const double res = std::sqrt(hs[3 * nv + v] / bn2[v]);
                if (!(res == res)) return fail(h, ASI_E_NONFINITE, "block pcg breakdown (non-finite residual)");
                iters[v] = it;
                relres[v] = res;
                if (res <= tol) act[v] = 0;
            }
            if (!any_active()) break;
            e = send_act();
            {
                Trace tr(h, ASI_K_DIAG, 0.0);
                if (e == hipSuccess) e = asi::launch_ldl_solve_m(L, nv, r, u, st);
                if (e == hipSuccess) e = asi::launch_dot_m(nn, nv, r, u, part, rhon, st);
                if (e == hipSuccess) e = asi::launch_xpby_ratio_m(nn, nv, u, rhon, rho, act_d, q, st);
                if (e == hipSuccess) e = asi::launch_copy_f64(nv, rhon, rho, st);
            }
            if (e != hipSuccess) return hip_fail(h, e, "block pcg preconditioner");
        }
        return asi_sync(h);
    }
    // simplified QMR, per vector as in asi_sqmr (restart from the last
    // iterate on a near-breakdown, at most kRestarts times per vector)
    constexpr int kRestarts = 8;
    std::vector<double> tau(nv, 0.0), theta(nv, 0.0);
    std::vector<int32_t> since(nv, 0), restarts(nv, 0);
    // restart the vectors flagged in need: r = b - Ah x, d = 0, q = M^-1 r,
    // rho = r.q, tau = ||r|| for those only (the others' vectors and scalars
    // are left as they are; t, u and the second rr slot are scratch)
    auto restart_flagged = [&](const std::vector<int32_t> &need) -> hipError_t {
        hipError_t e2 = hipMemcpyAsync(sel_d, need.data(), 4 * (size_t)nv, hipMemcpyHostToDevice, st);
        {
            Trace tr(h, ASI_K_DIAG, 0.0);
            if (e2 == hipSuccess)
                e2 = asi::launch_spmv_ahat_m(n, nv, A_rowptr, A_col, A_val, perm, h->iperm, X, t, st);
            if (e2 == hipSuccess) e2 = asi::launch_select_m(nn, nv, sel_d, 1, B, t, r, st);
            if (e2 == hipSuccess) e2 = asi::launch_select_m(nn, nv, sel_d, 2, nullptr, nullptr, d, st);
            if (e2 == hipSuccess) e2 = asi::launch_ldl_solve_m(L, nv, r, u, st);
            if (e2 == hipSuccess) e2 = asi::launch_select_m(nn, nv, sel_d, 0, nullptr, u, q, st);
            if (e2 == hipSuccess) e2 = asi::launch_dot_m(nn, nv, r, q, part, rr2, st);
            if (e2 == hipSuccess) e2 = asi::launch_select_m(1, nv, sel_d, 0, nullptr, rr2, rho, st);
            if (e2 == hipSuccess) e2 = asi::launch_dot_m(nn, nv, r, r, part, rr2, st);
        }
        if (e2 == hipSuccess) e2 = read(hs.data() + 5 * nv, rr2, nv);
        for (int32_t v = 0; v < nv; ++v) {
            if (!need[v]) continue;
            tau[v] = std::sqrt(hs[5 * nv + v]);
            theta[v] = 0.0;
            since[v] = 0;
        }
        return e2;
    };
    {
        Trace tr(h, ASI_K_DIAG, 0.0);
        e = asi::launch_spmv_ahat_m(n, nv, A_rowptr, A_col, A_val, perm, h->iperm, X, t, st);
        if (e == hipSuccess) e = asi::launch_sub(nnv, B, t, r, st);
        if (e == hipSuccess) e = asi::launch_fill_f64(nnv, 0.0, d, st);
        if (e == hipSuccess) e = asi::launch_ldl_solve_m(L, nv, r, q, st);
        if (e == hipSuccess) e = asi::launch_dot_m(nn, nv, r, q, part, rho, st);
        if (e == hipSuccess) e = asi::launch_dot_m(nn, nv, r, r, part, rr, st);
    }
    if (e == hipSuccess) e = read(hs.data(), sc, 4 * (size_t)nv);
    if (e != hipSuccess) return hip_fail(h, e, "block sqmr start");
    for (int32_t v = 0; v < nv; ++v) {
        tau[v] = std::sqrt(hs[3 * nv + v]);
        relres[v] = bn[v] > 0.0 ? tau[v] / bn[v] : 0.0;
    }
    std::vector<int32_t> need_true(nv, 0), need_restart(nv, 0);
    for (it = 1; it <= maxit; ++it) {
        {
            Trace tr(h, ASI_K_DIAG, 0.0);
            e = asi::launch_spmv_ahat_m(n, nv, A_rowptr, A_col, A_val, perm, h->iperm, q, t, st);
            if (e == hipSuccess) e = asi::launch_dot_m(nn, nv, q, t, part, sig, st);
            if (e == hipSuccess) e = asi::launch_axpy_ratio_m(nn, nv, rho, sig, act_d, -1.0, t, r, st);
            if (e == hipSuccess) e = asi::launch_dot_m(nn, nv, r, r, part, rr, st);
        }
        if (e == hipSuccess) e = read(hs.data(), sc, 4 * (size_t)nv);
        if (e != hipSuccess) return hip_fail(h, e, "block sqmr step");
        if (sweeps) *sweeps = it;
        bool any_true = false;
        for (int32_t v = 0; v < nv; ++v) {
            need_true[v] = need_restart[v] = 0;
            coef[2 * v] = coef[2 * v + 1] = 0.0;
            if (!act[v]) continue;
            iters[v] = it;
            const double rh = hs[v], sg = hs[2 * nv + v];
            const double alpha = rh / sg;
            const double theta_n = std::sqrt(hs[3 * nv + v]) / tau[v];
            const double c = 1.0 / std::sqrt(1.0 + theta_n * theta_n);
            const double tau_n = tau[v] * theta_n * c;
            const bool finite = std::isfinite(alpha) && std::isfinite(theta_n) && std::isfinite(tau_n) && c > 0.0;
            if (!finite || rh == 0.0 || sg == 0.0) {
                if (++restarts[v] > kRestarts)
                    return fail(h, ASI_E_NONFINITE, "block sqmr breakdown of vector " + std::to_string(v) +
                                                        " at step " + std::to_string(it) + " after " +
                                                        std::to_string(kRestarts) + " restarts");
                need_restart[v] = 1;  // coefficients (0, 0): d = 0 and x unchanged
                continue;
            }
            coef[2 * v] = c * c * theta[v] * theta[v];
            coef[2 * v + 1] = c * c * alpha;
            tau[v] = tau_n;
            theta[v] = theta_n;
            ++since[v];
            if (std::sqrt((double)since[v] + 1.0) * tau[v] <= tol * bn[v] || it == maxit) {
                need_true[v] = 1;
                any_true = true;
            }
        }
        e = hipMemcpyAsync(coef_d, coef.data(), 16 * (size_t)nv, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = asi::launch_qmr_update_m(nn, nv, coef_d, act_d, q, d, X, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // coef (host) may change after this
        if (e != hipSuccess) return hip_fail(h, e, "block sqmr update");
        if (any_true) {
            {
                Trace tr(h, ASI_K_DIAG, 0.0);
                e = asi::launch_spmv_ahat_m(n, nv, A_rowptr, A_col, A_val, perm, h->iperm, X, t, st);
                if (e == hipSuccess) e = asi::launch_sub(nnv, B, t, u, st);
                if (e == hipSuccess) e = asi::launch_dot_m(nn, nv, u, u, part, rr2, st);
            }
            if (e == hipSuccess) e = read(hs.data() + 5 * nv, rr2, nv);
            if (e != hipSuccess) return hip_fail(h, e, "block sqmr residual");
            for (int32_t v = 0; v < nv; ++v) {
                if (!need_true[v]) continue;
                relres[v] = std::sqrt(hs[5 * nv + v]) / bn[v];
                if (relres[v] <= tol)
                    act[v] = 0;
                else if (it < maxit)
                    need_restart[v] = 1;  // stalled recursion: a fresh one from the iterate, as in asi_sqmr
            }
        }
        if (!any_active()) break;
        e = send_act();
        {
            Trace tr(h, ASI_K_DIAG, 0.0);
            if (e == hipSuccess) e = asi::launch_ldl_solve_m(L, nv, r, u, st);
            if (e == hipSuccess) e = asi::launch_dot_m(nn, nv, r, u, part, rhon, st);
            if (e == hipSuccess) e = asi::launch_xpby_ratio_m(nn, nv, u, rhon, rho, act_d, q, st);
            if (e == hipSuccess) e = asi::launch_copy_f64(nv, rhon, rho, st);
        }
        if (e != hipSuccess) return hip_fail(h, e, "block sqmr preconditioner");
        bool any_restart = false;
        for (int32_t v = 0; v < nv; ++v) {
            need_restart[v] = need_restart[v] && act[v];
            any_restart = any_restart || need_restart[v];
        }
        if (any_restart) {
            e = restart_flagged(need_restart);
            if (e != hipSuccess) return hip_fail(h, e, "block sqmr restart");
        }
    }
    return asi_sync(h);
}

static asi_status block_solve_entry(asi_handle h, int method, const int64_t *A_rowptr, const int32_t *A_col,
                                    const double *A_val, const int32_t *perm, int32_t nrhs, const double *B,
                                    double *X, double tol, int32_t maxit, void *work, size_t work_bytes,
                                    int32_t *iters, double *relres) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!A_rowptr || !A_col || !A_val || !perm || !B || !X || !work || !iters || !relres)
        return fail(h, ASI_E_ARG, "null pointer");
    if (nrhs < 1 || nrhs > asi::kMaxRhs) return fail(h, ASI_E_ARG, "nrhs must be in 1..8");
    if (!(tol > 0.0) || maxit < 0) return fail(h, ASI_E_ARG, "tol must be > 0 and maxit >= 0");
    if (!h->factor_loaded) return fail(h, ASI_E_STATE, "no factor loaded (asi_load_factor)");
    if (h->A.s2u.empty() && h->A.nnzS > 0) return fail(h, ASI_E_UNSUPPORTED, "solves need |S| < 2^31");
    if ((reinterpret_cast<uintptr_t>(work) & 255) != 0) return fail(h, ASI_E_ARG, "work must be 256-byte aligned");
    if (work_bytes < block_layout(h->A.n, nrhs).total * 8)
        return fail(h, ASI_E_WORKSPACE, "work smaller than asi_block_solve_work_bytes(n, nrhs)");
    DeviceGuard g(h->device);
    s = ensure_ls(h);
    if (s != ASI_OK) return s;
    return block_krylov(h, method, A_rowptr, A_col, A_val, perm, nrhs, B, X, tol, maxit, static_cast<double *>(work),
                        iters, relres, nullptr);
}

asi_status asi_pcg_block(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                         const int32_t *perm, int32_t nrhs, const double *B, double *X, double tol, int32_t maxit,
                         void *work, size_t work_bytes, int32_t *iters, double *relres) {
    return block_solve_entry(h, 0, A_rowptr, A_col, A_val, perm, nrhs, B, X, tol, maxit, work, work_bytes, iters,
                             relres);
}

asi_status asi_sqmr_block(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                          const int32_t *perm, int32_t nrhs, const double *B, double *X, double tol, int32_t maxit,
                          void *work, size_t work_bytes, int32_t *iters, double *relres) {
    return block_solve_entry(h, 1, A_rowptr, A_col, A_val, perm, nrhs, B, X, tol, maxit, work, work_bytes, iters,
                             relres);
}

// ---- the eigen step: thick-restart (block) Lanczos --------------------------

// Work buffer of asi_eigs_error, in float64 slots, each region 256-byte aligned:
// two bases of m + b columns (the current one and the one a restart builds),
// the block X V_src, the Gram-Schmidt partials and coefficients, the Ritz
// coefficients sent for a restart or the result, the block solves' work.
struct EigLayout {
    size_t v0, v1, y, part, hc, Y, solve, total_bytes;
};

static EigLayout eig_layout(int64_t n, int32_t m, int32_t b) {
    EigLayout E{};
    const size_t cols = (size_t)m + b;
    size_t cur = 0;
    E.v0 = cur;
    cur += up32(cols * (size_t)n);
    E.v1 = cur;
    cur += up32(cols * (size_t)n);
    E.y = cur;
    cur += up32((size_t)b * n);
    E.part = cur;
    cur += up32(std::max(cols * (size_t)asi::gs_blocks(n), (size_t)asi::dot_blocks(n)));  // also launch_dot's partials
    E.hc = cur;
    cur += up32(2 * cols + 1);
    E.Y = cur;
    cur += up32((size_t)m * m);
    E.solve = cur;
    cur += block_layout(n, b).total;
    E.total_bytes = cur * 8;
    return E;
}

asi_status asi_eigs_work_bytes(int32_t n, int32_t m, int32_t block, size_t *bytes) {
    if (n < 2 || m < 1 || m > 256 || block < 1 || block > asi::kMaxRhs || !bytes) return ASI_E_ARG;
    *bytes = eig_layout(n, m, block).total_bytes;
    return ASI_OK;
}

asi_status asi_eigs_error(asi_handle h, const int64_t *A_rowptr, const int32_t *A_col, const double *A_val,
                          const int32_t *perm, const double *X_S, const double *v0, int32_t k, int32_t m,
                          int32_t block, double tol, int32_t max_restarts, int32_t method, double solve_tol,
                          int32_t solve_maxit, void *work, size_t work_bytes, double *lambda, double *V,
                          double *resid, double *stats) {
    asi_status s = need_ready(h);
    if (s != ASI_OK) return s;
    if (!A_rowptr || !A_col || !A_val || !perm || !X_S || !v0 || !work || !lambda || !V)
        return fail(h, ASI_E_ARG, "null pointer");
    if (!h->factor_loaded) return fail(h, ASI_E_STATE, "no factor loaded (asi_load_factor)");
    if (h->A.s2u.empty() && h->A.nnzS > 0) return fail(h, ASI_E_UNSUPPORTED, "solves need |S| < 2^31");
    const int32_t n = h->A.n, b = block;
    if (k < 1 || k > 64) return fail(h, ASI_E_ARG, "k must be in 1..64");
    if (b < 1 || b > asi::kMaxRhs) return fail(h, ASI_E_ARG, "block must be in 1..8");
    if (m < k + b + 1 || m > 256 || (int64_t)m + b > n)
        return fail(h, ASI_E_ARG, "the basis size m must satisfy k + block + 1 <= m <= 256 and m + block <= n");
    if (!(tol > 0.0) || max_restarts < 0 || (method != 0 && method != 1) || !(solve_tol > 0.0) || solve_maxit < 0)
        return fail(h, ASI_E_ARG, "tol > 0, max_restarts >= 0, method 0 or 1, solve_tol > 0, solve_maxit >= 0");
    if ((reinterpret_cast<uintptr_t>(work) & 255) != 0) return fail(h, ASI_E_ARG, "work must be 256-byte aligned");
    const EigLayout E = eig_layout(n, m, b);
    if (work_bytes < E.total_bytes)
        return fail(h, ASI_E_WORKSPACE, "work smaller than asi_eigs_work_bytes(n, m, block) = " +
                                             std::to_string(E.total_bytes));
    DeviceGuard g(h->device);
    s = ensure_ls(h);
    if (s != ASI_OK) return s;
    const int64_t nn = n;
    double *base = static_cast<double *>(work);
    double *Vc = base + E.v0, *Vn = base + E.v1, *y = base + E.y, *part = base + E.part, *hc = base + E.hc,
           *Yd = base + E.Y, *swork = base + E.solve;
    const int32_t cols = m + b;  // basis slots: m projected vectors, then the residual block
    hipStream_t st = h->stream;
    hipError_t e;
    auto read = [&](double *dst, const double *src, size_t cnt) {
        hipError_t e2 = hipMemcpyAsync(dst, src, 8 * cnt, hipMemcpyDeviceToHost, st);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
        return e2;
    };
    auto send = [&](double *dst, const double *src, size_t cnt) {
        hipError_t e2 = hipMemcpyAsync(dst, src, 8 * cnt, hipMemcpyHostToDevice, st);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
        return e2;
    };
    std::vector<double> coef(2 * (size_t)cols + 1);
    // orthogonalise column c of Vc against columns 0 .. c-1 (two classical
    // Gram-Schmidt passes); h receives the summed coefficients, returns ||w||^2
    auto orthogonalise = [&](int32_t c, double &norm2) -> hipError_t {
        double *w = Vc + (size_t)c * nn;
        hipError_t e2 = hipSuccess;
        {
            Trace t(h, ASI_K_DIAG, 0.0);
            if (c > 0) {
                e2 = asi::launch_gs_dots(nn, c, Vc, w, part, hc, st);
                if (e2 == hipSuccess) e2 = asi::launch_gs_update(nn, c, Vc, hc, w, st);
                if (e2 == hipSuccess) e2 = asi::launch_gs_dots(nn, c, Vc, w, part, hc + cols, st);
                if (e2 == hipSuccess) e2 = asi::launch_gs_update(nn, c, Vc, hc + cols, w, st);
            }
            if (e2 == hipSuccess) e2 = asi::launch_dot(nn, w, w, part, hc + 2 * cols, st);
        }
        if (e2 == hipSuccess) e2 = read(coef.data(), hc, 2 * (size_t)cols + 1);
        norm2 = coef[2 * cols];
        return e2;
    };
    // start block: the columns of v0, orthonormalised in order
    e = asi::launch_copy_f64((int64_t)b * nn, v0, Vc, st);
    if (e != hipSuccess) return hip_fail(h, e, "eigs start block");
    for (int32_t c = 0; c < b; ++c) {
        double nrm2 = 0.0, raw2 = 0.0;
        e = asi::launch_dot(nn, Vc + (size_t)c * nn, Vc + (size_t)c * nn, part, hc + 2 * cols, st);
        if (e == hipSuccess) e = read(&raw2, hc + 2 * cols, 1);
        if (e == hipSuccess) e = orthogonalise(c, nrm2);
        if (e != hipSuccess) return hip_fail(h, e, "eigs start block");
        if (!std::isfinite(raw2) || !(nrm2 > 1e-20 * raw2))
            return fail(h, ASI_E_ARG, "v0 must have finite, linearly independent columns");
        e = asi::launch_scale(nn, 1.0 / std::sqrt(nrm2), Vc + (size_t)c * nn, st);
        if (e != hipSuccess) return hip_fail(h, e, "eigs start block");
    }

    const size_t ct = (size_t)cols, mm = (size_t)m;
    std::vector<double> T(ct * ct, 0.0), Tm, theta(mm), Y(mm * mm), Ysel, res(mm);
    std::vector<int32_t> order(mm), its(b);
    std::vector<double> rel(b);
    double applications = 0.0, ksteps = 0.0, maxrel = 0.0, tnorm = 0.0;
    int32_t restarts = 0, q0 = b;
    for (;;) {
        int32_t meff = m;
        bool invariant = false;
        for (int32_t q = q0; q < cols && !invariant; q += b) {
            const int32_t nb = std::min(b, cols - q), src = q - b;
            double *Vs = Vc + (size_t)src * nn, *Wq = Vc + (size_t)q * nn;
            // W = A^-1 V_src - X V_src for the nb sources
            int32_t sweeps = 0;
            s = block_krylov(h, method, A_rowptr, A_col, A_val, perm, nb, Vs, Wq, solve_tol, solve_maxit, swork,
                             its.data(), rel.data(), &sweeps);
            if (s != ASI_OK) return s;
            applications += nb;
            ksteps += sweeps;
            for (int32_t v = 0; v < nb; ++v) maxrel = std::max(maxrel, rel[v]);
            {
                Trace t(h, ASI_K_DIAG, 0.0);
                e = asi::launch_spmv_s_m(n, nb, h->rowptr, h->col, X_S, Vs, y, st);
                if (e == hipSuccess) e = asi::launch_sub((int64_t)nb * nn, Wq, y, Wq, st);
            }
            if (e != hipSuccess) return hip_fail(h, e, "eigs application");
            for (int32_t v = 0; v < nb; ++v) {
                const int32_t c = q + v, sv = src + v;
                double nrm2 = 0.0;
                e = orthogonalise(c, nrm2);
                if (e != hipSuccess) return hip_fail(h, e, "eigs expansion");
                for (int32_t r = 0; r < c; ++r) {
                    const double val = coef[r] + coef[cols + r];
                    if (!std::isfinite(val)) return fail(h, ASI_E_NONFINITE, "eigs: non-finite projection");
                    T[(size_t)r * ct + sv] = T[(size_t)sv * ct + r] = val;
                    tnorm = std::max(tnorm, std::fabs(val));
                }
                const double beta = std::sqrt(nrm2);
                if (!std::isfinite(beta)) return fail(h, ASI_E_NONFINITE, "eigs: non-finite basis vector");
                tnorm = std::max(tnorm, beta);
                T[(size_t)c * ct + sv] = T[(size_t)sv * ct + c] = beta;
                if (beta <= 1e-13 * tnorm) {
                    if (b > 1)
                        return fail(h, ASI_E_NONFINITE, "eigs: the block became linearly dependent (use block 1 "
                                                        "or another v0)");
                    meff = c;  // E maps the basis into itself: the Ritz pairs are exact
                    invariant = true;
                    break;
                }
                e = asi::launch_scale(nn, 1.0 / beta, Vc + (size_t)c * nn, st);
                if (e != hipSuccess) return hip_fail(h, e, "eigs normalisation");
            }
        }
        // Rayleigh-Ritz on T(0:meff, 0:meff)
        Tm.assign((size_t)meff * meff, 0.0);
        for (int32_t r = 0; r < meff; ++r)
            for (int32_t c = 0; c < meff; ++c) Tm[(size_t)r * meff + c] = T[(size_t)r * ct + c];
        s = asi_dense_symeig(meff, Tm.data(), theta.data(), Y.data());
        if (s != ASI_OK) return fail(h, s, "eigs: projected eigenproblem failed");
        order.resize(meff);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t c) { return std::fabs(theta[a]) > std::fabs(theta[c]); });
        if (invariant && meff < k)
            return fail(h, ASI_E_NONFINITE, "eigs: invariant subspace of dimension " + std::to_string(meff) +
                                                " below k (choose another v0)");
        // residual of Ritz pair t: || C y_t ||, C = T(m : m + b, 0 : m) the
        // coupling of the residual block (zero for an invariant subspace)
        for (int32_t t = 0; t < meff; ++t) {
            double r2 = 0.0;
            if (!invariant)
                for (int32_t r = m; r < cols; ++r) {
                    double z = 0.0;
                    for (int32_t c = 0; c < m; ++c) z += T[(size_t)r * ct + c] * Y[(size_t)c * meff + order[t]];
                    r2 += z * z;
                }
            res[t] = std::sqrt(r2);
        }
        int32_t conv = 0;
        for (int32_t t = 0; t < k; ++t)
            if (res[t] <= tol * std::fabs(theta[order[t]])) ++conv;
        if (conv == k || restarts >= max_restarts || invariant) {
            Ysel.assign((size_t)meff * k, 0.0);
            for (int32_t r = 0; r < meff; ++r)
                for (int32_t t = 0; t < k; ++t) Ysel[(size_t)r * k + t] = Y[(size_t)r * meff + order[t]];
            e = send(Yd, Ysel.data(), Ysel.size());
            if (e == hipSuccess) e = asi::launch_basis_combine(nn, meff, k, Vc, Yd, V, true, st);
            if (e != hipSuccess) return hip_fail(h, e, "eigs result");
            for (int32_t t = 0; t < k; ++t) {
                lambda[t] = theta[order[t]];
                if (resid) resid[t] = theta[order[t]] != 0.0 ? res[t] / std::fabs(theta[order[t]]) : res[t];
            }
            if (stats) {
                stats[0] = applications;
                stats[1] = ksteps;
                stats[2] = restarts;
                stats[3] = conv;
                stats[4] = maxrel;
            }
            return asi_sync(h);
        }
        // thick restart: keep p Ritz vectors and the residual block
        const int32_t p = std::min(k + (m - k) / 2, m - b);
        Ysel.assign((size_t)m * p, 0.0);
        for (int32_t r = 0; r < m; ++r)
            for (int32_t t = 0; t < p; ++t) Ysel[(size_t)r * p + t] = Y[(size_t)r * mm + order[t]];
        e = send(Yd, Ysel.data(), Ysel.size());
        if (e == hipSuccess) e = asi::launch_basis_combine(nn, m, p, Vc, Yd, Vn, false, st);
        if (e == hipSuccess)
            e = asi::launch_copy_f64((int64_t)b * nn, Vc + (size_t)m * nn, Vn + (size_t)p * nn, st);
        if (e != hipSuccess) return hip_fail(h, e, "eigs restart");
        std::swap(Vc, Vn);
        std::fill(T.begin(), T.end(), 0.0);
        for (int32_t t = 0; t < p; ++t) T[(size_t)t * ct + t] = theta[order[t]];
        q0 = p + b;
        ++restarts;
    }
}

asi_status asi_sync(asi_handle h) {
    if (!h) return ASI_E_ARG;
    if (h->device < 0) return ASI_OK;
    DeviceGuard g(h->device);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");
    if (!h->ws_ready) return ASI_OK;
    int32_t st = 0;
    e = hipMemcpy(&st, h->status, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "read status");
    if (st != 0) {
        e = asi::launch_fill_i32(h->status, 1, 0, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "clear status");
        const char *what = st == asi::ST_PERM        ? "perm is not a permutation of 0..n-1"
                           : st == asi::ST_SINGULAR ? "singular D block"
                           : st == asi::ST_NONFINITE ? "non-finite value produced"
                           : st == asi::ST_POOL      ? "NInv pool exhausted: enlarge the workspace"
                           : st == asi::ST_TIMEOUT   ? "dataflow wait exceeded its poll limit"
                                                     : "a column exceeds a kernel limit";
        return fail(h, (asi_status)st, what);
    }
    return ASI_OK;
}

asi_status asi_profile(asi_handle h, int enable) {
    if (!h) return ASI_E_ARG;
    if (h->device < 0) return fail(h, ASI_E_STATE, "host-only handle");
    DeviceGuard g(h->device);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");
    for (auto &r : h->pending) {
        h->ev_free.push_back(r.a);
        h->ev_free.push_back(r.b);
    }
    h->pending.clear();
    for (int k = 0; k < ASI_K_COUNT; ++k) {
        h->prof_n[k] = 0;
        h->prof_ms[k] = 0.0;
        h->prof_bytes[k] = 0.0;
    }
    h->prof = enable != 0;
    return ASI_OK;
}

asi_status asi_profile_read(asi_handle h, int32_t kernel_class, int64_t *launches, double *total_ms,
                            double *bytes) {
    if (!h) return ASI_E_ARG;
    if (kernel_class < 0 || kernel_class >= ASI_K_COUNT) return fail(h, ASI_E_ARG, "unknown kernel class");
    if (h->device >= 0 && !h->pending.empty()) {
        DeviceGuard g(h->device);
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");
        for (auto &r : h->pending) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, r.a, r.b);
            if (e != hipSuccess) return hip_fail(h, e, "event elapsed time");
            h->prof_n[r.kind] += 1;
            h->prof_ms[r.kind] += ms;
            h->prof_bytes[r.kind] += r.bytes;
            h->ev_free.push_back(r.a);
            h->ev_free.push_back(r.b);
        }
        h->pending.clear();
    }
    if (launches) *launches = h->prof_n[kernel_class];
    if (total_ms) *total_ms = h->prof_ms[kernel_class];
    if (bytes) *bytes = h->prof_bytes[kernel_class];
    return ASI_OK;
}

}  // extern "C"
