// Internal declarations shared by the host analysis, the C ABI layer and the
// HIP kernels of libasi. Not part of the public interface (include/asi.h).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace asi {

// Per-slot record of a SelInv block, one per entry of a schedule, so that a
// wavefront finds everything it needs to start in one load.
struct BlockMeta {
    int64_t ub;      // u-start of the R_J entries of column last (the block's last column)
    int64_t ubj;     // u-start of L(R_J, j) (ub for a 1x1 block)
    int64_t h0;      // first hit word of the block
    int64_t pdl;     // S position of row last's first upper entry (diagpos[last] + 1)
    int64_t pdj;     // the same for row j (diagpos[j] + 2 for a 2x2 block, else pdl)
    int32_t j;       // first column of the block
    int32_t c;       // |R_J|
    int32_t nwords;  // hit words of the block
    int32_t two;     // 1 for a 2x2 block
    int64_t pad;
};
static_assert(sizeof(BlockMeta) == 64, "block records are 64 bytes");

// One row of a level of the preconditioner solves (forward: the lower part
// of row i of S, backward: its upper part): v_i -= sum of L v over the S
// positions [p0, p1), but for position skip (the other row of a 2x2 block,
// an explicit zero of L; -1 if none).
struct SolveRow {
    int32_t i, p0, p1, skip;
};
static_assert(sizeof(SolveRow) == 16, "solve rows are 16 bytes");

// Kernel limits (the analysis refuses patterns above them).
constexpr int kSmallCols = 128;   // |R_J| handled by one wavefront per block
constexpr int kBigCols = 2048;    // |R_J| handled by one 256-thread workgroup per block
constexpr int kSpaiMaxCols = 512; // entries per column of S for the SPAI kernel
constexpr int kMaxRank = 64;     // rank of the low-rank correction
constexpr int kRedBlocks = 512;   // blocks of the first stage of the diagonal-error reduction
constexpr int kMlpFeatures = 16;  // learned correction: inputs per entry
constexpr int kMlpHidden = 64;    //   hidden units per layer
constexpr int kMlpParams = kMlpHidden * kMlpFeatures + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpHidden + 1;  // 5313 float32 master parameters
constexpr int kMlpPackedBytes = 12944;      // bfloat16 weights + float32 biases

// Host-side result of the symbolic analysis. Positions index S's CSR arrays.
struct Analysis {
    int32_t n = 0;
    int64_t nnzL = 0;
    int64_t nnzS = 0;
    std::vector<int64_t> L_rowptr; // n+1: the input L's row pointers
    std::vector<int64_t> rowptr;   // n+1
    std::vector<int32_t> col;      // nnzS
    std::vector<int32_t> srow;     // nnzS: row of each position
    std::vector<int32_t> s2u;      // nnzS: u-index of L(max(i, j), min(i, j)) for (i, j), -1 on the diagonal
    std::vector<int64_t> diagpos;  // n: position of (i, i)
    std::vector<int64_t> mirror;   // nnzS: position of (j, i) for (i, j)
    // Upper triangle of S by rows ("u-space", the columns of L): the u-range of
    // row j is [ustart[j], ustart[j+1]) and holds R_J (after (j, j+1) when j
    // starts a 2x2 block).
    int64_t nnzU = 0;
    std::vector<int64_t> ustart;   // n+1
    std::vector<int32_t> ucol;     // nnzU: column r of the upper entry (j, r)
    std::vector<int64_t> lsrc_u;   // nnzU: index of L(r, j) in the input L arrays, -1 if absent
    std::vector<int32_t> q2u;      // nnzL: u-index of each input L entry (the inverse of lsrc_u)
    std::vector<int64_t> mirror_u; // nnzU: S position of the lower entry (r, j)
    std::vector<int64_t> useg_u;   // nnzU: ustart[r], start of row r's u-range (gather segment)
    // Hit lists of the SelInv gathers: for block J, every pair (r, l) in
    // R_J x R_J with r > l and (r, l) in S, as (a, b, off) with r = R_J[a],
    // l = R_J[b] and Z(r, l) at u-index ustart[l] + off, sorted by b then off.
    // Blocks with |R_J| <= kSmallCols use one word per hit,
    // a | b << 7 | off << 14; larger blocks use two, a | b << 16 and off.
    std::vector<int64_t> hit_ptr;  // n+1: words of block J are [hit_ptr[J], hit_ptr[J+1])
    std::vector<uint32_t> hits;
    std::vector<int8_t> piv;       // n
    std::vector<int32_t> level;    // n: DAG level of each unknown's block
    int32_t n_blocks = 0;
    int32_t n_levels = 0;
    int32_t max_cols = 0;
    // level-major schedules of block starts, split by column count
    std::vector<int32_t> sched_small, sched_big;
    std::vector<BlockMeta> meta_small, meta_big;  // records of the schedules' slots
    std::vector<int32_t> lvl_small, lvl_big;  // n_levels+1 offsets into the schedules
    std::vector<int32_t> lvl_maxc_big;        // per level: largest |R_J| of its large blocks
    std::vector<int32_t> lvl_heavy;           // per level: small blocks with more than kHeavyHits hits
                                              // (placed first in the level's small schedule)
    // rows of the preconditioner solves in level order (each level's blocks
    // as in the two schedules, both rows of a 2x2 block); empty when
    // |S| >= 2^31, where the solves are not offered
    std::vector<SolveRow> solve_fwd, solve_bwd;
    std::vector<int32_t> lvl_rows;            // n_levels+1 offsets into them
    int64_t gather_pairs = 0;
    int64_t gather_hits = 0;
    // algorithmic bytes of each level's launches, [0] float64 mode, [1] mixed
    std::vector<double> lvl_bytes_small[2], lvl_bytes_big[2];
};

// Algorithmic bytes of one SelInv block: L(R_J, J) read as index + value
// (12 B each), the h gathered Zhat entries (4 B index + w B value), the
// float64 outputs in both triangles (16 B per entry), the float32 working
// copy in mixed mode (4 B per entry) and Z(J, J).
inline double selinv_block_bytes(int64_t c, int ncols, int64_t hits, bool fp64) {
    const double w = fp64 ? 8.0 : 4.0;
    return 12.0 * c * ncols + (4.0 + w) * hits + (fp64 ? 16.0 : 20.0) * c * ncols + 8.0 * ncols * ncols;
}

// A small block with more hits than this takes more than two passes of a
// wavefront (4 hits per lane per pass); in a level run one wavefront per
// block such blocks get a whole 256-thread workgroup instead.
constexpr int32_t kHeavyHits = 512;

// The kernel variants of one level launch of the SelInv sweep (the same
// numbering as asi_sweep_variant in asi.h).
enum SweepVariant {
    SV_SMALL = 0,     // one wavefront per block, four per workgroup
    SV_SPLIT = 1,     // the same, the level's heavy blocks on 256-thread workgroups
    SV_GROUP128 = 2,  // one workgroup of 128 / 256 / 512 threads per block
    SV_GROUP256 = 3,
    SV_GROUP512 = 4,
    SV_BIG256 = 5,    // |R_J| > kSmallCols: 256 / 1024 threads per block
    SV_BIG1024 = 6,
    SV_COUNT = 7
};

// Variant for a level of nblk blocks with |R_J| <= kSmallCols, nheavy of them
// with more than kHeavyHits hits: enough lanes per block that the level keeps
// about 6144 wavefronts (256 CUs, 24 resident wavefronts each) busy, from one
// wavefront up to a 512-thread workgroup per block. The heavy-block split pays
// where a level is about one round of wavefronts (its tail is the longest hit
// list); on levels of many rounds the tail is amortised and the split
// kernel's lower occupancy costs more.
inline int small_level_variant(int64_t nblk, int64_t nheavy) {
    const int64_t waves = 6144;
    if (nblk * 2 > waves) return (nheavy > 0 && nblk <= 16384) ? SV_SPLIT : SV_SMALL;
    if (nblk * 4 > waves) return SV_GROUP128;
    if (nblk * 8 > waves) return SV_GROUP256;
    return SV_GROUP512;
}

// Variant for a level of nblk blocks with |R_J| > kSmallCols: few blocks get
// 1024 threads each (fewer passes over each block's hits), many get 256 (more
// blocks per compute unit).
inline int big_level_variant(int64_t nblk) { return nblk <= 1024 ? SV_BIG1024 : SV_BIG256; }

// Builds the analysis; returns 0 or an asi_status code with a message.
int analyze(int32_t n, const int64_t *Lp, const int32_t *Li, const int8_t *piv, Analysis &out,
            std::string &msg);

}  // namespace asi
