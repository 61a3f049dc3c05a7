// Learned per-entry correction of the Mix result (an addition to the paper's
// method): features on S, a 16 -> 64 -> 64 -> 1 ReLU network with
// bfloat16 weights and activations and float32 accumulation, its backward
// pass, the squared-error loss and Adam.
//
// Packed weights (MLP_PACKED_BYTES): W1 bf16 [64][32] (inputs 16..31 are
// zero padding), W2 bf16 [64][64], w3 bf16 [64], b1 f32 [64], b2 f32 [64],
// b3 f32. Master parameters (float32, 5313): W1 [64][16], b1, W2 [64][64],
// b2, w3, b3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace asi {
namespace dev {

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));
typedef short s16x4 __attribute__((__vector_size__(4 * sizeof(short))));

constexpr int NF = kMlpFeatures, NH = kMlpHidden;
constexpr int OFF_W1 = 0, OFF_W2 = 4096, OFF_W3 = 12288, OFF_B1 = 12416, OFF_B2 = 12672, OFF_B3 = 12928;
// master layout
constexpr int M_W1 = 0, M_B1 = 1024, M_W2 = 1088, M_B2 = 5184, M_W3 = 5248, M_B3 = 5312;

// float -> bfloat16 bits, round to nearest even (the gfx950 conversion
// instruction; bit-identical to the integer rounding b + 0x7FFF + lsb on
// finite values, denormals and ties included)
__device__ inline uint16_t to_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// A float64 value rounded to float32 and then to bfloat16, two separate
// roundings to nearest even as the features are defined. The second step is
// integer arithmetic: a compiler may otherwise fuse the float64 -> float32 ->
// bfloat16 chain into a single rounding from float64, which differs whenever
// the float32 value lies exactly halfway between two bfloat16 values.
__device__ inline uint16_t feat_bf16(double x) {
    const uint32_t b = __float_as_uint((float)x);
    if ((b & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((b >> 16) | 0x40u);  // NaN stays NaN
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
__device__ inline float round_bf16(float x) { return from_bf16(to_bf16(x)); }

// ---- features --------------------------------------------------------------
// Per-node record, computed once per call: the diagonals of M and Z, the
// node's bfloat16 features (log(|D^-1_ii| + 1e-30), log(||L(i,:)||_2 + 1e-30),
// log(||L(:,i)||_2 + 1e-30), level(i) / max level, log(1 + |R_i|)).
struct NodeRec {
    double m, z;
    uint16_t f[6];
    int32_t pad;
};
static_assert(sizeof(NodeRec) == 32, "node records are 32 bytes");

__device__ inline double dinv_diag(const double *dinv, const int8_t *piv, int32_t i) {
    // diagonal of D^-1 at i: 1x1 -> inv00; first of 2x2 -> inv00; second -> inv11
    return piv[i] == 2 ? dinv[3 * (int64_t)(i - 1) + 2] : dinv[3 * (int64_t)i];
}

// ||L(i, :)||_2 from the caller's CSR values (row order) into rn[i] and
// ||L(:, i)||_2 from the column layout (u-range of column i, padding is 0)
// into rn[n + i]; 16 lanes per unknown, strided over its entries. The row
// values read here are also copied to Lcopy (the loaded factor's row-order
// copy, read by the learned correction).
__global__ __launch_bounds__(256) void k_factor_norms(int32_t n, const int64_t *__restrict__ Lp,
                                                      const double *__restrict__ Lval,
                                                      const int64_t *__restrict__ ustart,
                                                      const double *__restrict__ Lu, double *__restrict__ rn,
                                                      double *__restrict__ Lcopy) {
    const int32_t i = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 4);
    const int sub = threadIdx.x & 15;
    double r = 0.0, c = 0.0;
    if (i < n) {
        for (int64_t q = Lp[i] + sub; q < Lp[i + 1]; q += 16) {
            const double v = Lval[q];
            r += v * v;
            Lcopy[q] = v;
        }
        for (int64_t u = ustart[i] + sub; u < ustart[i + 1]; u += 16) c += Lu[u] * Lu[u];
    }
#pragma unroll
    for (int k = 8; k >= 1; k >>= 1) {
        r += __shfl_xor(r, k, 64);
        c += __shfl_xor(c, k, 64);
    }
    if (i < n && sub == 0) {
        rn[i] = sqrt(r);
        rn[n + i] = sqrt(c);
    }
}

__global__ void k_node_feats(MlpFeatParams P) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const double maxlev = P.maxlevel > 0 ? (double)P.maxlevel : 1.0;
    NodeRec r;
    r.z = P.Z[P.diagpos[i]];
    if (P.fuse_mix) {
        const double nv = P.N[P.diagpos[i]];
        r.m = fabs(r.z) > P.eps * sqrt(fabs(r.z * r.z)) ? r.z : nv;  // Mix on the diagonal
    } else {
        r.m = P.M[P.diagpos[i]];
    }
    r.f[0] = feat_bf16(log(fabs(dinv_diag(P.dinv, P.piv, i)) + 1e-30));
    r.f[1] = feat_bf16(log(P.rn[i] + 1e-30));
    r.f[2] = feat_bf16(log(P.rn[P.n + i] + 1e-30));
    r.f[3] = feat_bf16(P.level[i] / maxlev);
    r.f[4] = feat_bf16(log1p((double)(P.ustart[i + 1] - P.ustart[i])));
    r.f[5] = 0;
    r.pad = 0;
    reinterpret_cast<NodeRec *>(P.node)[i] = r;
}

constexpr uint16_t kBf16One = 0x3F80;

// log(1 + x) for x >= 0 in float64 (+inf and NaN pass through), within a few
// units in the last place: 1 + x = u = 2^e m with m in [sqrt(1/2), sqrt(2)),
// log m = 2 atanh(t) = 2 t sum_k t^(2k) / (2k + 1) with t = (m - 1) / (m + 1)
// (|t| <= 0.1716, so 11 terms reach float64 precision), plus the rounding
// error of u, (x - (u - 1)) / u, which carries log1p's accuracy for small x.
// The features round the result to float32 and then bfloat16, which a
// last-place difference changes only for values within a few units of a
// float32 rounding boundary.
// coefficients 1 / (2k + 1), k = 10 .. 1, then ln 2 split so that e ln2_hi is
// exact for |e| < 2^11 (a table in constant memory keeps them in scalar registers)
__constant__ double kLog1pCoef[12] = {1.0 / 21.0, 1.0 / 19.0, 1.0 / 17.0, 1.0 / 15.0, 1.0 / 13.0, 1.0 / 11.0,
                                      1.0 / 9.0,  1.0 / 7.0,  1.0 / 5.0,  1.0 / 3.0,
                                      6.93147180369123816490e-01, 1.90821492927058770002e-10};

__device__ inline double log1p_pos(double x) {
    if (!(x < INFINITY)) return x;
    const double u = 1.0 + x;
    const double c = (x - (u - 1.0)) * __builtin_amdgcn_rcp(u);
    int e = __builtin_amdgcn_frexp_exp(u);
    double m = __builtin_amdgcn_frexp_mant(u);  // [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double t = (m - 1.0) / (m + 1.0);
    const double t2 = t * t;
    double q = kLog1pCoef[0];
#pragma unroll
    for (int k = 1; k < 10; ++k) q = fma(q, t2, kLog1pCoef[k]);
    const double logm = 2.0 * t + (2.0 * t) * (t2 * q);
    const double de = (double)e;
    return fma(de, kLog1pCoef[10], logm + fma(de, kLog1pCoef[11], c));
}

// The 16 features of entry p = (i, j) (order as in the header) from its
// values z = Z_ij, nv = N_ij, m = M_ij, the node records of i and j and
// lval = |L(max, min)| (0 on the diagonal); s = sqrt(|M_ii M_jj|) (1 where
// that is 0).
__device__ inline void features_of(const MlpFeatParams &P, int32_t i, int32_t j, const NodeRec &ni,
                                   const NodeRec &nj, double z, double nv, double m, double lval, uint16_t (&f)[NF],
                                   double &s) {
    s = sqrt(fabs(ni.m * nj.m));
    if (!(s > 0.0)) s = 1.0;
    const double rs = 1.0 / s;  // the four ratios below as products with 1 / s
    f[0] = feat_bf16(m * rs);
    f[1] = feat_bf16((z - nv) * rs);
    f[2] = fabs(z) > P.eps * sqrt(fabs(ni.z * nj.z)) ? kBf16One : (uint16_t)0;
    f[3] = i == j ? kBf16One : (uint16_t)0;
    f[4] = ni.f[0];
    f[5] = nj.f[0];
    f[6] = ni.f[1];
    f[7] = nj.f[1];
    f[8] = ni.f[2];
    f[9] = nj.f[2];
    f[10] = feat_bf16(lval);
    f[11] = feat_bf16(log1p_pos(fabs(nv) * rs));
    f[12] = feat_bf16(log1p_pos(fabs(z) * rs));
    f[13] = ni.f[3];
    f[14] = nj.f[3];
    f[15] = i < j ? ni.f[4] : nj.f[4];
}

// |L(max(i, j), min(i, j))| at u-index u (-1: diagonal, 0)
__device__ inline double lval_at(const MlpFeatParams &P, int32_t u) { return u >= 0 ? fabs(P.Lu[u]) : 0.0; }

// The same for entry p = (i, j) of S: below the diagonal, where the column
// layout would be a scattered gather, from the row-order copy of L when row i
// of L is the lower part of row i of S (position p - rowptr[i] in the row;
// past the row's end only the (i, i-1) entry of a 2x2 block, whose L value is
// 0); above it, from the column layout, which runs along the row.
__device__ inline double lval_of(const MlpFeatParams &P, int64_t p, int32_t i, int32_t j, int32_t u) {
    if (P.Lcsr && j < i) {
        const int64_t t = p - P.rowptr[i], l0 = P.Lp[i];
        return t < P.Lp[i + 1] - l0 ? fabs(P.Lcsr[l0 + t]) : 0.0;
    }
    return lval_at(P, u);
}

__device__ inline void store_features(uint16_t *dst16, const uint16_t (&f)[NF]) {
    uint4 *dst = reinterpret_cast<uint4 *>(dst16);
    dst[0] = make_uint4(f[0] | (uint32_t)f[1] << 16, f[2] | (uint32_t)f[3] << 16, f[4] | (uint32_t)f[5] << 16,
                        f[6] | (uint32_t)f[7] << 16);
    dst[1] = make_uint4(f[8] | (uint32_t)f[9] << 16, f[10] | (uint32_t)f[11] << 16,
                        f[12] | (uint32_t)f[13] << 16, f[14] | (uint32_t)f[15] << 16);
}

__global__ void k_features(MlpFeatParams P) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.nnz) return;
    const NodeRec *node = reinterpret_cast<const NodeRec *>(P.node);
    const int32_t i = P.srow[p], j = P.col[p];
    uint16_t f[NF];
    double sc;
    features_of(P, i, j, node[i], node[j], P.Z[p], P.N[p], P.M[p], lval_of(P, p, i, j, P.s2u[p]), f, sc);
    store_features(P.F + p * NF, f);
    P.scale[p] = (float)sc;
}

// ---- parameters --------------------------------------------------------------

__global__ void k_mlp_pack(const float *__restrict__ theta, uint8_t *__restrict__ W) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    uint16_t *w1 = reinterpret_cast<uint16_t *>(W + OFF_W1);
    uint16_t *w2 = reinterpret_cast<uint16_t *>(W + OFF_W2);
    uint16_t *w3 = reinterpret_cast<uint16_t *>(W + OFF_W3);
    float *b1 = reinterpret_cast<float *>(W + OFF_B1);
    float *b2 = reinterpret_cast<float *>(W + OFF_B2);
    float *b3 = reinterpret_cast<float *>(W + OFF_B3);
    if (t < NH * 32) {
        int n = t / 32, k = t % 32;
        w1[t] = k < NF ? to_bf16(theta[M_W1 + n * NF + k]) : (uint16_t)0;
    }
    if (t < NH * NH) w2[t] = to_bf16(theta[M_W2 + t]);
    if (t < NH) {
        w3[t] = to_bf16(theta[M_W3 + t]);
        b1[t] = theta[M_B1 + t];
        b2[t] = theta[M_B2 + t];
    }
    if (t == 0) b3[0] = theta[M_B3];
}

// ---- forward (bfloat16 MFMA, float32 accumulation) -----------------------------
// A wavefront handles 64 entries per tile as four blocks of 16. Each layer is
// computed transposed, units x entries = W x X^T, so that its result is
// already in the operand layout of the next layer. Operand layout of
// v_mfma_f32_16x16x32_bf16: lane l supplies row l % 16 of A and column l % 16
// of B with the 8 k values 8 (l / 16) ..; the result holds column l % 16 and
// rows 4 (l / 16) .. + 3. The first layer (16 inputs) uses
// v_mfma_f32_16x16x16_bf16, where lane l supplies the 4 k values 4 (l / 16) ..
// Lane (col = l % 16, g = l / 16) therefore ends a layer with entry col and
// units 16 nt + 4 g + r (nt, r = 0..3). The next layer's k slots are
// numbered so that these are exactly the values the lane supplies: slot s of
// k-block kb on lane group g is unit
//   sigma(kb, g, s) = 16 (2 kb + s / 4) + 4 g + s % 4,
// and the weights (A operand) are read in the same order. A sum over k does
// not depend on how its slots are numbered, so the activations never leave
// the registers. The last layer is an MFMA with w3 in every row of A. Biases
// are the accumulators' initial values. Only the tile's features go through
// LDS (lane = entry when computed, column layout for the first layer).

__device__ inline bf16x8 load8(const uint16_t *p) {
    uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

// units 32 kb + 4 g .. + 3 and 32 kb + 16 + 4 g .. + 3 of a bf16 row
__device__ inline bf16x8 load_sigma(const uint16_t *row, int kb, int g) {
    const uint2 lo = *reinterpret_cast<const uint2 *>(row + 32 * kb + 4 * g);
    const uint2 hi = *reinterpret_cast<const uint2 *>(row + 32 * kb + 16 + 4 * g);
    return __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
}

struct MlpRegs {
    s16x4 w1[4];  // layer 1 (16x16x16 MFMA): unit 16 nt + col, inputs 4 g .. + 3
    float b3;
};

// LDS tables of a workgroup: the biases b1, b2 (float32, 64 each; sb, read
// per block as f32x4) and the layer-2 and layer-3 weight fragments (sw,
// kMlpFragBytes), each lane's 16-byte fragment at ((f * 64) + lane) * 16 for
// fragment f = 2 nt + kb of layer 2 and f = 8 + kb of layer 3, so that a
// wavefront's read is one conflict-free 1 KiB row. Keeping them in LDS
// rather than registers leaves the registers to the feature computation (4
// wavefronts per SIMD without spills).
constexpr int kMlpFragBytes = 10 * 64 * 16;

// Layer-1 fragments into registers, the tables into LDS (filled by wavefront 0).
__device__ inline void load_mlp_regs(const uint8_t *W, int col, int g, MlpRegs &R, float *sb, uint8_t *sw) {
    const uint16_t *w1 = reinterpret_cast<const uint16_t *>(W + OFF_W1);
    const uint16_t *w2 = reinterpret_cast<const uint16_t *>(W + OFF_W2);
    const uint16_t *w3 = reinterpret_cast<const uint16_t *>(W + OFF_W3);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int n = nt * 16 + col;
        R.w1[nt] = *reinterpret_cast<const s16x4 *>(w1 + n * 32 + 4 * g);
        if (threadIdx.x < 64) {
            *reinterpret_cast<bf16x8 *>(sw + ((nt * 2 + 0) * 64 + threadIdx.x) * 16) = load_sigma(w2 + n * NH, 0, g);
            *reinterpret_cast<bf16x8 *>(sw + ((nt * 2 + 1) * 64 + threadIdx.x) * 16) = load_sigma(w2 + n * NH, 1, g);
        }
    }
    if (threadIdx.x < 64) {
        *reinterpret_cast<bf16x8 *>(sw + (8 * 64 + threadIdx.x) * 16) = load_sigma(w3, 0, g);
        *reinterpret_cast<bf16x8 *>(sw + (9 * 64 + threadIdx.x) * 16) = load_sigma(w3, 1, g);
    }
    R.b3 = reinterpret_cast<const float *>(W + OFF_B3)[0];
    // b1 then b2: OFF_B2 follows OFF_B1 directly
    const float *b = reinterpret_cast<const float *>(W + OFF_B1);
    for (int t = threadIdx.x; t < 2 * NH; t += blockDim.x) sb[t] = b[t];
    __syncthreads();
}

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// max(x, 0) as one integer maximum of the bit pattern (a negative float is a
// negative integer; -0 gives +0); a NaN with the sign bit clear passes through
__device__ inline float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// ReLU and bfloat16 rounding of two 16 x 16 result blocks (units of blocks
// 2 kb and 2 kb + 1), packed as the next layer's B operand for k-block kb
__device__ inline bf16x8 relu_pack(const f32x4 &a, const f32x4 &b) {
    uint16_t h[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        h[r] = to_bf16(relu(a[r]));
        h[4 + r] = to_bf16(relu(b[r]));
    }
    const uint4 v = make_uint4(h[0] | (uint32_t)h[1] << 16, h[2] | (uint32_t)h[3] << 16,
                               h[4] | (uint32_t)h[5] << 16, h[6] | (uint32_t)h[7] << 16);
    return __builtin_bit_cast(bf16x8, v);
}

// y for the 64 feature rows in Fs (LDS, row-major 64 x 16 bfloat16) into ys
// (LDS, 64 floats).
__device__ inline void mlp_tile(const MlpRegs &R, const float *sb, const uint8_t *sw, const uint16_t *Fs, float *ys,
                                int col, int g) {
    const int ln = col + 16 * g;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        // layer 1: [64 x 16] x [16 x 16]
        const s16x4 x = *reinterpret_cast<const s16x4 *>(Fs + (mt * 16 + col) * NF + 4 * g);
        f32x4 h1[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 b1 = *reinterpret_cast<const f32x4 *>(sb + 16 * nt + 4 * g);
            h1[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.w1[nt], x, b1, 0, 0, 0);
        }
        const bf16x8 x2[2] = {relu_pack(h1[0], h1[1]), relu_pack(h1[2], h1[3])};
        // layer 2: [64 x 64] x [64 x 16]
        f32x4 h2[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 b2 = *reinterpret_cast<const f32x4 *>(sb + NH + 16 * nt + 4 * g);
            const bf16x8 wa = *reinterpret_cast<const bf16x8 *>(sw + ((nt * 2 + 0) * 64 + ln) * 16);
            const bf16x8 wb = *reinterpret_cast<const bf16x8 *>(sw + ((nt * 2 + 1) * 64 + ln) * 16);
            h2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, x2[0], b2, 0, 0, 0);
            h2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb, x2[1], h2[nt], 0, 0, 0);
        }
        const bf16x8 x3[2] = {relu_pack(h2[0], h2[1]), relu_pack(h2[2], h2[3])};
        // layer 3: every row of A is w3, so every row of the result is y
        f32x4 y = {0.f, 0.f, 0.f, 0.f};
        const bf16x8 w3a = *reinterpret_cast<const bf16x8 *>(sw + (8 * 64 + ln) * 16);
        const bf16x8 w3b = *reinterpret_cast<const bf16x8 *>(sw + (9 * 64 + ln) * 16);
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3a, x3[0], y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3b, x3[1], y, 0, 0, 0);
        if (g == 0) ys[mt * 16 + col] = y[0] + R.b3;
    }
    wave_sync();
}

constexpr int kFwdWaves = 4;

__global__ __launch_bounds__(64 * kFwdWaves, 4) void k_mlp_forward(const uint8_t *__restrict__ W,
                                                                const uint16_t *__restrict__ F, int64_t rows,
                                                                float *__restrict__ y) {
    __shared__ __align__(16) uint16_t sF[kFwdWaves][64 * NF];
    __shared__ float sy[kFwdWaves][64];
    __shared__ __align__(16) float sb[2 * NH];
    __shared__ __align__(16) uint8_t sw[kMlpFragBytes];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4;
    MlpRegs R;
    load_mlp_regs(W, col, g, R, sb, sw);
    const int64_t ntiles = (rows + 63) / 64;
    for (int64_t tile = (int64_t)blockIdx.x * kFwdWaves + w; tile < ntiles; tile += (int64_t)gridDim.x * kFwdWaves) {
        const int64_t row = tile * 64 + lane;
        uint4 v0 = {0u, 0u, 0u, 0u}, v1 = {0u, 0u, 0u, 0u};
        if (row < rows) {
            v0 = reinterpret_cast<const uint4 *>(F + row * NF)[0];
            v1 = reinterpret_cast<const uint4 *>(F + row * NF)[1];
        }
        reinterpret_cast<uint4 *>(sF[w] + lane * NF)[0] = v0;
        reinterpret_cast<uint4 *>(sF[w] + lane * NF)[1] = v1;
        wave_sync();
        mlp_tile(R, sb, sw, sF[w], sy[w], col, g);
        if (row < rows) y[row] = sy[w][lane];
    }
}

// Features, network and correction in one pass: out = M + y s on S. The
// indices of the next tile (row, column, u-index) are loaded while the
// current tile's gathers and network run, so a tile waits for one round of
// memory accesses (node records, L value, Z, N, M) instead of two.
// FUSE: M = Mix(Z, N) is formed here (the test is the one the features
// already make, on the same values) and written to Mout when given.
template <bool FUSE>
__global__ __launch_bounds__(64 * kFwdWaves, 4) void k_mlp_correct(MlpFeatParams P, const uint8_t *__restrict__ W,
                                                                   double *out) {
    __shared__ __align__(16) uint16_t sF[kFwdWaves][64 * NF];
    __shared__ float sy[kFwdWaves][64];
    __shared__ __align__(16) float sb[2 * NH];
    __shared__ __align__(16) uint8_t sw[kMlpFragBytes];
    __shared__ double sM[FUSE ? kFwdWaves : 1][64];  // FUSE: the formed M value, kept across the network
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4;
    MlpRegs R;
    load_mlp_regs(W, col, g, R, sb, sw);
    const NodeRec *node = reinterpret_cast<const NodeRec *>(P.node);
    const int64_t ntiles = (P.nnz + 63) / 64;
    const int64_t stride = (int64_t)gridDim.x * kFwdWaves;
    int64_t tile = (int64_t)blockIdx.x * kFwdWaves + w;
    int32_t ci = 0, cj = 0, cu = -1;
    {
        const int64_t p = tile * 64 + lane;
        if (p < P.nnz) {
            ci = P.srow[p];
            cj = P.col[p];
            cu = P.s2u[p];
        }
    }
    for (; tile < ntiles; tile += stride) {
        const int64_t p = tile * 64 + lane;
        const bool valid = p < P.nnz;
        NodeRec ni{}, nj{};
        double z = 0.0, nv = 0.0, m = 0.0, lv = 0.0;
        if (valid) {
            ni = node[ci];
            nj = node[cj];
            lv = lval_of(P, p, ci, cj, cu);
            z = P.Z[p];
            nv = P.N[p];
            if constexpr (FUSE)
                m = fabs(z) > P.eps * sqrt(fabs(ni.z * nj.z)) ? z : nv;
            else
                m = P.M[p];
        }
        const int32_t i = ci, j = cj;
        const int64_t pn = p + stride * 64;
        if (pn < P.nnz) {
            ci = P.srow[pn];
            cj = P.col[pn];
            cu = P.s2u[pn];
        }
        uint16_t f[NF];
        double sc = 1.0;
        if (valid) {
            features_of(P, i, j, ni, nj, z, nv, m, lv, f, sc);
        } else {
#pragma unroll
            for (int k = 0; k < NF; ++k) f[k] = 0;
        }
        store_features(sF[w] + lane * NF, f);
        if constexpr (FUSE) sM[w][lane] = m;
        wave_sync();
        mlp_tile(R, sb, sw, sF[w], sy[w], col, g);
        if (valid) {
            if constexpr (FUSE) {
                const double mm = sM[w][lane];
                out[p] = mm + (double)sy[w][lane] * (double)(float)sc;
                if (P.Mout) P.Mout[p] = mm;
            } else {
                out[p] = m + (double)sy[w][lane] * (double)(float)sc;
            }
        }
    }
}

// ---- backward (bfloat16 MFMA, float32 accumulation) ------------------------------
// A wavefront takes 16 entries at a time and recomputes their forward pass in
// both orientations: transposed (units x entries, as the forward kernel does),
// whose results are the k operands of the next product over units, and direct
// (entries x units: the same MFMAs with A and B swapped), whose results hold
// for one unit the values of four consecutive entries, the operand layout of
// the gradient products, which contract over entries. So
//   dz2 = dy w3 [z2 > 0]                        (both layouts, elementwise)
//   dz1 = (dz2 W2) [z1 > 0]                     (direct; dz2 transposed as A)
//   gW2 += dz2^T h1, gW1 += dz1^T x             (K = the 16 entries)
//   gb2 += sum dz2, gb1 += sum dz1, gw3 += sum dy h2, gb3 += sum dy
// with no transpose through LDS. The activations and weights are bfloat16
// already, as in the forward pass; a float32 dz enters an MFMA as a bfloat16
// head and tail (dz = hi + lo to 2^-17 relative), two products each, so only
// the float32 sums round. The bfloat16 roundings of the forward pass count as
// identity in the derivative. At the end the workgroup adds its four
// wavefronts' sums in LDS (in wavefront order) and adds them to grad with one
// atomic per parameter.

constexpr int kBwdWaves = 4;
constexpr int kBwdBlocksPerWave = 4;   // at least this many 16-entry blocks per wavefront (amortises the final reduction)
constexpr int kBwdMaxGrid = 256;       // workgroups: one per compute unit

// W2 fragments of dz1 = dz2 W2 (B operand: k = output unit in slot order
// sigma, column = input unit 16 it + col), fragment f = 2 it + kb at
// (f * 64 + lane) * 16.
constexpr int kW2tFragBytes = 8 * 64 * 16;

__device__ inline void load_w2t_frags(const uint8_t *W, uint8_t *swt) {
    const uint16_t *w2 = reinterpret_cast<const uint16_t *>(W + OFF_W2);
    for (int t = threadIdx.x; t < 8 * 64; t += blockDim.x) {
        const int f = t >> 6, l = t & 63, it = f >> 1, kb = f & 1, c = l & 15, g = l >> 4;
        uint32_t h[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) h[s] = w2[(16 * (2 * kb + s / 4) + 4 * g + s % 4) * NH + 16 * it + c];
        *reinterpret_cast<uint4 *>(swt + t * 16) =
            make_uint4(h[0] | h[1] << 16, h[2] | h[3] << 16, h[4] | h[5] << 16, h[6] | h[7] << 16);
    }
}

// x = hi + lo, both bfloat16 (the difference x - hi is exact in float32)
__device__ inline void split2(float x, uint32_t &hi, uint32_t &lo) {
    const uint16_t h = to_bf16(x);
    hi = h;
    lo = to_bf16(x - from_bf16(h));
}

// two 16 x 16 blocks (slots 0..3 from a, 4..7 from b) as bfloat16 head and tail
__device__ inline void split_pack8(const f32x4 &a, const f32x4 &b, bf16x8 &hi, bf16x8 &lo) {
    uint32_t h[8], l[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        split2(a[r], h[r], l[r]);
        split2(b[r], h[4 + r], l[4 + r]);
    }
    hi = __builtin_bit_cast(bf16x8, make_uint4(h[0] | h[1] << 16, h[2] | h[3] << 16, h[4] | h[5] << 16,
                                               h[6] | h[7] << 16));
    lo = __builtin_bit_cast(bf16x8, make_uint4(l[0] | l[1] << 16, l[2] | l[3] << 16, l[4] | l[5] << 16,
                                               l[6] | l[7] << 16));
}

__device__ inline void split_pack4(const f32x4 &a, s16x4 &hi, s16x4 &lo) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) split2(a[r], h[r], l[r]);
    hi = __builtin_bit_cast(s16x4, make_uint2(h[0] | h[1] << 16, h[2] | h[3] << 16));
    lo = __builtin_bit_cast(s16x4, make_uint2(l[0] | l[1] << 16, l[2] | l[3] << 16));
}

__device__ inline s16x4 relu_pack4(const f32x4 &a) {
    uint32_t h[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) h[r] = to_bf16(relu(a[r]));
    return __builtin_bit_cast(s16x4, make_uint2(h[0] | h[1] << 16, h[2] | h[3] << 16));
}

__device__ inline float sum_groups(float v) {  // over the four lane groups g (lanes col + 16 g)
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

__global__ __launch_bounds__(64 * kBwdWaves, 2) void k_mlp_backward(const uint8_t *__restrict__ W,
                                                                    const uint16_t *__restrict__ F,
                                                                    const float *__restrict__ dy, int64_t rows,
                                                                    float *__restrict__ grad) {
    __shared__ __align__(16) float sb[2 * NH];
    __shared__ __align__(16) uint8_t sw[kMlpFragBytes];
    __shared__ __align__(16) uint8_t swt[kW2tFragBytes];
    __shared__ float sw3[NH];
    __shared__ __align__(16) uint16_t sX[kBwdWaves][16 * NF];
    __shared__ float sred[kMlpParams];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4;
    MlpRegs R;
    for (int t = threadIdx.x; t < kMlpParams; t += blockDim.x) sred[t] = 0.f;
    for (int t = threadIdx.x; t < NH; t += blockDim.x)
        sw3[t] = from_bf16(reinterpret_cast<const uint16_t *>(W + OFF_W3)[t]);
    load_w2t_frags(W, swt);
    load_mlp_regs(W, col, g, R, sb, sw);  // ends with a workgroup barrier

    f32x4 gW2[4][4], gW1[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    float gb1[4] = {0.f, 0.f, 0.f, 0.f}, gb2[4] = {0.f, 0.f, 0.f, 0.f}, gw3[4] = {0.f, 0.f, 0.f, 0.f};
    float gb3 = 0.f;
    float w3c[4];  // w3 of the lane's direct-layout units 16 nt + col
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) w3c[nt] = sw3[16 * nt + col];

    const int64_t nblk = (rows + 15) / 16;
    uint16_t *xs = sX[w];
    for (int64_t blk = (int64_t)blockIdx.x * kBwdWaves + w; blk < nblk; blk += (int64_t)gridDim.x * kBwdWaves) {
        const int64_t e0 = blk * 16;
        // the block's 16 feature rows (32 bytes each) into LDS; rows past the end are 0
        if (lane < 32) {
            const int64_t e = e0 + (lane >> 1);
            uint4 v = {0u, 0u, 0u, 0u};
            if (e < rows) v = reinterpret_cast<const uint4 *>(F + e * NF)[lane & 1];
            reinterpret_cast<uint4 *>(xs)[lane] = v;
        }
        wave_sync();
        // dy of entry col (transposed layout) and of entries 4 g + r (direct); 0 past the end
        const float dyt = e0 + col < rows ? dy[e0 + col] : 0.f;
        float dyn[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) dyn[r] = e0 + 4 * g + r < rows ? dy[e0 + 4 * g + r] : 0.f;
        const s16x4 x = *reinterpret_cast<const s16x4 *>(xs + col * NF + 4 * g);

        // layer 1, both orientations
        f32x4 z1t[4], z1n[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 b1t = *reinterpret_cast<const f32x4 *>(sb + 16 * nt + 4 * g);
            const float b1c = sb[16 * nt + col];
            z1t[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.w1[nt], x, b1t, 0, 0, 0);
            z1n[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, R.w1[nt], f32x4{b1c, b1c, b1c, b1c}, 0, 0, 0);
        }
        const bf16x8 h1t[2] = {relu_pack(z1t[0], z1t[1]), relu_pack(z1t[2], z1t[3])};
        s16x4 h1n[4];
        uint32_t m1 = 0;  // bit 4 it + r: z1 > 0 at entry 4 g + r, unit 16 it + col
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            h1n[it] = relu_pack4(z1n[it]);
#pragma unroll
            for (int r = 0; r < 4; ++r) m1 |= (uint32_t)(z1n[it][r] > 0.f) << (4 * it + r);
        }

        // layer 2, both orientations, and dz2
        f32x4 d2t[4], d2n[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 b2t = *reinterpret_cast<const f32x4 *>(sb + NH + 16 * nt + 4 * g);
            const float b2c = sb[NH + 16 * nt + col];
            const int ln = col + 16 * g;
            const bf16x8 wa = *reinterpret_cast<const bf16x8 *>(sw + ((nt * 2 + 0) * 64 + ln) * 16);
            const bf16x8 wb = *reinterpret_cast<const bf16x8 *>(sw + ((nt * 2 + 1) * 64 + ln) * 16);
            f32x4 zt = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, h1t[0], b2t, 0, 0, 0);
            zt = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb, h1t[1], zt, 0, 0, 0);
            f32x4 zn = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h1t[0], wa, f32x4{b2c, b2c, b2c, b2c}, 0, 0, 0);
            zn = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h1t[1], wb, zn, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                d2t[nt][r] = zt[r] > 0.f ? dyt * sw3[16 * nt + 4 * g + r] : 0.f;
                d2n[nt][r] = zn[r] > 0.f ? dyn[r] * w3c[nt] : 0.f;
                gw3[nt] += dyn[r] * round_bf16(relu(zn[r]));
                gb2[nt] += d2n[nt][r];
            }
        }
        if (col == 0) gb3 += (dyn[0] + dyn[1]) + (dyn[2] + dyn[3]);

        // gW2 += dz2^T h1 (K = the block's 16 entries)
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            s16x4 dh, dl;
            split_pack4(d2n[ob], dh, dl);
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) {
                gW2[ob][ib] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dh, h1n[ib], gW2[ob][ib], 0, 0, 0);
                gW2[ob][ib] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dl, h1n[ib], gW2[ob][ib], 0, 0, 0);
            }
        }

        // dz1 = (dz2 W2) [z1 > 0], direct layout: entries 4 g + r, input unit 16 it + col
        bf16x8 d2h[2], d2l[2];
        split_pack8(d2t[0], d2t[1], d2h[0], d2l[0]);
        split_pack8(d2t[2], d2t[3], d2h[1], d2l[1]);
        // x as the B operand of gW1: feature col of entries 4 g + r
        uint32_t xv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) xv[r] = xs[(4 * g + r) * NF + col];
        const s16x4 xn = __builtin_bit_cast(s16x4, make_uint2(xv[0] | xv[1] << 16, xv[2] | xv[3] << 16));
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int ln = col + 16 * g;
            const bf16x8 ta = *reinterpret_cast<const bf16x8 *>(swt + ((it * 2 + 0) * 64 + ln) * 16);
            const bf16x8 tb = *reinterpret_cast<const bf16x8 *>(swt + ((it * 2 + 1) * 64 + ln) * 16);
            f32x4 d1 = {0.f, 0.f, 0.f, 0.f};
            d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(d2h[0], ta, d1, 0, 0, 0);
            d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(d2h[1], tb, d1, 0, 0, 0);
            d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(d2l[0], ta, d1, 0, 0, 0);
            d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(d2l[1], tb, d1, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                d1[r] = (m1 >> (4 * it + r)) & 1u ? d1[r] : 0.f;
                gb1[it] += d1[r];
            }
            // gW1 += dz1^T x
            s16x4 dh, dl;
            split_pack4(d1, dh, dl);
            gW1[it] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dh, xn, gW1[it], 0, 0, 0);
            gW1[it] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dl, xn, gW1[it], 0, 0, 0);
        }
        wave_sync();  // xs is rewritten by the next block
    }

    // sums over the lane groups, then the workgroup's wavefronts in order into LDS
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        gb1[k] = sum_groups(gb1[k]);
        gb2[k] = sum_groups(gb2[k]);
        gw3[k] = sum_groups(gw3[k]);
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) gb3 += __shfl_xor(gb3, o, 64);
    for (int turn = 0; turn < kBwdWaves; ++turn) {
        if (w == turn) {
#pragma unroll
            for (int ob = 0; ob < 4; ++ob) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int n = 16 * ob + 4 * g + r;
#pragma unroll
                    for (int ib = 0; ib < 4; ++ib) sred[M_W2 + n * NH + 16 * ib + col] += gW2[ob][ib][r];
                    sred[M_W1 + n * NF + col] += gW1[ob][r];
                }
            }
            if (g == 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    sred[M_B1 + 16 * k + col] += gb1[k];
                    sred[M_B2 + 16 * k + col] += gb2[k];
                    sred[M_W3 + 16 * k + col] += gw3[k];
                }
            }
            if (lane == 0) sred[M_B3] += gb3;
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < kMlpParams; t += blockDim.x) atomicAdd(&grad[t], sred[t]);
}

// ---- loss, Adam, apply ------------------------------------------------------

__global__ void k_mlp_loss(const float *__restrict__ y, const float *__restrict__ t, int64_t rows,
                           float *__restrict__ dy, double *__restrict__ loss) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double sq = 0.0;
    if (e < rows) {
        float d = y[e] - t[e];
        dy[e] = 2.0f * d / (float)rows;
        sq = (double)d * (double)d;
    }
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss, sq / (double)rows);
}

__global__ void k_adam(float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int32_t np, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_mlp_apply(int64_t nnz, const double *__restrict__ M, const float *__restrict__ y,
                            const float *__restrict__ s, double *__restrict__ out) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) out[p] = M[p] + (double)y[p] * (double)s[p];
}

}  // namespace dev

hipError_t launch_factor_norms(int32_t n, const int64_t *Lp, const double *Lval, const int64_t *ustart,
                              const double *Lu, double *rn, double *Lcopy, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_factor_norms, dim3((unsigned)(((int64_t)n * 16 + 255) / 256)), dim3(256), 0, st, n, Lp,
                       Lval, ustart, Lu, rn, Lcopy);
    return hipGetLastError();
}

hipError_t launch_node_feats(const MlpFeatParams &P, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_node_feats, dim3((P.n + 255) / 256), dim3(256), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_mlp_features(const MlpFeatParams &P, hipStream_t st) {
    if (P.nnz > 0)
        hipLaunchKernelGGL(dev::k_features, dim3((unsigned)((P.nnz + 255) / 256)), dim3(256), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_mlp_correct(const MlpFeatParams &P, const void *W, double *out, hipStream_t st) {
    if (P.nnz <= 0) return hipSuccess;
    const int64_t tiles = (P.nnz + 63) / 64;
    const int64_t grid = std::min<int64_t>((tiles + dev::kFwdWaves - 1) / dev::kFwdWaves, 8192);
    if (P.fuse_mix)
        hipLaunchKernelGGL(dev::k_mlp_correct<true>, dim3((unsigned)grid), dim3(64 * dev::kFwdWaves), 0, st, P,
                           reinterpret_cast<const uint8_t *>(W), out);
    else
        hipLaunchKernelGGL(dev::k_mlp_correct<false>, dim3((unsigned)grid), dim3(64 * dev::kFwdWaves), 0, st, P,
                           reinterpret_cast<const uint8_t *>(W), out);
    return hipGetLastError();
}

hipError_t launch_mlp_pack(const float *theta, void *W, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_mlp_pack, dim3(16), dim3(256), 0, st, theta, reinterpret_cast<uint8_t *>(W));
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const void *W, const uint16_t *F, int64_t rows, float *y, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    const int64_t tiles = (rows + 63) / 64;
    const int64_t grid = std::min<int64_t>((tiles + dev::kFwdWaves - 1) / dev::kFwdWaves, 8192);
    hipLaunchKernelGGL(dev::k_mlp_forward, dim3((unsigned)grid), dim3(64 * dev::kFwdWaves), 0, st,
                       reinterpret_cast<const uint8_t *>(W), F, rows, y);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const void *W, const uint16_t *F, const float *dy, int64_t rows, float *grad,
                               hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    const int64_t blocks = (rows + 15) / 16;
    const int64_t per_wg = (int64_t)dev::kBwdWaves * dev::kBwdBlocksPerWave;
    const int64_t grid = std::min<int64_t>((blocks + per_wg - 1) / per_wg, dev::kBwdMaxGrid);
    hipLaunchKernelGGL(dev::k_mlp_backward, dim3((unsigned)grid), dim3(64 * dev::kBwdWaves), 0, st,
                       reinterpret_cast<const uint8_t *>(W), F, dy, rows, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_loss(const float *y, const float *t, int64_t rows, float *dy, double *loss, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_mlp_loss, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, y, t, rows, dy,
                       loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *theta, float *m, float *v, const float *g, int32_t np, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(dev::k_adam, dim3((np + 255) / 256), dim3(256), 0, st, theta, m, v, g, np, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_apply(int64_t nnz, const double *M, const float *y, const float *s, double *out,
                            hipStream_t st) {
    hipLaunchKernelGGL(dev::k_mlp_apply, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, nnz, M, y, s, out);
    return hipGetLastError();
}

}  // namespace asi
