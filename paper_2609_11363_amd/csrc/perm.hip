// Values on S moved from the factor ordering to A's own ordering.
//
// The factorization is of P^T A P (Section 2.1), so an approximation X on S
// in the factor ordering holds X(i, j) ~ (A^-1)(perm[i], perm[j]); the
// problem (Section 1) asks for entries of A^-1. Row perm[i] of the output is
// row i of S with every column j renamed perm[j] and the row sorted by the
// new column index. The position of an entry inside its output row is its
// rank among the row's renamed columns (they are distinct), so no sort pass
// and no scratch beyond the inverse permutation are needed.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace asi {
namespace dev {

__global__ void k_unperm_iperm(int32_t n, const int32_t *__restrict__ perm, int32_t *__restrict__ iperm,
                               int32_t *status) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t p = perm[i];
    if (p < 0 || p >= n) {
        atomicCAS(status, 0, ST_PERM);
        return;
    }
    iperm[p] = i;
}

// The factor row of output row r, or -1 when r has no preimage under perm
// (then perm is not a permutation: some index was hit twice or never).
__device__ inline int32_t source_row(int32_t n, const int32_t *perm, const int32_t *iperm, int32_t r) {
    const int32_t i = iperm[r];
    if (i < 0 || i >= n || perm[i] != r) return -1;
    return i;
}

__global__ void k_unperm_count(int32_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ perm,
                               const int32_t *__restrict__ iperm, int64_t *__restrict__ rowptr_out,
                               int32_t *status) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) rowptr_out[0] = 0;
    if (r >= n) return;
    const int32_t i = source_row(n, perm, iperm, r);
    if (i < 0) atomicCAS(status, 0, ST_PERM);
    rowptr_out[r + 1] = i < 0 ? 0 : rowptr[i + 1] - rowptr[i];
}

// One wavefront per output row; rows of up to kStage entries keep their
// renamed columns in LDS for the rank count, longer rows read them again
// from memory (perm is gathered through the row's column indices).
constexpr int kUnpermWaves = 4;
constexpr int kStage = 1024;

__global__ __launch_bounds__(64 * kUnpermWaves) void k_unperm_fill(
    int32_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col, const int32_t *__restrict__ perm,
    const int32_t *__restrict__ iperm, const double *__restrict__ X, const int64_t *__restrict__ rowptr_out,
    int32_t *__restrict__ col_out, double *__restrict__ val_out) {
    __shared__ int32_t keys[kUnpermWaves][kStage];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int32_t r = blockIdx.x * kUnpermWaves + w;
    if (r >= n) return;  // the whole wavefront leaves; no barrier follows
    const int32_t i = source_row(n, perm, iperm, r);
    if (i < 0) return;
    const int64_t p0 = rowptr[i];
    const int32_t c = (int32_t)(rowptr[i + 1] - p0);
    const int64_t o0 = rowptr_out[r];
    int32_t *kw = keys[w];
    const bool staged = c <= kStage;
    if (staged) {
        for (int32_t t = lane; t < c; t += 64) kw[t] = perm[col[p0 + t]];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    for (int32_t t = lane; t < c; t += 64) {
        const int32_t key = staged ? kw[t] : perm[col[p0 + t]];
        int32_t rank = 0;
        if (staged) {
            for (int32_t q = 0; q < c; ++q) rank += kw[q] < key;
        } else {
            for (int32_t q = 0; q < c; ++q) rank += perm[col[p0 + q]] < key;
        }
        col_out[o0 + rank] = key;
        val_out[o0 + rank] = X[p0 + t];
    }
}

// Scratch of the no-allocation variant: the inverse permutation (n int32)
// and the row-pointer scan's block sums (n / 1024 + 2 uint64) for n up to
// kUnpermStaticMaxN, one copy per device for the life of the process. Host
// code never uses this name as an address (on the host it is a stand-in, not
// device memory): it takes each device's address from hipGetSymbolAddress.
constexpr size_t kUnpermIpermBytes = (size_t)kUnpermStaticMaxN * 4;
constexpr size_t kUnpermBsumBytes = ((size_t)kUnpermStaticMaxN / 1024 + 2) * 8;
static __device__ __align__(256) unsigned char scratch[kUnpermIpermBytes + kUnpermBsumBytes];

}  // namespace dev

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
}  // namespace

hipError_t unpermute_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[device]) {
        // the caller has made `device` current
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(dev::scratch));
        g_scratch_err[device] = e;
        g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
        g_scratch_done[device] = true;
    }
    return g_scratch_err[device];
}

hipError_t launch_unpermute_static(int device, int32_t n, const int64_t *rowptr, const int32_t *col,
                                   const int32_t *perm, const double *X, int64_t *rowptr_out, int32_t *col_out,
                                   double *val_out, int32_t *status, hipStream_t st) {
    if (n < 0 || n > kUnpermStaticMaxN) return hipErrorInvalidValue;
    hipError_t e = unpermute_scratch_init(device);
    if (e != hipSuccess) return e;
    unsigned char *base;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = static_cast<unsigned char *>(g_scratch_ptr[device]);
    }
    int32_t *iperm = reinterpret_cast<int32_t *>(base);
    unsigned long long *bsum = reinterpret_cast<unsigned long long *>(base + dev::kUnpermIpermBytes);
    return launch_unpermute(n, rowptr, col, perm, X, iperm, bsum, rowptr_out, col_out, val_out, status, st);
}

hipError_t launch_unpermute(int32_t n, const int64_t *rowptr, const int32_t *col, const int32_t *perm,
                            const double *X, int32_t *iperm, unsigned long long *bsum, int64_t *rowptr_out,
                            int32_t *col_out, double *val_out, int32_t *status, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    hipLaunchKernelGGL(dev::k_unperm_iperm, g, b, 0, st, n, perm, iperm, status);
    hipLaunchKernelGGL(dev::k_unperm_count, g, b, 0, st, n, rowptr, perm, iperm, rowptr_out, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_scan_counts(n, reinterpret_cast<unsigned long long *>(rowptr_out), bsum, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dev::k_unperm_fill, dim3((unsigned)((n + dev::kUnpermWaves - 1) / dev::kUnpermWaves)),
                       dim3(64 * dev::kUnpermWaves), 0, st, n, rowptr, col, perm, iperm, X, rowptr_out, col_out,
                       val_out);
    return hipGetLastError();
}

}  // namespace asi
