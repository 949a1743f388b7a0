// measure.hip -- streaming kernels of known traffic: the HBM read ceiling the
// scans are priced against, and a copy whose bytes (n read, n written) scale
// the HBM byte counters of a profiled run.
//
// Both read with 16-byte non-temporal loads: each wave takes a run of
// kUnroll KiB (its 64 lanes side by side, kUnroll loads in flight per lane),
// the waves of the grid take consecutive runs, and a wave moves on by the
// grid's whole width. The copy writes with non-temporal stores of the same
// shape. No LDS in the loop and one atomic per workgroup at the end: nothing
// but the loads stands between them and the memory system.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/ac.h"
#include "automaton.h"
#include "scan.h"

namespace acm {
namespace {

using u32x4 = uint32_t __attribute__((ext_vector_type(4)));

constexpr uint32_t kThreads = 256;
constexpr uint32_t kWaves = kThreads / 64;
constexpr uint32_t kUnroll = 8;
constexpr uint64_t kRun = 64 * kUnroll;  // 16-byte words per wave run
constexpr uint32_t kBlocksPerCu = 1;

__device__ __forceinline__ uint32_t fold4(u32x4 v) { return v.x ^ v.y ^ v.z ^ v.w; }

// XOR of all 32-bit little-endian words of the n bytes (a short last word is
// zero-padded), accumulated into *fold.
__global__ void __launch_bounds__(kThreads) hbm_read_kernel(const u32x4 *p, uint64_t n16, const uint8_t *tail,
                                                            uint32_t n_tail, unsigned long long *fold) {
    __shared__ uint32_t s_acc[kWaves];
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t waves = uint64_t(gridDim.x) * kWaves;
    uint64_t r = uint64_t(blockIdx.x) * kWaves + threadIdx.x / 64;
    uint32_t acc = 0;
    for (; (r + 1) * kRun <= n16; r += waves) {
        const u32x4 *q = p + r * kRun + lane;
        u32x4 v[kUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(q + u * 64);
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) acc ^= fold4(v[u]);
    }
    // the one partial run (if any) falls to the wave whose turn it is
    for (uint64_t i = r * kRun + lane; i < n16; i += 64) acc ^= fold4(__builtin_nontemporal_load(p + i));
    if (blockIdx.x == 0 && threadIdx.x < n_tail) acc ^= uint32_t(tail[threadIdx.x]) << (8 * (threadIdx.x & 3));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc ^= __shfl_xor(acc, off);
    if (lane == 0) s_acc[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0;
        for (uint32_t w = 0; w < kWaves; ++w) a ^= s_acc[w];
        if (a) atomicXor(fold, (unsigned long long)a);
    }
}

__global__ void __launch_bounds__(kThreads) hbm_copy_kernel(u32x4 *dst, const u32x4 *p, uint64_t n16, uint8_t *dt,
                                                            const uint8_t *pt, uint32_t n_tail) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t waves = uint64_t(gridDim.x) * kWaves;
    uint64_t r = uint64_t(blockIdx.x) * kWaves + threadIdx.x / 64;
    for (; (r + 1) * kRun <= n16; r += waves) {
        const uint64_t i = r * kRun + lane;
        u32x4 v[kUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(p + i + u * 64);
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) __builtin_nontemporal_store(v[u], dst + i + u * 64);
    }
    for (uint64_t i = r * kRun + lane; i < n16; i += 64) __builtin_nontemporal_store(__builtin_nontemporal_load(p + i), dst + i);
    if (blockIdx.x == 0 && threadIdx.x < n_tail) dt[threadIdx.x] = pt[threadIdx.x];
}

// Workgroups for n bytes: `blocks` if given, else kBlocksPerCu per CU, never
// more than it takes to give every wave a run.
uint32_t grid_for(uint64_t n, uint32_t blocks) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    uint64_t g = blocks ? blocks : uint64_t(compute_units(dev)) * kBlocksPerCu;
    const uint64_t need = (n / 16 + kRun * kWaves - 1) / (kRun * kWaves);
    if (g > need) g = need;
    return uint32_t(g < 1 ? 1 : g);
}

}  // namespace
}  // namespace acm

extern "C" {

int ac_hbm_read(const void *d, uint64_t n, uint64_t *d_fold, uint32_t blocks, void *stream) {
    if (!d_fold || (n && !d)) return acm::set_error(AC_ERR_INVALID, "ac_hbm_read: NULL pointer");
    if (reinterpret_cast<uintptr_t>(d) & 15u) return acm::set_error(AC_ERR_INVALID, "ac_hbm_read: buffer not 16-byte aligned");
    if (n == 0) return AC_OK;
    const auto *p = static_cast<const uint8_t *>(d);
    const uint64_t n16 = n / 16;
    hipLaunchKernelGGL(acm::hbm_read_kernel, dim3(acm::grid_for(n, blocks)), dim3(acm::kThreads), 0,
                       static_cast<hipStream_t>(stream), reinterpret_cast<const acm::u32x4 *>(p), n16,
                       p + n16 * 16, uint32_t(n % 16), reinterpret_cast<unsigned long long *>(d_fold));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? AC_OK : acm::set_error(AC_ERR_HIP, std::string("ac_hbm_read: ") + hipGetErrorString(e));
}

int ac_hbm_copy(void *dst, const void *src, uint64_t n, uint32_t blocks, void *stream) {
    if (n && (!dst || !src)) return acm::set_error(AC_ERR_INVALID, "ac_hbm_copy: NULL pointer");
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15u)
        return acm::set_error(AC_ERR_INVALID, "ac_hbm_copy: buffers not 16-byte aligned");
    const auto *p = static_cast<const uint8_t *>(src);
    auto *q = static_cast<uint8_t *>(dst);
    if (n && p < q + n && q < p + n) return acm::set_error(AC_ERR_INVALID, "ac_hbm_copy: buffers overlap");
    if (n == 0) return AC_OK;
    const uint64_t n16 = n / 16;
    hipLaunchKernelGGL(acm::hbm_copy_kernel, dim3(acm::grid_for(n, blocks)), dim3(acm::kThreads), 0,
                       static_cast<hipStream_t>(stream), reinterpret_cast<acm::u32x4 *>(q),
                       reinterpret_cast<const acm::u32x4 *>(p), n16, q + n16 * 16, p + n16 * 16, uint32_t(n % 16));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? AC_OK : acm::set_error(AC_ERR_HIP, std::string("ac_hbm_copy: ") + hipGetErrorString(e));
}

}  // extern "C"
