// dfa.hip -- launch of the chunked full-DFA scan (kernels in dfa_kernel.h).
#include <algorithm>

#include "dfa_kernel.h"

namespace acm {
namespace {

// Threads per workgroup for a placement and walker count: one 1024-thread
// workgroup per CU holds the 16-bit image (768 threads when each lane runs 4
// walkers, whose registers would not fit 1024 lanes); 256 otherwise.
uint32_t block_for(uint32_t placement, uint32_t K) {
    if (placement == AC_PLACE_LDS_HOT) return K == 4 ? 768u : 1024u;
    return 256u;
}

}  // namespace

__global__ void copy_state_kernel(const uint32_t *in, uint32_t *out) { *out = in ? *in : 0u; }

int launch_copy_state(const uint32_t *in, uint32_t *out, hipStream_t stream, std::string &err) {
    hipLaunchKernelGGL(copy_state_kernel, dim3(1), dim3(1), 0, stream, in, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? AC_OK : hip_fail(e, "copy_state launch", err);
}

int launch_dfa_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                    uint64_t cap, uint64_t *count, const ScanConfig &cfg, hipStream_t stream,
                    std::string &err, const StreamArgs &st) {
    if (n == 0) return st.state_out ? launch_copy_state(st.state_in, st.state_out, stream, err) : AC_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const uint32_t cus = uint32_t(compute_units(dev));
    dfa::DfaArgs a{};
    a.text = text;
    a.n = uint32_t(n);
    dfa::fill_machine_args(dm, a);
    a.out = out;
    a.cap = cap;
    a.count = reinterpret_cast<unsigned long long *>(count);
    a.base = st.base;
    a.state_in = st.state_in;
    a.state_out = st.state_out;

    // default walkers per lane: two hide more lookup latency than one except
    // when every lookup goes to global memory
    const uint32_t K = cfg.walkers ? cfg.walkers : (cfg.placement == AC_PLACE_GLOBAL ? 1u : 2u);
    if (K < 1 || K > 4) {
        err = "ac_scan: walkers per lane must be 1, 2, 3 or 4";
        return AC_ERR_INVALID;
    }
    const uint32_t block = block_for(cfg.placement, K);
    uint32_t lds = (block / 64) * kQueueBytesPerWave + 256;
    if (cfg.placement == AC_PLACE_LDS_FULL) lds += a.table_words * 4u;
    if (cfg.placement == AC_PLACE_LDS_HOT) lds += ((dm.hot_states * dm.n_cols * 2u) + 15u) & ~15u;
    if (lds > kLdsPerWorkgroup) {
        err = "ac_scan: table image does not fit the LDS";
        return AC_ERR_INVALID;
    }
    if (cfg.block != 0 && cfg.block != block) {
        err = "ac_scan: this placement runs with " + std::to_string(block) + " threads per workgroup";
        return AC_ERR_INVALID;
    }
    // two-byte lookups from the states outside the image, where built
    const bool pair = cfg.placement == AC_PLACE_LDS_HOT && cfg.pair_steps && dm.pair_states > 0;
    // text block: whole cache lines (128 B, one buffer: a line is fetched
    // once) unless three or four walkers need the registers (64 B, one
    // buffer); the two-byte walk runs best on 64 B blocks in two buffers
    const uint32_t bb = cfg.block_bytes ? cfg.block_bytes : (K >= 3 || pair ? 64u : 128u);
    if (bb != 64 && bb != 128) {
        err = "ac_scan: block_bytes must be 64 or 128";
        return AC_ERR_INVALID;
    }
    dfa::DfaKernel kernel = nullptr;
    switch (cfg.placement) {
        case AC_PLACE_GLOBAL: kernel = dfa::select_global(dm, K, bb); break;
        case AC_PLACE_LDS_FULL: kernel = dfa::select_full(dm, K, bb); break;
        case AC_PLACE_LDS_HOT:
            kernel = pair ? dfa::select_hot_pair(dm, K, bb) : nullptr;
            if (!kernel) kernel = dfa::select_hot(dm, K, bb);
            break;
    }
    if (!kernel) {
        err = "ac_scan: no kernel for this placement / walker count";
        return AC_ERR_INVALID;
    }
    // resident workgroups per CU, as registers and LDS allow
    const uint32_t wg_per_cu = uint32_t(occupancy(reinterpret_cast<const void *>(kernel), block, lds));
    uint64_t chunk = cfg.chunk;
    if (chunk == 0) {
        // One chunk per walker the chip holds. Where that leaves chunks of at
        // least 4 * m_max (re-walked overlap under a quarter) they are rounded
        // to whole text blocks. A shorter text cannot fill the chip at that
        // length: its chunks stay short (down to 16 bytes) so that more lanes
        // share it and each walk, which is latency-bound, is short.
        const uint64_t walkers = uint64_t(cus) * wg_per_cu * block * K;
        const uint64_t fill = (n + walkers - 1) / walkers;
        if (fill >= 4ull * dm.m_max)
            chunk = (fill + bb - 1) & ~uint64_t(bb - 1);
        else
            chunk = std::max<uint64_t>(16, (fill + 15) & ~uint64_t(15));
        chunk = std::min<uint64_t>(chunk, 1u << 30);
    }
    if (chunk % 16 != 0 || chunk == 0 || chunk > (1u << 30)) {
        err = "ac_scan: chunk must be a positive multiple of 16, at most 2^30";
        return AC_ERR_INVALID;
    }
    a.chunk = uint32_t(chunk);
    a.n_chunks = uint32_t((n + chunk - 1) / chunk);
    const uint64_t lanes_needed = (uint64_t(a.n_chunks) + K - 1) / K;
    const uint64_t want = (lanes_needed + block - 1) / block;
    const uint64_t cap_grid = uint64_t(cus) * wg_per_cu;
    const uint32_t grid = uint32_t(std::max<uint64_t>(1, std::min(want, cap_grid)));
    return launch_kernel(kernel, grid, block, lds, stream, a, err);
}

}  // namespace acm
