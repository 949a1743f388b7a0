// scan.hip -- gfx950 kernels: failure-less (PFAC) per-start scan, the match
// counter reset, and an LSD radix sort of the match keys. The chunked DFA
// scan is in dfa.hip.
#include "scan.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/ac.h"
#include "device_common.h"
#include "machine.h"

namespace acm {
namespace {

__global__ void zero_count_kernel(unsigned long long *count) { *count = 0ull; }

// ------------------------------------------------------------------ PFAC scan
struct PfacArgs {
    const uint8_t *text;
    uint64_t n;
    uint32_t m_max;
    uint32_t n_cols;
    uint32_t hot_states;  // image rows used (a prefix of the machine's hot rows)
    uint32_t term_lo, term_end;  // states where a pattern ends exactly
    uint32_t table_words;
    uint32_t halo;  // text bytes staged past the tile's last start
    uint32_t no_class;  // byte-map value of bytes in no pattern
    const uint32_t *go;
    const uint16_t *hot;
    const uint8_t *cmap;
    const uint32_t *own_off, *own_ids;
    uint64_t *out;
    uint64_t cap;
    unsigned long long *count;
};

constexpr int kPfacStartsPerThread = 4;

template <int PLACE>
__device__ __forceinline__ uint32_t go_entry(uint32_t s, uint32_t c, const PfacArgs &a,
                                             const uint32_t *s_tab, const uint16_t *s_hot) {
    const uint32_t idx = s * a.n_cols + c;
    if constexpr (PLACE == AC_PLACE_LDS_FULL) {
        return s_tab[idx];
    } else if constexpr (PLACE == AC_PLACE_LDS_HOT) {
        if (s < a.hot_states) {
            // image entries are plain child ids (0 = no edge); a pattern ends
            // exactly at the child iff its id is in [term_lo, term_end)
            const uint32_t t = s_hot[idx];
            return t | (t - a.term_lo < a.term_end - a.term_lo ? kAccept : 0u);
        }
        return a.go[idx];
    } else {
        return a.go[idx];
    }
}

// One walk per start position (the failure-less machine of the paper's
// Sec. II.B): from the root along goto edges, reporting the patterns that end
// exactly at each state entered, until a byte has no edge.
template <int PLACE, int BLOCK>
__global__ void __launch_bounds__(BLOCK) pfac_scan_kernel(PfacArgs a) {
    // LDS: per-wave match queues | byte map | staged text classes | table image
    extern __shared__ __align__(16) uint8_t smem[];
    constexpr uint32_t kTile = BLOCK * kPfacStartsPerThread;
    constexpr uint32_t kQueues = (BLOCK / 64) * kQueueBytesPerWave;
    uint8_t *s_cmap = smem + kQueues;
    uint8_t *s_cls = smem + kQueues + 256;  // kTile + halo classes, padded to 16
    const uint32_t cls_bytes = (kTile + a.halo + 15u) & ~15u;
    uint32_t *s_tab = reinterpret_cast<uint32_t *>(smem + kQueues + 256 + cls_bytes);
    uint16_t *s_hot = reinterpret_cast<uint16_t *>(smem + kQueues + 256 + cls_bytes);
    const uint32_t tid = threadIdx.x;
    Emitter em;
    em.init(smem, a.out, a.cap, a.count);
    for (uint32_t i = tid; i < 64; i += BLOCK)
        reinterpret_cast<uint32_t *>(s_cmap)[i] = reinterpret_cast<const uint32_t *>(a.cmap)[i];
    if constexpr (PLACE == AC_PLACE_LDS_FULL) {
        for (uint32_t i = tid; i < a.table_words; i += BLOCK) s_tab[i] = a.go[i];
    } else if constexpr (PLACE == AC_PLACE_LDS_HOT) {
        const uint32_t halfwords = a.hot_states * a.n_cols;
        for (uint32_t i = tid; i < halfwords; i += BLOCK) s_hot[i] = a.hot[i];
    }
    __syncthreads();

    for (uint64_t base = uint64_t(blockIdx.x) * kTile; base < a.n; base += uint64_t(gridDim.x) * kTile) {
        const uint64_t staged = min(uint64_t(kTile + a.halo), a.n - base);
        for (uint32_t i = tid; i < staged; i += BLOCK) s_cls[i] = s_cmap[a.text[base + i]];
        __syncthreads();
        for (int r = 0; r < kPfacStartsPerThread; ++r) {
            const uint64_t p = base + uint64_t(r) * BLOCK + tid;
            if (p >= a.n) break;
            uint32_t s = 0;
            for (uint64_t j = p; j < a.n; ++j) {
                const uint64_t t = j - base;
                const uint32_t c = t < staged ? s_cls[t] : s_cmap[a.text[j]];
                if (c == a.no_class) break;
                const uint32_t e = go_entry<PLACE>(s, c, a, s_tab, s_hot);
                if (e == 0) break;
                s = e & kStateMask;
                if (__any(e & kAccept))
                    emit_set(em, (e & kAccept) != 0, s, j, a.own_off, a.own_ids);
            }
        }
        __syncthreads();
    }
    em.flush();
}

// ------------------------------------------------------------------ radix sort
constexpr int kSortBlock = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortBlock * kSortRounds;

__global__ void __launch_bounds__(kSortBlock) sort_hist_kernel(const uint64_t *keys, uint64_t n,
                                                               uint32_t shift, uint32_t *hist,
                                                               uint32_t nblocks) {
    __shared__ uint32_t h[256];
    const uint32_t tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const uint64_t base = uint64_t(blockIdx.x) * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const uint64_t i = base + uint64_t(r) * kSortBlock + tid;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[uint64_t(tid) * nblocks + blockIdx.x] = h[tid];
}

// Exclusive prefix sum of `total` counters, one workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) sort_scan_kernel(uint32_t *hist, uint32_t total) {
    __shared__ uint32_t part[1024];
    const uint32_t tid = threadIdx.x;
    const uint32_t seg = (total + 1023u) / 1024u;
    const uint32_t lo = min(total, tid * seg), hi = min(total, lo + seg);
    uint32_t sum = 0;
    for (uint32_t i = lo; i < hi; ++i) sum += hist[i];
    part[tid] = sum;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
        const uint32_t v = tid >= d ? part[tid - d] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t run = part[tid] - sum;
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t x = hist[i];
        hist[i] = run;
        run += x;
    }
}

// Stable scatter by one 8-bit digit: keys of equal digit keep their order
// (round, then wave, then lane) inside the tile, tiles keep block order.
__global__ void __launch_bounds__(kSortBlock) sort_scatter_kernel(const uint64_t *in, uint64_t *out,
                                                                  uint64_t n, uint32_t shift,
                                                                  const uint32_t *hist,
                                                                  uint32_t nblocks) {
    constexpr int kWaves = kSortBlock / 64;
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kWaves][256];
    const uint32_t tid = threadIdx.x, wave = tid / 64;
    run[tid] = hist[uint64_t(tid) * nblocks + blockIdx.x];
    const uint64_t base = uint64_t(blockIdx.x) * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const uint64_t i = base + uint64_t(r) * kSortBlock + tid;
        const bool valid = i < n;
        const uint64_t key = valid ? in[i] : 0ull;
        const uint32_t d = uint32_t(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = lane_rank(peers);
        for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        if (valid && rank == 0) wcnt[wave][d] = uint32_t(__popcll(peers));
        __syncthreads();
        if (valid) {
            uint32_t o = run[d] + rank;
            for (uint32_t w = 0; w < wave; ++w) o += wcnt[w][d];
            out[o] = key;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kWaves; ++w) add += wcnt[w][tid];
        run[tid] += add;
    }
}

}  // namespace

hipError_t allow_lds(const void *kernel, uint32_t lds) {
    if (lds <= 64u * 1024u) return hipSuccess;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, uint32_t> granted;
    std::lock_guard<std::mutex> g(mu);
    uint32_t &have = granted[{dev, kernel}];
    if (have >= lds) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e == hipSuccess) have = lds;
    return e;
}

int occupancy(const void *kernel, uint32_t block, uint32_t lds) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, uint32_t, uint32_t>, int> known;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = known.find({dev, kernel, block, lds});
        if (it != known.end()) return it->second;
    }
    int occ = 0;
    if (allow_lds(kernel, lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, int(block), size_t(lds)) != hipSuccess ||
        occ <= 0)
        occ = 1;
    std::lock_guard<std::mutex> g(mu);
    known[{dev, kernel, block, lds}] = occ;
    return occ;
}

int compute_units(int device) {
    static std::mutex mu;
    static std::vector<int> cache;
    std::lock_guard<std::mutex> g(mu);
    if (device < 0) device = 0;
    if (size_t(device) >= cache.size()) cache.resize(device + 1, 0);
    if (cache[device] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cache[device] = cus;
    }
    return cache[device];
}

int launch_zero_count(uint64_t *d_count, hipStream_t stream, std::string &err) {
    hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(1), 0, stream,
                       reinterpret_cast<unsigned long long *>(d_count));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? AC_OK : hip_fail(e, "zero_count launch", err);
}

int launch_pfac_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                     uint64_t cap, uint64_t *count, const ScanConfig &cfg, hipStream_t stream,
                     std::string &err) {
    if (n == 0) return AC_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const uint32_t cus = uint32_t(compute_units(dev));
    // 1024 threads: each walk is a chain of dependent lookups, and with the
    // image filling the LDS one workgroup per CU is all that fits, so its 16
    // waves are what hides the lookup latency
    constexpr uint32_t block = 1024;
    if (cfg.block != 0 && cfg.block != block) {
        err = "ac_scan: PFAC runs with 1024 threads per workgroup";
        return AC_ERR_INVALID;
    }
    PfacArgs a{};
    a.text = text;
    a.n = n;
    a.m_max = dm.m_max;
    a.n_cols = dm.n_cols;
    a.hot_states = dm.hot_states;
    a.term_lo = dm.hot_states;
    a.term_end = dm.term_end;
    a.table_words = dm.n_states * dm.n_cols;
    a.halo = std::min<uint32_t>(dm.m_max, 2048u);
    a.go = dm.go;
    a.hot = dm.hot_go;
    a.cmap = dm.cmap;
    a.no_class = dm.no_class;
    a.own_off = dm.own_off;
    a.own_ids = dm.own_ids;
    a.out = out;
    a.cap = cap;
    a.count = reinterpret_cast<unsigned long long *>(count);
    const uint32_t tile = block * kPfacStartsPerThread;
    uint32_t lds = (block / 64) * kQueueBytesPerWave + 256 + ((tile + a.halo + 15u) & ~15u);
    uint32_t place = cfg.placement;
    // the staged text shares the LDS with the table: a whole table that no
    // longer fits beside it is read from global memory instead
    if (place == AC_PLACE_LDS_FULL && uint64_t(lds) + uint64_t(a.table_words) * 4u > kLdsPerWorkgroup)
        place = AC_PLACE_GLOBAL;
    if (place == AC_PLACE_LDS_FULL) lds += a.table_words * 4u;
    if (place == AC_PLACE_LDS_HOT) {
        // any prefix of the hot rows is a valid image: keep the rows that fit
        // beside the staged text
        const uint32_t room = lds < kLdsPerWorkgroup ? kLdsPerWorkgroup - lds : 0u;
        a.hot_states = std::min(dm.hot_states, room / (2u * dm.n_cols));
        lds += a.hot_states * dm.n_cols * 2u;
    }
    if (lds > kLdsPerWorkgroup) {
        err = "ac_scan: goto table image does not fit the LDS";
        return AC_ERR_INVALID;
    }
    const uint64_t tiles = (n + tile - 1) / tile;
    const uint32_t wg_per_cu = std::max<uint32_t>(1, std::min<uint32_t>(8, kLdsPerWorkgroup / lds));
    uint64_t g = tiles;
    if (place != AC_PLACE_GLOBAL) g = std::min<uint64_t>(g, uint64_t(cus) * wg_per_cu);
    const uint32_t grid = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(g, 1u << 30)));
    switch (place) {
        case AC_PLACE_GLOBAL:
            return launch_kernel(pfac_scan_kernel<AC_PLACE_GLOBAL, block>, grid, block, lds, stream, a, err);
        case AC_PLACE_LDS_FULL:
            return launch_kernel(pfac_scan_kernel<AC_PLACE_LDS_FULL, block>, grid, block, lds, stream, a, err);
        case AC_PLACE_LDS_HOT:
            return launch_kernel(pfac_scan_kernel<AC_PLACE_LDS_HOT, block>, grid, block, lds, stream, a, err);
    }
    err = "ac_scan: unknown placement";
    return AC_ERR_INVALID;
}

uint64_t sort_scratch_bytes(uint64_t count) {
    const uint64_t blocks = (count + kSortTile - 1) / kSortTile;
    return count * 8 + blocks * 256 * 4 + 256;
}

int launch_sort(uint64_t *keys, uint64_t count, void *tmp, uint64_t tmp_bytes, hipStream_t stream,
                std::string &err) {
    if (count <= 1) return AC_OK;
    if (count >= (1ull << 32)) {
        err = "ac_sort_matches: at most 2^32 - 1 keys";
        return AC_ERR_TOO_LARGE;
    }
    if (tmp_bytes < sort_scratch_bytes(count)) {
        err = "ac_sort_matches: scratch smaller than ac_sort_scratch_bytes(count)";
        return AC_ERR_INVALID;
    }
    const uint32_t blocks = uint32_t((count + kSortTile - 1) / kSortTile);
    uint64_t *alt = reinterpret_cast<uint64_t *>(tmp);
    uint32_t *hist = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(tmp) + count * 8);
    uint64_t *src = keys, *dst = alt;
    for (uint32_t pass = 0; pass < 8; ++pass) {
        const uint32_t shift = pass * 8;
        hipLaunchKernelGGL(sort_hist_kernel, dim3(blocks), dim3(kSortBlock), 0, stream, src, count,
                           shift, hist, blocks);
        hipLaunchKernelGGL(sort_scan_kernel, dim3(1), dim3(1024), 0, stream, hist, blocks * 256u);
        hipLaunchKernelGGL(sort_scatter_kernel, dim3(blocks), dim3(kSortBlock), 0, stream, src, dst,
                           count, shift, hist, blocks);
        std::swap(src, dst);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? AC_OK : hip_fail(e, "sort launch", err);
}

}  // namespace acm
