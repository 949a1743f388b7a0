// scan.hip -- gfx950 kernels: chunked full-DFA scan, failure-less (PFAC)
// per-start scan, wave-level match compaction, and an LSD radix sort of the
// match keys.
#include "scan.h"

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/ac.h"
#include "machine.h"

namespace acm {
namespace {

constexpr uint32_t kNoClassDev = 0xffu;

// ------------------------------------------------------------------ compaction
// Rank of this lane among the set lanes of `mask` below it (mbcnt prefix).
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

// Append `key` for every active lane with `has`: one ballot, one atomic per
// wave, each lane writing at base + its rank. Keys past `cap` are counted but
// not stored.
__device__ __forceinline__ void emit_key(bool has, uint64_t key, uint64_t *out, uint64_t cap,
                                         unsigned long long *count) {
    const uint64_t mask = __ballot(has);
    if (mask == 0) return;
    const uint32_t rank = lane_rank(mask);
    unsigned long long base = 0;
    if (has && rank == 0) base = atomicAdd(count, (unsigned long long)__popcll(mask));
    base = __shfl(base, __ffsll((unsigned long long)mask) - 1);
    if (has) {
        const uint64_t idx = base + rank;
        if (idx < cap) out[idx] = key;
    }
}

// Every pattern id of the set ids[off[s] .. off[s+1]) as a match ending at pos.
__device__ __forceinline__ void emit_set(bool has, uint32_t s, uint64_t pos, const uint32_t *off,
                                         const uint32_t *ids, uint64_t *out, uint64_t cap,
                                         unsigned long long *count) {
    uint32_t k = 0, kend = 0;
    if (has) {
        k = off[s];
        kend = off[s + 1];
    }
    while (__any(k < kend)) {
        const bool h = k < kend;
        const uint32_t id = h ? ids[k] : 0u;
        emit_key(h, (pos << 32) | id, out, cap, count);
        k += h ? 1u : 0u;
    }
}

__global__ void zero_count_kernel(unsigned long long *count) { *count = 0ull; }

// ------------------------------------------------------------------ DFA scan
struct DfaArgs {
    const uint8_t *text;
    uint64_t n;
    uint64_t n_chunks;
    uint32_t chunk;
    uint32_t m_max;
    uint32_t n_cols;
    uint32_t hot_states;
    uint32_t table_words;  // LDS_FULL: n_states * n_cols
    const uint32_t *dfa;
    const uint16_t *hot;
    const uint8_t *cmap;
    const uint32_t *out_off, *out_ids;
    uint64_t *out;
    uint64_t cap;
    unsigned long long *count;
};

template <int PLACE>
__device__ __forceinline__ uint32_t dfa_entry(uint32_t s, uint32_t c, const DfaArgs &a,
                                              const uint32_t *s_tab, const uint16_t *s_hot) {
    const uint32_t idx = s * a.n_cols + c;
    if constexpr (PLACE == AC_PLACE_LDS_FULL) {
        return s_tab[idx];
    } else if constexpr (PLACE == AC_PLACE_LDS_HOT) {
        if (s < a.hot_states) {
            const uint32_t e = s_hot[idx];
            return (e & kHotMask) | ((e & kHotAccept) << 16);
        }
        return a.dfa[idx];
    } else {
        return a.dfa[idx];
    }
}

// One byte through the DFA: bytes outside the pattern alphabet send the
// walk back to the root; the table is still read (at column 0) so the
// lookup never leaves the table.
template <int PLACE>
__device__ __forceinline__ uint32_t dfa_byte(uint32_t s, uint32_t b, const DfaArgs &a,
                                             const uint8_t *s_cmap, const uint32_t *s_tab,
                                             const uint16_t *s_hot) {
    const uint32_t c = s_cmap[b];
    const bool valid = c != kNoClassDev;
    const uint32_t e = dfa_entry<PLACE>(s, valid ? c : 0u, a, s_tab, s_hot);
    return valid ? e : 0u;
}

// Chunk k owns end positions [kC, min(kC + C, n)). Its walker starts from the
// root at max(0, kC - m_max + 1) rounded down to 16 bytes: every occurrence
// ending in the chunk starts at or after kC - m_max + 1, and a walk from the
// root reports every occurrence starting at or after its first byte, so the
// walker sees exactly the occurrences it owns (plus some it discards).
template <int PLACE, int BLOCK>
__global__ void __launch_bounds__(BLOCK) dfa_scan_kernel(DfaArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint8_t *s_cmap = smem;
    uint32_t *s_tab = reinterpret_cast<uint32_t *>(smem + 256);
    uint16_t *s_hot = reinterpret_cast<uint16_t *>(smem + 256);
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < 64; i += BLOCK)
        reinterpret_cast<uint32_t *>(s_cmap)[i] = reinterpret_cast<const uint32_t *>(a.cmap)[i];
    if constexpr (PLACE == AC_PLACE_LDS_FULL) {
        for (uint32_t i = tid; i < a.table_words; i += BLOCK) s_tab[i] = a.dfa[i];
    } else if constexpr (PLACE == AC_PLACE_LDS_HOT) {
        const uint32_t halfwords = a.hot_states * a.n_cols;
        for (uint32_t i = tid; i < halfwords; i += BLOCK) s_hot[i] = a.hot[i];
    }
    __syncthreads();

    const uint64_t stride = uint64_t(gridDim.x) * BLOCK;
    for (uint64_t k = uint64_t(blockIdx.x) * BLOCK + tid; k < a.n_chunks; k += stride) {
        const uint64_t own_lo = k * a.chunk;
        const uint64_t own_hi = min(own_lo + a.chunk, a.n);
        const uint64_t back = a.m_max - 1;
        uint64_t pos = own_lo > back ? ((own_lo - back) & ~uint64_t(15)) : 0;
        const uint64_t full_end = own_hi & ~uint64_t(15);
        uint32_t s = 0;
        for (; pos < full_end; pos += 16) {
            const uint4 v = *reinterpret_cast<const uint4 *>(a.text + pos);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            const uint32_t s0 = s;
            uint32_t flag = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const uint32_t e = dfa_byte<PLACE>(s, (w[j >> 2] >> ((j & 3) * 8)) & 0xffu, a,
                                                   s_cmap, s_tab, s_hot);
                s = e & kStateMask;
                flag |= e;
            }
            if (flag & kAccept) {
                // some state in these 16 bytes is final: walk them again and report
                uint32_t r = s0;
                for (int j = 0; j < 16; ++j) {
                    const uint32_t e = dfa_byte<PLACE>(r, (w[j >> 2] >> ((j & 3) * 8)) & 0xffu, a,
                                                       s_cmap, s_tab, s_hot);
                    r = e & kStateMask;
                    const bool acc = (e & kAccept) && (pos + j >= own_lo);
                    emit_set(acc, r, pos + j, a.out_off, a.out_ids, a.out, a.cap, a.count);
                }
            }
        }
        for (; pos < own_hi; ++pos) {  // last bytes of a text whose length is not a multiple of 16
            const uint32_t e = dfa_byte<PLACE>(s, a.text[pos], a, s_cmap, s_tab, s_hot);
            s = e & kStateMask;
            emit_set((e & kAccept) && pos >= own_lo, s, pos, a.out_off, a.out_ids, a.out, a.cap,
                     a.count);
        }
    }
}

// ------------------------------------------------------------------ PFAC scan
struct PfacArgs {
    const uint8_t *text;
    uint64_t n;
    uint32_t m_max;
    uint32_t n_cols;
    uint32_t hot_states;
    uint32_t table_words;
    uint32_t halo;  // text bytes staged past the tile's last start
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
            const uint32_t e = s_hot[idx];
            return (e & kHotMask) | ((e & kHotAccept) << 16);
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
    extern __shared__ __align__(16) uint8_t smem[];
    constexpr uint32_t kTile = BLOCK * kPfacStartsPerThread;
    uint8_t *s_cmap = smem;
    uint8_t *s_cls = smem + 256;  // kTile + halo classes, padded to 16
    const uint32_t cls_bytes = (kTile + a.halo + 15u) & ~15u;
    uint32_t *s_tab = reinterpret_cast<uint32_t *>(smem + 256 + cls_bytes);
    uint16_t *s_hot = reinterpret_cast<uint16_t *>(smem + 256 + cls_bytes);
    const uint32_t tid = threadIdx.x;
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
                if (c == kNoClassDev) break;
                const uint32_t e = go_entry<PLACE>(s, c, a, s_tab, s_hot);
                if (e == 0) break;
                s = e & kStateMask;
                if (__any(e & kAccept))
                    emit_set((e & kAccept) != 0, s, j, a.own_off, a.own_ids, a.out, a.cap, a.count);
            }
        }
        __syncthreads();
    }
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

// ------------------------------------------------------------------ helpers
int hip_fail(hipError_t e, const char *what, std::string &err) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return AC_ERR_HIP;
}

template <typename K, typename A>
int launch(K kernel, uint32_t grid, uint32_t block, uint32_t lds, hipStream_t stream, const A &args,
           std::string &err) {
    if (lds > 64u * 1024u) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute", err);
    }
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, stream, args);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch", err);
    return AC_OK;
}

}  // namespace

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

int launch_dfa_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                    uint64_t cap, uint64_t *count, const ScanConfig &cfg, hipStream_t stream,
                    std::string &err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const uint32_t cus = uint32_t(compute_units(dev));
    DfaArgs a{};
    a.text = text;
    a.n = n;
    a.m_max = dm.m_max;
    a.n_cols = dm.n_cols;
    a.hot_states = dm.hot_states;
    a.table_words = dm.n_states * dm.n_cols;
    a.dfa = dm.dfa;
    a.hot = dm.hot_dfa;
    a.cmap = dm.cmap;
    a.out_off = dm.out_off;
    a.out_ids = dm.out_ids;
    a.out = out;
    a.cap = cap;
    a.count = reinterpret_cast<unsigned long long *>(count);

    uint32_t lds = 256;
    if (cfg.placement == AC_PLACE_LDS_FULL) lds += a.table_words * 4u;
    if (cfg.placement == AC_PLACE_LDS_HOT) lds += ((dm.hot_states * dm.n_cols * 2u) + 15u) & ~15u;
    if (lds > kLdsPerWorkgroup) {
        err = "ac_scan: table image does not fit the LDS";
        return AC_ERR_INVALID;
    }
    const uint32_t block = cfg.placement == AC_PLACE_LDS_HOT ? 1024u : 256u;
    if (cfg.block != 0 && cfg.block != block) {
        err = "ac_scan: this placement runs with " + std::to_string(block) + " threads per workgroup";
        return AC_ERR_INVALID;
    }
    const uint32_t wg_per_cu = std::max<uint32_t>(1, std::min<uint32_t>(2048 / block, kLdsPerWorkgroup / lds));
    // Chunk length: enough walkers to fill every lane the chip can hold, but at
    // least 4 * m_max so the overlap stays small.
    uint64_t chunk = cfg.chunk;
    if (chunk == 0) {
        const uint64_t walkers = uint64_t(cus) * wg_per_cu * block;
        chunk = (n + walkers - 1) / walkers;
        chunk = std::max<uint64_t>(chunk, 4ull * dm.m_max);
        chunk = std::max<uint64_t>(64, (chunk + 15) & ~uint64_t(15));
        chunk = std::min<uint64_t>(chunk, 1u << 30);
    }
    if (chunk % 16 != 0 || chunk == 0) {
        err = "ac_scan: chunk must be a positive multiple of 16";
        return AC_ERR_INVALID;
    }
    a.chunk = uint32_t(chunk);
    a.n_chunks = (n + chunk - 1) / chunk;
    if (a.n_chunks == 0) return AC_OK;
    const uint64_t want = (a.n_chunks + block - 1) / block;
    uint64_t cap_grid = want;
    if (cfg.placement != AC_PLACE_GLOBAL) cap_grid = uint64_t(cus) * wg_per_cu;
    const uint32_t grid = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(want, cap_grid)));
    switch (cfg.placement) {
        case AC_PLACE_GLOBAL:
            return launch(dfa_scan_kernel<AC_PLACE_GLOBAL, 256>, grid, block, lds, stream, a, err);
        case AC_PLACE_LDS_FULL:
            return launch(dfa_scan_kernel<AC_PLACE_LDS_FULL, 256>, grid, block, lds, stream, a, err);
        case AC_PLACE_LDS_HOT:
            return launch(dfa_scan_kernel<AC_PLACE_LDS_HOT, 1024>, grid, block, lds, stream, a, err);
    }
    err = "ac_scan: unknown placement";
    return AC_ERR_INVALID;
}

int launch_pfac_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                     uint64_t cap, uint64_t *count, const ScanConfig &cfg, hipStream_t stream,
                     std::string &err) {
    if (n == 0) return AC_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const uint32_t cus = uint32_t(compute_units(dev));
    constexpr uint32_t block = 256;
    if (cfg.block != 0 && cfg.block != block) {
        err = "ac_scan: PFAC runs with 256 threads per workgroup";
        return AC_ERR_INVALID;
    }
    PfacArgs a{};
    a.text = text;
    a.n = n;
    a.m_max = dm.m_max;
    a.n_cols = dm.n_cols;
    a.hot_states = dm.hot_states;
    a.table_words = dm.n_states * dm.n_cols;
    a.halo = std::min<uint32_t>(dm.m_max, 2048u);
    a.go = dm.go;
    a.hot = dm.hot_go;
    a.cmap = dm.cmap;
    a.own_off = dm.own_off;
    a.own_ids = dm.own_ids;
    a.out = out;
    a.cap = cap;
    a.count = reinterpret_cast<unsigned long long *>(count);
    const uint32_t tile = block * kPfacStartsPerThread;
    uint32_t lds = 256 + ((tile + a.halo + 15u) & ~15u);
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
            return launch(pfac_scan_kernel<AC_PLACE_GLOBAL, block>, grid, block, lds, stream, a, err);
        case AC_PLACE_LDS_FULL:
            return launch(pfac_scan_kernel<AC_PLACE_LDS_FULL, block>, grid, block, lds, stream, a, err);
        case AC_PLACE_LDS_HOT:
            return launch(pfac_scan_kernel<AC_PLACE_LDS_HOT, block>, grid, block, lds, stream, a, err);
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
