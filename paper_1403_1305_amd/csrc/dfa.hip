// dfa.hip -- chunked full-DFA scan for gfx950.
//
// The text is cut into chunks of C bytes. Chunk k owns the end positions
// [kC, min(kC + C, n)); its walker starts from the root exactly m_max - 1
// bytes before kC (or at 0) and reports only the matches that end inside the
// chunk. Every occurrence ending in the chunk starts at or after
// kC - m_max + 1, and a walk from the root reports every occurrence that
// starts at or after its first byte, so each match is reported exactly once.
//
// Each lane runs K walkers on K different chunks in lockstep, so K table
// lookups are in flight per lane per step. Text arrives in 16-byte groups
// that are prefetched two groups ahead. A walker only ORs the final-state
// flags of a group together; a flagged group is walked again and reported
// (final states are rare next to plain steps).
//
// Table placements:
//   LDS_FULL  the whole 32-bit table in LDS.
//   LDS_HOT   16-bit rows of the hot states [0, H) in LDS; a state >= H is
//             looked up in the 32-bit table in global memory (L2 resident).
//   GLOBAL    every lookup from the 32-bit table in global memory.
// Byte classes are either a bit field of the byte (small alphabets, checked
// four bytes at a time with v_perm against the letter of each field value) or
// a 256-entry map in LDS.
#include "scan.h"

#include <algorithm>

#include "../../include/ac.h"
#include "device_common.h"
#include "machine.h"

namespace acm {
namespace {

constexpr uint32_t kNoClassDev = 0xffu;

struct DfaArgs {
    const uint8_t *text;
    uint32_t n;            // text bytes (< 2^32)
    uint32_t chunk;        // bytes owned per walker (multiple of 16)
    uint32_t n_chunks;
    uint32_t back;         // m_max - 1
    uint32_t n_cols;
    uint32_t hot;          // H: states with rows in the LDS image
    uint32_t table_words;  // LDS_FULL: n_states * n_cols
    uint32_t hash_shift;   // hashed classes: column = (b >> shift) & (n_cols - 1)
    uint32_t letters_lo, letters_hi;  // the letter owning each hashed column
    const uint32_t *dfa;
    const uint16_t *hot_rows;
    const uint8_t *cmap;
    const uint32_t *out_off, *out_ids;
    uint64_t *out;
    uint64_t cap;
    unsigned long long *count;
};

// Entry of (s, c) in the canonical 32-bit form: successor | kAccept if final.
template <int PLACE, int LOG2C>
__device__ __forceinline__ uint32_t lookup(uint32_t s, uint32_t c, const DfaArgs &a,
                                           const uint32_t *s_tab, const uint16_t *s_hot) {
    const uint32_t idx = LOG2C >= 0 ? ((s << (LOG2C >= 0 ? LOG2C : 0)) | c) : (s * a.n_cols + c);
    if constexpr (PLACE == AC_PLACE_LDS_FULL) {
        return s_tab[idx];
    } else if constexpr (PLACE == AC_PLACE_LDS_HOT) {
        if (s < a.hot) {
            const uint32_t e = s_hot[idx];
            return (e & kHotMask) | ((e & kHotAccept) << 16);
        }
        return a.dfa[idx];
    } else {
        return a.dfa[idx];
    }
}

// One byte with the general byte map: bytes in no pattern reset to the root.
template <int PLACE, int LOG2C>
__device__ __forceinline__ uint32_t step_byte(uint32_t s, uint32_t b, const DfaArgs &a,
                                              const uint8_t *s_cmap, const uint32_t *s_tab,
                                              const uint16_t *s_hot) {
    const uint32_t c = s_cmap[b];
    const bool valid = c != kNoClassDev;
    const uint32_t e = lookup<PLACE, LOG2C>(s & kStateMask, valid ? c : 0u, a, s_tab, s_hot);
    return valid ? e : 0u;
}

__device__ __forceinline__ uint32_t word_of(const uint4 &v, int d) {
    return d == 0 ? v.x : d == 1 ? v.y : d == 2 ? v.z : v.w;
}

// Walk 16 bytes from state s with the byte map; report final states at
// positions >= own_lo when `report`. Returns the state after the last byte.
// (Bytes are taken from each word by shifting, never by a runtime index,
// so the group stays in registers.)
template <int PLACE, int LOG2C>
__device__ __forceinline__ uint32_t walk_group_slow(uint32_t s, const uint4 &v, uint32_t pos,
                                                    uint32_t own_lo, bool report, const DfaArgs &a,
                                                    const uint8_t *s_cmap, const uint32_t *s_tab,
                                                    const uint16_t *s_hot, Emitter &em) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        uint32_t w = word_of(v, d);
#pragma unroll 1
        for (uint32_t j = 0; j < 4; ++j, w >>= 8) {
            const uint32_t e = step_byte<PLACE, LOG2C>(s, w & 0xffu, a, s_cmap, s_tab, s_hot);
            s = e & kStateMask;
            const uint32_t p = pos + 4u * d + j;
            emit_set(em, report && (e & kAccept) && p >= own_lo, s, uint64_t(p), a.out_off, a.out_ids);
        }
    }
    return s;
}

struct Block64 {
    uint4 g[4];
};

__device__ __forceinline__ void load_block(Block64 &b, const uint8_t *text, uint32_t p, bool ok) {
    if (ok) {
        const uint4 *q = reinterpret_cast<const uint4 *>(text + p);
        b.g[0] = q[0];
        b.g[1] = q[1];
        b.g[2] = q[2];
        b.g[3] = q[3];
    }
}

// The walkers of one lane, stepping K chunks in lockstep.
template <int PLACE, int K, int LOG2C, bool HASHED>
struct Walkers {
    const DfaArgs &a;
    const uint8_t *s_cmap;
    const uint32_t *s_tab;
    const uint16_t *s_hot;
    Emitter &em;

    // One 16-byte group per walker. Dead walkers (live false) keep their state.
    __device__ __forceinline__ void group(uint32_t (&s)[K], const uint4 (&v)[K],
                                          const uint32_t (&gpos)[K], const bool (&live)[K],
                                          const uint32_t (&own)[K]) const {
        uint32_t s0[K], flag[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            s0[k] = s[k];
            flag[k] = 0;
        }
        bool slow = true;
        uint4 h[K];
        if constexpr (HASHED) {
            const uint32_t mask4 = ((1u << LOG2C) - 1u) * 0x01010101u;
            bool bad = false;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                h[k].x = (v[k].x >> a.hash_shift) & mask4;
                h[k].y = (v[k].y >> a.hash_shift) & mask4;
                h[k].z = (v[k].z >> a.hash_shift) & mask4;
                h[k].w = (v[k].w >> a.hash_shift) & mask4;
                // a byte is in the alphabet iff it equals the letter owning its bit field
                const uint32_t d = (__builtin_amdgcn_perm(a.letters_hi, a.letters_lo, h[k].x) ^ v[k].x) |
                                   (__builtin_amdgcn_perm(a.letters_hi, a.letters_lo, h[k].y) ^ v[k].y) |
                                   (__builtin_amdgcn_perm(a.letters_hi, a.letters_lo, h[k].z) ^ v[k].z) |
                                   (__builtin_amdgcn_perm(a.letters_hi, a.letters_lo, h[k].w) ^ v[k].w);
                bad |= live[k] && d != 0;
            }
            slow = __any(bad);
        }
        if (slow) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    uint32_t w = word_of(v[k], d);
#pragma unroll 1
                    for (uint32_t j = 0; j < 4; ++j, w >>= 8) {
                        const uint32_t e = step_byte<PLACE, LOG2C>(s[k], w & 0xffu, a, s_cmap, s_tab, s_hot);
                        s[k] = e & kStateMask;
                        flag[k] |= e;
                    }
                }
            }
        } else if constexpr (HASHED) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const uint32_t sh = (j & 3) * 8;
                uint32_t c[K], e[K];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t hw = j < 4 ? h[k].x : j < 8 ? h[k].y : j < 12 ? h[k].z : h[k].w;
                    c[k] = (hw >> sh) & ((1u << LOG2C) - 1u);
                }
                if constexpr (PLACE == AC_PLACE_LDS_HOT) {
                    bool cold = false;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const bool hk = s[k] < a.hot;
                        cold |= !hk;
                        const uint32_t t = s_hot[((hk ? s[k] : 0u) << LOG2C) | c[k]];
                        e[k] = (t & kHotMask) | ((t & kHotAccept) << 16);
                    }
                    if (__any(cold)) {
#pragma unroll
                        for (int k = 0; k < K; ++k)
                            if (s[k] >= a.hot) e[k] = a.dfa[(s[k] << LOG2C) | c[k]];
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < K; ++k) e[k] = lookup<PLACE, LOG2C>(s[k], c[k], a, s_tab, s_hot);
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    s[k] = e[k] & kStateMask;
                    flag[k] |= e[k];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!live[k]) s[k] = s0[k];
            // the group passed a final state: walk it again and report
            const bool rep = live[k] && (flag[k] & kAccept);
            if (__any(rep))
                walk_group_slow<PLACE, LOG2C>(s0[k], v[k], gpos[k], own[k], rep, a, s_cmap, s_tab, s_hot, em);
        }
    }

    // The four groups of the 64-byte block in X, then refill X with the block
    // after the one the other buffer holds.
    __device__ __forceinline__ void block(Block64 (&X)[K], uint32_t (&s)[K], const uint32_t (&own)[K],
                                          const uint32_t (&wstart)[K], uint32_t (&bpos)[K],
                                          const uint32_t (&bend)[K]) const {
#pragma unroll
        for (int gi = 0; gi < 4; ++gi) {
            uint4 v[K];
            uint32_t gpos[K];
            bool live[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                v[k] = X[k].g[gi];
                gpos[k] = bpos[k] + 16u * gi;
                live[k] = bpos[k] < bend[k] && gpos[k] >= wstart[k];
            }
            group(s, v, gpos, live, own);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool more = bpos[k] < bend[k];
            bpos[k] += more ? 64u : 0u;
            load_block(X[k], a.text, bpos[k] + 64, more && bend[k] > 64 && bpos[k] < bend[k] - 64);
        }
    }
};

// Text is read in 64-byte blocks (one half cache line per lane, four
// back-to-back 16-byte loads) into two register buffers used in turn, so one
// block is in flight while the other is walked.
template <int PLACE, int K, int LOG2C, bool HASHED, int BLOCK>
__global__ void __launch_bounds__(BLOCK) dfa_kernel(DfaArgs a) {
    // LDS: per-wave match queues | byte map (256 B) | table image
    extern __shared__ __align__(16) uint8_t smem[];
    constexpr uint32_t kQueues = (BLOCK / 64) * kQueueBytesPerWave;
    uint8_t *s_cmap = smem + kQueues;
    uint32_t *s_tab = reinterpret_cast<uint32_t *>(smem + kQueues + 256);
    uint16_t *s_hot = reinterpret_cast<uint16_t *>(smem + kQueues + 256);
    const uint32_t tid = threadIdx.x;
    Emitter em;
    em.init(smem, a.out, a.cap, a.count);
    for (uint32_t i = tid; i < 64; i += BLOCK)
        reinterpret_cast<uint32_t *>(s_cmap)[i] = reinterpret_cast<const uint32_t *>(a.cmap)[i];
    if constexpr (PLACE == AC_PLACE_LDS_FULL) {
        for (uint32_t i = tid; i < a.table_words; i += BLOCK) s_tab[i] = a.dfa[i];
    } else if constexpr (PLACE == AC_PLACE_LDS_HOT) {
        const uint32_t words = (a.hot * a.n_cols + 1) / 2;  // image is padded to 4 bytes
        const uint32_t *src = reinterpret_cast<const uint32_t *>(a.hot_rows);
        for (uint32_t i = tid; i < words; i += BLOCK) reinterpret_cast<uint32_t *>(s_hot)[i] = src[i];
    }
    __syncthreads();

    const Walkers<PLACE, K, LOG2C, HASHED> W{a, s_cmap, s_tab, s_hot, em};
    const uint32_t lanes = gridDim.x * BLOCK;
    const uint32_t lane = blockIdx.x * BLOCK + tid;

    for (uint32_t base = 0; base < a.n_chunks; base += K * lanes) {
        // walker k: chunk `base + k * lanes + lane`, owning [own, hi); it walks
        // [wstart, hi) with wstart = own - m_max + 1 rounded down to 16 bytes
        // (starting earlier than needed only repeats warm-up steps).
        uint32_t s[K], own[K], hi[K], wstart[K], bpos[K], bend[K];
        Block64 A[K], B[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t ch = base + k * lanes + lane;
            const bool act = ch < a.n_chunks;
            own[k] = act ? ch * a.chunk : 0u;
            hi[k] = act ? uint32_t(min(uint64_t(own[k]) + a.chunk, uint64_t(a.n))) : 0u;
            wstart[k] = (own[k] > a.back ? own[k] - a.back : 0u) & ~15u;
            bpos[k] = wstart[k] & ~63u;
            bend[k] = hi[k] & ~63u;
            s[k] = 0;
            load_block(A[k], a.text, bpos[k], bpos[k] < bend[k]);
            load_block(B[k], a.text, bpos[k] + 64, bend[k] > 64 && bpos[k] < bend[k] - 64);
        }
        while (true) {
            bool any_left = false;
#pragma unroll
            for (int k = 0; k < K; ++k) any_left |= bpos[k] < bend[k];
            if (!__any(any_left)) break;
            W.block(A, s, own, wstart, bpos, bend);
            any_left = false;
#pragma unroll
            for (int k = 0; k < K; ++k) any_left |= bpos[k] < bend[k];
            if (!__any(any_left)) break;
            W.block(B, s, own, wstart, bpos, bend);
        }
        // bytes past the last full block (chunks whose end is not 64-aligned),
        // or the whole walk when the chunk has no full block
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (base + k * lanes + lane < a.n_chunks) {
                for (uint32_t p = max(bend[k], wstart[k]); p < hi[k]; ++p) {
                    const uint32_t e = step_byte<PLACE, LOG2C>(s[k], a.text[p], a, s_cmap, s_tab, s_hot);
                    s[k] = e & kStateMask;
                    emit_set(em, (e & kAccept) && p >= own[k], s[k], uint64_t(p), a.out_off, a.out_ids);
                }
            }
        }
    }
    em.flush();
}

template <typename Kern>
int run(Kern kernel, uint32_t grid, uint32_t block, uint32_t lds, hipStream_t stream,
        const DfaArgs &args, std::string &err) {
    return launch_kernel(kernel, grid, block, lds, stream, args, err);
}

// Instantiate the kernels for one placement and class scheme.
template <int PLACE, int BLOCK>
int dispatch(const DeviceMachine &dm, uint32_t K, uint32_t grid, uint32_t lds, hipStream_t stream,
             const DfaArgs &a, std::string &err) {
    const bool hashed = dm.hashed;
    const int l2 = hashed ? int(dm.log2_cols) : -1;
#define AC_DFA_CASE(KK, LL, HH)                                                                   \
    if (K == KK && l2 == LL && hashed == HH)                                                      \
        return run(dfa_kernel<PLACE, KK, LL, HH, BLOCK>, grid, BLOCK, lds, stream, a, err);
#define AC_DFA_KS(LL, HH) AC_DFA_CASE(1, LL, HH) AC_DFA_CASE(2, LL, HH) AC_DFA_CASE(4, LL, HH)
    AC_DFA_KS(-1, false)
    AC_DFA_KS(0, true)
    AC_DFA_KS(1, true)
    AC_DFA_KS(2, true)
    AC_DFA_KS(3, true)
#undef AC_DFA_KS
#undef AC_DFA_CASE
    err = "ac_scan: unsupported walker count";
    return AC_ERR_INVALID;
}

}  // namespace

int launch_dfa_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                    uint64_t cap, uint64_t *count, const ScanConfig &cfg, hipStream_t stream,
                    std::string &err) {
    if (n == 0) return AC_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const uint32_t cus = uint32_t(compute_units(dev));
    DfaArgs a{};
    a.text = text;
    a.n = uint32_t(n);
    a.back = dm.m_max - 1;
    a.n_cols = dm.n_cols;
    a.hot = dm.hot_states;
    a.table_words = dm.n_states * dm.n_cols;
    a.hash_shift = dm.hash_shift;
    a.letters_lo = uint32_t(dm.hash_letter[0]) | uint32_t(dm.hash_letter[1]) << 8 |
                   uint32_t(dm.hash_letter[2]) << 16 | uint32_t(dm.hash_letter[3]) << 24;
    a.letters_hi = uint32_t(dm.hash_letter[4]) | uint32_t(dm.hash_letter[5]) << 8 |
                   uint32_t(dm.hash_letter[6]) << 16 | uint32_t(dm.hash_letter[7]) << 24;
    a.dfa = dm.dfa;
    a.hot_rows = dm.hot_dfa;
    a.cmap = dm.cmap;
    a.out_off = dm.out_off;
    a.out_ids = dm.out_ids;
    a.out = out;
    a.cap = cap;
    a.count = reinterpret_cast<unsigned long long *>(count);

    const uint32_t block = cfg.placement == AC_PLACE_LDS_HOT ? 1024u : 256u;
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
    const uint32_t K = cfg.walkers ? cfg.walkers : 2u;
    if (K != 1 && K != 2 && K != 4) {
        err = "ac_scan: walkers per lane must be 1, 2 or 4";
        return AC_ERR_INVALID;
    }
    if (block == 1024 && K > 2) {  // 128 registers per lane at 1024 threads: 4 walkers would spill
        err = "ac_scan: the LDS_HOT placement runs 1 or 2 walkers per lane";
        return AC_ERR_INVALID;
    }
    const uint32_t wg_per_cu = std::max<uint32_t>(1, std::min<uint32_t>(2048 / block, kLdsPerWorkgroup / lds));
    uint64_t chunk = cfg.chunk;
    if (chunk == 0) {
        // enough walkers for every lane the chip holds, but chunks of at least
        // 4 * m_max so that the re-walked overlap stays small
        const uint64_t walkers = uint64_t(cus) * wg_per_cu * block * K;
        chunk = (n + walkers - 1) / walkers;
        chunk = std::max<uint64_t>(chunk, 4ull * dm.m_max);
        chunk = std::max<uint64_t>(64, (chunk + 63) & ~uint64_t(63));
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
    switch (cfg.placement) {
        case AC_PLACE_GLOBAL: return dispatch<AC_PLACE_GLOBAL, 256>(dm, K, grid, lds, stream, a, err);
        case AC_PLACE_LDS_FULL: return dispatch<AC_PLACE_LDS_FULL, 256>(dm, K, grid, lds, stream, a, err);
        case AC_PLACE_LDS_HOT: return dispatch<AC_PLACE_LDS_HOT, 1024>(dm, K, grid, lds, stream, a, err);
    }
    err = "ac_scan: unknown placement";
    return AC_ERR_INVALID;
}

}  // namespace acm
