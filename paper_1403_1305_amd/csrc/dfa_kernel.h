// dfa_kernel.h -- the chunked full-DFA scan kernel for gfx950 (templates;
// instantiated per table placement in dfa_place_*.hip, launched from dfa.hip).
//
// The text is cut into chunks of C bytes. Chunk k owns the end positions
// [kC, min(kC + C, n)); its walker starts from the root m_max - 1 bytes
// before kC, rounded down to 16 (or at 0), and reports only the matches that
// end inside the chunk. Every occurrence ending in the chunk starts at or
// after kC - m_max + 1, and a walk from the root reports every occurrence
// that starts at or after its first byte, so each match is reported exactly
// once.
//
// Each lane runs K walkers on K different chunks in lockstep, so K table
// lookups are in flight per lane per step. Each walker holds its text in
// registers, a block of 64 or 128 bytes at a time (the next block is read as
// the current one is walked, or in a second buffer). A walker only notes
// whether a 16-byte group passed a final state; a flagged group is walked
// again and reported (final states are rare next to plain steps).
//
// Table placements:
//   LDS_FULL  the whole 32-bit table in LDS.
//   LDS_HOT   16-bit rows of the hot states [0, H) in LDS; a state >= H is
//             looked up in the 32-bit table in global memory (L2 resident).
//             One offset per step addresses both tables. With two-byte rows
//             built, a walker outside the image looks up two bytes at once.
//   GLOBAL    every lookup from the 32-bit table in global memory.
// Byte classes are either a bit field of the byte (small alphabets, checked
// four bytes at a time with v_perm against the letter of each field value) or
// a 256-entry map in LDS.
#pragma once

#include <algorithm>

#include "../../include/ac.h"
#include "device_common.h"
#include "machine.h"
#include "scan.h"

namespace acm {
namespace dfa {

struct DfaArgs {
    const uint8_t *text;
    uint32_t n;            // text bytes (< 2^32)
    uint32_t chunk;        // bytes owned per walker (multiple of 16)
    uint32_t n_chunks;
    uint32_t back;         // m_max - 1
    uint32_t n_cols;
    uint32_t hot;          // H: states with rows in the LDS image
    uint32_t acc_end;      // final states are exactly [H, acc_end) when H > 0
    uint32_t table_words;  // LDS_FULL: n_states * n_cols
    uint32_t hash_shift;   // hashed classes: column = (b >> shift) & (n_cols - 1)
    uint32_t pair_base;    // word of dfa where the two-byte rows of states >= hot start
    uint32_t letters_lo, letters_hi;  // the letter owning each hashed column
    uint32_t no_class;     // byte-map value of bytes in no pattern (DeviceMachine::no_class)
    const uint32_t *dfa;
    const uint16_t *hot_rows;
    const uint8_t *cmap;
    const uint32_t *out_off, *out_ids;
    uint64_t *out;
    uint64_t cap;
    unsigned long long *count;
    uint64_t base;              // added to every reported end position
    const uint32_t *state_in;   // state before byte 0 (NULL = the root)
    uint32_t *state_out;        // receives the state after byte n-1 (NULL = not wanted)
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
            const uint32_t t = s_hot[idx];
            return t | (t - a.hot < a.acc_end - a.hot ? kAccept : 0u);
        }
        return a.dfa[idx];
    } else {
        return a.dfa[idx];
    }
}

// 16-bit image entry at a byte offset into the image.
__device__ __forceinline__ uint32_t lds_u16(const uint16_t *image, uint32_t byte_off) {
    return *reinterpret_cast<const uint16_t *>(reinterpret_cast<const uint8_t *>(image) + byte_off);
}

// One byte with the general byte map: bytes in no pattern reset to the root.
template <int PLACE, int LOG2C>
__device__ __forceinline__ uint32_t step_byte(uint32_t s, uint32_t b, const DfaArgs &a,
                                              const uint8_t *s_cmap, const uint32_t *s_tab,
                                              const uint16_t *s_hot) {
    const uint32_t c = s_cmap[b];
    const bool valid = c != a.no_class;
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
            emit_set(em, report && (e & kAccept) && p >= own_lo, s, a.base + p, a.out_off, a.out_ids);
        }
    }
    return s;
}

// A block of G 16-byte groups of text held in registers.
template <int G>
struct TextBlock {
    uint4 g[G];
};

template <int G>
__device__ __forceinline__ void load_block(TextBlock<G> &b, const uint8_t *text, uint32_t p, bool ok) {
    if (ok) {
        const uint4 *q = reinterpret_cast<const uint4 *>(text + p);
#pragma unroll
        for (int i = 0; i < G; ++i) b.g[i] = q[i];
    }
}

// The first block of a walk: groups wholly before the walk's first byte are
// not read (zeros stand in; those groups are never walked). A chunk's
// lead-in then requests only the end of the line before it, which the
// neighbouring walker reads again much later.
template <int G>
__device__ __forceinline__ void load_first_block(TextBlock<G> &b, const uint8_t *text, uint32_t p, bool ok,
                                                 uint32_t from) {
    if (ok) {
        const uint4 *q = reinterpret_cast<const uint4 *>(text + p);
#pragma unroll
        for (int i = 0; i < G; ++i) b.g[i] = p + 16u * (i + 1) > from ? q[i] : make_uint4(0u, 0u, 0u, 0u);
    }
}

// The walkers of one lane, stepping K chunks in lockstep. With PAIR (LDS_HOT,
// four hashed columns, two-byte rows built) a walker outside the image looks
// up two bytes at once.
template <int PLACE, int K, int LOG2C, bool HASHED, bool PAIR = false>
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
        } else if constexpr (HASHED && PAIR) {
            static_assert(PLACE == AC_PLACE_LDS_HOT && LOG2C == 2, "two-byte rows exist for the 4-column image only");
            // Two bytes per step. A walker in an image state takes the first
            // byte from the image; a walker outside it reads its two-byte row
            // in global memory, and one that leaves the image on the first byte
            // reads the second byte's row there: at most one global load per
            // walker per two bytes, so half the waits on global memory.
#pragma unroll
            for (int j = 0; j < 16; j += 2) {
                const uint32_t sh = (j & 3) * 8;
                uint32_t c1[K], c2[K], e1[K], e2[K], g[K];
                bool cs[K];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t hw = j < 4 ? h[k].x : j < 8 ? h[k].y : j < 12 ? h[k].z : h[k].w;
                    c1[k] = (hw >> sh) & 3u;
                    c2[k] = (hw >> (sh + 8)) & 3u;
                    cs[k] = s[k] >= a.hot;
                    e1[k] = lds_u16(s_hot, (min(s[k], a.hot - 1u) << 3) | (c1[k] << 1));
                }
                bool need = false;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    // second byte from the image, read before any global wait
                    e2[k] = lds_u16(s_hot, (min(e1[k], a.hot - 1u) << 3) | (c2[k] << 1));
                    need |= cs[k] || e1[k] >= a.hot;
                    g[k] = 0;
                }
                if (__any(need)) {
                    // image walkers read entry 0, one shared line
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const bool ce = !cs[k] && e1[k] >= a.hot;
                        const uint32_t idx = cs[k] ? (s[k] << 4) + (a.pair_base - (a.hot << 4)) + (c1[k] | (c2[k] << 2))
                                                   : ce ? ((e1[k] << 2) | c2[k]) : 0u;
                        g[k] = a.dfa[idx];
                    }
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        // final states: the one a walker outside the image stands
                        // in (entered at byte j-1) and the one after byte j
                        if (cs[k] && j > 0 && s[k] < a.acc_end) flag[k] |= kAccept;
                        if (cs[k])
                            flag[k] |= g[k] & kAccept;
                        else if (e1[k] - a.hot < a.acc_end - a.hot)
                            flag[k] |= kAccept;
                    }
                }
#pragma unroll
                for (int k = 0; k < K; ++k) s[k] = (cs[k] || e1[k] >= a.hot) ? (g[k] & kStateMask) : e2[k];
            }
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (s[k] - a.hot < a.acc_end - a.hot) flag[k] |= kAccept;
        } else if constexpr (HASHED && PLACE == AC_PLACE_LDS_HOT) {
            // Classes pre-scaled to the 2-byte entries of an image row: one
            // shift per word, then the step's offset u = s * row + 2c serves
            // both tables (image: u clamped to its last entry, since a lane
            // outside the image discards what it reads there; 32-bit table:
            // byte offset 2u from its base).
            uint4 h2[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                h2[k].x = h[k].x << 1;
                h2[k].y = h[k].y << 1;
                h2[k].z = h[k].z << 1;
                h2[k].w = h[k].w << 1;
                // hide the known-zero bits, so that each class below stays one
                // bit-field extract instead of a shift and a mask (no code)
                asm volatile("" : "+v"(h2[k].x), "+v"(h2[k].y), "+v"(h2[k].z), "+v"(h2[k].w));
            }
            const uint32_t last = (a.hot << (LOG2C + 1)) - 2u;
            const uint8_t *img = reinterpret_cast<const uint8_t *>(s_hot);
            const uint8_t *tab = reinterpret_cast<const uint8_t *>(a.dfa);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const uint32_t sh = (j & 3) * 8;
                uint32_t u[K], e[K];
                bool cold = false;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t hw = j < 4 ? h2[k].x : j < 8 ? h2[k].y : j < 12 ? h2[k].z : h2[k].w;
                    u[k] = (s[k] << (LOG2C + 1)) | __builtin_amdgcn_ubfe(hw, sh, LOG2C + 1);
                    cold |= s[k] >= a.hot;
                    e[k] = *reinterpret_cast<const uint16_t *>(img + min(u[k], last));
                }
                if (__any(cold)) {
                    // all K loads go out before any is waited on; image lanes
                    // read entry 0, one shared line
                    uint32_t g[K];
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        g[k] = *reinterpret_cast<const uint32_t *>(tab + (s[k] >= a.hot ? u[k] << 1 : 0u));
                    // every lane issues its load (kept out of a branch on the
                    // lane's own state, which measured slower; no code)
#pragma unroll
                    for (int k = 0; k < K; ++k) asm volatile("" ::"v"(g[k]));
                    // Every final state is outside the image, so a walker that
                    // entered one at byte j-1 is here: its matches are reported
                    // at once (no second walk of the group).
                    bool fin[K];
                    bool any_fin = false;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const bool ck = s[k] >= a.hot;
                        fin[k] = s[k] - a.hot < a.acc_end - a.hot;  // final (and so outside the image)
                        any_fin |= fin[k];
                        e[k] = ck ? (g[k] & kStateMask) : e[k];
                    }
                    if (j > 0 && __builtin_expect(__any(any_fin), 0)) {
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            const uint32_t p = gpos[k] + uint32_t(j - 1);
                            const bool has = fin[k] && live[k] && p >= own[k];
                            if (__any(has)) emit_set(em, has, s[k], a.base + p, a.out_off, a.out_ids);
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < K; ++k) s[k] = e[k];
            }
            // the state after byte 15
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool fin = s[k] - a.hot < a.acc_end - a.hot;
                if (__builtin_expect(__any(fin), 0)) {
                    const bool has = fin && live[k] && gpos[k] + 15u >= own[k];
                    if (__any(has)) emit_set(em, has, s[k], a.base + gpos[k] + 15u, a.out_off, a.out_ids);
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
                // the whole table in LDS, or every lookup from global memory
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    e[k] = lookup<PLACE, LOG2C>(s[k], c[k], a, s_tab, s_hot);
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

    template <int GI, int G>
    __device__ __forceinline__ void group_of(const TextBlock<G> (&X)[K], uint32_t (&s)[K],
                                             const uint32_t (&own)[K], const uint32_t (&wstart)[K],
                                             const uint32_t (&bpos)[K], const uint32_t (&bend)[K]) const {
        uint4 v[K];
        uint32_t gpos[K];
        bool live[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            v[k] = X[k].g[GI];
            gpos[k] = bpos[k] + 16u * GI;
            live[k] = bpos[k] < bend[k] && gpos[k] >= wstart[k];
        }
        group(s, v, gpos, live, own);
    }

    // The groups of the block in X (G groups of 16 bytes), then refill X with
    // the block `ahead` bytes on (two blocks on when another buffer holds the
    // next one, one block on when X is the only buffer).
    template <int G>
    __device__ __forceinline__ void block(TextBlock<G> (&X)[K], uint32_t (&s)[K], const uint32_t (&own)[K],
                                          const uint32_t (&wstart)[K], uint32_t (&bpos)[K],
                                          const uint32_t (&bend)[K], uint32_t ahead) const {
        // (groups written out one by one: a runtime group index would push X to scratch)
        group_of<0>(X, s, own, wstart, bpos, bend);
        group_of<1>(X, s, own, wstart, bpos, bend);
        group_of<2>(X, s, own, wstart, bpos, bend);
        group_of<3>(X, s, own, wstart, bpos, bend);
        if constexpr (G == 8) {
            group_of<4>(X, s, own, wstart, bpos, bend);
            group_of<5>(X, s, own, wstart, bpos, bend);
            group_of<6>(X, s, own, wstart, bpos, bend);
            group_of<7>(X, s, own, wstart, bpos, bend);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool more = bpos[k] < bend[k];
            const bool fetch = more && bend[k] - bpos[k] > ahead;  // bpos + ahead < bend
            const uint32_t next = bpos[k] + ahead;
            bpos[k] += more ? uint32_t(16 * G) : 0u;
            load_block(X[k], a.text, next, fetch);
        }
    }
};

// Copy `bytes` (a multiple of 4) from global memory to LDS, both 16-byte
// aligned: 16-byte pieces with four loads in flight per thread before their
// stores, then the last words.
template <int BLOCK>
__device__ __forceinline__ void copy_to_lds(void *dst, const void *src, uint32_t bytes) {
    const uint32_t tid = threadIdx.x;
    const uint32_t n16 = bytes / 16;
    const uint4 *s = reinterpret_cast<const uint4 *>(src);
    uint4 *d = reinterpret_cast<uint4 *>(dst);
    uint32_t i = tid;
    for (; i + 3 * BLOCK < n16; i += 4 * BLOCK) {
        const uint4 v0 = s[i], v1 = s[i + BLOCK], v2 = s[i + 2 * BLOCK], v3 = s[i + 3 * BLOCK];
        d[i] = v0;
        d[i + BLOCK] = v1;
        d[i + 2 * BLOCK] = v2;
        d[i + 3 * BLOCK] = v3;
    }
    for (; i < n16; i += BLOCK) d[i] = s[i];
    for (uint32_t w = n16 * 4 + tid; w < bytes / 4; w += BLOCK)
        static_cast<uint32_t *>(dst)[w] = static_cast<const uint32_t *>(src)[w];
}

// The byte map and, for the LDS placements, the table image of `a` into LDS.
// Every thread of the workgroup takes part; ends with a barrier.
template <int PLACE, int BLOCK>
__device__ __forceinline__ void load_tables(const DfaArgs &a, uint8_t *s_cmap, uint32_t *s_tab,
                                            uint16_t *s_hot) {
    copy_to_lds<BLOCK>(s_cmap, a.cmap, 256);
    if constexpr (PLACE == AC_PLACE_LDS_FULL)
        copy_to_lds<BLOCK>(s_tab, a.dfa, a.table_words * 4u);
    else if constexpr (PLACE == AC_PLACE_LDS_HOT)
        copy_to_lds<BLOCK>(s_hot, a.hot_rows, ((a.hot * a.n_cols + 1) / 2) * 4u);  // image padded to 4 bytes
    __syncthreads();
}

// Text is read per walker in blocks of G 16-byte groups (64 or 128 bytes: a
// half or a whole cache line, loaded back to back). With NBUF = 2 two register
// buffers are used in turn, so one block is in flight while the other is
// walked; with NBUF = 1 the next block is requested as soon as a block is
// finished (fewer registers, and whole lines are never fetched twice).
//
// Walker k owns end positions [own[k], hi[k]) and walks [wstart[k], hi[k])
// (wstart a multiple of 16) from state s[k]; a walker without a chunk has
// own = hi = wstart = 0 and walks nothing. On return s[k] is the state after
// byte hi[k] - 1.
template <int PLACE, int K, int LOG2C, bool HASHED, int NBUF, int G, bool PAIR = false>
__device__ __forceinline__ void walk_chunks(const Walkers<PLACE, K, LOG2C, HASHED, PAIR> &W, const DfaArgs &a,
                                            Emitter &em, const uint8_t *s_cmap, const uint32_t *s_tab,
                                            const uint16_t *s_hot, uint32_t (&s_io)[K],
                                            const uint32_t (&own_in)[K], const uint32_t (&hi_in)[K],
                                            const uint32_t (&wstart_in)[K]) {
    constexpr uint32_t BB = 16u * G;  // bytes per block
    // Local copies: the compiler simplifies this function before inlining it,
    // and walking through the callers' arrays then costs enough registers to
    // spill the hashed two-walker kernels.
    uint32_t s[K], own[K], hi[K], wstart[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        s[k] = s_io[k];
        own[k] = own_in[k];
        hi[k] = hi_in[k];
        wstart[k] = wstart_in[k];
    }
    uint32_t bpos[K], bend[K];
    TextBlock<G> A[K], B[NBUF == 2 ? K : 1];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        bpos[k] = wstart[k] & ~(BB - 1);
        bend[k] = hi[k] & ~(BB - 1);
        load_first_block(A[k], a.text, bpos[k], bpos[k] < bend[k], wstart[k]);
        if constexpr (NBUF == 2)
            load_block(B[k], a.text, bpos[k] + BB, bend[k] > BB && bpos[k] < bend[k] - BB);
    }
    while (true) {
        bool any_left = false;
#pragma unroll
        for (int k = 0; k < K; ++k) any_left |= bpos[k] < bend[k];
        if (!__any(any_left)) break;
        W.block(A, s, own, wstart, bpos, bend, NBUF * BB);
        if constexpr (NBUF == 2) {
            any_left = false;
#pragma unroll
            for (int k = 0; k < K; ++k) any_left |= bpos[k] < bend[k];
            if (!__any(any_left)) break;
            W.block(B, s, own, wstart, bpos, bend, 2 * BB);
        }
    }
    // bytes past the last full block (chunks whose end is not block-aligned),
    // or the whole walk when the chunk has no full block
#pragma unroll
    for (int k = 0; k < K; ++k) {
        for (uint32_t p = max(bend[k], wstart[k]); p < hi[k]; ++p) {
            const uint32_t e = step_byte<PLACE, LOG2C>(s[k], a.text[p], a, s_cmap, s_tab, s_hot);
            s[k] = e & kStateMask;
            emit_set(em, (e & kAccept) && p >= own[k], s[k], a.base + p, a.out_off, a.out_ids);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) s_io[k] = s[k];
}

template <int PLACE, int K, int LOG2C, bool HASHED, int BLOCK, int NBUF, int G, bool PAIR = false>
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
    load_tables<PLACE, BLOCK>(a, s_cmap, s_tab, s_hot);

    const Walkers<PLACE, K, LOG2C, HASHED, PAIR> W{a, s_cmap, s_tab, s_hot, em};
    const uint32_t lanes = gridDim.x * BLOCK;
    const uint32_t lane = blockIdx.x * BLOCK + tid;

    for (uint32_t base = 0; base < a.n_chunks; base += K * lanes) {
        // walker k: chunk `base + k * lanes + lane`, owning [own, hi); it walks
        // [wstart, hi) with wstart = own - m_max + 1 rounded down to 16 bytes
        // (starting earlier than needed only repeats warm-up steps).
        uint32_t s[K], own[K], hi[K], wstart[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t ch = base + k * lanes + lane;
            const bool act = ch < a.n_chunks;
            own[k] = act ? ch * a.chunk : 0u;
            hi[k] = act ? uint32_t(min(uint64_t(own[k]) + a.chunk, uint64_t(a.n))) : 0u;
            wstart[k] = (own[k] > a.back ? own[k] - a.back : 0u) & ~15u;
            // a walk that would start before byte 0 starts there instead, in the
            // state the text's earlier pieces ended in (the root for a new text)
            s[k] = (act && own[k] <= a.back && a.state_in) ? *a.state_in : 0u;
        }
        walk_chunks<PLACE, K, LOG2C, HASHED, NBUF, G, PAIR>(W, a, em, s_cmap, s_tab, s_hot, s, own, hi, wstart);
        // the last chunk's walker ends exactly in the text's final state: it
        // walked at least m_max bytes or started from the carried state
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (base + k * lanes + lane == a.n_chunks - 1 && a.state_out) *a.state_out = s[k];
    }
    em.flush();
}

// ------------------------------------------------------------------ batches
// Many texts in one buffer, each with its own automaton. The host cuts every
// text into work items (chunks) and groups the items of one automaton into
// tasks of at most one item per walker. Workgroups take tasks from a shared
// counter, so tasks are handed out in increasing order: a workgroup meets the
// automata in order and reloads its LDS image at most once per automaton,
// while fast and slow automata still balance across the grid.
struct BatchItem {
    uint32_t own_lo, own_hi;  // end positions this item reports, in the batch buffer
    uint32_t text_lo;         // first byte of its text (a multiple of 16)
    uint32_t pad;
};
struct BatchTask {
    uint32_t item_begin, item_end;  // items [item_begin, item_end) of one automaton,
                                    // at most one per walker of a workgroup
    uint32_t automaton;
    uint32_t pad;
};
struct BatchArgs {
    const uint8_t *text;
    const BatchItem *items;
    const BatchTask *tasks;
    uint32_t n_tasks;
    const DfaArgs *autos;  // per automaton: tables, sizes and class scheme
    uint64_t *out;
    uint64_t cap;
    unsigned long long *count;
    uint32_t *next_task;   // task counter, zero at launch
    const uint32_t *n_tasks_dev;  // if set, the task count is read here (a plan built on the device)
};

template <int PLACE, int K, int LOG2C, bool HASHED, int BLOCK, int NBUF, int G>
__global__ void __launch_bounds__(BLOCK) batch_kernel(BatchArgs b) {
    extern __shared__ __align__(16) uint8_t smem[];
    constexpr uint32_t kQueues = (BLOCK / 64) * kQueueBytesPerWave;
    uint8_t *s_cmap = smem + kQueues;
    uint32_t *s_tab = reinterpret_cast<uint32_t *>(smem + kQueues + 256);
    uint16_t *s_hot = reinterpret_cast<uint16_t *>(smem + kQueues + 256);
    const uint32_t tid = threadIdx.x;
    __shared__ uint32_t s_task;
    Emitter em;
    em.init(smem, b.out, b.cap, b.count);
    const uint32_t n_tasks = b.n_tasks_dev ? __builtin_amdgcn_readfirstlane(*b.n_tasks_dev) : b.n_tasks;
    uint32_t loaded = 0xffffffffu;
    while (true) {
        // the first barrier also ends every thread's previous task, so the
        // LDS image may be replaced below; the second lets thread 0 reuse s_task
        if (tid == 0) s_task = atomicAdd(b.next_task, 1u);
        __syncthreads();
        // uniform across the workgroup: keeps the task and its automaton's
        // arguments in scalar registers
        const uint32_t t = __builtin_amdgcn_readfirstlane(s_task);
        __syncthreads();
        if (t >= n_tasks) break;
        const BatchTask task = b.tasks[t];
        DfaArgs a = b.autos[task.automaton];
        a.text = b.text;
        a.out = b.out;
        a.cap = b.cap;
        a.count = b.count;
        a.base = 0;
        a.state_in = nullptr;
        a.state_out = nullptr;
        if (task.automaton != loaded) {
            load_tables<PLACE, BLOCK>(a, s_cmap, s_tab, s_hot);
            loaded = task.automaton;
        }
        const Walkers<PLACE, K, LOG2C, HASHED> W{a, s_cmap, s_tab, s_hot, em};
        // a task holds at most one item per walker (K x BLOCK)
        uint32_t s[K], own[K], hi[K], wstart[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t i = task.item_begin + k * BLOCK + tid;
            const BatchItem it = i < task.item_end ? b.items[i] : BatchItem{0, 0, 0, 0};
            own[k] = it.own_lo;
            hi[k] = it.own_hi;
            // the walk never starts before its own text
            wstart[k] = (own[k] - it.text_lo > a.back ? own[k] - a.back : it.text_lo) & ~15u;
            s[k] = 0;
        }
        walk_chunks<PLACE, K, LOG2C, HASHED, NBUF, G>(W, a, em, s_cmap, s_tab, s_hot, s, own, hi, wstart);
    }
    em.flush();
}

// Table pointers, sizes and class scheme of a machine (the text, output and
// chunking fields are left for the caller).
inline void fill_machine_args(const DeviceMachine &dm, DfaArgs &a) {
    a.back = dm.m_max - 1;
    a.n_cols = dm.n_cols;
    a.hot = dm.hot_states;
    a.acc_end = dm.acc_end;
    a.table_words = dm.n_states * dm.n_cols;
    a.hash_shift = dm.hash_shift;
    a.pair_base = dm.pair_base;
    a.letters_lo = uint32_t(dm.hash_letter[0]) | uint32_t(dm.hash_letter[1]) << 8 |
                   uint32_t(dm.hash_letter[2]) << 16 | uint32_t(dm.hash_letter[3]) << 24;
    a.letters_hi = uint32_t(dm.hash_letter[4]) | uint32_t(dm.hash_letter[5]) << 8 |
                   uint32_t(dm.hash_letter[6]) << 16 | uint32_t(dm.hash_letter[7]) << 24;
    a.dfa = dm.dfa;
    a.hot_rows = dm.hot_dfa;
    a.cmap = dm.cmap;
    a.no_class = dm.no_class;
    a.out_off = dm.out_off;
    a.out_ids = dm.out_ids;
}

using DfaKernel = void (*)(DfaArgs);

// Kernel for one walker count, block size and class scheme of a placement.
// One or two walkers: 128-byte blocks in one buffer, or 64-byte blocks in two;
// three or four walkers: 64-byte blocks in one buffer (the registers for
// longer blocks would spill). ONLY_K != 0 instantiates that walker count
// only (the image kernels are split over translation units by walker count,
// which compile in parallel).
template <int PLACE, int ONLY_K = 0>
DfaKernel select_for(const DeviceMachine &dm, uint32_t K, uint32_t block_bytes) {
    const bool hashed = dm.hashed;
    const int l2 = hashed ? int(dm.log2_cols) : -1;
    constexpr bool kHot = PLACE == AC_PLACE_LDS_HOT;
#define AC_DFA_V(KK, LL, HH, NB, GG)                                                                \
    return dfa_kernel<PLACE, KK, LL, HH, (kHot ? (KK == 4 ? 768 : 1024) : 256), NB, GG>;
#define AC_DFA_CASE(KK, LL, HH)                                                                     \
    if constexpr (ONLY_K == 0 || ONLY_K == KK) {                                                    \
        if (K == KK && l2 == LL && hashed == HH) {                                                  \
            if constexpr (KK >= 3) { AC_DFA_V(KK, LL, HH, 1, 4) }                                   \
            else if (block_bytes == 128) { AC_DFA_V(KK, LL, HH, 1, 8) }                             \
            else { AC_DFA_V(KK, LL, HH, 2, 4) }                                                     \
        }                                                                                           \
    }
#define AC_DFA_KS(LL, HH) \
    AC_DFA_CASE(1, LL, HH) AC_DFA_CASE(2, LL, HH) AC_DFA_CASE(3, LL, HH) AC_DFA_CASE(4, LL, HH)
    AC_DFA_KS(-1, false)
    AC_DFA_KS(0, true)
    AC_DFA_KS(1, true)
    AC_DFA_KS(2, true)
    AC_DFA_KS(3, true)
#undef AC_DFA_KS
#undef AC_DFA_CASE
#undef AC_DFA_V
    return nullptr;
}

using BatchKernel = void (*)(BatchArgs);

// Batch kernel for a placement (LDS_HOT or GLOBAL), walker count, block size
// and class scheme (shared by every automaton of the batch); ONLY_K as for
// select_for.
template <int PLACE, int ONLY_K = 0>
BatchKernel select_batch_for(bool hashed, int l2, uint32_t K, uint32_t block_bytes) {
    constexpr bool kHot = PLACE == AC_PLACE_LDS_HOT;
#define AC_B_V(KK, LL, HH, NB, GG)                                                                  \
    return batch_kernel<PLACE, KK, LL, HH, (kHot ? (KK == 4 ? 768 : 1024) : 256), NB, GG>;
#define AC_B_CASE(KK, LL, HH)                                                                       \
    if constexpr (ONLY_K == 0 || ONLY_K == KK) {                                                    \
        if (K == KK && l2 == LL && hashed == HH) {                                                  \
            if constexpr (KK >= 3) { AC_B_V(KK, LL, HH, 1, 4) }                                     \
            else { AC_B_V(KK, LL, HH, 1, 8) }                                                       \
        }                                                                                           \
    }
#define AC_B_KS(LL, HH) AC_B_CASE(1, LL, HH) AC_B_CASE(2, LL, HH) AC_B_CASE(3, LL, HH) AC_B_CASE(4, LL, HH)
    AC_B_KS(-1, false)
    AC_B_KS(0, true)
    AC_B_KS(1, true)
    AC_B_KS(2, true)
    AC_B_KS(3, true)
#undef AC_B_KS
#undef AC_B_CASE
#undef AC_B_V
    return nullptr;
}

BatchKernel select_batch_hot(bool hashed, int l2, uint32_t K, uint32_t block_bytes);
BatchKernel select_batch_global(bool hashed, int l2, uint32_t K, uint32_t block_bytes);

DfaKernel select_global(const DeviceMachine &dm, uint32_t K, uint32_t block_bytes);
DfaKernel select_full(const DeviceMachine &dm, uint32_t K, uint32_t block_bytes);
DfaKernel select_hot(const DeviceMachine &dm, uint32_t K, uint32_t block_bytes);
// select_hot for two, three and four walkers (translation units of their own)
DfaKernel select_hot_k2(const DeviceMachine &dm, uint32_t block_bytes);
DfaKernel select_hot_k3(const DeviceMachine &dm, uint32_t block_bytes);
DfaKernel select_hot_k4(const DeviceMachine &dm, uint32_t block_bytes);
BatchKernel select_batch_hot_k2(bool hashed, int l2, uint32_t block_bytes);
BatchKernel select_batch_hot_k3(bool hashed, int l2, uint32_t block_bytes);
BatchKernel select_batch_hot_k4(bool hashed, int l2, uint32_t block_bytes);
// LDS_HOT with two-byte rows (four hashed columns); nullptr for other machines.
DfaKernel select_hot_pair(const DeviceMachine &dm, uint32_t K, uint32_t block_bytes);

}  // namespace dfa
}  // namespace acm
