// gate.hip -- the failure-less scan from gated start positions (AC_ALGO_GATED).
//
// Every occurrence of a pattern begins at exactly one start position, and the
// failure-less machine (the goto function with the patterns that end at each
// state, the paper's Sec. II.B and IV.A) walked from that position finds every
// pattern that begins there. Most positions begin no pattern at all, and the
// bytes from the position on decide it: the 2-bit classes of the next
// kGateQ bytes form a 20-bit code, and a bitmap over every code, held in
// LDS, marks those some pattern can begin with. A start that passes is
// checked once more against a small hashed bitmap (also in LDS) over the
// classes of kGateQ + 2 bytes, and only then walked; a table over the 20-bit
// codes takes the walk's first kGateQ steps in one lookup.
//
// A wave step reads 1 KiB of text, 16 bytes per lane in one coalesced load,
// and owns the last 1008 of them: lane 0 holds the 16 bytes before, so that
// every lane finds the 9 bytes before its own in the lane below it and tests
// the 16 windows that end in its bytes. Steps are handed to the waves of the
// grid in turn. Starts that pass the first level go to a per-wave queue in
// LDS; there they are tested against the second level 64 at a time, and
// whenever 63 or more have passed both, the wave walks 64 of them, one per
// lane.
// Every start position belongs to the one window that begins at it, so each
// occurrence is found once.
#include <algorithm>
#include <cstring>

#include "device_common.h"
#include "machine.h"
#include "scan.h"

namespace acm {
namespace {

constexpr uint32_t kGateBlock = 1024;
constexpr uint32_t kGateWaves = kGateBlock / 64;
constexpr uint32_t kLaneBytes = 16;
constexpr uint32_t kOwnBytes = 63 * kLaneBytes;  // text a wave step owns
constexpr uint32_t kPrefetch = 4;                // wave steps loaded ahead
constexpr uint32_t kStartQueue = 125;            // queued start positions per wave: 62 + 63
constexpr uint32_t kEmitSlots = 8;               // matches queued per lane (a wave flushes up to 512)
constexpr uint32_t kBatchEmitSlots = 4;          // the same in the batched kernel (fewer registers free)
constexpr uint32_t kBitmapBytes = kGateCodes / 8;
constexpr uint32_t kBitmapWords = kGateCodes / 32;
constexpr uint32_t kBitmap2Words = kGate2Bits / 32;
constexpr uint32_t kGateLds =
    kBitmapBytes + kBitmap2Words * 4 + kGateWaves * (kStartQueue * 8 + kQueueBytesPerWave) + (kGateWaves + 2) * 4;
static_assert(kGateLds <= kLdsPerWorkgroup, "gate kernel LDS");
static_assert(kGateQ == 10 && kGateQ2 == 12, "the window extraction below assumes 10- and 12-byte windows");

struct GateArgs {
    const uint8_t *text;
    uint32_t n;
    uint32_t base;            // added to every reported end position
    uint32_t shift;           // class of byte b = (b >> shift) & 3
    uint32_t letters;         // byte c = the letter of class c
    const uint32_t *bits, *bits2, *node, *go, *own_off, *own_ids, *path_off, *path_ids, *pat_len;
    const uint32_t *own_one, *path_one;  // the single pattern of a state or path, or kOneMany
    uint64_t *out;
    uint64_t cap;
    unsigned long long *count;
    Completion done;
};

// Classes of 16 bytes, byte i in bits 2i and 2i+1. A dot product with the
// weights 1, 4, 16, 64 gathers the four (still shifted) classes of a word.
__device__ __forceinline__ uint32_t pack_classes(const uint4 &v, uint32_t shift) {
    const uint32_t m = 0x03030303u << shift;
    const uint32_t w = 0x40100401u;
    const uint32_t p0 = __builtin_amdgcn_udot4(v.x & m, w, 0u, false);
    const uint32_t p1 = __builtin_amdgcn_udot4(v.y & m, w, 0u, false);
    const uint32_t p2 = __builtin_amdgcn_udot4(v.z & m, w, 0u, false);
    const uint32_t p3 = __builtin_amdgcn_udot4(v.w & m, w, 0u, false);
    return (p0 >> shift) | (p1 << (8 - shift)) | (p2 << (16 - shift)) | (p3 << (24 - shift));
}

// 16 bytes the text streams past once (non-temporal: they need not stay in
// the caches, which then keep the walks' tables).
__device__ __forceinline__ uint4 load_stream(const uint8_t *p) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    return make_uint4(x[0], x[1], x[2], x[3]);
}

// Bytes [p, p + 12) as three words (p < n; bytes at or past n are garbage).
__device__ __forceinline__ void load12(const GateArgs &a, uint32_t p, uint32_t (&b)[3]) {
    const uint32_t last = (a.n - 1) & ~3u;
    const uint32_t *t = reinterpret_cast<const uint32_t *>(a.text);
    const uint32_t a0 = p & ~3u;
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = t[min(a0 + 4u * i, last) >> 2];
    const uint32_t sh = p & 3u;
#pragma unroll
    for (int i = 0; i < 3; ++i) b[i] = __builtin_amdgcn_alignbyte(w[i + 1], w[i], sh);
}

// How many of the (at most 12) bytes in b are letters of the alphabet before
// the first that is not.
__device__ __forceinline__ uint32_t letter_run(const GateArgs &a, const uint32_t (&b)[3]) {
    uint32_t run = 12;
#pragma unroll
    for (int i = 2; i >= 0; --i) {
        const uint32_t cls = (b[i] >> a.shift) & 0x03030303u;
        const uint32_t bad = __builtin_amdgcn_perm(0u, a.letters, cls) ^ b[i];
        if (bad) run = 4u * i + (uint32_t(__builtin_ctz(bad)) >> 3);
    }
    return run;
}

// Goto walks from node x of the lanes with `active`, over the bytes from i
// on: each step into a state where patterns end reports them at that byte.
// A walk ends at the first missing edge, a byte outside the alphabet or the
// end of the text.
template <class Em>
__device__ __forceinline__ void walk_on(const GateArgs &a, bool active, uint32_t x, uint32_t i,
                                        Em &em) {
    while (__any(active)) {
        uint32_t g = 0;
        if (active) {
            if (i >= a.n) {
                active = false;
            } else {
                const uint32_t b = a.text[i];
                const uint32_t c = (b >> a.shift) & 3u;
                const bool letter = ((a.letters >> (8u * c)) & 0xffu) == b;
                g = letter ? a.go[x * 4u + c] : 0u;
                active = g != 0u;
                if (active) x = g & kStateMask;
            }
        }
        emit_set(em, active && (g & kAccept), x, i + a.base, a.own_off, a.own_ids);
        ++i;
    }
}

// The goto entry for byte B at position i from state x (lanes with `active`):
// 0 past the text's end, for a byte outside the alphabet or a missing edge.
__device__ __forceinline__ uint32_t go_entry(const GateArgs &a, bool active, uint32_t x, uint32_t B, uint32_t i) {
    if (!active || i >= a.n) return 0u;
    const uint32_t c = (B >> a.shift) & 3u;
    return ((a.letters >> (8u * c)) & 0xffu) == B ? a.go[x * 4u + c] : 0u;
}

// One step of the walks beyond the window: g is each lane's goto entry for the
// byte at i (0 once its walk has ended), B1 the byte at i + 1. The state's
// single pattern and the next goto entry are both requested before the match
// is reported, so a step waits for one lookup, not three. Returns false once
// every walk of the wave has ended.
template <class Em>
__device__ __forceinline__ bool walk_step(const GateArgs &a, uint32_t &g, uint32_t &x, uint32_t i, uint32_t B1,
                                          Em &em) {
    if (!__any(g != 0u)) return false;
    const bool active = g != 0u;
    if (active) x = g & kStateMask;
    const bool acc = active && (g & kAccept);
    const uint32_t one = acc ? a.own_one[x] : 0u;
    const uint32_t gn = go_entry(a, active, x, B1, i + 1u);
    // the patterns ending here: the state's single one, or its list
    const bool many = acc && one == kOneMany;
    uint32_t k = 0, ke = acc ? 1u : 0u;
    if (__any(many) && many) {
        k = a.own_off[x];
        ke = a.own_off[x + 1];
    }
    while (__any(k < ke)) {
        const bool h = k < ke;
        const uint32_t id = !h ? 0u : many ? a.own_ids[k] : one;
        em.emit(h, (uint64_t(i + a.base) << 32) | id);
        k += h ? 1u : 0u;
    }
    g = gn;
    return true;
}

// Walk the start positions p (lanes with `has`), whose window code is `code`:
// the patterns that end within the window come from the gate table's node
// (its single pattern, or its list), the longer ones from the goto walk
// beyond it. The walk's bytes are loaded a step ahead, so a step waits for
// its goto lookup alone.
template <class Em>
__device__ __forceinline__ void walk_starts(const GateArgs &a, bool has, uint32_t p, uint32_t code,
                                            Em &em) {
    const uint32_t e = has ? a.node[code] : 0u;
    uint32_t b[3] = {0u, 0u, 0u};
    if (has) load12(a, p, b);
    const uint32_t d = (e >> kGateNodeBits) & 31u;
    uint32_t x = e & kGateNodeMask;
    const uint32_t run = has ? min(letter_run(a, b), d) : 0u;
    const bool hp = has && (e & kGatePathFlag);
    const uint32_t one = hp ? a.path_one[x] : kOneMany;
    const bool deep = has && d == kGateQ && run == kGateQ;
    static_assert(kGateQ == 10, "bytes 10 and 11 of the start are the last two of b");
    uint32_t g = go_entry(a, deep, x, (b[2] >> 16) & 0xffu, p + kGateQ);
    // patterns ending within the window that lie within the letters read:
    // the path's single one, or its list
    const bool many = hp && one == kOneMany;
    uint32_t k = 0, ke = hp ? 1u : 0u;
    if (__any(many) && many) {
        k = a.path_off[x];
        ke = a.path_off[x + 1];
    }
    while (__any(k < ke)) {
        const bool h = k < ke;
        const uint32_t id = !h ? 0u : many ? a.path_ids[k] : one & 0x0fffffffu;
        const uint32_t len = !h ? 0u : many ? a.pat_len[id] : one >> 28;
        em.emit(h && len <= run, (uint64_t(p + len - 1 + a.base) << 32) | id);
        k += h ? 1u : 0u;
    }
    // the walks beyond the window
    uint32_t B1 = b[2] >> 24;  // byte 11
    for (uint32_t i = p + kGateQ;; ++i) {
        const uint32_t B2 = g != 0u && i + 2u < a.n ? uint32_t(a.text[i + 2u]) : 0u;
        if (!walk_step(a, g, x, i, B1, em)) break;
        B1 = B2;
    }
}

// Queue entries are {start, classes of the 12 bytes from the start (first
// byte in the lowest bits) | kNoSecond when the second level does not apply}.
constexpr uint32_t kNoSecond = 0x80000000u;

// Walk up to 64 of the qn starts queued at q, one per lane; returns how many
// wait afterwards.
template <class Em>
__device__ __forceinline__ uint32_t drain_starts(const GateArgs &a, const uint2 *q, uint32_t qn, Em &em) {
    const uint32_t lane = __lane_id();
    const uint32_t took = min(qn, 64u);
    __builtin_amdgcn_wave_barrier();
    const uint2 e = lane < took ? q[qn - took + lane] : make_uint2(0u, 0u);
    __builtin_amdgcn_wave_barrier();
    walk_starts(a, lane < took, e.x, e.y & (kGateCodes - 1u), em);
    return qn - took;
}

// Test the queued starts [qf, qn) against the second level, 64 at a time (one
// LDS read for all of them), and keep those that pass, in order, from qf on;
// returns the queue's new length. A round reads all its entries before it
// writes any, and writes only at or below the lowest index it read.
__device__ __forceinline__ uint32_t filter_starts(const uint32_t *s_bits2, uint2 *q, uint32_t qf, uint32_t qn) {
    const uint32_t lane = __lane_id();
    uint32_t wr = qf;
    for (uint32_t rd = qf; rd < qn; rd += 64u) {
        const uint32_t t = min(qn - rd, 64u);
        __builtin_amdgcn_wave_barrier();
        const uint2 e = lane < t ? q[rd + lane] : make_uint2(0u, 0u);
        bool keep = false;
        if (lane < t) {
            const uint32_t y = e.y & 0xffffffu, h = gate2_hash(y), h2 = gate2_hash2(y);
            keep = (e.y & kNoSecond) != 0u || (__builtin_amdgcn_ubfe(s_bits2[h >> 5], h, 1u) &
                                                __builtin_amdgcn_ubfe(s_bits2[h2 >> 5], h2, 1u)) != 0u;
        }
        const uint64_t ks = __ballot(keep);
        __builtin_amdgcn_wave_barrier();
        if (keep) q[wr + lane_rank(ks)] = e;
        wr += uint32_t(__popcll(ks));
    }
    return wr;
}

// The windows of one wave step. Lane l (l >= 1) owns the 16 bytes at pos and
// holds their classes in W; P holds the lane below's (the 16 bytes before),
// Wn the lane above's. Bit j of the result is set when the window ending at
// the lane's byte j passes the first level.
__device__ __forceinline__ uint32_t test_windows(const uint32_t *s_bits, uint32_t W, uint32_t P) {
    // window ending at byte j of the lane: classes of bytes j-9 .. j, bits
    // 14 + 2j on in the 64-bit word P:W
    uint32_t m = 0;
#pragma unroll
    for (uint32_t j = 0; j < 16; ++j) {
        const uint32_t r = j <= 8 ? __builtin_amdgcn_alignbit(W, P, 14u + 2u * j) : (W >> (2u * j - 18u));
        const uint32_t word = s_bits[(r >> 5) & (kBitmapWords - 1u)];
        // bit r mod 32 of the word (the field offset takes r's low 5 bits)
        m |= __builtin_amdgcn_ubfe(word, r, 1u) << j;
    }
    return m;
}

// Queue the starts of the windows in m (as test_windows gives them) at q with
// their 12-byte class string (qn queued, the first qf of them already through
// the second level; the same in every lane), taking their bits out of m.
// With SECOND the second level applies where the lane holds those 12 bytes.
// Whenever 63 or more wait (a queue below 63 takes a round's at most 63 new
// ones) the new ones are filtered; if 63 or more remain, it returns false,
// and the caller walks 64 of them and calls again with what is left in m.
// There is no LDS read per window: the second level is tested on 64 queued
// starts at once (filter_starts).
template <bool SECOND>
__device__ __forceinline__ bool push_starts(const uint32_t *s_bits2, uint32_t W, uint32_t P, uint32_t Wn,
                                            uint32_t pos, uint32_t &m, uint2 *q, uint32_t &qn, uint32_t &qf) {
    const uint32_t lane = __lane_id();
    while (true) {
        const uint64_t has = __ballot(m != 0);
        if (has == 0) return true;
        if (m) {
            const uint32_t j = uint32_t(__builtin_ctz(m));
            m &= m - 1u;
            // classes of bytes j-9 .. j+6 of the lane (the window and what follows)
            const uint32_t r = j <= 8 ? __builtin_amdgcn_alignbit(W, P, 14u + 2u * j)
                                      : __builtin_amdgcn_alignbit(Wn, W, 2u * j - 18u);
            const bool second = SECOND && (lane < 63 || j < 14);
            q[qn + lane_rank(has)] = make_uint2(pos + j - (kGateQ - 1), (r & 0xffffffu) | (second ? 0u : kNoSecond));
        }
        qn += uint32_t(__popcll(has));
        if (qn >= 63) {
            qn = filter_starts(s_bits2, q, qf, qn);
            qf = qn;
            if (qn >= 63) return false;
        }
    }
}

// Copy an automaton's two bitmaps into LDS (every thread of the workgroup
// takes part; the caller synchronises).
__device__ __forceinline__ void load_bitmaps(const GateArgs &a, uint32_t *s_bits, uint32_t *s_bits2) {
    const uint4 *src = reinterpret_cast<const uint4 *>(a.bits);
    uint4 *dst = reinterpret_cast<uint4 *>(s_bits);
    for (uint32_t i = threadIdx.x; i < kBitmapWords / 4; i += kGateBlock) dst[i] = src[i];
    const uint4 *src2 = reinterpret_cast<const uint4 *>(a.bits2);
    uint4 *dst2 = reinterpret_cast<uint4 *>(s_bits2);
    for (uint32_t i = threadIdx.x; i < kBitmap2Words / 4; i += kGateBlock) dst2[i] = src2[i];
}

// The start positions of tiles [t0, t1) of the text (tile t = the 1,008
// starts from t * 1008), taken by this wave (gw) of W waves in turn: every
// start of the range is tested, the passing ones walked, and with the text's
// last tile also the starts too close to its end for a whole window. The
// wave's queue is empty again on return.
template <class Em>
__device__ __forceinline__ void gate_range(const GateArgs &a, const uint32_t *s_bits, const uint32_t *s_bits2,
                                           uint2 *q, Em &em, uint32_t t0, uint32_t t1, uint32_t gw,
                                           uint32_t W) {
    const uint32_t lane = __lane_id();
    uint32_t qn = 0, qf = 0;  // queued starts, and how many passed the second level (the same in every lane)
    const uint32_t n_tiles = uint32_t((uint64_t(a.n) + kOwnBytes - 1) / kOwnBytes);
    // tiles whose 1 KiB lies inside the text, the first excepted (its lane 0
    // would read before byte 0): [lo, hi), wave gw taking lo + gw, lo + gw + W, ...
    const uint32_t full = a.n / kOwnBytes;
    const uint32_t lo = max(t0, 1u), hi = min(t1, full);
    const uint32_t first = lo + gw;
    const uint32_t cnt = hi > first ? (hi - first + W - 1) / W : 0u;
    const uint8_t *lane_text = a.text + lane * kLaneBytes;  // + t * kOwnBytes - 16
    uint4 buf[kPrefetch];  // the next kPrefetch tiles of this wave, in flight
#pragma unroll
    for (uint32_t k = 0; k < kPrefetch; ++k)
        buf[k] = k < cnt ? load_stream(lane_text + (first + k * W) * kOwnBytes - 16) : make_uint4(0u, 0u, 0u, 0u);
    for (uint32_t i = 0; i < cnt; i += kPrefetch) {
        // the ring's entries in turn, each in a register of its own (a fold,
        // not a loop the compiler may leave rolled and index at run time)
        for_each_while(
            [&](auto kc) -> bool {
                constexpr uint32_t k = decltype(kc)::value;
                if (i + k >= cnt) return false;
                const uint32_t t = first + (i + k) * W;
                const uint4 v = buf[k];
                if (i + k + kPrefetch < cnt) buf[k] = load_stream(lane_text + (t + kPrefetch * W) * kOwnBytes - 16);
                const uint32_t Wd = pack_classes(v, a.shift);
                const uint32_t P = __shfl_up(Wd, 1);
                const uint32_t Wn = __shfl_down(Wd, 1);
                const uint32_t pos = t * kOwnBytes + (lane - 1u) * kLaneBytes;
                uint32_t m = lane ? test_windows(s_bits, Wd, P) : 0u;
                while (!push_starts<true>(s_bits2, Wd, P, Wn, pos, m, q, qn, qf)) {
                    qn = drain_starts(a, q, qn, em);
                    qf = qn;
                }
                return true;
            },
            std::make_integer_sequence<uint32_t, kPrefetch>{});
    }
    // the first tile and a last, partial one, where they lie in the range:
    // loads and windows checked against the text's ends, second level left
    // out; taken by the last two waves, which have the fewest tiles above
#pragma unroll 1
    for (uint32_t e = 0; e < 2; ++e) {
        const uint32_t t = e == 0 ? 0u : n_tiles - 1u;
        if (n_tiles == 0 || t < t0 || t >= t1 || (e == 1 && (t < full || t == 0)) || gw != W - 1 - e % W) continue;
        const int64_t base = int64_t(t) * kOwnBytes - 16 + int64_t(lane) * kLaneBytes;
        const uint4 v = base >= 0 && base < int64_t(a.n) ? *reinterpret_cast<const uint4 *>(a.text + base)
                                                          : make_uint4(0u, 0u, 0u, 0u);
        const uint32_t Wd = pack_classes(v, a.shift);
        const uint32_t P = __shfl_up(Wd, 1);
        const uint32_t Wn = __shfl_down(Wd, 1);
        // window ends base + j must lie in [kGateQ - 1, n)
        uint32_t valid = 0;
        if (lane > 0) {
            for (uint32_t j = 0; j < 16; ++j)
                if (base + j >= kGateQ - 1 && base + j < int64_t(a.n)) valid |= 1u << j;
        }
        uint32_t me = test_windows(s_bits, Wd, P) & valid;
        while (!push_starts<false>(s_bits2, Wd, P, Wn, uint32_t(base), me, q, qn, qf)) {
            qn = drain_starts(a, q, qn, em);
            qf = qn;
        }
    }
    qn = filter_starts(s_bits2, q, qf, qn);
    while (qn) qn = drain_starts(a, q, qn, em);
    // starts too close to the end for a whole window: walked from the root
    // (by the last wave, as the last tile)
    if (t1 >= n_tiles && gw == W - 1) {
        const uint32_t from = a.n > kGateQ - 1 ? a.n - (kGateQ - 1) : 0u;
        walk_on(a, from + lane < a.n, 0u, from + lane, em);
    }
}

template <class Em>
__global__ void __launch_bounds__(kGateBlock) gate_kernel(GateArgs a) {
    // static LDS: the bitmaps' addresses are then constants the lookups fold in
    __shared__ __align__(16) uint32_t s_bits[kBitmapWords];
    __shared__ __align__(16) uint32_t s_bits2[kBitmap2Words];
    __shared__ __align__(16) uint2 s_queue[kGateWaves * kStartQueue];
    __shared__ uint32_t s_flush[kGateWaves + 2];
    __shared__ __align__(16) uint8_t s_emit[EmitterLds<Em>::bytes(kGateWaves)];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    Em em;
    init_emitter(em, s_emit, a.out, a.cap, a.count);
    load_bitmaps(a, s_bits, s_bits2);
    __syncthreads();
    const uint32_t n_tiles = uint32_t((uint64_t(a.n) + kOwnBytes - 1) / kOwnBytes);
    gate_range(a, s_bits, s_bits2, s_queue + wave * kStartQueue, em, 0u, n_tiles,
               blockIdx.x * kGateWaves + wave, gridDim.x * kGateWaves);
    em.flush_group(s_flush);
    complete_launch(a.done, a.count);
}

// Many texts against several automata in one persistent launch: workgroups
// take tasks (a range of tiles of one text, and its automaton) in increasing
// order from a device counter and load an automaton's bitmaps into LDS only
// when it differs from the previous task's. Tasks are ordered by automaton.
struct BatchLaunch {
    const uint8_t *base;            // task offsets are from here
    const GateTask *tasks;
    uint32_t n_tasks;
    const GateArgs *autos;          // per automaton: tables and class scheme
    uint64_t *out;                  // the batch's one match list
    uint64_t cap;
    unsigned long long *count;
    uint32_t *next_task;            // zero at launch
};

// A value the same in every lane, in scalar registers.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
    return uint64_t(uniform_u32(uint32_t(x))) | uint64_t(uniform_u32(uint32_t(x >> 32))) << 32;
}
// A pointer to global memory, the same in every lane. One loaded from memory
// (not a kernel argument) has no known address space, and the compiler would
// reach it with flat loads, whose waits also take in the LDS reads in flight;
// the cast lets it use global loads.
template <class T>
__device__ __forceinline__ T *uniform_global(T *p) {
    const uint64_t u = uniform_u64(reinterpret_cast<uint64_t>(p));
#if defined(__HIP_DEVICE_COMPILE__)
    return (T *)(__attribute__((address_space(1))) T *)u;
#else
    return reinterpret_cast<T *>(u);
#endif
}

// *p, the same for the whole workgroup, field by field into scalar registers
// (a plain copy would hold it in vector registers, which the scan needs).
__device__ __forceinline__ GateArgs uniform_args(const GateArgs *p) {
    const GateArgs s = *p;
    GateArgs a;
    a.text = uniform_global(s.text);
    a.n = uniform_u32(s.n);
    a.base = uniform_u32(s.base);
    a.shift = uniform_u32(s.shift);
    a.letters = uniform_u32(s.letters);
    a.bits = uniform_global(s.bits);
    a.bits2 = uniform_global(s.bits2);
    a.node = uniform_global(s.node);
    a.go = uniform_global(s.go);
    a.own_off = uniform_global(s.own_off);
    a.own_ids = uniform_global(s.own_ids);
    a.path_off = uniform_global(s.path_off);
    a.path_ids = uniform_global(s.path_ids);
    a.pat_len = uniform_global(s.pat_len);
    a.own_one = uniform_global(s.own_one);
    a.path_one = uniform_global(s.path_one);
    a.out = uniform_global(s.out);
    a.cap = uniform_u64(s.cap);
    a.count = uniform_global(s.count);
    a.done = Completion{uniform_global(s.done.finished), uniform_global(s.done.word), uniform_u64(s.done.seq)};
    return a;
}

template <class Em>
__global__ void __launch_bounds__(kGateBlock) gate_batch_kernel(BatchLaunch b) {
    __shared__ __align__(16) uint32_t s_bits[kBitmapWords];
    __shared__ __align__(16) uint32_t s_bits2[kBitmap2Words];
    __shared__ __align__(16) uint2 s_queue[kGateWaves * kStartQueue];
    __shared__ uint32_t s_task;
    __shared__ uint32_t s_flush[kGateWaves + 2];
    __shared__ __align__(16) uint8_t s_emit[EmitterLds<Em>::bytes(kGateWaves)];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    Em em;
    init_emitter(em, s_emit, b.out, b.cap, b.count);
    uint32_t cur = ~0u;  // automaton whose bitmaps are in LDS
    while (true) {
        __syncthreads();  // every wave done with the previous task (and its bitmaps)
        if (threadIdx.x == 0) s_task = atomicAdd(b.next_task, 1u);
        __syncthreads();
        const uint32_t k = __builtin_amdgcn_readfirstlane(s_task);
        if (k >= b.n_tasks) break;
        const GateTask task = b.tasks[k];
        GateArgs a = uniform_args(b.autos + task.automaton);
        if (task.automaton != cur) {
            load_bitmaps(a, s_bits, s_bits2);
            __syncthreads();
            cur = task.automaton;
        }
        a.text = b.base + task.off;
        a.n = task.len;
        a.base = task.pos_base;
        a.out = b.out;
        a.cap = b.cap;
        a.count = b.count;
        a.done = Completion{nullptr, nullptr, 0};
        gate_range(a, s_bits, s_bits2, s_queue + wave * kStartQueue, em, task.t0, task.t1, wave, kGateWaves);
    }
    em.flush_group(s_flush);
}

// The grouped served launch (requests passed by value, at most kGroupMax).
struct GroupLaunch {
    const GateArgs *autos;
    uint32_t *counters;  // next task, workgroups finished
    uint32_t n_req, per;
    GroupReq req[kGroupMax];
};

template <class Em>
__global__ void __launch_bounds__(kGateBlock) gate_group_kernel(GroupLaunch g) {
    __shared__ __align__(16) uint32_t s_bits[kBitmapWords];
    __shared__ __align__(16) uint32_t s_bits2[kBitmap2Words];
    __shared__ __align__(16) uint2 s_queue[kGateWaves * kStartQueue];
    __shared__ uint32_t s_task;
    __shared__ uint32_t s_flush[kGateWaves + 2];
    __shared__ __align__(16) uint8_t s_emit[EmitterLds<Em>::bytes(kGateWaves)];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    Em em;
    uint32_t cur = ~0u;  // automaton whose bitmaps are in LDS
    uint32_t total = g.req[0].task_end;
#pragma unroll
    for (uint32_t i = 1; i < kGroupMax; ++i)
        if (i < g.n_req) total = g.req[i].task_end;
    while (true) {
        __syncthreads();  // every wave done with the previous task (and its bitmaps)
        if (threadIdx.x == 0) s_task = atomicAdd(g.counters, 1u);
        __syncthreads();
        const uint32_t k = __builtin_amdgcn_readfirstlane(s_task);
        if (k >= total) break;
        // the task's request, found with fixed indices (the argument block
        // stays in the kernel-argument segment)
        GroupReq q = g.req[0];
        uint32_t first = 0;
#pragma unroll
        for (uint32_t i = 1; i < kGroupMax; ++i)
            if (i < g.n_req && k >= g.req[i - 1].task_end) {
                q = g.req[i];
                first = g.req[i - 1].task_end;
            }
        const uint32_t tiles = (q.n + kOwnBytes - 1) / kOwnBytes;
        const uint32_t t0 = (k - first) * g.per, t1 = min(t0 + g.per, tiles);
        GateArgs a = uniform_args(g.autos + q.automaton);
        if (q.automaton != cur) {
            load_bitmaps(a, s_bits, s_bits2);
            __syncthreads();
            cur = q.automaton;
        }
        a.text = uniform_global(q.text);
        a.n = q.n;
        a.base = 0;
        a.out = uniform_global(q.out);
        a.cap = q.cap;
        a.count = uniform_global(q.count);
        a.done = Completion{nullptr, nullptr, 0};
        init_emitter(em, s_emit, a.out, a.cap, a.count);
        gate_range(a, s_bits, s_bits2, s_queue + wave * kStartQueue, em, t0, t1, wave, kGateWaves);
        em.flush_group(s_flush);
        // the request's last task to finish publishes its total
        if (threadIdx.x == 0) {
            __threadfence();  // this workgroup's matches and count updates first
            if (atomicAdd(q.finished, 1u) == q.task_end - first - 1u) {
                __threadfence();  // the request's other workgroups', seen through the counter
                const uint64_t n_matches = __hip_atomic_load(q.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(q.count, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(q.finished, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(q.word, n_matches, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(q.word + 1, q.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
    // the launch's last workgroup leaves the counters zero for the next launch
    if (threadIdx.x == 0 && atomicAdd(g.counters + 1, 1u) == gridDim.x - 1) {
        __hip_atomic_store(g.counters, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(g.counters + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace

namespace {

// The machine's tables and class scheme (text, output and completion fields
// left empty).
GateArgs machine_args(const DeviceMachine &dm) {
    GateArgs a{};
    a.shift = dm.hash_shift;
    a.letters = uint32_t(dm.hash_letter[0]) | uint32_t(dm.hash_letter[1]) << 8 |
                uint32_t(dm.hash_letter[2]) << 16 | uint32_t(dm.hash_letter[3]) << 24;
    a.bits = dm.gate_bits;
    a.bits2 = dm.gate2_bits;
    a.node = dm.gate_node;
    a.go = dm.go;
    a.own_off = dm.own_off;
    a.own_ids = dm.own_ids;
    a.path_off = dm.path_off;
    a.path_ids = dm.path_ids;
    a.pat_len = dm.pat_len;
    a.own_one = dm.own_one;
    a.path_one = dm.path_one;
    return a;
}

}  // namespace

int launch_gate_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                     uint64_t cap, uint64_t *count, hipStream_t stream, std::string &err, const Completion *done,
                     uint32_t wave_tiles) {
    wave_tiles = std::max(1u, wave_tiles);
    if (!dm.gate_bits) {
        err = "ac_scan: this automaton has no start-position gate";
        return AC_ERR_INVALID;
    }
    if (n == 0) return AC_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const uint32_t cus = uint32_t(compute_units(dev));
    GateArgs a = machine_args(dm);
    a.text = text;
    a.n = uint32_t(n);
    a.base = 0;
    a.out = out;
    a.cap = cap;
    a.count = reinterpret_cast<unsigned long long *>(count);
    a.done = done ? *done : Completion{nullptr, nullptr, 0};
    // one workgroup per CU (the bitmaps fill the LDS), fewer for short texts
    const uint64_t tiles = (n + kOwnBytes - 1) / kOwnBytes;
    const uint32_t grid = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>((tiles + kGateWaves * wave_tiles - 1) / (kGateWaves * wave_tiles), cus)));
    return dm.dense ? launch_kernel(gate_kernel<RegEmitter<kEmitSlots>>, grid, kGateBlock, 0u, stream, a, err)
                    : launch_kernel(gate_kernel<Emitter>, grid, kGateBlock, 0u, stream, a, err);
}

size_t gate_batch_auto_bytes() { return sizeof(GateArgs); }

void fill_gate_batch_auto(const DeviceMachine &dm, void *dst) {
    const GateArgs a = machine_args(dm);
    std::memcpy(dst, &a, sizeof(a));
}

uint32_t gate_batch_tile_bytes() { return kOwnBytes; }

int launch_gate_batch(const uint8_t *base, const GateTask *tasks, uint32_t n_tasks, const void *autos,
                      uint64_t *out, uint64_t cap, uint64_t *count, uint32_t *next_task, uint32_t grid,
                      bool dense, hipStream_t stream, std::string &err) {
    BatchLaunch b{};
    b.base = base;
    b.tasks = tasks;
    b.n_tasks = n_tasks;
    b.autos = static_cast<const GateArgs *>(autos);
    b.out = out;
    b.cap = cap;
    b.count = reinterpret_cast<unsigned long long *>(count);
    b.next_task = next_task;
    return dense ? launch_kernel(gate_batch_kernel<RegEmitter<kBatchEmitSlots>>, grid, kGateBlock, 0u, stream, b, err)
                 : launch_kernel(gate_batch_kernel<Emitter>, grid, kGateBlock, 0u, stream, b, err);
}

int launch_gate_group(const void *autos, const GroupReq *reqs, uint32_t n_req, uint32_t per,
                      uint32_t *counters, uint32_t grid, bool dense, hipStream_t stream, std::string &err) {
    if (n_req == 0 || n_req > kGroupMax || per == 0) {
        err = "grouped scan: 1 to 16 requests and a task size are needed";
        return AC_ERR_INVALID;
    }
    GroupLaunch g{};
    g.autos = static_cast<const GateArgs *>(autos);
    g.counters = counters;
    g.n_req = n_req;
    g.per = per;
    for (uint32_t i = 0; i < n_req; ++i) g.req[i] = reqs[i];
    return dense ? launch_kernel(gate_group_kernel<RegEmitter<kBatchEmitSlots>>, grid, kGateBlock, 0u, stream, g, err)
                 : launch_kernel(gate_group_kernel<Emitter>, grid, kGateBlock, 0u, stream, g, err);
}

}  // namespace acm
