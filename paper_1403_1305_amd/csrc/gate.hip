// gate.hip -- the failure-less scan from gated start positions (AC_ALGO_GATED).
//
// Every occurrence of a pattern begins at exactly one start position, and the
// failure-less machine (the goto function with the patterns that end at each
// state, the paper's Sec. II.B and IV.A) walked from that position finds every
// pattern that begins there. Most positions begin no pattern at all, and the
// next kGateQ bytes decide it: their 2-bit classes form a 20-bit code, and a
// bitmap over every code, held in LDS, marks those some pattern can begin
// with. Only marked positions are walked, and a table over the codes takes a
// walk's first kGateQ steps in one lookup.
//
// A wave takes 1 KiB of text per step, 16 bytes per lane in one coalesced
// load. Each lane packs its bytes into one word of classes; the word of the
// lane before (of the wave's previous step, for lane 0) supplies the 9 bytes
// before them, so the lane tests the 16 windows that end in its bytes. Marked
// start positions go to a per-wave queue in LDS; whenever it holds 64 the
// whole wave walks them, one per lane. Windows and starts line up one to
// one, so each start (and each match) is handled once, with no overlap
// between waves beyond the 9 bytes a lane borrows from its neighbour.
#include <algorithm>

#include "device_common.h"
#include "machine.h"
#include "scan.h"

namespace acm {
namespace {

constexpr uint32_t kGateBlock = 1024;
constexpr uint32_t kGateWaves = kGateBlock / 64;
constexpr uint32_t kLaneBytes = 16;
constexpr uint32_t kTileBytes = 64 * kLaneBytes;  // text of one wave step
constexpr uint32_t kPrefetch = 4;                 // wave steps loaded ahead
constexpr uint32_t kStartQueue = 128;             // queued start positions per wave
constexpr uint32_t kBitmapBytes = kGateCodes / 8;
constexpr uint32_t kBitmapWords = kGateCodes / 32;
constexpr uint32_t kGateLds = kBitmapBytes + kGateWaves * (kStartQueue * 8 + kQueueBytesPerWave);
static_assert(kGateLds <= kLdsPerWorkgroup, "gate kernel LDS");
static_assert(kGateQ == 10, "the window extraction below assumes 10-byte windows");

struct GateArgs {
    const uint8_t *text;
    uint32_t n;
    uint32_t n_tiles;         // ceil(n / kTileBytes)
    uint32_t tiles_per_wave;  // consecutive tiles each wave takes
    uint32_t shift;           // class of byte b = (b >> shift) & 3
    uint32_t letters;         // byte c = the letter of class c
    const uint32_t *bits, *node, *go, *own_off, *own_ids, *path_off, *path_ids, *pat_len;
    uint64_t *out;
    uint64_t cap;
    unsigned long long *count;
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

// The 16 bytes at `pos` (16-byte aligned). A block that holds byte pos < n
// lies on a mapped page, so it is read whole; bytes past n are never used.
__device__ __forceinline__ uint4 load_lane(const uint8_t *text, uint32_t pos, uint32_t n) {
    if (pos >= n) return make_uint4(0u, 0u, 0u, 0u);
    return *reinterpret_cast<const uint4 *>(text + pos);
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
__device__ __forceinline__ void walk_on(const GateArgs &a, bool active, uint32_t x, uint32_t i,
                                        Emitter &em) {
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
        emit_set(em, active && (g & kAccept), x, i, a.own_off, a.own_ids);
        ++i;
    }
}

// Walk the start positions p (lanes with `has`), whose window code is `code`:
// the patterns that end within the window come from the gate table's node,
// the longer ones from the goto walk beyond it.
__device__ __forceinline__ void walk_starts(const GateArgs &a, bool has, uint32_t p, uint32_t code,
                                            Emitter &em) {
    const uint32_t g = has ? a.node[code] : 0u;
    const uint32_t d = (g >> kGateNodeBits) & 31u;
    const uint32_t x = g & kGateNodeMask;
    uint32_t run = 0;
    if (has) {
        uint32_t b[3];
        load12(a, p, b);
        run = min(letter_run(a, b), d);
    }
    // patterns ending on the path to x that lie within the letters read
    const bool hp = has && (g & kGatePathFlag);
    uint32_t k = hp ? a.path_off[x] : 0u;
    const uint32_t ke = hp ? a.path_off[x + 1] : 0u;
    while (__any(k < ke)) {
        const bool h = k < ke;
        const uint32_t id = h ? a.path_ids[k] : 0u;
        const uint32_t len = h ? a.pat_len[id] : 0u;
        em.emit(h && len <= run, (uint64_t(p + len - 1) << 32) | id);
        k += h ? 1u : 0u;
    }
    walk_on(a, has && d == kGateQ && run == kGateQ, x, p + kGateQ, em);
}

__global__ void __launch_bounds__(kGateBlock) gate_kernel(GateArgs a) {
    // static LDS: the bitmap's address is then a constant the lookups fold in
    __shared__ __align__(16) uint32_t s_bits[kBitmapWords];
    __shared__ __align__(16) uint2 s_queue[kGateWaves * kStartQueue];
    __shared__ __align__(16) uint8_t s_emit[kGateWaves * kQueueBytesPerWave];
    const uint32_t wave = threadIdx.x / 64, lane = threadIdx.x & 63u;
    uint2 *q = s_queue + wave * kStartQueue;
    Emitter em;
    em.init(s_emit, a.out, a.cap, a.count);
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.bits);
        uint4 *dst = reinterpret_cast<uint4 *>(s_bits);
        for (uint32_t i = threadIdx.x; i < kBitmapBytes / 16; i += kGateBlock) dst[i] = src[i];
    }
    __syncthreads();

    const uint32_t gw = blockIdx.x * kGateWaves + wave;
    const uint32_t t0 = min(gw * a.tiles_per_wave, a.n_tiles);
    const uint32_t t1 = min(t0 + a.tiles_per_wave, a.n_tiles);
    uint32_t qn = 0;  // queued starts (the same in every lane)
    if (t0 < t1) {
        // classes of the 16 bytes before the first tile: lane 0's left neighbour
        uint32_t carry = 0;
        if (t0 > 0) carry = pack_classes(*reinterpret_cast<const uint4 *>(a.text + t0 * kTileBytes - 16), a.shift);
        uint4 buf[kPrefetch];
#pragma unroll
        for (uint32_t k = 0; k < kPrefetch; ++k)
            buf[k] = t0 + k < t1 ? load_lane(a.text, (t0 + k) * kTileBytes + lane * kLaneBytes, a.n)
                                 : make_uint4(0u, 0u, 0u, 0u);
        for (uint32_t t = t0; t < t1; t += kPrefetch) {
#pragma unroll
            for (uint32_t k = 0; k < kPrefetch; ++k) {
                const uint32_t tile = t + k;
                if (tile >= t1) break;
                const uint4 v = buf[k];
                const uint32_t ahead = tile + kPrefetch;
                buf[k] = ahead < t1 ? load_lane(a.text, ahead * kTileBytes + lane * kLaneBytes, a.n)
                                    : make_uint4(0u, 0u, 0u, 0u);
                const uint32_t pos = tile * kTileBytes + lane * kLaneBytes;
                const uint32_t W = pack_classes(v, a.shift);
                const uint32_t up = __shfl_up(W, 1);
                const uint32_t P = lane == 0 ? carry : up;
                carry = __builtin_amdgcn_readlane(W, 63);
                // window ending at byte j of this lane: classes of bytes j-9 .. j,
                // bits 14 + 2j on in the 64-bit word P:W
                uint32_t m = 0;
#pragma unroll
                for (uint32_t j = 0; j < 16; ++j) {
                    const uint32_t r = j <= 8 ? __builtin_amdgcn_alignbit(W, P, 14u + 2u * j) : (W >> (2u * j - 18u));
                    const uint32_t word = s_bits[(r >> 5) & (kBitmapWords - 1u)];
                    // bit r mod 32 of the word (the field offset takes r's low 5 bits)
                    m |= __builtin_amdgcn_ubfe(word, r, 1u) << j;
                }
                // windows must start at byte 0 or later and end before byte n
                if (pos < kGateQ - 1) m &= 0xffffu << (kGateQ - 1 - pos);
                if (pos + kLaneBytes > a.n) m &= pos < a.n ? (1u << (a.n - pos)) - 1u : 0u;
                // queue the marked starts; walk 64 of them whenever that many wait
                while (true) {
                    const uint64_t has = __ballot(m != 0);
                    if (has == 0) break;
                    if (m) {
                        const uint32_t j = uint32_t(__builtin_ctz(m));
                        m &= m - 1u;
                        const uint32_t r = j <= 8 ? __builtin_amdgcn_alignbit(W, P, 14u + 2u * j) : (W >> (2u * j - 18u));
                        q[qn + lane_rank(has)] = make_uint2(pos + j - (kGateQ - 1), r & (kGateCodes - 1u));
                    }
                    qn += uint32_t(__popcll(has));
                    if (qn >= 64) {
                        __builtin_amdgcn_wave_barrier();
                        const uint2 e = q[qn - 64 + lane];
                        __builtin_amdgcn_wave_barrier();
                        qn -= 64;
                        walk_starts(a, true, e.x, e.y, em);
                    }
                }
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    {
        const bool has = lane < qn;
        const uint2 e = has ? q[lane] : make_uint2(0u, 0u);
        walk_starts(a, has, e.x, e.y, em);
    }
    // starts too close to the end for a whole window: walked from the root
    if (blockIdx.x == 0 && wave == 0) {
        const uint32_t first = a.n > kGateQ - 1 ? a.n - (kGateQ - 1) : 0u;
        walk_on(a, first + lane < a.n, 0u, first + lane, em);
    }
    em.flush();
}

}  // namespace

int launch_gate_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                     uint64_t cap, uint64_t *count, hipStream_t stream, std::string &err) {
    if (!dm.gate_bits) {
        err = "ac_scan: this automaton has no start-position gate";
        return AC_ERR_INVALID;
    }
    if (n == 0) return AC_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const uint32_t cus = uint32_t(compute_units(dev));
    GateArgs a{};
    a.text = text;
    a.n = uint32_t(n);
    a.n_tiles = uint32_t((n + kTileBytes - 1) / kTileBytes);
    // one workgroup per CU (the bitmap fills the LDS), fewer for short texts
    const uint32_t want = (a.n_tiles + kGateWaves - 1) / kGateWaves;
    const uint32_t grid = std::max<uint32_t>(1, std::min(want, cus));
    a.tiles_per_wave = (a.n_tiles + grid * kGateWaves - 1) / (grid * kGateWaves);
    a.shift = dm.hash_shift;
    a.letters = uint32_t(dm.hash_letter[0]) | uint32_t(dm.hash_letter[1]) << 8 |
                uint32_t(dm.hash_letter[2]) << 16 | uint32_t(dm.hash_letter[3]) << 24;
    a.bits = dm.gate_bits;
    a.node = dm.gate_node;
    a.go = dm.go;
    a.own_off = dm.own_off;
    a.own_ids = dm.own_ids;
    a.path_off = dm.path_off;
    a.path_ids = dm.path_ids;
    a.pat_len = dm.pat_len;
    a.out = out;
    a.cap = cap;
    a.count = reinterpret_cast<unsigned long long *>(count);
    return launch_kernel(gate_kernel, grid, kGateBlock, 0u, stream, a, err);
}

}  // namespace acm
