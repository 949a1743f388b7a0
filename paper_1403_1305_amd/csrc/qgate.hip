// qgate.hip -- the failure-less scan from start positions a hashed gate passes
// (AC_ALGO_GATED on machines without the class gate whose patterns are all
// at least kQgQ bytes long).
//
// Every occurrence begins at exactly one start position, and the failure-less
// machine (the goto function with the patterns that end at each state, the
// paper's Sec. II.B and IV.A) walked from there finds every pattern that
// begins at it. A pattern can begin at p only if the kQgQ bytes from p are
// the first kQgQ bytes of some pattern. A blocked Bloom filter over those
// windows, 2^20 bits in LDS, tests each start with one LDS read: two bits of
// one word, picked by a multiplicative hash of the window. A start that
// passes is looked up in a table of the windows (in global memory, small
// enough to stay in L2; each window in one of two slots, both read at once),
// which rejects the filter's false positives and gives the goto state after
// the window; the walk goes on from there.
//
// A wave step reads 1 KiB of text, 16 bytes per lane in one coalesced load,
// and owns the last 1008 of them: lane 0 holds the 16 bytes before, so that
// every lane finds the 5 bytes before its own in the lane below and tests the
// 16 windows that end in its bytes. Steps are handed to the waves of the grid
// in turn. Passing starts go to a per-wave queue in LDS; whenever kDrainAt or
// more wait, the wave looks up and walks all of them, kWalks per lane at once
// (so that their dependent loads overlap), then goes on streaming. Starts in
// the last kQgQ - 1 bytes of the text begin no pattern and are not tested.
#include <algorithm>
#include <utility>

#include "device_common.h"
#include "machine.h"
#include "scan.h"

namespace acm {
namespace {

constexpr uint32_t kQgBlock = 1024;
constexpr uint32_t kQgWaves = kQgBlock / 64;
constexpr uint32_t kLaneBytes = 16;
constexpr uint32_t kOwnBytes = 63 * kLaneBytes;  // text a wave step owns
constexpr uint32_t kPrefetch = 4;                // wave steps loaded ahead
constexpr uint32_t kWalks = 2;                   // queued starts a lane walks at once
constexpr uint32_t kStartQueue = 125;            // queued starts per wave (position and window, 12 bytes)
constexpr uint32_t kDrainAt = kStartQueue - 63;  // queue length that triggers a drain
static_assert(kStartQueue <= 64 * kWalks, "a drain takes the whole queue");
constexpr uint32_t kQgLds = kQgWords * 4 + 256 + kQgWaves * (kStartQueue * 12 + kQueueBytesPerWave);
// Matches queued per lane: a wave reserves room in the list once per up to
// 64 times as many.
constexpr uint32_t kQgEmitSlots = 8;
using QgEmitter = RegEmitter<kQgEmitSlots>;
static_assert(kQgLds <= kLdsPerWorkgroup, "hashed gate kernel LDS");
static_assert(kQgQ == 6, "the window extraction below assumes 6-byte windows");

struct QgArgs {
    const uint8_t *text;
    uint32_t n;
    uint32_t n_cols;
    const uint32_t *bits;  // kQgWords words
    const uint4 *tab;      // the window table
    uint32_t tab_shift;    // 32 - log2 of its slots
    uint32_t no_class;     // byte-map value of bytes in no pattern
    const uint32_t *go, *own_off, *own_ids;
    const uint8_t *cmap;
    uint64_t *out;
    uint64_t cap;
    unsigned long long *count;
    Completion done;
};

// Low 32 bits of the product of the low 24 bits of a and b (one full-rate
// multiply). HIP's __umul24 returns int, which would make a later right
// shift arithmetic; this returns the unsigned value.
__device__ __forceinline__ uint32_t mul_u24(uint32_t a, uint32_t b) { return uint32_t(__umul24(a, b)); }

// 16 bytes of the text stream. Ordinary (temporal) loads: the starts a
// step queues read their window again a few steps later, and one in 30 or
// so of the positions of protein-like text is queued, so keeping the text
// in L2 for that long beats keeping the tables there alone (measured 4%).
__device__ __forceinline__ uint4 load_stream(const uint8_t *p) { return *reinterpret_cast<const uint4 *>(p); }

template <class Em, uint32_t... K>
__device__ __forceinline__ void emit_walks(const QgArgs &a, Em &em, const bool (&active)[kWalks],
                                           const uint32_t (&g)[kWalks], const uint32_t (&x)[kWalks],
                                           const uint32_t (&i)[kWalks], std::integer_sequence<uint32_t, K...>) {
    (emit_set(em, active[K] && (g[K] & kAccept), x[K], i[K], a.own_off, a.own_ids), ...);
}

template <class Em, uint32_t... K>
__device__ __forceinline__ void emit_found(const QgArgs &a, Em &em, const bool (&hit)[kWalks],
                                           const uint32_t (&own)[kWalks], const uint32_t (&x)[kWalks],
                                           const uint32_t (&p)[kWalks], std::integer_sequence<uint32_t, K...>) {
    (emit_set(em, hit[K] && own[K], x[K], p[K] + kQgQ - 1u, a.own_off, a.own_ids), ...);
}

// Goto walks of kWalks starts per lane from states x[k] (those with
// active[k]), over the bytes from i[k] on: each step into a state where
// patterns end reports them at that byte. A walk ends at the first missing
// edge, a byte in no pattern or the end of the text. The walks of a lane
// advance together, so their loads are in flight at once.
template <class Em>
__device__ __forceinline__ void walk_on(const QgArgs &a, const uint8_t *s_cmap, bool (&active)[kWalks],
                                        uint32_t (&x)[kWalks], uint32_t (&i)[kWalks], Em &em) {
    while (true) {
        bool any = false;
#pragma unroll
        for (uint32_t k = 0; k < kWalks; ++k) {
            if (active[k] && i[k] >= a.n) active[k] = false;
            any |= active[k];
        }
        if (!__any(any)) break;
        uint32_t b[kWalks], g[kWalks];
#pragma unroll
        for (uint32_t k = 0; k < kWalks; ++k) b[k] = active[k] ? a.text[i[k]] : 0u;
#pragma unroll
        for (uint32_t k = 0; k < kWalks; ++k) {
            const uint32_t c = s_cmap[b[k]];
            g[k] = active[k] && c != a.no_class ? a.go[x[k] * a.n_cols + c] : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < kWalks; ++k) {
            active[k] = g[k] != 0u;
            if (active[k]) x[k] = g[k] & kStateMask;
        }
        // matches are rare: one wave-wide test before the per-walk emits (one
        // call per walk, written out: a loop around the wave-wide emits would
        // not be unrolled and would index the arrays at run time)
        bool acc = false;
#pragma unroll
        for (uint32_t k = 0; k < kWalks; ++k) acc |= active[k] && (g[k] & kAccept);
        if (__any(acc)) emit_walks(a, em, active, g, x, i, std::make_integer_sequence<uint32_t, kWalks>());
        for (uint32_t k = 0; k < kWalks; ++k) ++i[k];
    }
}

// Look up the windows (bytes p .. p + 3 in lo, p + 4 and p + 5 in hi) at the
// start positions p[k] (those with has[k]; p[k] + kQgQ <= n) in the table
// and walk on from the states of those found.
template <class Em>
__device__ __forceinline__ void walk_starts(const QgArgs &a, const uint8_t *s_cmap, const bool (&has)[kWalks],
                                            const uint32_t (&p)[kWalks], const uint32_t (&lo)[kWalks],
                                            const uint32_t (&hi)[kWalks], Em &em) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    // the window's two slots; it is in one of them or not in the table
    uint32_t k1[kWalks], sa[kWalks], sb[kWalks];
#pragma unroll
    for (uint32_t k = 0; k < kWalks; ++k) {
        k1[k] = hi[k] | kQgUsed;
        const uint32_t wx = lo[k] & 0xffffffu, wy = (lo[k] >> 24) | hi[k] << 8;
        sa[k] = (mul_u24(wx, kQgK3) ^ mul_u24(wy, kQgK4)) >> a.tab_shift;
        sb[k] = (mul_u24(wx, kQgK5) ^ mul_u24(wy, kQgK6)) >> a.tab_shift;
    }
    u32x4 ea[kWalks], eb[kWalks];
#pragma unroll
    for (uint32_t k = 0; k < kWalks; ++k) {
        ea[k] = has[k] ? *reinterpret_cast<const u32x4 *>(a.tab + sa[k]) : u32x4{0u, 0u, 0u, 0u};
        eb[k] = has[k] ? *reinterpret_cast<const u32x4 *>(a.tab + sb[k]) : u32x4{0u, 0u, 0u, 0u};
    }
    bool hit[kWalks], go_on[kWalks];
    uint32_t x[kWalks], own[kWalks];
#pragma unroll
    for (uint32_t k = 0; k < kWalks; ++k) {
        const bool ma = ea[k].x == lo[k] && (ea[k].y & ~kQgOwn) == k1[k];
        const bool mb = eb[k].x == lo[k] && (eb[k].y & ~kQgOwn) == k1[k];
        hit[k] = has[k] && (ma || mb);
        x[k] = ma ? ea[k].z : eb[k].z;
        own[k] = (ma ? ea[k].y : eb[k].y) & kQgOwn;
        // the walk goes on only if the next byte's class is one of the
        // state's children (most walks end here without a goto lookup)
        const uint32_t kids = ma ? ea[k].w : eb[k].w;
        const uint32_t nx = p[k] + kQgQ;
        const uint32_t c = hit[k] && nx < a.n ? s_cmap[a.text[nx]] : a.no_class;
        go_on[k] = hit[k] && c != a.no_class && ((kids >> (c & 31u)) & 1u);
    }
    bool found = false;
#pragma unroll
    for (uint32_t k = 0; k < kWalks; ++k) found |= hit[k] && own[k];
    if (__any(found)) emit_found(a, em, hit, own, x, p, std::make_integer_sequence<uint32_t, kWalks>());
    uint32_t i[kWalks];
#pragma unroll
    for (uint32_t k = 0; k < kWalks; ++k) i[k] = p[k] + kQgQ;
    walk_on(a, s_cmap, go_on, x, i, em);
}

// The per-wave queue of passing starts: position, window bytes 0..3, window
// bytes 4..5 (three LDS arrays).
struct StartQueue {
    uint32_t *p, *lo, *hi;
};

// Walk the qn starts queued at q (at most 64 * kWalks), kWalks per lane;
// returns how many wait afterwards.
template <class Em>
__device__ __forceinline__ uint32_t drain_starts(const QgArgs &a, const uint8_t *s_cmap, const StartQueue &q,
                                                 uint32_t qn, Em &em) {
    const uint32_t lane = __lane_id();
    const uint32_t took = min(qn, 64u * kWalks);
    bool has[kWalks];
    uint32_t p[kWalks], lo[kWalks], hi[kWalks];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (uint32_t k = 0; k < kWalks; ++k) {
        const uint32_t e = qn - took + lane + 64u * k;
        has[k] = lane + 64u * k < took;
        p[k] = has[k] ? q.p[e] : 0u;
        lo[k] = has[k] ? q.lo[e] : 0u;
        hi[k] = has[k] ? q.hi[e] : 0u;
    }
    __builtin_amdgcn_wave_barrier();
    walk_starts(a, s_cmap, has, p, lo, hi, em);
    return qn - took;
}

// Four bytes from byte o of the lane's window registers r (r[0] holds bytes
// -8 .. -5, ..., r[5] bytes 12 .. 15; o + 3 may pass byte 15, those bytes are
// unused).
template <int O>
__device__ __forceinline__ uint32_t bytes_at(const uint32_t (&r)[6]) {
    constexpr int k = (O + 8) >> 2, sh = (O + 8) & 3;
    if constexpr (sh == 0) return r[k];
    else return __builtin_amdgcn_alignbyte(r[k + 1 < 6 ? k + 1 : 5], r[k], sh);
}

template <int J>
__device__ __forceinline__ uint32_t test_window(const uint32_t *s_bits, const uint32_t (&r)[6]) {
    // the window ending at byte J: X = bytes J-5 .. J-3, Y = bytes J-2 .. J
    const uint32_t h = mul_u24(bytes_at<J - 5>(r), kQgK1) + mul_u24(bytes_at<J - 2>(r), kQgK2);
    const uint32_t word = s_bits[h >> 17];
    // bits (h >> 12) mod 32 and h mod 32 (the field offsets take the low 5 bits)
    return (__builtin_amdgcn_ubfe(word, h >> 12, 1u) & __builtin_amdgcn_ubfe(word, h, 1u)) << J;
}

template <int... J>
__device__ __forceinline__ uint32_t test_windows(const uint32_t *s_bits, const uint32_t (&r)[6],
                                                 std::integer_sequence<int, J...>) {
    return (test_window<J>(s_bits, r) | ...);
}

// The windows of one wave step. Lane l (l >= 1) owns the 16 bytes at pos (v);
// P2, P3 are the last 8 bytes of the lane below. `valid` masks the windows
// (by their last byte) that lie inside the text. Passing starts are queued at
// q (qn of them waiting, the same in every lane); whenever kDrainAt or more
// wait, all are walked (a queue below kDrainAt takes a round's at most 63 new
// ones, and a drain takes up to 64 * kWalks).
template <class Em>
__device__ __forceinline__ void step_windows(const QgArgs &a, const uint32_t *s_bits, const uint8_t *s_cmap,
                                             const uint4 &v, uint32_t P2, uint32_t P3, uint32_t pos, uint32_t valid,
                                             const StartQueue &q, uint32_t &qn, Em &em) {
    const uint32_t r[6] = {P2, P3, v.x, v.y, v.z, v.w};
    uint32_t m = test_windows(s_bits, r, std::make_integer_sequence<int, 16>()) & valid;
    while (true) {
        const uint64_t has = __ballot(m != 0);
        if (has == 0) break;
        if (m) {
            const uint32_t j = uint32_t(__builtin_ctz(m));
            m &= m - 1u;
            // the window's first byte is byte j + 3 of r: words g .. g + 2
            // (g = (j + 3) / 4 in 0..4), picked by the bits of g in three
            // stages of selects; for g = 4 the third word is not needed
            const uint32_t g = (j + 3u) >> 2, sh = (j + 3u) & 3u;
            const bool g4 = g >= 4u, g2 = (g & 2u) != 0u, g1 = (g & 1u) != 0u;
            const uint32_t t0 = g4 ? r[4] : r[0], t1 = g4 ? r[5] : r[1];
            const uint32_t u0 = g2 ? r[2] : t0, u1 = g2 ? r[3] : t1, u2 = g2 ? r[4] : r[2], u3 = g2 ? r[5] : r[3];
            const uint32_t w0 = g1 ? u1 : u0, w1 = g1 ? u2 : u1, w2 = g1 ? u3 : u2;
            const uint32_t e = qn + lane_rank(has);
            q.p[e] = pos + j - (kQgQ - 1u);
            q.lo[e] = __builtin_amdgcn_alignbyte(w1, w0, sh);
            q.hi[e] = __builtin_amdgcn_alignbyte(w2, w1, sh) & 0xffffu;
        }
        qn += uint32_t(__popcll(has));
        if (qn >= kDrainAt) qn = drain_starts(a, s_cmap, q, qn, em);
    }
}

template <class Em>
__global__ void __launch_bounds__(kQgBlock) qgate_kernel(QgArgs a) {
    // static LDS: the bitmap's address is then a constant the lookups fold in
    __shared__ __align__(16) uint32_t s_bits[kQgWords];
    __shared__ __align__(16) uint8_t s_cmap[256];
    __shared__ __align__(16) uint32_t s_queue[kQgWaves * kStartQueue * 3];
    __shared__ __align__(16) uint8_t s_emit[EmitterLds<Em>::bytes(kQgWaves)];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x & 63u;
    Em em;
    init_emitter(em, s_emit, a.out, a.cap, a.count);
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.bits);
        uint4 *dst = reinterpret_cast<uint4 *>(s_bits);
        for (uint32_t i = threadIdx.x; i < kQgWords / 4; i += kQgBlock) dst[i] = src[i];
        if (threadIdx.x < 256) s_cmap[threadIdx.x] = a.cmap[threadIdx.x];
    }
    __syncthreads();
    const StartQueue q{s_queue + wave * kStartQueue * 3, s_queue + wave * kStartQueue * 3 + kStartQueue,
                       s_queue + wave * kStartQueue * 3 + 2 * kStartQueue};
    uint32_t qn = 0;  // queued starts (the same in every lane)

    const uint32_t W = gridDim.x * kQgWaves, gw = blockIdx.x * kQgWaves + wave;
    const uint32_t n_tiles = uint32_t((uint64_t(a.n) + kOwnBytes - 1) / kOwnBytes);
    // tiles whose 1 KiB lies inside the text, the first excepted (its lane 0
    // would read before byte 0): t = first, first + W, ... < full
    const uint32_t full = a.n / kOwnBytes;
    const uint32_t first = gw == 0 ? W : gw;
    const uint32_t cnt = full > first ? (full - first + W - 1) / W : 0u;
    const uint8_t *lane_text = a.text + lane * kLaneBytes;  // + t * kOwnBytes - 16
    uint4 buf[kPrefetch];  // the next kPrefetch tiles of this wave, in flight
#pragma unroll
    for (uint32_t k = 0; k < kPrefetch; ++k)
        buf[k] = k < cnt ? load_stream(lane_text + (first + k * W) * kOwnBytes - 16) : make_uint4(0u, 0u, 0u, 0u);
    for (uint32_t i = 0; i < cnt; i += kPrefetch) {
        // the ring's entries in turn, each in a register of its own
        for_each_while(
            [&](auto kc) -> bool {
                constexpr uint32_t k = decltype(kc)::value;
                if (i + k >= cnt) return false;
                const uint32_t t = first + (i + k) * W;
                const uint4 v = buf[k];
                if (i + k + kPrefetch < cnt) buf[k] = load_stream(lane_text + (t + kPrefetch * W) * kOwnBytes - 16);
                const uint32_t P2 = __shfl_up(v.z, 1), P3 = __shfl_up(v.w, 1);
                const uint32_t pos = t * kOwnBytes + (lane - 1u) * kLaneBytes;
                step_windows(a, s_bits, s_cmap, v, P2, P3, pos, lane ? 0xffffu : 0u, q, qn, em);
                return true;
            },
            std::make_integer_sequence<uint32_t, kPrefetch>{});
    }
    // the first tile and a last, partial one: loads and windows checked
    // against the text's ends
    for (uint32_t e = 0; e < 2; ++e) {
        const uint32_t t = e == 0 ? 0u : n_tiles - 1u;
        if (n_tiles == 0 || (e == 1 && (t < full || t == 0)) || gw != t % W) continue;
        const int64_t base = int64_t(t) * kOwnBytes - 16 + int64_t(lane) * kLaneBytes;
        const uint4 v = base >= 0 && base < int64_t(a.n) ? *reinterpret_cast<const uint4 *>(a.text + base)
                                                          : make_uint4(0u, 0u, 0u, 0u);
        const uint32_t P2 = __shfl_up(v.z, 1), P3 = __shfl_up(v.w, 1);
        // window ends base + j must lie in [kQgQ - 1, n)
        uint32_t valid = 0;
        if (lane > 0) {
            for (uint32_t j = 0; j < 16; ++j)
                if (base + j >= kQgQ - 1 && base + j < int64_t(a.n)) valid |= 1u << j;
        }
        step_windows(a, s_bits, s_cmap, v, P2, P3, uint32_t(base), valid, q, qn, em);
    }
    while (qn) qn = drain_starts(a, s_cmap, q, qn, em);
    em.flush_group(s_queue);  // every queue is empty by now
    complete_launch(a.done, a.count);
}

}  // namespace

int launch_qgate_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                      uint64_t cap, uint64_t *count, hipStream_t stream, std::string &err, const Completion *done,
                      uint32_t wave_tiles) {
    wave_tiles = std::max(1u, wave_tiles);
    if (!dm.qg_bits) {
        err = "ac_scan: this automaton has no hashed start-position gate";
        return AC_ERR_INVALID;
    }
    if (uint64_t(dm.n_states) * dm.n_cols >= (1ull << 32)) {
        err = "ac_scan: goto table too large for the gated scan's 32-bit indexing";
        return AC_ERR_TOO_LARGE;
    }
    if (n < kQgQ) return AC_OK;  // no start has a whole window: nothing can match
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const uint32_t cus = uint32_t(compute_units(dev));
    QgArgs a{};
    a.text = text;
    a.n = uint32_t(n);
    a.n_cols = dm.n_cols;
    a.bits = dm.qg_bits;
    a.tab = reinterpret_cast<const uint4 *>(dm.qg_tab);
    a.tab_shift = 32u - dm.qg_tab_bits;
    a.go = dm.go;
    a.own_off = dm.own_off;
    a.own_ids = dm.own_ids;
    a.cmap = dm.cmap;
    a.no_class = dm.no_class;
    a.out = out;
    a.cap = cap;
    a.count = reinterpret_cast<unsigned long long *>(count);
    a.done = done ? *done : Completion{nullptr, nullptr, 0};
    // one workgroup per CU (the bitmap fills most of the LDS), fewer for short texts
    const uint64_t tiles = (n + kOwnBytes - 1) / kOwnBytes;
    const uint32_t grid = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>((tiles + kQgWaves * wave_tiles - 1) / (kQgWaves * wave_tiles), cus)));
    return dm.dense ? launch_kernel(qgate_kernel<QgEmitter>, grid, kQgBlock, 0u, stream, a, err)
                    : launch_kernel(qgate_kernel<Emitter>, grid, kQgBlock, 0u, stream, a, err);
}

}  // namespace acm
