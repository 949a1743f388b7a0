// machine.h -- host-side construction of the Aho-Corasick machine (internal).
//
// Step 1 of the method (the paper's Sec. II): from the pattern set, build the
// goto function (a trie), the failure function and the output function
// (Sec. II.A). The failure transitions are then folded into ordinary ones,
// so every (state, byte class) pair has exactly one successor: the full-DFA
// form the paper's Sec. III cites as faster to search than the original.
// The goto function alone is also kept: it is the failure-less machine of
// Sec. II.B that the per-start-position (PFAC) matcher walks.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace acm {

// 32-bit table entries: successor state id, top bit set when the successor's
// output set is non-empty (it is a final state).
constexpr uint32_t kAccept = 0x80000000u;
constexpr uint32_t kStateMask = 0x7fffffffu;
// 16-bit LDS image entries hold plain successor ids, which must be < 2^16.
constexpr uint32_t kHotIdLimit = 1u << 16;
// An image squeezed below this many rows (to fit the id limit) is dropped.
constexpr uint32_t kMinHotStates = 256;
// byte -> column map value for bytes that occur in no pattern
constexpr uint8_t kNoClass = 0xffu;
// Two-byte rows are built for at most this many states outside the image
// (16 four-byte entries each: 64 MiB at the limit).
constexpr uint32_t kPairMaxStates = 1u << 20;

// Start-position gate (4-column machines with bit-field classes). A window
// of kGateQ text bytes is coded as kGateQ 2-bit classes, the first byte in
// the lowest bits: kGateCodes codes in all.
constexpr uint32_t kGateQ = 10;
constexpr uint32_t kGateCodes = 1u << (2 * kGateQ);
// gate_node entries: node id in the low bits, its depth above it, and the
// top bit set when some pattern ends on the path from the root to the node.
constexpr uint32_t kGateNodeBits = 26;
constexpr uint32_t kGateNodeMask = (1u << kGateNodeBits) - 1u;
constexpr uint32_t kGatePathFlag = 0x80000000u;
// Expected matches per text byte above which a gated scan stages its matches
// in registers: fewer reservations in the list, whose counter every
// workgroup updates, against more registers held. Below it the reservations
// are spread out enough to overlap with the scan, and the LDS queue's lighter
// emits win.
constexpr double kDenseMatches = 4e-3;
// own_one / path_one: not exactly one pattern (the lists then apply).
constexpr uint32_t kOneMany = 0xffffffffu;
// Second gate level: a bitmap of kGate2Bits bits over a hash of the classes
// of kGateQ2 bytes (the window and the two bytes after it).
constexpr uint32_t kGateQ2 = kGateQ + 2;
constexpr uint32_t kGate2Bits = 1u << 16;
// Bit of the second level for the class string code (first byte in the
// lowest two bits): the top 16 bits of a multiplicative hash.
inline constexpr uint32_t gate2_hash(uint32_t code24) { return (code24 * 0x9E3779B1u) >> 16; }
// The second bit of a class string (two bits per string: a string passes when
// both are set, which halves the strings that pass by chance at the headline
// set's fill).
inline constexpr uint32_t gate2_hash2(uint32_t code24) { return (code24 * 0x85EBCA77u) >> 16; }

// Hashed start-position gate (machines whose patterns are all at least kQgQ
// bytes long and that have no class gate). A window is the kQgQ bytes from a
// start position on, read as X = bytes 0..2 and Y = bytes 3..5 (each little
// endian, 24 bits). qg_hash(X, Y) (32-bit arithmetic) picks a word of a 2^20-bit bitmap (bits 17
// and up) and two bits in it (bits 12..16 and 0..4): a blocked Bloom filter
// over the windows that begin some pattern. A table of those windows, each
// in one of its two slots (cuckoo hashing: qg_slot_a / qg_slot_b), gives the
// goto state each one leads to.
constexpr uint32_t kQgQ = 6;
constexpr uint32_t kQgWords = 1u << 15;
constexpr uint32_t kQgK1 = 0x9E3779u, kQgK2 = 0x85EBCBu;  // odd, below 2^24
constexpr uint32_t kQgK3 = 0xC2B2AFu, kQgK4 = 0x27D4EBu;
constexpr uint32_t kQgK5 = 0x165667u, kQgK6 = 0xD3A2E5u;
constexpr uint32_t kQgUsed = 0x80000000u;  // table entry word 1: slot in use
constexpr uint32_t kQgOwn = 0x40000000u;   // table entry word 1: patterns end at the state
inline constexpr uint32_t qg_hash(uint32_t x, uint32_t y) { return x * kQgK1 + y * kQgK2; }
inline constexpr uint32_t qg_slot_a(uint32_t x, uint32_t y) { return x * kQgK3 ^ y * kQgK4; }
inline constexpr uint32_t qg_slot_b(uint32_t x, uint32_t y) { return x * kQgK5 ^ y * kQgK6; }
inline constexpr uint32_t qg_word(uint32_t h) { return h >> 17; }
inline constexpr uint32_t qg_mask(uint32_t h) { return 1u << ((h >> 12) & 31u) | 1u << (h & 31u); }

struct Machine {
    uint32_t n_patterns = 0;
    uint32_t m_max = 0;
    uint32_t n_states = 0;
    uint32_t sigma = 0;       // distinct pattern bytes
    uint32_t n_cols = 0;      // table width
    uint32_t log2_cols = 0;   // valid when cols_pow2
    bool cols_pow2 = false;
    bool hashed = false;      // column = (b >> hash_shift) & (n_cols - 1)
    uint32_t hash_shift = 0;
    uint8_t hash_letter[8] = {0};  // the pattern byte owning each hashed column (hashed only)
    uint8_t cmap[256];        // byte -> column, kNoClass if absent from all patterns

    bool goto_only = false;   // built without failure function and DFA (dfa is empty)
    // Full DFA: dfa[s * n_cols + c] = delta(s, c) | kAccept if it is final.
    std::vector<uint32_t> dfa;
    // Output sets in CSR form, ids ascending: out(s) = out_ids[out_off[s] .. out_off[s+1]).
    std::vector<uint32_t> out_off, out_ids;
    // Goto function: go[s * n_cols + c] = child | kAccept if the child ends a
    // pattern itself, or 0 where there is no edge (the root is nobody's child).
    std::vector<uint32_t> go;
    // Patterns ending exactly at each state (no failure-chain outputs).
    std::vector<uint32_t> own_off, own_ids;

    // State ids come in ranges: [0, H) non-final states with image rows,
    // [H, term_end) final states where a pattern ends exactly, [term_end,
    // acc_end) final states with inherited outputs only, then the other
    // non-final states. H = hot_states (at least 1 for the numbering even
    // without an image, since the root comes first).
    uint32_t term_end = 0, acc_end = 0;
    // States [0, hot_states) form the LDS image; every successor of a hot
    // row is numbered below kHotIdLimit so that it fits 16 bits.
    uint32_t hot_states = 0;
    std::vector<uint16_t> hot_dfa;  // hot_states * n_cols successor ids
    std::vector<uint16_t> hot_go;   // hot_states * n_cols goto children, 0 = no edge
    // Two-byte rows of the states outside the image, for 4-column hashed
    // machines with an image: pair[(s - H) * 16 + (c1 | c2 << 2)] is the state
    // after bytes of classes c1 then c2 from s, | kAccept if the state after
    // c1 is final. Empty when not built (pair_states == 0).
    std::vector<uint32_t> pair;
    uint32_t pair_states = 0;
    // Start-position gate for the failure-less scan (empty unless built):
    //   gate_bits  kGateCodes bits (32 per word): bit x is set when some
    //              pattern can begin with a window of code x, i.e. x starts
    //              with the classes of a pattern shorter than kGateQ bytes, or
    //              x is the class string of the first kGateQ bytes of one;
    //   gate_node  per code, the deepest goto node its class string reaches
    //              from the root (the walk stops at the first missing edge):
    //              node | depth << kGateNodeBits | kGatePathFlag if a pattern
    //              ends on the path to it;
    //   path_off, path_ids  per node of depth <= kGateQ (CSR over all states),
    //              the patterns ending on its path from the root, ascending;
    //   pat_len    every pattern's length.
    //   gate2_bits kGate2Bits bits: bits gate2_hash(y) and gate2_hash2(y) are
    //              set for every class string y of kGateQ2 bytes a pattern can
    //              begin with (its first kGateQ2 classes, or every extension of
    //              a shorter one);
    //   path_one   per state, the one pattern ending on its path when there is
    //              exactly one and its id is below 2^28: id | length << 28;
    //              else kOneMany.
    std::vector<uint32_t> gate_bits, gate2_bits, gate_node, path_off, path_ids, pat_len, path_one;
    // Per state (built with either gate, else empty): the id of the one
    // pattern ending exactly at s, kOneMany when none or several do.
    std::vector<uint32_t> own_one;
    // Hashed gate (empty unless built; never beside the class gate):
    //   qg_bits  kQgWords words, the blocked Bloom filter: for the window
    //            (X, Y) of every pattern's first kQgQ bytes, both bits of
    //            qg_mask(h) are set in word qg_word(h), h = qg_hash(X, Y);
    //   qg_tab   2^qg_tab_bits slots of 4 words, one per distinct window:
    //            {X | (Y & 0xff) << 24, Y >> 8 | kQgUsed | kQgOwn if
    //            patterns end at the state, the goto state the window leads
    //            to from the root, its children: bit c set when it has an
    //            edge of class c (all bits when the machine has more than 32
    //            classes)};
    //            a window sits in slot qg_slot_a(X, Y) >> (32 - qg_tab_bits)
    //            or slot qg_slot_b(X, Y) >> (32 - qg_tab_bits); unused
    //            slots are all zero.
    std::vector<uint32_t> qg_bits, qg_tab;
    uint32_t qg_tab_bits = 0;
    // Expected fraction of start positions the gate passes: for the class
    // gate, the share of window codes whose bit is set; for the hashed gate,
    // the chance that a window drawn from the patterns' byte frequencies
    // begins a pattern, plus the filter's false-positive rate.
    double gate_pass = 1.0;
    // Expected matches per text byte, for text whose bytes are drawn
    // independently with the patterns' own byte frequencies (the sum over the
    // patterns of the product of their bytes' frequencies); 0 without a gate.
    // The gated scans stage matches per lane in registers above kDenseMatches.
    double match_rate = 0.0;
    double build_ms = 0.0;
};

// What to plan the 16-bit LDS image for.
struct HotPlan {
    uint32_t lds_bytes = 0;      // bytes the image may take, 256 of them for the byte map; 0 = none
    uint32_t max_states = 0;     // cap on its rows, 0 = none
    bool only_if_needed = true;  // skip it when the whole 32-bit table fits lds_bytes
    // Build the goto function and the patterns ending at each state only: no
    // failure function, no output unions, no full DFA (the failure-less machine
    // of Sec. II.B, all that the per-start-position matcher needs).
    bool goto_only = false;
    uint32_t threads = 0;        // host threads for the build, 0 = hardware threads (at most 16)
    bool pair_rows = false;      // also build Machine::pair where it applies
    bool gate = true;            // build the start-position gate where it applies
};

// Returns 0 or a negative AC_ERR_* code with `err` set. Without an image,
// states are numbered in plain breadth-first order.
int build_machine(const uint8_t *pat, const uint64_t *off, uint32_t n, const HotPlan &plan,
                  Machine &m, std::string &err);

}  // namespace acm
