// scan.h -- device-side machine image and kernel launchers (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace acm {

// Device copy of a Machine (see machine.h); all pointers are device memory
// owned by the automaton.
struct DeviceMachine {
    uint32_t n_states = 0, n_cols = 0, m_max = 0, hot_states = 0;
    uint32_t term_end = 0, acc_end = 0;  // state id ranges (see Machine)
    uint32_t log2_cols = 0, hash_shift = 0;
    // Value of a byte-map entry for bytes in no pattern: 0xff, or 0x100 (which
    // no entry equals) when every byte value occurs in some pattern and the
    // 256 columns use all entry values.
    uint32_t no_class = 0xffu;
    bool cols_pow2 = false, hashed = false;
    uint8_t hash_letter[8] = {0};
    const uint32_t *dfa = nullptr, *go = nullptr;
    const uint32_t *out_off = nullptr, *out_ids = nullptr;
    const uint32_t *own_off = nullptr, *own_ids = nullptr;
    const uint16_t *hot_dfa = nullptr, *hot_go = nullptr;
    const uint8_t *cmap = nullptr;  // 256 bytes
    // Two-byte rows (Machine::pair) live in the dfa allocation from word
    // pair_base on (a multiple of 16); pair_states == 0 when there are none.
    uint32_t pair_states = 0, pair_base = 0;
    // Start-position gate (Machine::gate_bits and its tables); gate_bits is
    // NULL when the machine has none.
    const uint32_t *gate_bits = nullptr, *gate2_bits = nullptr, *gate_node = nullptr;
    const uint32_t *path_off = nullptr, *path_ids = nullptr, *pat_len = nullptr, *path_one = nullptr;
    // Machine::own_one (NULL without a gate).
    const uint32_t *own_one = nullptr;
    // Hashed gate (Machine::qg_bits, qg_tab); qg_bits is NULL without it.
    const uint32_t *qg_bits = nullptr, *qg_tab = nullptr;
    uint32_t qg_tab_bits = 0;
    double gate_pass = 1.0;
    bool dense = false;  // Machine::match_rate above kDenseMatches: gated scans stage matches in registers
};

struct ScanConfig {
    uint32_t algo = 0;       // AC_ALGO_*
    uint32_t chunk = 0;      // DFA chunk bytes (multiple of 16), 0 = auto
    uint32_t block = 0;      // threads per workgroup, 0 = auto
    uint32_t walkers = 0;    // DFA chunks walked per lane (1 to 4), 0 = auto
    uint32_t block_bytes = 0;  // DFA text bytes per walker load (64, 128), 0 = auto
    uint32_t placement = 0;  // resolved AC_PLACE_* (never AUTO here)
    bool pair_steps = true;  // LDS_HOT: two-byte lookups from cold states when built
};

// LDS bytes a workgroup may use on gfx950.
constexpr uint32_t kLdsPerWorkgroup = 160u * 1024u;

int compute_units(int device);

// Each returns AC_OK or an AC_ERR_* code with `err` set. Nothing is
// launched when an error is returned before the first launch.
int launch_zero_count(uint64_t *d_count, hipStream_t stream, std::string &err);
// Continuation of a text scanned in pieces (the per-buffer search with carried
// state of the paper's Alg. 1): positions are reported as base + local
// position, the walk of byte 0 continues from *state_in, and the state after
// the last byte is written to *state_out. Both pointers are device memory and
// may be NULL.
struct StreamArgs {
    uint64_t base = 0;
    const uint32_t *state_in = nullptr;
    uint32_t *state_out = nullptr;
};

int launch_dfa_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                    uint64_t cap, uint64_t *count, const ScanConfig &cfg, hipStream_t stream,
                    std::string &err, const StreamArgs &st = StreamArgs());
int launch_copy_state(const uint32_t *in, uint32_t *out, hipStream_t stream, std::string &err);
// Failure-less walks from the start positions the gate passes (dm.gate_bits
// must be set).
struct Completion;
// With `done` (n > 0) the launch reports its own completion (device_common.h).
// wave_tiles: each wavefront takes at least that many 1,008-byte tiles (fewer
// workgroups for short texts): 1 for the shortest time alone; more where
// launches run side by side, since every workgroup first loads 136 KiB of
// bitmaps into LDS.
int launch_gate_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                     uint64_t cap, uint64_t *count, hipStream_t stream, std::string &err,
                     const Completion *done = nullptr, uint32_t wave_tiles = 1);
// Failure-less walks from the start positions the hashed gate passes
// (dm.qg_bits must be set).
// With `done` (n >= 6) the launch reports its own completion.
int launch_qgate_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                      uint64_t cap, uint64_t *count, hipStream_t stream, std::string &err,
                      const Completion *done = nullptr, uint32_t wave_tiles = 1);
// The gated scan with whichever gate the machine has.
inline int launch_gated_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                             uint64_t cap, uint64_t *count, hipStream_t stream, std::string &err,
                             const Completion *done = nullptr, uint32_t wave_tiles = 1) {
    return dm.gate_bits ? launch_gate_scan(dm, text, n, out, cap, count, stream, err, done, wave_tiles)
                        : launch_qgate_scan(dm, text, n, out, cap, count, stream, err, done, wave_tiles);
}
// Whether launch_gated_scan launches a kernel for n bytes (and so can report
// a completion).
inline bool gated_scan_launches(const DeviceMachine &dm, uint64_t n) { return dm.gate_bits ? n > 0 : n >= 6; }
// The batched gated scan: a task is tiles [t0, t1) of the text of `len` bytes
// at `off` bytes past the launch's base pointer (tile t = the start positions
// [1008 t, 1008 t + 1008) of the text), matched against automaton
// `automaton`, its matches reported at end position + pos_base into the one
// list; tasks are ordered by automaton. The per-automaton argument blocks
// (gate_batch_auto_bytes() each, filled by fill_gate_batch_auto) sit in one
// device array. next_task must be zero at launch. `dense`: stage the matches
// in registers (some automaton's DeviceMachine::dense), else in LDS.
struct GateTask {
    uint64_t off;
    uint32_t len, t0, t1, automaton, pos_base, pad;
};
// The served form's grouped launch: up to kGroupMax requests, each a text
// against an automaton with the class gate (its argument block at `automaton`
// in the same per-automaton array as the batched scan's), cut into tasks of
// `per` tiles; task_end is the running total of tasks up to and including the
// request. Each request has its own list, count and completion word: the
// workgroup that finishes its last task writes {total, seq} to `word` and
// clears count and finished (both zero before the launch).
constexpr uint32_t kGroupMax = 16;
struct GroupReq {
    const uint8_t *text;
    uint64_t *out;
    unsigned long long *count;
    unsigned int *finished;
    uint64_t *word;
    uint64_t cap;
    uint64_t seq;
    uint32_t n, automaton, task_end, pad;
};
// counters: two words on the device, zero before the first launch on a
// stream; each launch leaves them zero for the next one on the same stream.
int launch_gate_group(const void *autos, const GroupReq *reqs, uint32_t n_req, uint32_t per,
                      uint32_t *counters, uint32_t grid, bool dense, hipStream_t stream, std::string &err);
size_t gate_batch_auto_bytes();
void fill_gate_batch_auto(const DeviceMachine &dm, void *dst);
uint32_t gate_batch_tile_bytes();
int launch_gate_batch(const uint8_t *base, const GateTask *tasks, uint32_t n_tasks, const void *autos,
                      uint64_t *out, uint64_t cap, uint64_t *count, uint32_t *next_task, uint32_t grid,
                      bool dense, hipStream_t stream, std::string &err);
int launch_pfac_scan(const DeviceMachine &dm, const uint8_t *text, uint64_t n, uint64_t *out,
                     uint64_t cap, uint64_t *count, const ScanConfig &cfg, hipStream_t stream,
                     std::string &err);

// LSD radix sort of uint64 keys (ascending), using d_tmp scratch.
uint64_t sort_scratch_bytes(uint64_t count);
int launch_sort(uint64_t *keys, uint64_t count, void *tmp, uint64_t tmp_bytes, hipStream_t stream,
                std::string &err);

}  // namespace acm
