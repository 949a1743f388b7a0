// api.hip -- the extern "C" surface declared in include/ac.h.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>

#include "../../include/ac.h"
#include "automaton.h"
#include "device_common.h"
#include "machine.h"
#include "scan.h"

namespace {
thread_local std::string g_err;
}  // namespace

int acm::set_error(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

namespace {

int fail(int code, const std::string &msg) { return acm::set_error(code, msg); }

// Largest LDS image, in bytes, a build may plan for: the LDS of a workgroup
// less the match queues of 16 waves and some slack.
uint32_t lds_budget(const ac_build_opts *o) {
    const uint32_t dflt = acm::kLdsPerWorkgroup - 9 * 1024;
    if (!o || o->lds_bytes == 0) return dflt;
    return std::min(o->lds_bytes, dflt);
}

template <typename T>
int upload(ac_automaton *a, const std::vector<T> &v, const T **dst, hipStream_t stream) {
    *dst = nullptr;
    if (v.empty()) return AC_OK;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, v.size() * sizeof(T));
    if (e != hipSuccess) return fail(AC_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    a->allocations.push_back(p);
    e = hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return fail(AC_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    *dst = static_cast<const T *>(p);
    return AC_OK;
}

// The DFA table, followed (from a word offset that is a multiple of 16) by
// the two-byte rows when the machine has them, in one device allocation.
int upload_dfa(ac_automaton *a, const acm::Machine &m, acm::DeviceMachine &dm, hipStream_t stream) {
    dm.dfa = nullptr;
    dm.pair_states = 0;
    dm.pair_base = 0;
    if (m.dfa.empty()) return AC_OK;
    const size_t base = m.pair.empty() ? m.dfa.size() : (m.dfa.size() + 15) & ~size_t(15);
    const size_t words = base + m.pair.size();
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, words * sizeof(uint32_t));
    if (e != hipSuccess) return fail(AC_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    a->allocations.push_back(p);
    uint32_t *d = static_cast<uint32_t *>(p);
    e = hipMemcpyAsync(d, m.dfa.data(), m.dfa.size() * sizeof(uint32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !m.pair.empty())
        e = hipMemcpyAsync(d + base, m.pair.data(), m.pair.size() * sizeof(uint32_t), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return fail(AC_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    dm.dfa = d;
    if (!m.pair.empty()) {
        dm.pair_states = m.pair_states;
        dm.pair_base = uint32_t(base);
    }
    return AC_OK;
}

void release(ac_automaton *a) {
    for (void *p : a->allocations) (void)hipFree(p);
    a->allocations.clear();
}

int build_common(const uint8_t *pat, const uint64_t *off, uint32_t n, const ac_build_opts *opts,
                 ac_automaton **out, ac_automaton *&a) {
    if (!out) return fail(AC_ERR_INVALID, "ac_build: out is NULL");
    *out = nullptr;
    const uint32_t place = opts ? opts->placement : AC_PLACE_AUTO;
    if (place > AC_PLACE_LDS_HOT) return fail(AC_ERR_INVALID, "ac_build: unknown placement");
    const uint32_t flags = opts ? opts->flags : 0u;
    if (flags & ~uint32_t(AC_BUILD_GOTO_ONLY | AC_BUILD_PAIR_ROWS | AC_BUILD_NO_GATE))
        return fail(AC_ERR_INVALID, "ac_build: unknown flags");
    a = new (std::nothrow) ac_automaton();
    if (!a) return fail(AC_ERR_NOMEM, "ac_build: out of host memory");
    const uint32_t budget = lds_budget(opts);
    acm::HotPlan plan;
    if (place == AC_PLACE_AUTO || place == AC_PLACE_LDS_HOT) {
        plan.lds_bytes = budget;
        plan.max_states = opts ? opts->hot_states : 0;
        plan.only_if_needed = place == AC_PLACE_AUTO;
    }
    plan.goto_only = (flags & AC_BUILD_GOTO_ONLY) != 0;
    plan.pair_rows = (flags & AC_BUILD_PAIR_ROWS) != 0;
    plan.gate = (flags & AC_BUILD_NO_GATE) == 0;
    plan.threads = opts ? opts->threads : 0u;
    std::string err;
    int rc;
    try {
        rc = acm::build_machine(pat, off, n, plan, a->m, err);
    } catch (const std::bad_alloc &) {
        rc = AC_ERR_NOMEM;
        err = "ac_build: out of host memory";
    } catch (const std::exception &e) {  // e.g. a build thread that cannot start
        rc = AC_ERR_NOMEM;
        err = std::string("ac_build: ") + e.what();
    }
    if (rc != AC_OK) {
        delete a;
        a = nullptr;
        return fail(rc, err);
    }
    const uint64_t full = 256ull + uint64_t(a->m.n_states) * a->m.n_cols * 4ull;
    if (place == AC_PLACE_LDS_FULL && full > budget) {
        delete a;
        a = nullptr;
        return fail(AC_ERR_TOO_LARGE, "ac_build: table does not fit the LDS (placement LDS_FULL)");
    }
    if (place == AC_PLACE_AUTO)
        a->placement = full <= budget ? AC_PLACE_LDS_FULL
                                      : (a->m.hot_states > 0 ? AC_PLACE_LDS_HOT : AC_PLACE_GLOBAL);
    else
        a->placement = place;
    if (a->placement == AC_PLACE_LDS_HOT && a->m.hot_states == 0) a->placement = AC_PLACE_GLOBAL;
    return AC_OK;
}

bool resolve_placement(const ac_automaton *a, uint32_t want, uint32_t &place) {
    place = want == AC_PLACE_AUTO ? a->placement : want;
    if (place == AC_PLACE_LDS_HOT && a->m.hot_states == 0) return false;
    // the whole-table kernels run 256 threads: 4 waves of match queues beside the table
    if (place == AC_PLACE_LDS_FULL &&
        256ull + uint64_t(a->m.n_states) * a->m.n_cols * 4ull + 4ull * acm::kQueueBytesPerWave >
            acm::kLdsPerWorkgroup)
        return false;
    return place <= AC_PLACE_LDS_HOT;
}

}  // namespace

extern "C" {

const char *ac_last_error(void) { return g_err.c_str(); }

int ac_build(const uint8_t *pat_bytes, const uint64_t *pat_off, uint32_t n_patterns,
             const ac_build_opts *opts, void *stream, ac_automaton **out) {
    ac_automaton *a = nullptr;
    int rc = build_common(pat_bytes, pat_off, n_patterns, opts, out, a);
    if (rc != AC_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        delete a;
        return fail(AC_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    a->device = dev;
    acm::DeviceMachine &dm = a->dm;
    const acm::Machine &m = a->m;
    dm.n_states = m.n_states;
    dm.n_cols = m.n_cols;
    dm.m_max = m.m_max;
    dm.hot_states = m.hot_states;
    dm.term_end = m.term_end;
    dm.acc_end = m.acc_end;
    dm.log2_cols = m.log2_cols;
    dm.cols_pow2 = m.cols_pow2;
    dm.hashed = m.hashed;
    dm.hash_shift = m.hash_shift;
    std::memcpy(dm.hash_letter, m.hash_letter, sizeof(dm.hash_letter));
    dm.gate_pass = m.gate_pass;
    dm.dense = m.match_rate > acm::kDenseMatches;
    dm.qg_tab_bits = m.qg_tab_bits;
    dm.no_class = m.sigma == 256 ? 0x100u : uint32_t(acm::kNoClass);
    std::vector<uint8_t> cmap(m.cmap, m.cmap + 256);
    if ((rc = upload_dfa(a, m, dm, s)) || (rc = upload(a, m.go, &dm.go, s)) ||
        (rc = upload(a, m.out_off, &dm.out_off, s)) || (rc = upload(a, m.out_ids, &dm.out_ids, s)) ||
        (rc = upload(a, m.own_off, &dm.own_off, s)) || (rc = upload(a, m.own_ids, &dm.own_ids, s)) ||
        (rc = upload(a, m.hot_dfa, &dm.hot_dfa, s)) || (rc = upload(a, m.hot_go, &dm.hot_go, s)) ||
        (rc = upload(a, cmap, &dm.cmap, s)) || (rc = upload(a, m.gate_bits, &dm.gate_bits, s)) || (rc = upload(a, m.gate2_bits, &dm.gate2_bits, s)) ||
        (rc = upload(a, m.gate_node, &dm.gate_node, s)) || (rc = upload(a, m.path_off, &dm.path_off, s)) ||
        (rc = upload(a, m.path_ids, &dm.path_ids, s)) || (rc = upload(a, m.pat_len, &dm.pat_len, s)) ||
        (rc = upload(a, m.path_one, &dm.path_one, s)) || (rc = upload(a, m.own_one, &dm.own_one, s)) ||
        (rc = upload(a, m.qg_bits, &dm.qg_bits, s)) || (rc = upload(a, m.qg_tab, &dm.qg_tab, s))) {
        (void)hipStreamSynchronize(s);
        release(a);
        delete a;
        return rc;
    }
    // out_ids may be empty only if no pattern exists, which build rejects
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        release(a);
        delete a;
        return fail(AC_ERR_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    }
    a->on_device = true;
    *out = a;
    return AC_OK;
}

int ac_build_host(const uint8_t *pat_bytes, const uint64_t *pat_off, uint32_t n_patterns,
                  const ac_build_opts *opts, ac_automaton **out) {
    ac_automaton *a = nullptr;
    int rc = build_common(pat_bytes, pat_off, n_patterns, opts, out, a);
    if (rc != AC_OK) return rc;
    *out = a;
    return AC_OK;
}

void ac_free(ac_automaton *a) {
    if (!a) return;
    release(a);
    delete a;
}

int ac_info(const ac_automaton *a, ac_info_t *info) {
    if (!a || !info) return fail(AC_ERR_INVALID, "ac_info: NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->n_states = a->m.n_states;
    info->n_patterns = a->m.n_patterns;
    info->sigma = a->m.sigma;
    info->n_cols = a->m.n_cols;
    info->m_max = a->m.m_max;
    info->placement = a->placement;
    info->hot_states = a->m.hot_states;
    info->class_shift = a->m.hash_shift;
    info->class_hashed = a->m.hashed ? 1u : 0u;
    info->table_bytes = a->m.goto_only ? 0ull : uint64_t(a->m.n_states) * a->m.n_cols * 4ull;
    info->goto_only = a->m.goto_only ? 1u : 0u;
    info->pair_states = a->m.pair_states;
    info->out_entries = a->m.out_ids.size();
    info->build_ms = a->m.build_ms;
    info->has_gate = !a->m.gate_bits.empty() ? 1u : !a->m.qg_bits.empty() ? 2u : 0u;
    info->gate_pass = a->m.gate_pass;
    info->match_rate = a->m.match_rate;
    return AC_OK;
}

int ac_get_table(const ac_automaton *a, uint32_t which, void *dst, uint64_t dst_bytes,
                 uint64_t *bytes) {
    if (!a || !bytes) return fail(AC_ERR_INVALID, "ac_get_table: NULL argument");
    const void *src = nullptr;
    uint64_t sz = 0;
    const acm::Machine &m = a->m;
    switch (which) {
        case AC_TABLE_DFA: src = m.dfa.data(); sz = m.dfa.size() * 4; break;
        case AC_TABLE_GO: src = m.go.data(); sz = m.go.size() * 4; break;
        case AC_TABLE_OUT_OFF: src = m.out_off.data(); sz = m.out_off.size() * 4; break;
        case AC_TABLE_OUT_IDS: src = m.out_ids.data(); sz = m.out_ids.size() * 4; break;
        case AC_TABLE_OWN_OFF: src = m.own_off.data(); sz = m.own_off.size() * 4; break;
        case AC_TABLE_OWN_IDS: src = m.own_ids.data(); sz = m.own_ids.size() * 4; break;
        case AC_TABLE_HOT_DFA: src = m.hot_dfa.data(); sz = m.hot_dfa.size() * 2; break;
        case AC_TABLE_HOT_GO: src = m.hot_go.data(); sz = m.hot_go.size() * 2; break;
        case AC_TABLE_CMAP: src = m.cmap; sz = 256; break;
        case AC_TABLE_PAIR: src = m.pair.data(); sz = m.pair.size() * 4; break;
        case AC_TABLE_GATE_BITS: src = m.gate_bits.data(); sz = m.gate_bits.size() * 4; break;
        case AC_TABLE_GATE_NODE: src = m.gate_node.data(); sz = m.gate_node.size() * 4; break;
        case AC_TABLE_PATH_OFF: src = m.path_off.data(); sz = m.path_off.size() * 4; break;
        case AC_TABLE_PATH_IDS: src = m.path_ids.data(); sz = m.path_ids.size() * 4; break;
        case AC_TABLE_GATE2_BITS: src = m.gate2_bits.data(); sz = m.gate2_bits.size() * 4; break;
        case AC_TABLE_QGATE_BITS: src = m.qg_bits.data(); sz = m.qg_bits.size() * 4; break;
        case AC_TABLE_QGATE_TAB: src = m.qg_tab.data(); sz = m.qg_tab.size() * 4; break;
        case AC_TABLE_OWN_ONE: src = m.own_one.data(); sz = m.own_one.size() * 4; break;
        case AC_TABLE_PATH_ONE: src = m.path_one.data(); sz = m.path_one.size() * 4; break;
        default: return fail(AC_ERR_INVALID, "ac_get_table: unknown table");
    }
    *bytes = sz;
    if (!dst) return AC_OK;
    if (dst_bytes < sz) return fail(AC_ERR_INVALID, "ac_get_table: destination too small");
    if (sz) std::memcpy(dst, src, sz);
    return AC_OK;
}

int ac_scan(const ac_automaton *a, const uint8_t *d_text, uint64_t n, uint64_t *d_matches,
            uint64_t capacity, uint64_t *d_count, const ac_scan_opts *opts, void *stream) {
    if (!a || !d_count) return fail(AC_ERR_INVALID, "ac_scan: NULL automaton or count");
    if (!a->on_device) return fail(AC_ERR_INVALID, "ac_scan: automaton has no device tables");
    if (n > 0 && !d_text) return fail(AC_ERR_INVALID, "ac_scan: NULL text");
    if (capacity > 0 && !d_matches) return fail(AC_ERR_INVALID, "ac_scan: NULL match buffer");
    if (n >= (1ull << 32)) return fail(AC_ERR_TOO_LARGE, "ac_scan: text of 2^32 bytes or more");
    if (n > 0 && (reinterpret_cast<uintptr_t>(d_text) & 15u))
        return fail(AC_ERR_INVALID, "ac_scan: text must be 16-byte aligned");
    acm::ScanConfig cfg;
    uint32_t want = AC_PLACE_AUTO;
    bool append = false;
    if (opts) {
        cfg.algo = opts->algo;
        cfg.chunk = opts->chunk;
        cfg.block = opts->block;
        cfg.walkers = opts->walkers;
        cfg.block_bytes = opts->block_bytes;
        cfg.pair_steps = opts->pair_steps == AC_PAIR_AUTO;
        want = opts->placement;
        if (opts->pair_steps > AC_PAIR_OFF) return fail(AC_ERR_INVALID, "ac_scan: unknown pair_steps");
        if (opts->append > 1) return fail(AC_ERR_INVALID, "ac_scan: append must be 0 or 1");
        append = opts->append != 0;
    }
    if (cfg.algo > AC_ALGO_GATED) return fail(AC_ERR_INVALID, "ac_scan: unknown algo");
    if (cfg.algo == AC_ALGO_AUTO) cfg.algo = acm::auto_algo(a);
    if (cfg.algo == AC_ALGO_DFA && a->m.goto_only)
        return fail(AC_ERR_INVALID, "ac_scan: a goto-only automaton has no DFA (use AC_ALGO_PFAC or AC_ALGO_GATED)");
    if (cfg.algo == AC_ALGO_GATED && !a->dm.gate_bits && !a->dm.qg_bits)
        return fail(AC_ERR_INVALID, "ac_scan: this automaton has no start-position gate (AC_ALGO_GATED)");
    if (!resolve_placement(a, want, cfg.placement))
        return fail(AC_ERR_INVALID, "ac_scan: placement not available for this automaton");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != a->device) return fail(AC_ERR_INVALID, "ac_scan: automaton lives on another device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::string err;
    int rc = append ? AC_OK : acm::launch_zero_count(d_count, s, err);
    if (rc == AC_OK) {
        if (cfg.algo == AC_ALGO_DFA)
            rc = acm::launch_dfa_scan(a->dm, d_text, n, d_matches, capacity, d_count, cfg, s, err);
        else if (cfg.algo == AC_ALGO_GATED)
            rc = acm::launch_gated_scan(a->dm, d_text, n, d_matches, capacity, d_count, s, err);
        else
            rc = acm::launch_pfac_scan(a->dm, d_text, n, d_matches, capacity, d_count, cfg, s, err);
    }
    return rc == AC_OK ? AC_OK : fail(rc, err);
}

int ac_scan_stream(const ac_automaton *a, const uint8_t *d_text, uint64_t n, uint64_t base,
                   const uint32_t *d_state_in, uint32_t *d_state_out, uint64_t *d_matches,
                   uint64_t capacity, uint64_t *d_count, int append, const ac_scan_opts *opts,
                   void *stream) {
    if (!a || !d_count) return fail(AC_ERR_INVALID, "ac_scan_stream: NULL automaton or count");
    if (!a->on_device) return fail(AC_ERR_INVALID, "ac_scan_stream: automaton has no device tables");
    if (a->m.goto_only) return fail(AC_ERR_INVALID, "ac_scan_stream: a goto-only automaton has no DFA");
    if (n > 0 && !d_text) return fail(AC_ERR_INVALID, "ac_scan_stream: NULL text");
    if (capacity > 0 && !d_matches) return fail(AC_ERR_INVALID, "ac_scan_stream: NULL match buffer");
    if (base + n >= (1ull << 32) || base >= (1ull << 32))
        return fail(AC_ERR_TOO_LARGE, "ac_scan_stream: positions must stay below 2^32");
    if (n > 0 && (reinterpret_cast<uintptr_t>(d_text) & 15u))
        return fail(AC_ERR_INVALID, "ac_scan_stream: text must be 16-byte aligned");
    if (d_state_in && d_state_in == d_state_out)
        return fail(AC_ERR_INVALID, "ac_scan_stream: state_in and state_out must differ");
    acm::ScanConfig cfg;
    uint32_t want = AC_PLACE_AUTO;
    if (opts) {
        if (opts->algo != AC_ALGO_DFA && opts->algo != AC_ALGO_AUTO)
            return fail(AC_ERR_INVALID, "ac_scan_stream: only the DFA scan carries state");
        cfg.chunk = opts->chunk;
        cfg.block = opts->block;
        cfg.walkers = opts->walkers;
        cfg.block_bytes = opts->block_bytes;
        cfg.pair_steps = opts->pair_steps == AC_PAIR_AUTO;
        want = opts->placement;
        if (opts->pair_steps > AC_PAIR_OFF) return fail(AC_ERR_INVALID, "ac_scan_stream: unknown pair_steps");
        if (opts->append > 1) return fail(AC_ERR_INVALID, "ac_scan_stream: append must be 0 or 1");
        append = append || opts->append;
    }
    if (!resolve_placement(a, want, cfg.placement))
        return fail(AC_ERR_INVALID, "ac_scan_stream: placement not available for this automaton");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != a->device)
        return fail(AC_ERR_INVALID, "ac_scan_stream: automaton lives on another device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::string err;
    int rc = append ? AC_OK : acm::launch_zero_count(d_count, s, err);
    acm::StreamArgs st;
    st.base = base;
    st.state_in = d_state_in;
    st.state_out = d_state_out;
    if (rc == AC_OK)
        rc = acm::launch_dfa_scan(a->dm, d_text, n, d_matches, capacity, d_count, cfg, s, err, st);
    return rc == AC_OK ? AC_OK : fail(rc, err);
}

int ac_scan_sync(const ac_automaton *a, const uint8_t *d_text, uint64_t n, uint64_t *d_matches,
                 uint64_t capacity, uint64_t *d_count, const ac_scan_opts *opts, void *stream,
                 uint64_t *h_count) {
    if (!h_count) return fail(AC_ERR_INVALID, "ac_scan_sync: NULL host count");
    int rc = ac_scan(a, d_text, n, d_matches, capacity, d_count, opts, stream);
    if (rc != AC_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(h_count, d_count, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(AC_ERR_HIP, std::string("ac_scan_sync: ") + hipGetErrorString(e));
    if (*h_count > capacity)
        return fail(AC_ERR_OVERFLOW, "ac_scan_sync: " + std::to_string(*h_count) +
                                         " matches exceed capacity " + std::to_string(capacity));
    return AC_OK;
}

uint64_t ac_sort_scratch_bytes(uint64_t count) { return acm::sort_scratch_bytes(count); }

int ac_sort_matches(uint64_t *d_keys, uint64_t count, void *d_tmp, uint64_t tmp_bytes, void *stream) {
    if (count > 1 && (!d_keys || !d_tmp)) return fail(AC_ERR_INVALID, "ac_sort_matches: NULL buffer");
    std::string err;
    int rc = acm::launch_sort(d_keys, count, d_tmp, tmp_bytes, static_cast<hipStream_t>(stream), err);
    return rc == AC_OK ? AC_OK : fail(rc, err);
}

}  // extern "C"
