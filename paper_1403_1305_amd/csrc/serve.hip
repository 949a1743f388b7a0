// serve.hip -- the served form (the ac_serve_* entry points of include/ac.h):
// the scheduler of serve_sched.h over a HIP device.
//
// Each slot owns one HIP stream. A request's work is queued on its slot's
// stream alone, in order: the copy of a host text into the pool, then the
// scan, whose last workgroup publishes the match total and the run's
// sequence number to the slot's completion word in pinned host memory and
// clears the slot's device counters for its next run (one launch per request;
// the DFA path and texts too short for a launch publish with a one-thread
// kernel instead). So nothing on one slot ever waits on another, and the
// scheduler sees completions by reading host memory, with no runtime call in
// its polling.
//
// The scan: automata whose start-position gate passes few windows are
// scanned in one gated launch (AC_ALGO_GATED); the others with the DFA, in
// pieces with the state carried on the device from piece to piece (the
// per-buffer search of the paper's Alg. 1).
//
// Short requests against automata with the class gate that one pass of the
// scheduler issues together share a launch (gate_group_kernel): up to 16
// requests, cut into tasks of 64 tiles, on one of a few group streams. Each
// request keeps its own list, count and completion word, written by the
// workgroup that finishes its last task; its slot's stream is not used.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "automaton.h"
#include "device_common.h"
#include "scan.h"
#include "serve_sched.h"

namespace {

using acm::set_error;
using acm::serve::Device;
using acm::serve::Request;
using acm::serve::Scheduler;
using acm::serve::SlotWork;

// The run's total and sequence number to the slot's completion word (count,
// then sequence, the sequence stored last with release order at system
// scope), and the count back to zero for the slot's next run.
__global__ void publish_kernel(unsigned long long *count, uint64_t *word, uint64_t seq) {
    const uint64_t c = *count;
    __hip_atomic_store(word, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(word + 1, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    *count = 0;
}

__global__ void zero_slot_kernel(unsigned long long *count, unsigned int *finished) {
    *count = 0;
    *finished = 0;
}

constexpr size_t kSlotWordBytes = 32;
constexpr uint32_t kGroupStreams = 4;                 // streams that take grouped launches in turn
constexpr uint64_t kGroupBytes = 4ull << 20;          // requests up to this length may be grouped
constexpr uint64_t kLargeBytes = 4ull << 20;          // a gated launch this long fills the GPU
// Tiles per wavefront at least, in a request's own gated launch: requests run
// side by side, so fewer workgroups each (less LDS filling per byte) give
// more throughput than the shortest time alone would. Shorter requests keep
// more workgroups: with a slot each, their latency bounds the rate.
constexpr uint32_t kServeWaveTiles = 16;
constexpr uint32_t kServeWaveTilesShort = 4;
// Tiles of 1,008 start positions per task of a grouped launch (its requests
// are all short): the same share per wavefront of its 16.
constexpr uint32_t kGroupTiles = 16 * kServeWaveTilesShort;

class HipDevice final : public Device {
public:
    struct Slot {
        hipStream_t stream = nullptr;
        unsigned long long *d_count = nullptr;  // device: the run's match count
        uint32_t *d_state = nullptr;            // device: two carried-state words, used in turn
        unsigned int *d_finished = nullptr;     // device: workgroups of the run's scan done
    };

    int device = -1;
    uint64_t piece = 0;
    uint8_t *pool_base = nullptr;
    std::vector<Slot> slots;
    void *words = nullptr;      // device words of every slot (count, two state words, finish counter)
    uint64_t *h_words = nullptr;  // pinned host: two completion words per slot (total, sequence)
    const ac_automaton *autos[acm::serve::kMaxAutos] = {};
    bool groupable[acm::serve::kMaxAutos] = {};  // gated scan with the class gate
    std::atomic<uint32_t> n_autos{0};
    void *d_autos = nullptr;       // device: per automaton, the gated scan's argument block
    uint32_t *d_gcount = nullptr;  // device: two counters per group stream
    hipStream_t gstream[kGroupStreams] = {};
    uint32_t next_group = 0;

    ~HipDevice() override {
        for (Slot &sl : slots)
            if (sl.stream) {
                (void)hipStreamSynchronize(sl.stream);
                (void)hipStreamDestroy(sl.stream);
            }
        for (hipStream_t g : gstream)
            if (g) {
                (void)hipStreamSynchronize(g);
                (void)hipStreamDestroy(g);
            }
        if (d_autos) (void)hipFree(d_autos);
        if (d_gcount) (void)hipFree(d_gcount);
        if (words) (void)hipFree(words);
        if (h_words) (void)hipHostFree(h_words);
        if (pool_base) (void)hipFree(pool_base);
    }

    hipError_t init(uint64_t budget, uint32_t n_slots) {
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&pool_base), budget);
        if (e != hipSuccess) {
            pool_base = nullptr;
            return e;
        }
        // per slot: count (8 bytes), two state words, the finish counter
        e = hipMalloc(&words, size_t(n_slots) * kSlotWordBytes);
        if (e == hipSuccess) e = hipMemset(words, 0, size_t(n_slots) * kSlotWordBytes);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&h_words), size_t(n_slots) * 16, hipHostMallocCoherent);
        if (e != hipSuccess) return e;
        std::memset(h_words, 0, size_t(n_slots) * 16);
        slots.resize(n_slots);
        for (uint32_t i = 0; i < n_slots && e == hipSuccess; ++i) {
            Slot &sl = slots[i];
            uint8_t *base = static_cast<uint8_t *>(words) + kSlotWordBytes * i;
            sl.d_count = reinterpret_cast<unsigned long long *>(base);
            sl.d_state = reinterpret_cast<uint32_t *>(base + 8);
            sl.d_finished = reinterpret_cast<unsigned int *>(base + 16);
            e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        }
        if (e == hipSuccess) e = hipMalloc(&d_autos, acm::serve::kMaxAutos * acm::gate_batch_auto_bytes());
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&d_gcount), kGroupStreams * 2 * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMemset(d_gcount, 0, kGroupStreams * 2 * sizeof(uint32_t));
        for (uint32_t g = 0; g < kGroupStreams && e == hipSuccess; ++g)
            e = hipStreamCreateWithFlags(&gstream[g], hipStreamNonBlocking);
        return e;
    }

    bool add(const ac_automaton *a, uint32_t *id) {
        const uint32_t k = n_autos.load();
        if (k >= acm::serve::kMaxAutos) return false;
        autos[k] = a;
        groupable[k] = false;
        if (a->dm.gate_bits && acm::auto_algo(a) == AC_ALGO_GATED) {
            // the group kernel's argument block (copied before the
            // automaton can be named by a request)
            bind_thread();
            std::vector<uint8_t> blob(acm::gate_batch_auto_bytes());
            acm::fill_gate_batch_auto(a->dm, blob.data());
            groupable[k] = hipMemcpy(static_cast<uint8_t *>(d_autos) + size_t(k) * blob.size(), blob.data(),
                                     blob.size(), hipMemcpyHostToDevice) == hipSuccess;
        }
        n_autos.store(k + 1);
        *id = k;
        return true;
    }

    bool grouped(const SlotWork &w) const {
        return groupable[w.automaton] && w.n > 0 && w.n <= kGroupBytes;
    }

    // One grouped launch for the items `idx` of w (at most kGroupMax).
    int run_group(const uint32_t *slot_of, const SlotWork *w, const std::vector<size_t> &idx, std::string &err) {
        hipStream_t gs = gstream[next_group];
        uint32_t *counters = d_gcount + 2 * next_group;
        next_group = (next_group + 1) % kGroupStreams;
        acm::GroupReq reqs[acm::kGroupMax] = {};
        uint32_t tasks = 0;
        bool dense = false;
        const uint64_t tile = acm::gate_batch_tile_bytes();
        for (size_t j = 0; j < idx.size(); ++j) {
            const SlotWork &x = w[idx[j]];
            const Slot &sl = slots[slot_of[idx[j]]];
            if (x.src) {
                const hipError_t e = hipMemcpyAsync(const_cast<uint8_t *>(x.d_text), x.src, x.n, hipMemcpyHostToDevice, gs);
                if (e != hipSuccess) {
                    err = std::string("text copy: ") + hipGetErrorString(e);
                    return AC_ERR_HIP;
                }
            }
            acm::GroupReq &r = reqs[j];
            r.text = x.d_text;
            r.out = x.d_out;
            r.count = sl.d_count;
            r.finished = sl.d_finished;
            r.word = h_words + 2 * slot_of[idx[j]];
            r.cap = x.cap;
            r.seq = x.seq;
            r.n = uint32_t(x.n);
            r.automaton = x.automaton;
            tasks += uint32_t((x.n + tile * kGroupTiles - 1) / (tile * kGroupTiles));
            r.task_end = tasks;
            dense |= autos[x.automaton]->dm.dense;
        }
        const uint32_t grid = std::min<uint32_t>(tasks, uint32_t(acm::compute_units(device)));
        return acm::launch_gate_group(d_autos, reqs, uint32_t(idx.size()), kGroupTiles, counters, grid, dense, gs, err);
    }

    void run_many(const uint32_t *slot_of, const SlotWork *w, size_t n, uint32_t *pieces,
                  std::pair<int, std::string> *rc) override {
        bind_thread();
        std::vector<size_t> group, rest;
        for (size_t k = 0; k < n; ++k) (grouped(w[k]) ? group : rest).push_back(k);
        if (group.size() < 2) {
            rest.insert(rest.end(), group.begin(), group.end());
            group.clear();
        }
        // by automaton, shortest first: fewer bitmap loads, early completions
        std::sort(group.begin(), group.end(), [&](size_t x, size_t y) {
            return w[x].automaton != w[y].automaton ? w[x].automaton < w[y].automaton : w[x].n < w[y].n;
        });
        for (size_t b = 0; b < group.size(); b += acm::kGroupMax) {
            const std::vector<size_t> part(group.begin() + b, group.begin() + std::min(group.size(), b + acm::kGroupMax));
            std::string err;
            const int r = run_group(slot_of, w, part, err);
            for (size_t k : part) {
                pieces[k] = 1;
                rc[k].first = r;
                rc[k].second = err;
            }
            if (r != AC_OK)
                for (size_t k : part) recover(slot_of[k]);
        }
        for (size_t k : rest) {
            rc[k].first = run(slot_of[k], w[k], &pieces[k], rc[k].second);
            if (rc[k].first != AC_OK) recover(slot_of[k]);
        }
    }

    void bind_thread() {
        thread_local int bound = -1;
        if (bound != device) {
            (void)hipSetDevice(device);
            bound = device;
        }
    }

    int run(uint32_t slot, const SlotWork &w, uint32_t *pieces, std::string &err) override {
        bind_thread();
        Slot &sl = slots[slot];
        const ac_automaton *a = autos[w.automaton];
        *pieces = 0;
        if (w.src) {
            const hipError_t e = hipMemcpyAsync(const_cast<uint8_t *>(w.d_text), w.src, w.n, hipMemcpyHostToDevice,
                                                sl.stream);
            if (e != hipSuccess) {
                err = std::string("text copy: ") + hipGetErrorString(e);
                return AC_ERR_HIP;
            }
        }
        uint64_t *count = reinterpret_cast<uint64_t *>(sl.d_count);
        int rc = AC_OK;
        bool published = false;
        if (acm::auto_algo(a) == AC_ALGO_GATED) {
            *pieces = 1;
            if (acm::gated_scan_launches(a->dm, w.n)) {
                const acm::Completion c{sl.d_finished, h_words + 2 * slot, w.seq};
                rc = acm::launch_gated_scan(a->dm, w.d_text, w.n, w.d_out, w.cap, count, sl.stream, err, &c,
                                            w.n >= kLargeBytes ? kServeWaveTiles : kServeWaveTilesShort);
                published = true;
            } else {
                rc = acm::launch_gated_scan(a->dm, w.d_text, w.n, w.d_out, w.cap, count, sl.stream, err, nullptr,
                                            w.n >= kLargeBytes ? kServeWaveTiles : kServeWaveTilesShort);
            }
        } else {
            acm::ScanConfig cfg;
            cfg.algo = AC_ALGO_DFA;
            cfg.placement = a->placement;
            const uint64_t P = piece;
            *pieces = uint32_t((w.n + P - 1) / P);
            for (uint32_t p = 0; p < *pieces && rc == AC_OK; ++p) {
                const uint64_t off = uint64_t(p) * P, len = std::min(P, w.n - off);
                acm::StreamArgs st;
                st.base = off;
                st.state_in = p ? sl.d_state + ((p - 1) & 1u) : nullptr;
                st.state_out = p + 1 < *pieces ? sl.d_state + (p & 1u) : nullptr;
                rc = acm::launch_dfa_scan(a->dm, w.d_text + off, len, w.d_out, w.cap, count, cfg, sl.stream, err, st);
            }
        }
        if (rc != AC_OK) return rc;
        if (published) return AC_OK;
        hipLaunchKernelGGL(publish_kernel, dim3(1), dim3(1), 0, sl.stream, sl.d_count, h_words + 2 * slot, w.seq);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            err = std::string("completion launch: ") + hipGetErrorString(e);
            return AC_ERR_HIP;
        }
        return AC_OK;
    }

    bool done(uint32_t slot, uint64_t seq, uint64_t *count) override {
        if (__atomic_load_n(h_words + 2 * slot + 1, __ATOMIC_ACQUIRE) != seq) return false;
        *count = __atomic_load_n(h_words + 2 * slot, __ATOMIC_RELAXED);
        return true;
    }

    void recover(uint32_t slot) override {
        bind_thread();
        Slot &sl = slots[slot];
        (void)hipStreamSynchronize(sl.stream);
        for (hipStream_t g : gstream) (void)hipStreamSynchronize(g);  // grouped launches write the slot too
        hipLaunchKernelGGL(zero_slot_kernel, dim3(1), dim3(1), 0, sl.stream, sl.d_count, sl.d_finished);
        (void)hipStreamSynchronize(sl.stream);
    }

    uint8_t *pool_at(uint64_t off) override { return pool_base + off; }
};

}  // namespace

struct ac_server {
    std::unique_ptr<HipDevice> dev;
    std::unique_ptr<Scheduler> sched;
};

namespace {

bool usable(const ac_automaton *a, int dev) {
    return a && a->on_device && a->device == dev && !a->m.goto_only;
}

}  // namespace

extern "C" {

int ac_serve_create(const ac_automaton *const *autos, uint32_t n_autos, const ac_serve_opts *opts,
                    ac_server **out) {
    if (!out) return set_error(AC_ERR_INVALID, "ac_serve_create: out is NULL");
    *out = nullptr;
    if (!autos || n_autos == 0) return set_error(AC_ERR_INVALID, "ac_serve_create: no automata");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(AC_ERR_HIP, "ac_serve_create: hipGetDevice failed");
    for (uint32_t i = 0; i < n_autos; ++i)
        if (!usable(autos[i], dev))
            return set_error(AC_ERR_INVALID, "ac_serve_create: automaton " + std::to_string(i) +
                                                 " is NULL, host-only, goto-only or on another device");
    const uint64_t budget = opts && opts->hbm_budget ? opts->hbm_budget : (4ull << 30);
    const uint32_t slots = opts && opts->max_inflight ? opts->max_inflight : 8u;
    const uint64_t piece = opts && opts->piece_bytes ? opts->piece_bytes : (16u << 20);
    const double rate = (opts && opts->match_ppm ? opts->match_ppm : 20000u) * 1e-6;
    if (piece % 16 != 0) return set_error(AC_ERR_INVALID, "ac_serve_create: piece_bytes must be a multiple of 16");
    if (slots > acm::serve::kMaxSlots) return set_error(AC_ERR_INVALID, "ac_serve_create: at most 64 slots");
    if (n_autos > acm::serve::kMaxAutos) return set_error(AC_ERR_INVALID, "ac_serve_create: at most 256 automata");
    if (opts && opts->flags) return set_error(AC_ERR_INVALID, "ac_serve_create: unknown flags");
    if (opts && opts->reserved) return set_error(AC_ERR_INVALID, "ac_serve_create: reserved must be 0");
    const uint32_t max_large = opts ? opts->max_large : 0u;  // 0: no limit

    ac_server *s = new (std::nothrow) ac_server();
    if (!s) return set_error(AC_ERR_NOMEM, "ac_serve_create: out of host memory");
    s->dev.reset(new (std::nothrow) HipDevice());
    if (!s->dev) {
        delete s;
        return set_error(AC_ERR_NOMEM, "ac_serve_create: out of host memory");
    }
    HipDevice &d = *s->dev;
    d.device = dev;
    d.piece = piece;
    const hipError_t e = d.init(budget, slots);
    if (e != hipSuccess) {
        const int code = d.pool_base ? AC_ERR_HIP : AC_ERR_NOMEM;
        delete s;
        return set_error(code, std::string("ac_serve_create: ") + hipGetErrorString(e));
    }
    uint32_t id = 0;
    for (uint32_t i = 0; i < n_autos; ++i) d.add(autos[i], &id);
    try {
        s->sched.reset(new Scheduler(&d, budget, slots, std::vector<double>(n_autos, rate), rate, kLargeBytes, max_large));
        s->sched->start();
    } catch (...) {
        s->sched.reset();
        delete s;
        return set_error(AC_ERR_NOMEM, "ac_serve_create: cannot start the scheduler thread");
    }
    *out = s;
    return AC_OK;
}

int ac_serve_add(ac_server *s, const ac_automaton *a, uint32_t *id) {
    if (!s || !a || !id) return set_error(AC_ERR_INVALID, "ac_serve_add: NULL argument");
    if (!usable(a, s->dev->device))
        return set_error(AC_ERR_INVALID, "ac_serve_add: automaton is host-only, goto-only or on another device");
    // the device table first: a ticket can name the automaton only once the
    // scheduler counts it
    uint32_t k = 0;
    if (!s->dev->add(a, &k)) return set_error(AC_ERR_INVALID, "ac_serve_add: at most 256 automata");
    *id = s->sched->add_automaton();
    return AC_OK;
}

int ac_serve_submit(ac_server *s, uint32_t automaton, const uint8_t *text, uint64_t n, int text_on_device,
                    uint64_t arrival_ns, uint64_t *ticket) {
    if (!s || !ticket) return set_error(AC_ERR_INVALID, "ac_serve_submit: NULL server or ticket");
    if (n > 0 && !text) return set_error(AC_ERR_INVALID, "ac_serve_submit: NULL text");
    if (n >= (1ull << 32)) return set_error(AC_ERR_TOO_LARGE, "ac_serve_submit: text of 2^32 bytes or more");
    if (text_on_device && n > 0 && (reinterpret_cast<uintptr_t>(text) & 15u))
        return set_error(AC_ERR_INVALID, "ac_serve_submit: device text must be 16-byte aligned");
    std::string err;
    const int rc = s->sched->submit(automaton, text, n, text_on_device != 0, arrival_ns, ticket, err);
    return rc == AC_OK ? AC_OK : set_error(rc, err);
}

int ac_serve_wait(ac_server *s, uint64_t ticket, int64_t timeout_ms, ac_serve_result *res) {
    if (!s || !res) return set_error(AC_ERR_INVALID, "ac_serve_wait: NULL server or result");
    Request r;
    std::string err;
    const int rc = s->sched->wait(ticket, timeout_ms, &r, err);
    if (rc == AC_OK || r.id == ticket) {
        res->status = r.status;
        res->automaton = r.automaton;
        res->n = r.n;
        res->d_matches = r.d_out;
        res->n_matches = r.n_matches;
        res->t_submit_ns = r.t_submit;
        res->t_admit_ns = r.t_admit;
        res->t_done_ns = r.t_done;
        res->pieces = r.pieces;
        res->rescans = r.rescans;
    }
    return rc == AC_OK ? AC_OK : set_error(rc, err);
}

int ac_serve_release(ac_server *s, uint64_t ticket) {
    if (!s) return set_error(AC_ERR_INVALID, "ac_serve_release: NULL server");
    std::string err;
    const int rc = s->sched->release(ticket, err);
    return rc == AC_OK ? AC_OK : set_error(rc, err);
}

int ac_serve_stats(ac_server *s, ac_serve_stats_t *st) {
    if (!s || !st) return set_error(AC_ERR_INVALID, "ac_serve_stats: NULL argument");
    s->sched->stats(st);
    return AC_OK;
}

uint64_t ac_serve_now_ns(const ac_server *s) { return s ? s->sched->now_ns() : 0; }

void ac_serve_destroy(ac_server *s) {
    if (!s) return;
    s->sched->stop();  // finishes the device work, fails what still waits
    s->sched.reset();
    s->dev.reset();
    delete s;
}

}  // extern "C"
