// serve.hip -- the served form (the ac_serve_* entry points of include/ac.h).
//
// A scheduler thread admits scan requests into a fixed number of slots as
// slots and device memory free up (continuous batching): each request holds
// a slot (a HIP stream and a few device words) while it is on the device, and
// bytes of one device pool for its text copy and its match list. Requests on
// different slots overlap on the GPU. A request is scanned in pieces with the
// DFA state carried on the device from piece to piece (the per-buffer search
// of the paper's Alg. 1), so a long request never occupies the whole device
// in one launch and host texts can be copied in while earlier pieces scan.
//
// With AC_SERVE_MERGED, requests of the same kernel shape admitted together
// are scanned together:
// one launch of the served kernel covers all their texts (chunks of every
// request in one work list, tasks taken from a device counter), its keys
// carry the request's slot, and a second kernel hands each key to its
// request's list. That keeps the device busy when requests are too short to
// fill it alone. Requests of 64 MiB or more, and reruns, use the per-request
// path above.
//
// The match list is sized before the count is known: the reservation is the
// text length times a per-automaton match rate learnt from finished requests.
// A request whose count exceeds its reservation is scanned again into a list
// of the exact size (its text is still on the device), so results are exact
// whatever the estimate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "automaton.h"
#include "device_common.h"
#include "dfa_kernel.h"
#include "scan.h"

namespace {

using acm::set_error;
using Clock = std::chrono::steady_clock;
constexpr uint64_t kNone = ~0ull;
constexpr uint64_t kAlign = 256;
constexpr uint32_t kPieceEvents = 8;   // copy -> scan hand-off events per slot, reused in turn
constexpr uint32_t kMaxBypass = 16;    // later requests admitted ahead of a waiting head, at most
constexpr size_t kLatencyRing = 65536;  // finished requests kept for the latency percentiles
constexpr uint32_t kLaunches = 3;          // merged launches in flight at once
constexpr uint32_t kMaxTasks = 1u << 16;   // served tasks per merged launch
constexpr uint64_t kLaunchBytes = 512ull << 20;  // text bytes per merged launch (a larger request goes alone)
constexpr uint32_t kMaxAutos = 256;        // automata a server holds
constexpr uint32_t kMaxSlots = 1u << (32 - acm::dfa::kSlotShift);

// Where the demultiplexing kernel puts the keys of one slot.
struct DemuxSlot {
    uint64_t *list;
    uint64_t cap;
    unsigned long long *count;
    uint64_t used;  // nonzero: the slot's request is in the launch
};

// Zero the launch's key count and task counter and the counts of its requests.
__global__ void merged_prepare_kernel(unsigned long long *launch_count, uint32_t *next_task,
                                      const DemuxSlot *slots) {
    const uint32_t i = threadIdx.x;
    if (i == 0) {
        *launch_count = 0;
        *next_task = 0;
    }
    if (i < kMaxSlots && slots[i].used) *slots[i].count = 0;
}

// Hand every key of the launch's list to its request: the slot is the top of
// the position field, the rest is the end position within the request. A
// wave takes 64 keys at a time and, for each slot among them, reserves room
// with one atomic and places its keys by their rank (keys of one request
// mostly arrive together, so that is usually a single atomic per wave).
__global__ void merged_demux_kernel(const uint64_t *keys, const unsigned long long *n_keys, uint64_t cap,
                                    const DemuxSlot *slots) {
    const uint64_t n = min(uint64_t(*n_keys), cap);
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    // whole waves step together, so every ballot sees all 64 lanes
    for (uint64_t base = uint64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u); base < n; base += stride) {
        const uint64_t i = base + lane;
        const bool has = i < n;
        const uint64_t k = has ? keys[i] : 0ull;
        const uint32_t pos = uint32_t(k >> 32);
        const uint32_t slot = pos >> acm::dfa::kSlotShift;
        uint64_t todo = __ballot(has);
        while (todo) {
            const uint32_t leader = uint32_t(__ffsll((unsigned long long)todo) - 1);
            const uint32_t lslot = __shfl(slot, int(leader));
            const bool mine = has && slot == lslot;
            const uint64_t same = __ballot(mine);
            const DemuxSlot d = slots[lslot];
            unsigned long long first = 0;
            if (lane == leader) first = atomicAdd(d.count, (unsigned long long)__popcll(same));
            first = __shfl(first, int(leader));
            if (mine) {
                const uint64_t at = first + acm::lane_rank(same);
                const uint64_t end = pos & ((1u << acm::dfa::kSlotShift) - 1u);
                if (at < d.cap) d.list[at] = (end << 32) | (k & 0xffffffffull);
            }
            todo &= ~same;
        }
    }
}


// First-fit allocator over one device allocation (offsets, 256-byte aligned).
class DevicePool {
public:
    void init(uint64_t bytes) {
        size_ = bytes;
        free_.clear();
        if (bytes) free_[0] = bytes;
        used_ = peak_ = 0;
    }
    uint64_t alloc(uint64_t bytes) {
        bytes = std::max<uint64_t>(kAlign, (bytes + kAlign - 1) & ~(kAlign - 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const uint64_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            taken_[off] = bytes;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return off;
        }
        return kNone;
    }
    void release(uint64_t off) {
        auto t = taken_.find(off);
        if (t == taken_.end()) return;
        uint64_t start = off, len = t->second;
        used_ -= len;
        taken_.erase(t);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && start + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }
    // Keep the first `bytes` of the block at `off` and free the rest.
    void shrink(uint64_t off, uint64_t bytes) {
        auto t = taken_.find(off);
        if (t == taken_.end()) return;
        bytes = std::max<uint64_t>(kAlign, (bytes + kAlign - 1) & ~(kAlign - 1));
        if (bytes >= t->second) return;
        uint64_t tail = off + bytes, len = t->second - bytes;
        t->second = bytes;
        used_ -= len;
        auto next = free_.lower_bound(tail);
        if (next != free_.end() && tail + len == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[tail] = len;
    }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }

private:
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> length, coalesced
    std::unordered_map<uint64_t, uint64_t> taken_;
};

enum class Phase { Queued, Running, WaitMemory, Done };

struct Request {
    uint64_t id = 0;
    uint32_t automaton = 0;
    const uint8_t *src = nullptr;
    uint64_t n = 0;
    bool on_device = false;
    Phase phase = Phase::Queued;
    int slot = -1;
    uint64_t text_off = kNone, out_off = kNone, cap = 0;
    const uint8_t *d_text = nullptr;
    uint64_t *d_out = nullptr;
    uint64_t n_matches = 0;
    uint32_t pieces = 0, rescans = 0, bypassed = 0;
    bool merged = false;    // scanned in a merged launch (else on its slot's stream)
    bool launched = false;  // merged: in a launch
    int status = AC_OK;
    std::string message;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
};

struct Slot {
    hipStream_t scan = nullptr, copy = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t piece[kPieceEvents] = {};
    uint64_t *d_count = nullptr;  // device: match count
    uint32_t *d_state = nullptr;  // device: two carried-state words, used in turn
    uint64_t *h_count = nullptr;  // pinned host copy of the count
    Request *req = nullptr;
};

// One launch of the served kernel over several requests.
struct MergedLaunch {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    acm::dfa::ServedTask *h_tasks = nullptr, *d_tasks = nullptr;  // pinned staging, device copy
    DemuxSlot *h_demux = nullptr, *d_demux = nullptr;
    unsigned long long *d_count = nullptr;  // keys of the launch
    uint32_t *d_next = nullptr;             // task counter
    uint64_t *h_count = nullptr;            // pinned: the launch's key count
    uint64_t *h_words = nullptr;            // pinned mirror of every slot's device words
    uint64_t out_off = kNone, out_cap = 0;
    std::vector<Request *> reqs;
    bool busy = false;
};

}  // namespace

struct ac_server {
    int device = -1;
    std::vector<const ac_automaton *> autos;
    std::vector<double> rate;  // matches per text byte, per automaton
    double rate0 = 0.0;        // the first guess, for automata added later
    uint64_t piece = 0;
    uint8_t *pool_base = nullptr;
    DevicePool pool;
    std::vector<Slot> slots;
    std::vector<MergedLaunch> launches;
    acm::dfa::DfaArgs *d_autos = nullptr;  // every automaton's tables, for the served kernel
    bool merge = false;
    uint64_t merged_launches = 0;
    void *words = nullptr;       // device words of every slot
    uint64_t *h_counts = nullptr;  // pinned count words of every slot
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::vector<Request *> running;  // Running or WaitMemory
    std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
    uint64_t next_id = 1;
    uint64_t submitted = 0, completed = 0, rescans = 0, failed = 0, running_peak = 0;
    uint64_t bytes_done = 0, first_arrival = ~0ull, last_done = 0;
    std::vector<uint64_t> latency;  // ring of the last kLatencyRing finished requests, ns
    size_t latency_next = 0;
    bool stop = false;
    Clock::time_point t0;
    std::thread worker;
};

namespace {

uint64_t now_ns(const ac_server *s) {
    return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - s->t0).count());
}

// Match-list keys reserved for a request: its length times the automaton's
// learnt rate, with a quarter of headroom.
uint64_t reservation(const ac_server *s, const Request *r) {
    const double keys = double(r->n) * s->rate[r->automaton] * 1.25 + 1024.0;
    const uint64_t text = r->on_device ? 0 : (r->n + kAlign - 1) & ~(kAlign - 1);
    const uint64_t room = s->pool.size() > text + kAlign ? (s->pool.size() - text - kAlign) / sizeof(uint64_t) : 0;
    // never more than the pool could hold beside the text: a larger count
    // is found by the rescan, which then needs exactly that much
    return std::min<uint64_t>(keys < double(room) ? uint64_t(keys) : room, room);
}

// Bytes a request needs at once for its text copy and `keys` match keys.
uint64_t footprint(const Request *r, uint64_t keys) {
    const uint64_t text = r->on_device ? 0 : (r->n + kAlign - 1) & ~(kAlign - 1);
    return text + ((std::max<uint64_t>(keys, 1) * sizeof(uint64_t) + kAlign - 1) & ~(kAlign - 1));
}

void finish(ac_server *s, Request *r, int status, const std::string &msg) {
    r->status = status;
    r->message = msg;
    r->phase = Phase::Done;
    r->t_done = now_ns(s);
    if (r->text_off != kNone) {
        s->pool.release(r->text_off);
        r->text_off = kNone;
        r->d_text = r->on_device ? r->d_text : nullptr;
    }
    if (status != AC_OK && r->out_off != kNone) {
        s->pool.release(r->out_off);
        r->out_off = kNone;
        r->d_out = nullptr;
        ++s->failed;
    }
    if (r->slot >= 0) {
        s->slots[size_t(r->slot)].req = nullptr;
        r->slot = -1;
    }
    if (status == AC_OK) {
        s->bytes_done += r->n;
        s->first_arrival = std::min(s->first_arrival, r->t_submit);
        s->last_done = std::max(s->last_done, r->t_done);
        const uint64_t lat = r->t_done - r->t_submit;
        if (s->latency.size() < kLatencyRing)
            s->latency.push_back(lat);
        else
            s->latency[s->latency_next] = lat;
        s->latency_next = (s->latency_next + 1) % kLatencyRing;
    }
    ++s->completed;
    s->cv_done.notify_all();
}

// Queue the request's scans (and, for host texts, its copy) on its slot.
int issue(ac_server *s, Request *r, bool copy_text, std::string &err) {
    Slot &sl = s->slots[size_t(r->slot)];
    const ac_automaton *a = s->autos[r->automaton];
    acm::ScanConfig cfg;
    cfg.algo = AC_ALGO_DFA;
    cfg.placement = a->placement;
    int rc = acm::launch_zero_count(sl.d_count, sl.scan, err);
    if (rc != AC_OK) return rc;
    const uint64_t P = s->piece;
    r->pieces = uint32_t((r->n + P - 1) / P);
    for (uint32_t p = 0; p < r->pieces; ++p) {
        const uint64_t off = uint64_t(p) * P, len = std::min(P, r->n - off);
        if (copy_text) {
            hipError_t e = hipMemcpyAsync(const_cast<uint8_t *>(r->d_text) + off, r->src + off, len,
                                          hipMemcpyHostToDevice, sl.copy);
            if (e == hipSuccess) e = hipEventRecord(sl.piece[p % kPieceEvents], sl.copy);
            if (e == hipSuccess) e = hipStreamWaitEvent(sl.scan, sl.piece[p % kPieceEvents], 0);
            if (e != hipSuccess) {
                err = std::string("text copy: ") + hipGetErrorString(e);
                return AC_ERR_HIP;
            }
        }
        acm::StreamArgs st;
        st.base = off;
        st.state_in = p ? sl.d_state + ((p - 1) & 1u) : nullptr;
        st.state_out = p + 1 < r->pieces ? sl.d_state + (p & 1u) : nullptr;
        rc = acm::launch_dfa_scan(a->dm, r->d_text + off, len, r->d_out, r->cap, sl.d_count, cfg, sl.scan, err,
                                  st);
        if (rc != AC_OK) return rc;
    }
    hipError_t e = hipMemcpyAsync(sl.h_count, sl.d_count, sizeof(uint64_t), hipMemcpyDeviceToHost, sl.scan);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.scan);
    if (e != hipSuccess) {
        err = std::string("completion record: ") + hipGetErrorString(e);
        return AC_ERR_HIP;
    }
    return AC_OK;
}

// Device memory for the request's text copy and match list; false if the
// pool cannot hold them now.
bool reserve(ac_server *s, Request *r) {
    uint64_t t = kNone;
    if (!r->on_device) {
        t = s->pool.alloc(r->n);
        if (t == kNone) return false;
    }
    const uint64_t cap = reservation(s, r);
    const uint64_t o = s->pool.alloc(cap * sizeof(uint64_t));
    if (o == kNone) {
        if (t != kNone) s->pool.release(t);
        return false;
    }
    if (!r->on_device) {
        r->text_off = t;
        r->d_text = s->pool_base + t;
    }
    r->out_off = o;
    r->d_out = reinterpret_cast<uint64_t *>(s->pool_base + o);
    r->cap = cap;
    return true;
}

// The request can join merged launches: its end positions fit below the
// slot field and its slot fits the field.
bool mergeable(const ac_server *s, const Request *r) {
    return s->merge && r->n < (1ull << acm::dfa::kSlotShift) && uint32_t(r->slot) < kMaxSlots &&
           s->autos[r->automaton]->m.m_max < (1u << 20);
}

void start(ac_server *s, Request *r, int slot) {
    r->slot = slot;
    s->slots[size_t(slot)].req = r;
    r->phase = Phase::Running;
    r->t_admit = now_ns(s);
    std::string err;
    if (mergeable(s, r)) {
        // the text goes to the device at once; the next merged launch waits for it
        r->merged = true;
        r->launched = false;
        r->pieces = 1;
        int rc = AC_OK;
        if (!r->on_device) {
            Slot &sl = s->slots[size_t(slot)];
            hipError_t e = hipMemcpyAsync(const_cast<uint8_t *>(r->d_text), r->src, r->n, hipMemcpyHostToDevice, sl.copy);
            if (e == hipSuccess) e = hipEventRecord(sl.piece[0], sl.copy);
            if (e != hipSuccess) {
                rc = AC_ERR_HIP;
                err = std::string("text copy: ") + hipGetErrorString(e);
            }
        }
        if (rc != AC_OK) {
            (void)hipStreamSynchronize(s->slots[size_t(slot)].copy);
            finish(s, r, rc, err);
        } else {
            s->running.push_back(r);
            s->running_peak = std::max<uint64_t>(s->running_peak, s->running.size());
        }
        return;
    }
    const int rc = issue(s, r, !r->on_device, err);
    if (rc != AC_OK) {
        // nothing after the failing call was queued; let the slot drain first
        (void)hipStreamSynchronize(s->slots[size_t(slot)].scan);
        (void)hipStreamSynchronize(s->slots[size_t(slot)].copy);
        finish(s, r, rc, err);
    } else {
        s->running.push_back(r);
        s->running_peak = std::max<uint64_t>(s->running_peak, s->running.size());
    }
}

void admit(ac_server *s) {
    std::vector<int> free_slots;
    for (size_t i = 0; i < s->slots.size(); ++i)
        if (!s->slots[i].req) free_slots.push_back(int(i));
    const uint64_t now = now_ns(s);
    auto it = s->queue.begin();
    while (it != s->queue.end() && !free_slots.empty()) {
        Request *r = *it;
        if (r->t_submit > now) break;  // not arrived yet (the queue is in arrival order)
        if (r->n == 0) {
            r->t_admit = now_ns(s);
            r->pieces = 0;
            finish(s, r, AC_OK, "");
            it = s->queue.erase(it);
            continue;
        }
        if (reserve(s, r)) {
            if (it != s->queue.begin()) ++s->queue.front()->bypassed;
            start(s, r, free_slots.back());
            free_slots.pop_back();
            it = s->queue.erase(it);
            continue;
        }
        // the head waits for memory; later requests may pass it a bounded
        // number of times, then admission holds until the head fits
        if (it == s->queue.begin() && r->bypassed >= kMaxBypass) break;
        ++it;
    }
}

// A slot's scans have finished: check the count against the reservation.
void complete(ac_server *s, Request *r) {
    Slot &sl = s->slots[size_t(r->slot)];
    const uint64_t count = *sl.h_count;
    if (count <= r->cap) {
        r->n_matches = count;
        // a finished list keeps only its own bytes of the budget
        s->pool.shrink(r->out_off, count * sizeof(uint64_t));
        r->cap = count;
        const double seen = double(count) / double(std::max<uint64_t>(1, r->n));
        double &est = s->rate[r->automaton];
        est = std::max(seen, 0.9 * est + 0.1 * seen);
        finish(s, r, AC_OK, "");
        return;
    }
    // too many matches for the reservation: rescan into an exact list
    s->pool.release(r->out_off);
    r->out_off = kNone;
    r->d_out = nullptr;
    r->cap = count;
    r->n_matches = count;
    s->rate[r->automaton] = std::max(s->rate[r->automaton], double(count) / double(r->n));
    r->phase = Phase::WaitMemory;
    ++r->rescans;
    ++s->rescans;
}

bool retry_rescan(ac_server *s, Request *r) {
    if (footprint(r, r->cap) > s->pool.size()) {
        finish(s, r, AC_ERR_TOO_LARGE,
               "the match list (" + std::to_string(r->cap) + " keys) does not fit the HBM budget");
        return false;
    }
    const uint64_t o = s->pool.alloc(r->cap * sizeof(uint64_t));
    if (o == kNone) return false;
    r->out_off = o;
    r->d_out = reinterpret_cast<uint64_t *>(s->pool_base + o);
    r->phase = Phase::Running;
    std::string err;
    const int rc = issue(s, r, false, err);
    if (rc != AC_OK) {
        (void)hipStreamSynchronize(s->slots[size_t(r->slot)].scan);
        finish(s, r, rc, err);
        return false;
    }
    return true;
}

// A request admitted for merging scans on its own slot's stream instead (its
// text is on the device, or being copied there on the slot's copy stream).
void go_alone(ac_server *s, Request *r) {
    r->merged = false;
    Slot &sl = s->slots[size_t(r->slot)];
    std::string err;
    const hipError_t e = r->on_device ? hipSuccess : hipStreamWaitEvent(sl.scan, sl.piece[0], 0);
    const int rc = e == hipSuccess ? issue(s, r, false, err) : AC_ERR_HIP;
    if (rc != AC_OK) {
        (void)hipStreamSynchronize(sl.scan);
        finish(s, r, rc, err.empty() ? std::string("text copy wait failed") : err);
    }
}

// Kernel shape of a request's automaton: LDS image or global table, and
// the byte-class scheme (all requests of one merged launch share it).
uint64_t shape_of(const ac_server *s, const Request *r) {
    const acm::Machine &m = s->autos[r->automaton]->m;
    const uint64_t hot = m.hot_states > 0 ? 1 : 0;
    return hot << 40 | uint64_t(m.hashed ? 1 : 0) << 32 | (m.hashed ? m.log2_cols : 0xffu);
}

// Form and queue one merged launch on an idle launch slot, from requests
// waiting for one (in admission order, one kernel shape). False if none.
bool merge_one(ac_server *s, MergedLaunch &L) {
    std::vector<Request *> cand;
    for (Request *r : s->running)
        if (r->merged && !r->launched && r->phase == Phase::Running) cand.push_back(r);
    if (cand.empty()) return false;
    const uint64_t shape = shape_of(s, cand.front());
    std::vector<Request *> pick;
    uint64_t bytes = 0;
    for (Request *r : cand) {
        if (shape_of(s, r) != shape) continue;
        if (!pick.empty() && bytes + r->n > kLaunchBytes) continue;
        pick.push_back(r);
        bytes += r->n;
    }
    const acm::Machine &m0 = s->autos[pick.front()->automaton]->m;
    const bool hot = m0.hot_states > 0;
    const uint32_t K = 1u, bb = 128u;  // one walker per lane: the served kernels spill with two
    const uint32_t block = hot ? 1024u : 256u;
    const int l2 = m0.hashed ? int(m0.log2_cols) : -1;
    acm::dfa::ServedKernel kernel = hot ? acm::dfa::select_served_hot(m0.hashed, l2, K, bb)
                                        : acm::dfa::select_served_global(m0.hashed, l2, K, bb);
    if (!kernel) {  // no such kernel: these requests go their own way
        for (Request *r : pick) go_alone(s, r);
        return true;
    }
    uint32_t image = 0;
    for (Request *r : pick)
        if (hot) image = std::max<uint32_t>(image, (s->autos[r->automaton]->m.hot_states *
                                                    s->autos[r->automaton]->m.n_cols * 2u + 15u) & ~15u);
    const uint32_t lds = (block / 64) * acm::kQueueBytesPerWave + 256 + image;
    const uint64_t grid_max =
        uint64_t(acm::compute_units(s->device)) * uint64_t(acm::occupancy(reinterpret_cast<const void *>(kernel), block, lds));
    const uint64_t walkers = grid_max * block * K;
    const uint64_t per_task = uint64_t(block) * K;
    // chunks: one per walker the chip holds over the whole launch, as for a
    // plain scan of that many bytes; lengthened if the task list would not fit
    uint32_t n_tasks = 0;
    uint64_t out_cap = 0;
    auto plan = [&](const std::vector<Request *> &reqs) {
        uint64_t total = 0;
        for (Request *r : reqs) total += r->n;
        uint64_t fill = std::max<uint64_t>(1, (total + walkers - 1) / walkers);
        while (true) {
            n_tasks = 0;
            out_cap = 0;
            for (Request *r : reqs) {
                const uint32_t mm = s->autos[r->automaton]->m.m_max;
                uint64_t chunk = fill >= 4ull * mm ? (fill + bb - 1) & ~uint64_t(bb - 1)
                                                   : std::max<uint64_t>(16, (fill + 15) & ~uint64_t(15));
                chunk = std::min<uint64_t>(chunk, 1u << 30);
                const uint64_t items = (r->n + chunk - 1) / chunk;
                for (uint64_t i0 = 0; i0 < items; i0 += per_task) {
                    if (n_tasks < kMaxTasks) {
                        acm::dfa::ServedTask &t = L.h_tasks[n_tasks];
                        t.text = r->d_text;
                        t.own_first = uint32_t(i0 * chunk);
                        t.n_items = uint32_t(std::min<uint64_t>(per_task, items - i0));
                        t.chunk = uint32_t(chunk);
                        t.text_len = uint32_t(r->n);
                        t.automaton = r->automaton;
                        t.slot = uint32_t(r->slot);
                    }
                    ++n_tasks;
                }
                out_cap += std::max<uint64_t>(1, r->cap);
            }
            if (n_tasks <= kMaxTasks) return;
            fill *= 2;
        }
    };
    plan(pick);
    uint64_t out_off = s->pool.alloc(out_cap * sizeof(uint64_t));
    if (out_off == kNone && pick.size() > 1) {
        pick.resize(1);
        plan(pick);
        out_off = s->pool.alloc(out_cap * sizeof(uint64_t));
    }
    if (out_off == kNone) {
        // no room for a launch list beside the requests' own lists: the first
        // request scans on its own stream, which needs only its own list
        go_alone(s, pick.front());
        return true;
    }
    for (uint32_t i = 0; i < kMaxSlots; ++i) L.h_demux[i] = DemuxSlot{nullptr, 0, nullptr, 0};
    for (Request *r : pick) {
        Slot &sl = s->slots[size_t(r->slot)];
        L.h_demux[r->slot] = DemuxSlot{r->d_out, r->cap, reinterpret_cast<unsigned long long *>(sl.d_count), 1};
    }
    uint64_t *d_out = reinterpret_cast<uint64_t *>(s->pool_base + out_off);
    std::string err;
    hipError_t e = hipSuccess;
    for (Request *r : pick)
        if (!r->on_device && e == hipSuccess) e = hipStreamWaitEvent(L.stream, s->slots[size_t(r->slot)].piece[0], 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(L.d_tasks, L.h_tasks, size_t(n_tasks) * sizeof(acm::dfa::ServedTask), hipMemcpyHostToDevice,
                           L.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(L.d_demux, L.h_demux, kMaxSlots * sizeof(DemuxSlot), hipMemcpyHostToDevice, L.stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(merged_prepare_kernel, dim3(1), dim3(kMaxSlots), 0, L.stream, L.d_count, L.d_next,
                           L.d_demux);
        e = hipGetLastError();
    }
    int rc = e == hipSuccess ? AC_OK : AC_ERR_HIP;
    if (rc == AC_OK) {
        acm::dfa::ServedArgs args{L.d_tasks, n_tasks, s->d_autos, d_out, out_cap, L.d_count, L.d_next};
        const uint32_t grid = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(grid_max, n_tasks)));
        rc = acm::launch_kernel(kernel, grid, block, lds, L.stream, args, err);
    }
    if (rc == AC_OK) {
        hipLaunchKernelGGL(merged_demux_kernel, dim3(512), dim3(256), 0, L.stream, d_out, L.d_count, out_cap,
                           L.d_demux);
        e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(L.h_count, L.d_count, sizeof(uint64_t), hipMemcpyDeviceToHost, L.stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(L.h_words, s->words, s->slots.size() * 16, hipMemcpyDeviceToHost, L.stream);
        if (e == hipSuccess) e = hipEventRecord(L.done, L.stream);
        if (e != hipSuccess) {
            rc = AC_ERR_HIP;
            err = std::string("merged launch: ") + hipGetErrorString(e);
        }
    }
    if (rc != AC_OK) {
        (void)hipStreamSynchronize(L.stream);
        s->pool.release(out_off);
        for (Request *r : pick) finish(s, r, rc, err.empty() ? std::string("merged launch failed") : err);
        return true;
    }
    for (Request *r : pick) r->launched = true;
    L.reqs = pick;
    L.out_off = out_off;
    L.out_cap = out_cap;
    L.busy = true;
    ++s->merged_launches;
    return true;
}

// A merged launch has finished: settle each of its requests.
void settle_launch(ac_server *s, MergedLaunch &L) {
    const bool overflow = *L.h_count > L.out_cap;
    for (Request *r : L.reqs) {
        r->merged = false;  // from here on any rerun uses its slot's stream
        if (overflow) {
            // the launch's list was too short: keys are missing, so scan again
            // on the request's own stream (its text is on the device)
            std::string err;
            const int rc = issue(s, r, false, err);
            if (rc != AC_OK) {
                (void)hipStreamSynchronize(s->slots[size_t(r->slot)].scan);
                finish(s, r, rc, err);
            } else {
                ++r->rescans;
                ++s->rescans;
            }
            continue;
        }
        Slot &sl = s->slots[size_t(r->slot)];
        *sl.h_count = L.h_words[size_t(r->slot) * 2];
        complete(s, r);
        if (r->phase == Phase::WaitMemory) retry_rescan(s, r);
    }
    s->pool.release(L.out_off);
    L.out_off = kNone;
    L.out_cap = 0;
    L.reqs.clear();
    L.busy = false;
}

void worker_main(ac_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        bool progress = false;
        for (size_t i = 0; i < s->running.size();) {
            Request *r = s->running[i];
            bool drop = false;
            if (r->merged) {
                drop = r->phase == Phase::Done;  // settled by its launch
            } else if (r->phase == Phase::Running) {
                const hipError_t q = hipEventQuery(s->slots[size_t(r->slot)].done);
                if (q == hipSuccess) {
                    complete(s, r);
                    progress = true;
                    if (r->phase == Phase::WaitMemory) {
                        retry_rescan(s, r);
                    }
                    drop = r->phase == Phase::Done;
                } else if (q != hipErrorNotReady) {
                    finish(s, r, AC_ERR_HIP, std::string("request scan: ") + hipGetErrorString(q));
                    drop = true;
                }
            } else if (r->phase == Phase::WaitMemory) {
                if (retry_rescan(s, r)) progress = true;
                drop = r->phase == Phase::Done;
            }
            if (drop) {
                s->running[i] = s->running.back();
                s->running.pop_back();
            } else {
                ++i;
            }
        }
        for (MergedLaunch &L : s->launches)
            if (L.busy) {
                const hipError_t q = hipEventQuery(L.done);
                if (q == hipSuccess) {
                    settle_launch(s, L);
                    progress = true;
                } else if (q != hipErrorNotReady) {
                    for (Request *r : L.reqs) finish(s, r, AC_ERR_HIP, std::string("merged launch: ") + hipGetErrorString(q));
                    s->pool.release(L.out_off);
                    L.reqs.clear();
                    L.busy = false;
                    progress = true;
                }
            }
        // drop requests their launches finished
        s->running.erase(std::remove_if(s->running.begin(), s->running.end(),
                                        [](const Request *r) { return r->phase == Phase::Done; }),
                         s->running.end());
        const size_t queued = s->queue.size();
        admit(s);
        progress |= s->queue.size() != queued;
        for (MergedLaunch &L : s->launches)
            if (!L.busy && merge_one(s, L)) progress = true;
        s->running.erase(std::remove_if(s->running.begin(), s->running.end(),
                                        [](const Request *r) { return r->phase == Phase::Done; }),
                         s->running.end());
        bool on_device = false;  // some request has work queued on the GPU
        for (const Request *r : s->running) on_device |= r->phase == Phase::Running && !(r->merged && !r->launched);
        for (const MergedLaunch &L : s->launches) on_device |= L.busy;
        if (s->stop && !on_device) {
            // shutting down with nothing on the device: whatever still waits
            // for memory can no longer get it
            for (Request *r : s->running) finish(s, r, AC_ERR_BUSY, "server shut down before the request could run");
            s->running.clear();
            for (Request *r : s->queue) finish(s, r, AC_ERR_BUSY, "server shut down before admission");
            s->queue.clear();
            break;
        }
        if (progress) continue;
        // sleep until a completion may have happened (poll), the next
        // scheduled arrival, or a submit / release / stop
        const uint64_t now = now_ns(s);
        uint64_t wake = on_device ? now + 20000 : kNone;
        if (!s->queue.empty() && s->queue.front()->t_submit > now)
            wake = std::min(wake, s->queue.front()->t_submit);
        if (wake == kNone)
            s->cv_work.wait(lk);
        else if (wake > now)
            s->cv_work.wait_for(lk, std::chrono::nanoseconds(std::min<uint64_t>(wake - now, 20000)));
    }
}

void destroy(ac_server *s) {
    for (Slot &sl : s->slots) {
        if (sl.scan) (void)hipStreamDestroy(sl.scan);
        if (sl.copy) (void)hipStreamDestroy(sl.copy);
        if (sl.done) (void)hipEventDestroy(sl.done);
        for (hipEvent_t &e : sl.piece)
            if (e) (void)hipEventDestroy(e);
    }
    for (MergedLaunch &L : s->launches) {
        if (L.stream) (void)hipStreamDestroy(L.stream);
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.h_tasks) (void)hipHostFree(L.h_tasks);
        if (L.d_tasks) (void)hipFree(L.d_tasks);
        if (L.h_demux) (void)hipHostFree(L.h_demux);
        if (L.d_demux) (void)hipFree(L.d_demux);
        if (L.d_count) (void)hipFree(L.d_count);
        if (L.h_count) (void)hipHostFree(L.h_count);
        if (L.h_words) (void)hipHostFree(L.h_words);
    }
    if (s->d_autos) (void)hipFree(s->d_autos);
    if (s->words) (void)hipFree(s->words);
    if (s->h_counts) (void)hipHostFree(s->h_counts);
    if (s->pool_base) (void)hipFree(s->pool_base);
    delete s;
}

// Upload automaton i's tables to the served kernel's array.
hipError_t upload_auto(ac_server *s, uint32_t i) {
    acm::dfa::DfaArgs a{};
    acm::dfa::fill_machine_args(s->autos[i]->dm, a);
    return hipMemcpy(s->d_autos + i, &a, sizeof(a), hipMemcpyHostToDevice);
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
        if (!autos[i] || !autos[i]->on_device || autos[i]->device != dev || autos[i]->m.goto_only)
            return set_error(AC_ERR_INVALID, "ac_serve_create: automaton " + std::to_string(i) +
                                                 " is NULL, host-only, goto-only or on another device");
    const uint64_t budget = opts && opts->hbm_budget ? opts->hbm_budget : (4ull << 30);
    const uint32_t slots = opts && opts->max_inflight ? opts->max_inflight : 8u;
    const uint64_t piece = opts && opts->piece_bytes ? opts->piece_bytes : (16u << 20);
    const double rate = (opts && opts->match_ppm ? opts->match_ppm : 20000u) * 1e-6;
    if (piece % 16 != 0) return set_error(AC_ERR_INVALID, "ac_serve_create: piece_bytes must be a multiple of 16");
    if (slots > kMaxSlots) return set_error(AC_ERR_INVALID, "ac_serve_create: at most 64 slots");
    if (n_autos > kMaxAutos) return set_error(AC_ERR_INVALID, "ac_serve_create: at most 256 automata");
    if (opts && (opts->flags & ~uint32_t(AC_SERVE_MERGED)))
        return set_error(AC_ERR_INVALID, "ac_serve_create: unknown flags");

    ac_server *s = new (std::nothrow) ac_server();
    if (!s) return set_error(AC_ERR_NOMEM, "ac_serve_create: out of host memory");
    s->device = dev;
    s->autos.assign(autos, autos + n_autos);
    s->rate.assign(n_autos, rate);
    s->rate0 = rate;
    s->piece = piece;
    s->merge = opts && (opts->flags & AC_SERVE_MERGED);
    s->t0 = Clock::now();
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&s->pool_base), budget);
    if (e != hipSuccess) {
        s->pool_base = nullptr;
        destroy(s);
        return set_error(AC_ERR_NOMEM, std::string("ac_serve_create: device pool: ") + hipGetErrorString(e));
    }
    s->pool.init(budget);
    // per slot: count (8 bytes) and two state words, 16 bytes in all
    e = hipMalloc(&s->words, size_t(slots) * 16);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&s->h_counts), size_t(slots) * 8, 0);
    s->slots.resize(slots);
    for (uint32_t i = 0; i < slots && e == hipSuccess; ++i) {
        Slot &sl = s->slots[i];
        sl.d_count = reinterpret_cast<uint64_t *>(static_cast<uint8_t *>(s->words) + 16 * i);
        sl.d_state = reinterpret_cast<uint32_t *>(static_cast<uint8_t *>(s->words) + 16 * i + 8);
        sl.h_count = s->h_counts + i;
        e = hipStreamCreateWithFlags(&sl.scan, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.copy, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        for (uint32_t k = 0; k < kPieceEvents && e == hipSuccess; ++k)
            e = hipEventCreateWithFlags(&sl.piece[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&s->d_autos), kMaxAutos * sizeof(acm::dfa::DfaArgs));
    for (uint32_t i = 0; i < n_autos && e == hipSuccess; ++i) e = upload_auto(s, i);
    s->launches.resize(kLaunches);
    for (MergedLaunch &L : s->launches) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&L.h_tasks), kMaxTasks * sizeof(acm::dfa::ServedTask), 0);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&L.d_tasks), kMaxTasks * sizeof(acm::dfa::ServedTask));
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&L.h_demux), kMaxSlots * sizeof(DemuxSlot), 0);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&L.d_demux), kMaxSlots * sizeof(DemuxSlot));
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&L.d_count), 16);  // count, then task counter
        if (e == hipSuccess) L.d_next = reinterpret_cast<uint32_t *>(L.d_count + 1);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&L.h_count), sizeof(uint64_t), 0);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&L.h_words), size_t(slots) * 16, 0);
    }
    if (e != hipSuccess) {
        destroy(s);
        return set_error(AC_ERR_HIP, std::string("ac_serve_create: ") + hipGetErrorString(e));
    }
    try {
        s->worker = std::thread(worker_main, s);
    } catch (...) {
        destroy(s);
        return set_error(AC_ERR_NOMEM, "ac_serve_create: cannot start the scheduler thread");
    }
    *out = s;
    return AC_OK;
}

int ac_serve_add(ac_server *s, const ac_automaton *a, uint32_t *id) {
    if (!s || !a || !id) return set_error(AC_ERR_INVALID, "ac_serve_add: NULL argument");
    if (!a->on_device || a->device != s->device || a->m.goto_only)
        return set_error(AC_ERR_INVALID, "ac_serve_add: automaton is host-only, goto-only or on another device");
    std::lock_guard<std::mutex> g(s->mu);
    if (s->autos.size() >= kMaxAutos) return set_error(AC_ERR_INVALID, "ac_serve_add: at most 256 automata");
    *id = uint32_t(s->autos.size());
    s->autos.push_back(a);
    s->rate.push_back(s->rate0);
    const hipError_t e = upload_auto(s, *id);
    if (e != hipSuccess) {
        s->autos.pop_back();
        s->rate.pop_back();
        return set_error(AC_ERR_HIP, std::string("ac_serve_add: ") + hipGetErrorString(e));
    }
    return AC_OK;
}

int ac_serve_submit(ac_server *s, uint32_t automaton, const uint8_t *text, uint64_t n, int text_on_device,
                    uint64_t arrival_ns, uint64_t *ticket) {
    if (!s || !ticket) return set_error(AC_ERR_INVALID, "ac_serve_submit: NULL server or ticket");
    if (n > 0 && !text) return set_error(AC_ERR_INVALID, "ac_serve_submit: NULL text");
    if (n >= (1ull << 32)) return set_error(AC_ERR_TOO_LARGE, "ac_serve_submit: text of 2^32 bytes or more");
    if (text_on_device && n > 0 && (reinterpret_cast<uintptr_t>(text) & 15u))
        return set_error(AC_ERR_INVALID, "ac_serve_submit: device text must be 16-byte aligned");
    auto r = std::make_unique<Request>();
    r->automaton = automaton;
    r->src = text;
    r->n = n;
    r->on_device = text_on_device != 0;
    if (r->on_device) r->d_text = text;
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return set_error(AC_ERR_INVALID, "ac_serve_submit: server is shutting down");
    if (automaton >= s->autos.size()) return set_error(AC_ERR_INVALID, "ac_serve_submit: no such automaton");
    if (footprint(r.get(), 1024) > s->pool.size())
        return set_error(AC_ERR_TOO_LARGE, "ac_serve_submit: the request alone exceeds the HBM budget");
    r->id = s->next_id++;
    r->t_submit = std::max(arrival_ns, now_ns(s));
    *ticket = r->id;
    // the queue is kept in arrival order (FIFO among equal times)
    auto pos = s->queue.end();
    while (pos != s->queue.begin() && (*std::prev(pos))->t_submit > r->t_submit) --pos;
    s->queue.insert(pos, r.get());
    s->requests.emplace(r->id, std::move(r));
    ++s->submitted;
    s->cv_work.notify_one();
    return AC_OK;
}

int ac_serve_wait(ac_server *s, uint64_t ticket, int64_t timeout_ms, ac_serve_result *res) {
    if (!s || !res) return set_error(AC_ERR_INVALID, "ac_serve_wait: NULL server or result");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->requests.find(ticket) == s->requests.end())
        return set_error(AC_ERR_INVALID, "ac_serve_wait: unknown ticket");
    // look the ticket up again after every wake-up: another thread may have
    // released it meanwhile
    auto done = [&] {
        auto f = s->requests.find(ticket);
        return f == s->requests.end() || f->second->phase == Phase::Done;
    };
    if (timeout_ms < 0)
        s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done))
        return set_error(AC_ERR_BUSY, "ac_serve_wait: request not finished within the timeout");
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return set_error(AC_ERR_INVALID, "ac_serve_wait: ticket released meanwhile");
    Request *r = it->second.get();
    res->status = r->status;
    res->automaton = r->automaton;
    res->n = r->n;
    res->d_matches = r->d_out;
    res->n_matches = r->n_matches;
    res->t_submit_ns = r->t_submit;
    res->t_admit_ns = r->t_admit;
    res->t_done_ns = r->t_done;
    res->pieces = r->pieces;
    res->rescans = r->rescans;
    if (r->status != AC_OK) return set_error(r->status, "ac_serve_wait: request failed: " + r->message);
    return AC_OK;
}

int ac_serve_release(ac_server *s, uint64_t ticket) {
    if (!s) return set_error(AC_ERR_INVALID, "ac_serve_release: NULL server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return set_error(AC_ERR_INVALID, "ac_serve_release: unknown ticket");
    Request *r = it->second.get();
    if (r->phase != Phase::Done) return set_error(AC_ERR_BUSY, "ac_serve_release: request still running");
    if (r->out_off != kNone) s->pool.release(r->out_off);
    s->requests.erase(it);
    s->cv_work.notify_one();  // memory came free
    return AC_OK;
}

int ac_serve_stats(ac_server *s, ac_serve_stats_t *st) {
    if (!s || !st) return set_error(AC_ERR_INVALID, "ac_serve_stats: NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->failed = s->failed;
    st->queued = s->queue.size();
    st->running = s->running.size();
    st->rescans = s->rescans;
    st->pool_bytes = s->pool.size();
    st->pool_used = s->pool.used();
    st->pool_peak = s->pool.peak();
    st->running_peak = s->running_peak;
    st->merged_launches = s->merged_launches;
    st->bytes_done = s->bytes_done;
    st->p50_ms = st->p99_ms = st->gbps = 0.0;
    if (!s->latency.empty()) {
        std::vector<uint64_t> l(s->latency);
        std::sort(l.begin(), l.end());
        // nearest rank
        auto pct = [&](double q) { return double(l[std::min(l.size() - 1, size_t(q * double(l.size())))]) * 1e-6; };
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
    }
    if (s->last_done > s->first_arrival)
        st->gbps = double(s->bytes_done) / double(s->last_done - s->first_arrival);
    return AC_OK;
}

uint64_t ac_serve_now_ns(const ac_server *s) { return s ? now_ns(s) : 0; }

void ac_serve_destroy(ac_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv_work.notify_one();
    }
    if (s->worker.joinable()) s->worker.join();
    destroy(s);
}

}  // extern "C"
