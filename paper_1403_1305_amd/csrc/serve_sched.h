// serve_sched.h -- the served form's scheduler, host side only (no HIP).
//
// Requests arrive (ac_serve_submit), wait in arrival order, and are admitted
// into a fixed number of slots as slots and bytes of one device pool free up
// (continuous batching): a request holds a slot while its work is on the
// device, and pool bytes for its text copy (host texts) and its match list.
// Requests on different slots overlap on the device.
//
// The device side is reached only through the Device interface below, which
// the library implements with HIP (serve.hip) and the tests with a model that
// completes work on host threads. Its contract keeps the scheduler free of
// cross-slot waits: a slot's work is queued in order on that slot alone, and
// completion is observed by reading a word the device writes (no call that
// waits on device progress). Device calls are made without the scheduler's
// lock held.
//
// The match list is sized before the count is known: the reservation is the
// text length times a per-automaton match rate learnt from finished requests.
// A request whose count exceeds its reservation is scanned again into a list
// of the exact size (its text is still on the device), so results are exact
// whatever the estimate.
#pragma once

#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ac.h"

namespace acm {
namespace serve {

using Clock = std::chrono::steady_clock;
constexpr uint64_t kNone = ~0ull;
constexpr uint64_t kAlign = 256;
constexpr uint32_t kMaxBypass = 16;     // later requests admitted ahead of a waiting head, at most
constexpr size_t kLatencyRing = 65536;  // finished requests kept for the latency percentiles
constexpr uint32_t kMaxSlots = 64;
constexpr uint32_t kMaxAutos = 256;

// First-fit allocator over one device allocation (offsets, 256-byte aligned).
class DevicePool {
public:
    void init(uint64_t bytes) {
        size_ = bytes;
        free_.clear();
        taken_.clear();
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
    std::map<uint64_t, uint64_t> free_;  // offset -> length, coalesced
    std::unordered_map<uint64_t, uint64_t> taken_;
};

// One request's device work, queued in order on its slot: copy a host text
// in (src != nullptr), scan it into the list, then publish the match total
// with the sequence number `seq` on the slot's completion word.
struct SlotWork {
    uint32_t automaton = 0;
    const uint8_t *src = nullptr;  // host text to copy in, or nullptr
    const uint8_t *d_text = nullptr;  // device text (the copy's destination for host texts)
    uint64_t n = 0;
    uint64_t *d_out = nullptr;  // match list, room for cap keys
    uint64_t cap = 0;
    uint64_t seq = 0;
};

// What the scheduler needs from the device.
class Device {
public:
    virtual ~Device() = default;
    // Queue `w` on the slot. May block the calling thread (a copy from pageable
    // host memory), never on another slot's work. On an error nothing more
    // of `w` runs, but part of it may still be queued.
    virtual int run(uint32_t slot, const SlotWork &w, uint32_t *pieces, std::string &err) = 0;
    // Queue the work of several slots at once, as one pass of the scheduler
    // issues it; the device may give several of them one launch. Per item:
    // rc[k] as run() returns it (an item that fails has been recovered) and
    // pieces[k]. By default run() for each.
    virtual void run_many(const uint32_t *slots, const SlotWork *w, size_t n, uint32_t *pieces,
                          std::pair<int, std::string> *rc) {
        for (size_t k = 0; k < n; ++k) {
            rc[k].first = run(slots[k], w[k], &pieces[k], rc[k].second);
            if (rc[k].first != AC_OK) recover(slots[k]);
        }
    }
    // Non-blocking: true once the slot's work with sequence `seq` is done, with
    // its match total in *count.
    virtual bool done(uint32_t slot, uint64_t seq, uint64_t *count) = 0;
    // Bring a slot back to a clean state after a failed run (its queued work
    // drains first).
    virtual void recover(uint32_t slot) = 0;
    // Device address of pool offset `off`.
    virtual uint8_t *pool_at(uint64_t off) = 0;
};

enum class Phase { Queued, Issuing, Running, WaitMemory, Done };

struct Request {
    uint64_t id = 0;
    uint32_t automaton = 0;
    const uint8_t *src = nullptr;
    uint64_t n = 0;
    bool on_device = false;
    Phase phase = Phase::Queued;
    int slot = -1;
    uint64_t seq = 0;  // completion sequence of the run in flight
    uint64_t text_off = kNone, out_off = kNone, cap = 0;
    const uint8_t *d_text = nullptr;
    uint64_t *d_out = nullptr;
    uint64_t n_matches = 0;
    uint32_t pieces = 0, rescans = 0, bypassed = 0;
    bool copy_text = false;  // the next run copies the host text in
    int status = AC_OK;
    std::string message;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
};

struct Stats {
    uint64_t submitted = 0, completed = 0, failed = 0, rescans = 0, running_peak = 0;
    uint64_t bytes_done = 0, first_arrival = ~0ull, last_done = 0;
};

class Scheduler {
public:
    // max_large > 0: at most that many requests of large_bytes or more on the
    // device at once (each fills the chip by itself); shorter ones may pass a
    // large one that waits for this.
    Scheduler(Device *dev, uint64_t pool_bytes, uint32_t slots, std::vector<double> rates, double rate0,
              uint64_t large_bytes = 0, uint32_t max_large = 0)
        : dev_(dev), slots_(slots, nullptr), rate_(std::move(rates)), rate0_(rate0), t0_(Clock::now()),
          large_bytes_(large_bytes), max_large_(max_large) {
        pool_.init(pool_bytes);
    }
    ~Scheduler() { stop(); }

    void start() { worker_ = std::thread([this] { loop(); }); }

    // Finish what is on the device, fail what is still queued, stop the thread.
    void stop() {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
            cv_work_.notify_one();
        }
        if (worker_.joinable()) worker_.join();
    }

    uint64_t now_ns() const {
        return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0_).count());
    }

    uint32_t add_automaton() {
        std::lock_guard<std::mutex> g(mu_);
        rate_.push_back(rate0_);
        return uint32_t(rate_.size() - 1);
    }
    uint32_t automata() {
        std::lock_guard<std::mutex> g(mu_);
        return uint32_t(rate_.size());
    }

    int submit(uint32_t automaton, const uint8_t *text, uint64_t n, bool on_device, uint64_t arrival_ns,
               uint64_t *ticket, std::string &err) {
        auto r = std::make_unique<Request>();
        r->automaton = automaton;
        r->src = text;
        r->n = n;
        r->on_device = on_device;
        if (on_device) r->d_text = text;
        std::lock_guard<std::mutex> g(mu_);
        if (stop_) return fail(err, AC_ERR_INVALID, "ac_serve_submit: server is shutting down");
        if (automaton >= rate_.size()) return fail(err, AC_ERR_INVALID, "ac_serve_submit: no such automaton");
        if (footprint(r.get(), 1024) > pool_.size())
            return fail(err, AC_ERR_TOO_LARGE, "ac_serve_submit: the request alone exceeds the HBM budget");
        r->id = next_id_++;
        r->t_submit = std::max(arrival_ns, now_ns());
        *ticket = r->id;
        // the queue is kept in arrival order (FIFO among equal times)
        auto pos = queue_.end();
        while (pos != queue_.begin() && (*std::prev(pos))->t_submit > r->t_submit) --pos;
        queue_.insert(pos, r.get());
        requests_.emplace(r->id, std::move(r));
        ++st_.submitted;
        cv_work_.notify_one();
        return AC_OK;
    }

    // Block until the request is done (timeout_ms < 0: no limit); copy it out.
    int wait(uint64_t ticket, int64_t timeout_ms, Request *out, std::string &err) {
        std::unique_lock<std::mutex> lk(mu_);
        if (requests_.find(ticket) == requests_.end()) return fail(err, AC_ERR_INVALID, "ac_serve_wait: unknown ticket");
        // look the ticket up again after every wake-up: another thread may have
        // released it meanwhile
        auto done = [&] {
            auto f = requests_.find(ticket);
            return f == requests_.end() || f->second->phase == Phase::Done;
        };
        if (timeout_ms < 0) {
            cv_done_.wait(lk, done);
        } else if (!cv_done_.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
            return fail(err, AC_ERR_BUSY, "ac_serve_wait: request not finished within the timeout; " + describe(ticket));
        }
        auto it = requests_.find(ticket);
        if (it == requests_.end()) return fail(err, AC_ERR_INVALID, "ac_serve_wait: ticket released meanwhile");
        *out = *it->second;
        if (out->status != AC_OK) return fail(err, out->status, "ac_serve_wait: request failed: " + out->message);
        return AC_OK;
    }

    int release(uint64_t ticket, std::string &err) {
        std::lock_guard<std::mutex> g(mu_);
        auto it = requests_.find(ticket);
        if (it == requests_.end()) return fail(err, AC_ERR_INVALID, "ac_serve_release: unknown ticket");
        Request *r = it->second.get();
        if (r->phase != Phase::Done) return fail(err, AC_ERR_BUSY, "ac_serve_release: request still running");
        if (r->out_off != kNone) pool_.release(r->out_off);
        requests_.erase(it);
        cv_work_.notify_one();  // memory came free
        return AC_OK;
    }

    void stats(ac_serve_stats_t *s) {
        std::lock_guard<std::mutex> g(mu_);
        *s = ac_serve_stats_t{};
        s->submitted = st_.submitted;
        s->completed = st_.completed;
        s->failed = st_.failed;
        s->queued = queue_.size();
        s->running = running_.size();
        s->rescans = st_.rescans;
        s->pool_bytes = pool_.size();
        s->pool_used = pool_.used();
        s->pool_peak = pool_.peak();
        s->running_peak = st_.running_peak;
        s->bytes_done = st_.bytes_done;
        if (!latency_.empty()) {
            std::vector<uint64_t> l(latency_);
            std::sort(l.begin(), l.end());
            // nearest rank
            auto pct = [&](double q) { return double(l[std::min(l.size() - 1, size_t(q * double(l.size())))]) * 1e-6; };
            s->p50_ms = pct(0.50);
            s->p99_ms = pct(0.99);
        }
        if (st_.last_done > st_.first_arrival)
            s->gbps = double(st_.bytes_done) / double(st_.last_done - st_.first_arrival);
    }

private:
    static int fail(std::string &err, int code, const std::string &msg) {
        err = msg;
        return code;
    }

    // State of a ticket, for the message of a wait that timed out.
    std::string describe(uint64_t ticket) {
        auto f = requests_.find(ticket);
        if (f == requests_.end()) return "released";
        const Request *r = f->second.get();
        static const char *names[] = {"queued", "issuing", "running", "waiting for memory", "done"};
        std::string s = "phase " + std::string(names[int(r->phase)]) + ", slot " + std::to_string(r->slot) +
                        ", run " + std::to_string(r->seq) + ", " + std::to_string(r->n) + " bytes, reserved " +
                        std::to_string(r->cap) + " keys, " + std::to_string(queue_.size()) + " queued, " +
                        std::to_string(running_.size()) + " on the device, pool " + std::to_string(pool_.used()) +
                        " of " + std::to_string(pool_.size()) + " bytes in use, " +
                        std::to_string(std::count(slots_.begin(), slots_.end(), nullptr)) + " free slots";
        if (!queue_.empty())
            s += ", queue head arrives at " + std::to_string(queue_.front()->t_submit) + " ns (now " +
                 std::to_string(now_ns()) + ", passed " + std::to_string(queue_.front()->bypassed) + " times)";
        if (r->slot >= 0) {
            uint64_t c = 0;
            s += dev_->done(uint32_t(r->slot), r->seq, &c) ? ", its slot reports it done" : ", its slot has not reported";
        }
        return s;
    }

    // Match-list keys reserved for a request: its length times the automaton's
    // learnt rate, with a quarter of headroom.
    uint64_t reservation(const Request *r) const {
        const double keys = double(r->n) * rate_[r->automaton] * 1.25 + 1024.0;
        const uint64_t text = r->on_device ? 0 : (r->n + kAlign - 1) & ~(kAlign - 1);
        const uint64_t room = pool_.size() > text + kAlign ? (pool_.size() - text - kAlign) / sizeof(uint64_t) : 0;
        // never more than the pool could hold beside the text: a larger count
        // is found by the rescan, which then needs exactly that much
        return std::min<uint64_t>(keys < double(room) ? uint64_t(keys) : room, room);
    }

    // Bytes a request needs at once for its text copy and `keys` match keys.
    static uint64_t footprint(const Request *r, uint64_t keys) {
        const uint64_t text = r->on_device ? 0 : (r->n + kAlign - 1) & ~(kAlign - 1);
        return text + ((std::max<uint64_t>(keys, 1) * sizeof(uint64_t) + kAlign - 1) & ~(kAlign - 1));
    }

    void finish(Request *r, int status, const std::string &msg) {
        r->status = status;
        r->message = msg;
        r->phase = Phase::Done;
        r->t_done = now_ns();
        if (r->text_off != kNone) {
            pool_.release(r->text_off);
            r->text_off = kNone;
            if (!r->on_device) r->d_text = nullptr;
        }
        if (status != AC_OK) {
            if (r->out_off != kNone) {
                pool_.release(r->out_off);
                r->out_off = kNone;
                r->d_out = nullptr;
            }
            ++st_.failed;
        }
        if (r->slot >= 0) {
            slots_[size_t(r->slot)] = nullptr;
            r->slot = -1;
        }
        if (status == AC_OK) {
            st_.bytes_done += r->n;
            st_.first_arrival = std::min(st_.first_arrival, r->t_submit);
            st_.last_done = std::max(st_.last_done, r->t_done);
            const uint64_t lat = r->t_done - r->t_submit;
            if (latency_.size() < kLatencyRing)
                latency_.push_back(lat);
            else
                latency_[latency_next_] = lat;
            latency_next_ = (latency_next_ + 1) % kLatencyRing;
        }
        ++st_.completed;
        cv_done_.notify_all();
    }

    // Device memory for the request's text copy and match list; false if the
    // pool cannot hold them now.
    bool reserve(Request *r) {
        uint64_t t = kNone;
        if (!r->on_device) {
            t = pool_.alloc(r->n);
            if (t == kNone) return false;
        }
        const uint64_t cap = reservation(r);
        const uint64_t o = pool_.alloc(cap * sizeof(uint64_t));
        if (o == kNone) {
            if (t != kNone) pool_.release(t);
            return false;
        }
        if (!r->on_device) {
            r->text_off = t;
            r->d_text = dev_->pool_at(t);
        }
        r->out_off = o;
        r->d_out = reinterpret_cast<uint64_t *>(dev_->pool_at(o));
        r->cap = cap;
        return true;
    }

    // Admit the requests that have arrived by `now` (in arrival order, a head
    // waiting for memory passed at most kMaxBypass times) into free slots;
    // they are issued after the lock is dropped.
    void admit(uint64_t now, std::vector<Request *> &to_issue) {
        std::vector<int> free_slots;
        for (size_t i = slots_.size(); i-- > 0;)
            if (!slots_[i]) free_slots.push_back(int(i));
        uint32_t large = 0;  // large requests holding a slot
        for (const Request *r : running_) large += is_large(r) ? 1u : 0u;
        auto it = queue_.begin();
        while (it != queue_.end() && !free_slots.empty()) {
            Request *r = *it;
            if (r->t_submit > now) break;  // not arrived yet (the queue is in arrival order)
            if (is_large(r) && large >= max_large_) {
                ++it;  // waits for a large one to finish; shorter ones go ahead
                continue;
            }
            if (r->n == 0) {
                r->t_admit = now;
                r->pieces = 0;
                finish(r, AC_OK, "");
                it = queue_.erase(it);
                continue;
            }
            if (reserve(r)) {
                if (it != queue_.begin()) ++queue_.front()->bypassed;
                r->slot = free_slots.back();
                free_slots.pop_back();
                slots_[size_t(r->slot)] = r;
                r->t_admit = now;
                r->copy_text = !r->on_device;
                r->phase = Phase::Issuing;
                r->seq = ++seq_;
                running_.push_back(r);
                large += is_large(r) ? 1u : 0u;
                st_.running_peak = std::max<uint64_t>(st_.running_peak, running_.size());
                to_issue.push_back(r);
                it = queue_.erase(it);
                continue;
            }
            // the head waits for memory; later requests may pass it a bounded
            // number of times, then admission holds until the head fits
            if (it == queue_.begin() && r->bypassed >= kMaxBypass) break;
            ++it;
        }
    }

    // A run has finished: check the count against the reservation.
    void complete(Request *r, uint64_t count) {
        if (count <= r->cap) {
            r->n_matches = count;
            // a finished list keeps only its own bytes of the budget
            pool_.shrink(r->out_off, count * sizeof(uint64_t));
            r->cap = count;
            const double seen = double(count) / double(std::max<uint64_t>(1, r->n));
            double &est = rate_[r->automaton];
            est = std::max(seen, 0.9 * est + 0.1 * seen);
            finish(r, AC_OK, "");
            return;
        }
        // too many matches for the reservation: rescan into an exact list
        pool_.release(r->out_off);
        r->out_off = kNone;
        r->d_out = nullptr;
        r->cap = count;
        r->n_matches = count;
        rate_[r->automaton] = std::max(rate_[r->automaton], double(count) / double(r->n));
        r->phase = Phase::WaitMemory;
        ++r->rescans;
        ++st_.rescans;
    }

    // A rescan's exact list; the request is issued again once it fits.
    bool retry_rescan(Request *r, std::vector<Request *> &to_issue) {
        if (footprint(r, r->cap) > pool_.size()) {
            finish(r, AC_ERR_TOO_LARGE, "the match list (" + std::to_string(r->cap) + " keys) does not fit the HBM budget");
            return true;
        }
        const uint64_t o = pool_.alloc(r->cap * sizeof(uint64_t));
        if (o == kNone) return false;
        r->out_off = o;
        r->d_out = reinterpret_cast<uint64_t *>(dev_->pool_at(o));
        r->copy_text = false;  // the text is still on the device
        r->phase = Phase::Issuing;
        r->seq = ++seq_;
        to_issue.push_back(r);
        return true;
    }

    void loop() {
        // the completion polls sleep a few microseconds: ask the kernel for a
        // wake-up close to that rather than its default 50 us slack
        (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
        std::unique_lock<std::mutex> lk(mu_);
        std::vector<Request *> to_issue;
        struct Issue {
            Request *r;
            uint32_t slot;
            SlotWork w;
        };
        std::vector<Issue> work;
        while (true) {
            bool progress = false;
            to_issue.clear();
            // One clock reading decides both which requests have arrived and,
            // below, how long to sleep: a request that arrives between two
            // readings would otherwise be left out of admission by the first
            // and counted as arrived by the second, and with nothing on the
            // device the scheduler would then sleep until the next submit or
            // release, which a client waiting for that request never makes.
            const uint64_t now = now_ns();
            // completions (a word per slot, no device call that waits)
            for (size_t i = 0; i < running_.size();) {
                Request *r = running_[i];
                uint64_t count = 0;
                if (r->phase == Phase::Running && dev_->done(uint32_t(r->slot), r->seq, &count)) {
                    complete(r, count);
                    progress = true;
                }
                if (r->phase == Phase::WaitMemory && retry_rescan(r, to_issue)) progress = true;
                if (r->phase == Phase::Done) {
                    running_[i] = running_.back();
                    running_.pop_back();
                } else {
                    ++i;
                }
            }
            const size_t queued = queue_.size();
            if (!stop_) admit(now, to_issue);
            progress |= queue_.size() != queued;

            if (!to_issue.empty()) {
                // queue the device work without the lock: a copy from pageable
                // host memory may block this thread until the slot's stream
                // takes it, and submit / wait / release must not wait for that
                work.clear();
                for (Request *r : to_issue) {
                    SlotWork w;
                    w.automaton = r->automaton;
                    w.src = r->copy_text ? r->src : nullptr;
                    w.d_text = r->d_text;
                    w.n = r->n;
                    w.d_out = r->d_out;
                    w.cap = r->cap;
                    w.seq = r->seq;
                    work.push_back({r, uint32_t(r->slot), w});
                }
                lk.unlock();
                std::vector<std::pair<int, std::string>> rc(work.size());
                std::vector<uint32_t> pieces(work.size(), 0);
                std::vector<uint32_t> slots(work.size());
                std::vector<SlotWork> works(work.size());
                for (size_t k = 0; k < work.size(); ++k) {
                    slots[k] = work[k].slot;
                    works[k] = work[k].w;
                }
                dev_->run_many(slots.data(), works.data(), work.size(), pieces.data(), rc.data());
                lk.lock();
                for (size_t k = 0; k < work.size(); ++k) {
                    Request *r = work[k].r;
                    r->pieces = pieces[k];
                    if (rc[k].first == AC_OK)
                        r->phase = Phase::Running;
                    else
                        finish(r, rc[k].first, rc[k].second);
                }
                running_.erase(std::remove_if(running_.begin(), running_.end(),
                                              [](const Request *q) { return q->phase == Phase::Done; }),
                               running_.end());
                progress = true;
            }
            bool on_device = false;
            for (const Request *r : running_) on_device |= r->phase == Phase::Running;
            if (stop_ && !on_device) {
                // shutting down with nothing on the device: whatever still waits
                // for memory or admission can no longer run
                for (Request *r : running_) finish(r, AC_ERR_BUSY, "server shut down before the request could run");
                running_.clear();
                for (Request *r : queue_) finish(r, AC_ERR_BUSY, "server shut down before admission");
                queue_.clear();
                break;
            }
            if (progress) continue;
            // nothing changed: poll again shortly while work is on the device,
            // else sleep until the next scheduled arrival (every request that
            // had arrived by `now` was considered above) or a submit / release / stop
            uint64_t wake = on_device ? now + kPollNs : kNone;
            if (!stop_ && !queue_.empty() && queue_.front()->t_submit > now)
                wake = std::min(wake, queue_.front()->t_submit);
            if (wake == kNone)
                cv_work_.wait(lk);
            else if (wake > now)
                cv_work_.wait_for(lk, std::chrono::nanoseconds(std::min<uint64_t>(wake - now, kPollNs)));
        }
    }

    bool is_large(const Request *r) const { return max_large_ > 0 && r->n >= large_bytes_; }

    static constexpr uint64_t kPollNs = 4000;  // completion polling period while work is on the device

    Device *dev_;
    DevicePool pool_;
    std::vector<Request *> slots_;
    std::vector<double> rate_;  // matches per text byte, per automaton
    double rate0_;
    Clock::time_point t0_;
    uint64_t large_bytes_;
    uint32_t max_large_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<Request *> queue_;
    std::vector<Request *> running_;  // Issuing, Running or WaitMemory
    std::unordered_map<uint64_t, std::unique_ptr<Request>> requests_;
    uint64_t next_id_ = 1, seq_ = 0;
    Stats st_;
    std::vector<uint64_t> latency_;
    size_t latency_next_ = 0;
    bool stop_ = false;
    std::thread worker_;
};

}  // namespace serve
}  // namespace acm
