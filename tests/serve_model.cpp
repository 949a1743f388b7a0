// Host-only model of the served form's scheduler (serve_sched.h) for tests:
// a fake device completes each slot's work on host threads after random
// delays, in order per slot, and writes the completion word as the HIP
// device does. The scenarios replay the request sequences the served form
// runs (saturated replays then Poisson arrivals; host and device texts in
// small pieces; many slots; memory-bound admission, rescans, lists that
// never fit, shutdown with requests waiting). Every ticket must end within
// a bounded wait with the expected count. Built with ThreadSanitizer by
// tests/test_serve_model.py.
//
//   serve_model <scenario> <seed>     prints "ok ..." or "FAIL ..." and exits 0 / 1
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "serve_sched.h"

using namespace acm::serve;

namespace {

// Matches a fake automaton reports for a text of n bytes: a fixed rate per
// automaton, so that a request's expected count is known in advance.
uint64_t fake_count(uint32_t automaton, uint64_t n) { return n * (automaton % 4) / 64 + (n % 7); }

class FakeDevice final : public Device {
public:
    // large: requests of this many bytes or more are counted while on the
    // "device" (large_peak(): the most at once)
    explicit FakeDevice(uint32_t slots, uint64_t seed, int fail_every, uint64_t large = ~0ull)
        : q_(slots), words_(slots), rng_(seed), fail_every_(fail_every), large_(large) {
        for (auto &w : words_) {
            w.count.store(0);
            w.seq.store(0);
        }
        for (uint32_t s = 0; s < slots; ++s) threads_.emplace_back([this, s] { engine(s); });
    }
    ~FakeDevice() override {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : threads_) t.join();
    }

    int run(uint32_t slot, const SlotWork &w, uint32_t *pieces, std::string &err) override {
        uint64_t delay, copy_us;
        bool fail;
        {
            std::lock_guard<std::mutex> g(mu_);
            delay = 1 + rng_() % 300 + w.n / (1 << 20);  // microseconds on the "device"
            copy_us = w.src ? rng_() % 200 : 0;          // a pageable copy blocks the caller
            fail = fail_every_ > 0 && rng_() % uint64_t(fail_every_) == 0;
        }
        if (copy_us) std::this_thread::sleep_for(std::chrono::microseconds(copy_us));
        *pieces = 1;
        if (fail) {
            err = "injected launch failure";
            return AC_ERR_HIP;
        }
        {
            std::lock_guard<std::mutex> g(mu_);
            const bool large = w.n >= large_;
            q_[slot].push_back(Job{w.seq, fake_count(w.automaton, w.n), delay, large});
            ++queued_;
            if (large) large_peak_ = std::max(large_peak_, ++large_now_);
        }
        cv_.notify_all();
        return AC_OK;
    }
    bool done(uint32_t slot, uint64_t seq, uint64_t *count) override {
        if (words_[slot].seq.load(std::memory_order_acquire) != seq) return false;
        *count = words_[slot].count.load(std::memory_order_relaxed);
        return true;
    }
    void recover(uint32_t slot) override {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return q_[slot].empty() && !busy_[slot]; });
    }
    uint8_t *pool_at(uint64_t off) override { return reinterpret_cast<uint8_t *>(uintptr_t(0x100000) + off); }
    uint32_t large_peak() {
        std::lock_guard<std::mutex> g(mu_);
        return large_peak_;
    }

private:
    struct Job {
        uint64_t seq, count, delay_us;
        bool large;
    };
    struct Word {
        std::atomic<uint64_t> count, seq;
    };
    void engine(uint32_t s) {
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            cv_.wait(lk, [&] { return stop_ || !q_[s].empty(); });
            if (q_[s].empty()) return;
            const Job j = q_[s].front();
            q_[s].pop_front();
            busy_[s] = true;
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(j.delay_us));
            lk.lock();
            if (j.large) --large_now_;  // before its completion can be seen
            lk.unlock();
            words_[s].count.store(j.count, std::memory_order_relaxed);
            words_[s].seq.store(j.seq, std::memory_order_release);
            lk.lock();
            busy_[s] = false;
            cv_.notify_all();
        }
    }
    std::mutex mu_;
    std::condition_variable cv_;
    std::vector<std::deque<Job>> q_;
    std::vector<Word> words_;
    std::map<uint32_t, bool> busy_;
    std::vector<std::thread> threads_;
    std::mt19937_64 rng_;
    int fail_every_;
    uint64_t large_;
    uint32_t large_now_ = 0, large_peak_ = 0;
    uint64_t queued_ = 0;
    bool stop_ = false;
};

struct Spec {
    uint64_t n;
    uint32_t automaton;
    bool host;
    uint64_t arrival;  // ns after the replay's start (0: at once)
};

int failures = 0;
void check(bool ok, const char *what, uint64_t a = 0, uint64_t b = 0) {
    if (!ok) {
        std::printf("FAIL %s (%llu, %llu)\n", what, (unsigned long long)a, (unsigned long long)b);
        ++failures;
    }
}

// Submit the requests, wait for each in turn (bounded), check and release.
// With `expect_errors` a request may fail with an injected error.
void replay(Scheduler &s, const std::vector<Spec> &reqs, bool expect_errors, int64_t wait_ms = 20000) {
    static std::vector<uint8_t> host(1 << 16, 'A');
    const uint64_t t0 = s.now_ns() + 2'000'000;
    std::vector<uint64_t> tickets;
    for (const Spec &r : reqs) {
        uint64_t t = 0;
        std::string err;
        const uint8_t *text = r.host ? host.data() : reinterpret_cast<const uint8_t *>(uintptr_t(0x4000));
        const int rc = s.submit(r.automaton, text, r.n, !r.host, r.arrival ? t0 + r.arrival : t0, &t, err);
        check(rc == AC_OK, "submit", rc);
        tickets.push_back(t);
    }
    for (size_t i = 0; i < tickets.size(); ++i) {
        Request out;
        std::string err;
        const int rc = s.wait(tickets[i], wait_ms, &out, err);
        if (rc == AC_ERR_BUSY) {
            std::printf("FAIL ticket %llu not done within %lld ms: %s\n", (unsigned long long)tickets[i],
                        (long long)wait_ms, err.c_str());
            ++failures;
            return;
        }
        if (rc == AC_OK)
            check(out.n_matches == fake_count(reqs[i].automaton, reqs[i].n), "count", out.n_matches,
                  fake_count(reqs[i].automaton, reqs[i].n));
        else
            check(expect_errors && rc == AC_ERR_HIP, "unexpected failure", uint64_t(rc));
        std::string e2;
        check(s.release(tickets[i], e2) == AC_OK, "release");
    }
}

std::vector<Spec> log_uniform(std::mt19937_64 &rng, int count, double lo, double hi, uint32_t autos, bool host_half,
                              uint64_t max_host = 1 << 16) {
    std::uniform_real_distribution<double> u(0.0, 1.0);
    std::vector<Spec> v;
    for (int i = 0; i < count; ++i) {
        Spec s;
        s.n = uint64_t(std::exp(std::log(lo) + (std::log(hi) - std::log(lo)) * u(rng)));
        s.automaton = uint32_t(rng() % autos);
        s.host = host_half && (i % 2 == 0);
        if (s.host) s.n = std::min<uint64_t>(s.n, max_host);
        s.arrival = 0;
        v.push_back(s);
    }
    return v;
}

}  // namespace

int main(int argc, char **argv) {
    const std::string scenario = argc > 1 ? argv[1] : "saturated";
    const uint64_t seed = argc > 2 ? std::strtoull(argv[2], nullptr, 10) : 1;
    std::mt19937_64 rng(seed);
    if (scenario == "saturated") {
        // 512 requests (device texts), two saturated replays then Poisson
        // arrivals at half the service rate, 8 slots, a 4 GiB budget
        FakeDevice dev(8, seed, 0);
        Scheduler s(&dev, 4ull << 30, 8, std::vector<double>(8, 0.02), 0.02);
        s.start();
        auto reqs = log_uniform(rng, 512, 1024, 64 << 20, 8, false);
        replay(s, reqs, false);
        replay(s, reqs, false);
        std::exponential_distribution<double> gap(1.0 / 150e3);  // ns between arrivals
        double at = 0;
        for (Spec &r : reqs) r.arrival = uint64_t(at += gap(rng)) + 1;
        replay(s, reqs, false);
        ac_serve_stats_t st;
        s.stats(&st);
        check(st.completed == 3 * 512 && st.failed == 0 && st.pool_used == 0, "stats", st.completed, st.pool_used);
        check(st.running_peak > 1, "overlap", st.running_peak);
    } else if (scenario == "mix") {
        // 40 requests, half host texts (the copy blocks the scheduler), 64 MiB
        // budget, 8 slots; then each alone
        FakeDevice dev(8, seed, 0);
        Scheduler s(&dev, 64ull << 20, 8, std::vector<double>(4, 0.02), 0.02);
        s.start();
        auto reqs = log_uniform(rng, 40, 16, 1 << 18, 4, true);
        replay(s, reqs, false);
        for (const Spec &r : reqs) replay(s, {r}, false);
        ac_serve_stats_t st;
        s.stats(&st);
        check(st.completed == 80 && st.failed == 0 && st.pool_used == 0, "stats", st.completed, st.failed);
    } else if (scenario == "slots16") {
        // many small requests over 16 slots, with launch failures injected;
        // at most 2 of 16 KiB or more on the device at once
        FakeDevice dev(16, seed, 23, 16 << 10);
        Scheduler s(&dev, 256ull << 20, 16, std::vector<double>(6, 0.02), 0.02, 16 << 10, 2);
        s.start();
        auto reqs = log_uniform(rng, 600, 16, 1 << 16, 6, true);
        replay(s, reqs, true);
        ac_serve_stats_t st;
        s.stats(&st);
        check(st.completed == 600 && st.pool_used == 0, "stats", st.completed, st.pool_used);
        check(dev.large_peak() >= 1 && dev.large_peak() <= 2, "large requests at once", dev.large_peak());
    } else if (scenario == "memory") {
        // a 1 MiB budget (admission waits for memory), a match-rate guess far
        // too low (rescans), one list that can never fit, then shutdown while
        // requests wait for memory behind results that are never released
        FakeDevice dev(4, seed, 0, 8 << 10);
        Scheduler s(&dev, 1 << 20, 4, std::vector<double>(4, 1e-6), 1e-6, 8 << 10, 1);
        s.start();
        auto reqs = log_uniform(rng, 120, 16, 1 << 16, 4, true);
        // largest first: the first admitted overflow before any finished
        // request can teach the scheduler a better rate
        std::sort(reqs.begin(), reqs.end(), [](const Spec &a, const Spec &b) { return a.n > b.n; });
        replay(s, reqs, false);
        ac_serve_stats_t st;
        s.stats(&st);
        check(st.rescans > 0, "rescans", st.rescans);
        check(st.pool_peak <= (1u << 20) && st.pool_used == 0, "memory stats", st.pool_peak, st.pool_used);
        check(dev.large_peak() <= 1, "large requests at once", dev.large_peak());
        // automaton 3 makes n * 3 / 64 keys: 8 MiB of text gives 3 MiB of keys
        uint64_t t = 0;
        std::string err;
        check(s.submit(3, reinterpret_cast<const uint8_t *>(uintptr_t(0x4000)), 8 << 20, true, 0, &t, err) == AC_OK, "big");
        Request out;
        check(s.wait(t, 20000, &out, err) == AC_ERR_TOO_LARGE, "too large");
        check(s.release(t, err) == AC_OK, "release big");
        std::vector<uint64_t> held;
        for (int i = 0; i < 8; ++i) {
            // 1 MiB of text makes 48 Ki keys (384 KiB): two lists fill the pool
            check(s.submit(3, reinterpret_cast<const uint8_t *>(uintptr_t(0x4000)), 1 << 20, true, 0, &t, err) == AC_OK,
                  "held");
            held.push_back(t);
        }
        s.wait(held[0], 20000, &out, err);  // its list is never released
        s.stop();
        for (uint64_t h : held) {
            const int rc = s.wait(h, 20000, &out, err);
            check(rc == AC_OK || rc == AC_ERR_BUSY, "after stop", uint64_t(rc));
            check(rc != AC_ERR_BUSY || out.status == AC_ERR_BUSY, "stopped request", uint64_t(out.status));
        }
    } else {
        std::printf("FAIL unknown scenario %s\n", scenario.c_str());
        return 2;
    }
    if (failures) return 1;
    std::printf("ok %s seed %llu\n", scenario.c_str(), (unsigned long long)seed);
    return 0;
}
