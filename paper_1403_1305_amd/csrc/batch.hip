// batch.hip -- many texts against several resident automata in one persistent
// launch (the ac_batch_* entry points of include/ac.h).
//
// The plan cuts every text into work items of `chunk` end positions (each
// walked from at most m_max - 1 bytes before its first owned byte, never from
// before its own text), orders the items by automaton, and groups them into
// tasks of one item per walker of a workgroup. One launch of batch_kernel then
// covers the whole batch: workgroups take tasks in increasing order from a
// device counter, so each loads a new LDS image at most once per automaton.
// The counter reset and the launch can be captured once into a hipGraph and
// replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "automaton.h"
#include "dfa_kernel.h"

struct ac_batch {
    int device = -1;
    uint32_t placement = AC_PLACE_GLOBAL, walkers = 1, block_bytes = 128, chunk = 0;
    uint32_t block = 256, lds = 0, grid = 1;
    uint32_t n_items = 0, n_tasks = 0, n_texts = 0, n_autos = 0;
    uint64_t text_bytes = 0;  // sum of the text lengths
    acm::dfa::BatchKernel kernel = nullptr;
    acm::dfa::BatchItem *d_items = nullptr;
    acm::dfa::BatchTask *d_tasks = nullptr;
    acm::dfa::DfaArgs *d_autos = nullptr;
    uint32_t *d_next = nullptr;  // task counter of the persistent launch
    // graph of (counter reset, batch kernel) for one set of buffers
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *g_text = nullptr;
    const void *g_out = nullptr;
    const void *g_count = nullptr;
    uint64_t g_cap = 0;
};

namespace {

using acm::set_error;

void release(ac_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_tasks) (void)hipFree(b->d_tasks);
    if (b->d_autos) (void)hipFree(b->d_autos);
    if (b->d_next) (void)hipFree(b->d_next);
    b->exec = nullptr;
    b->graph = nullptr;
    b->capture = nullptr;
    b->d_items = nullptr;
    b->d_tasks = nullptr;
    b->d_autos = nullptr;
    b->d_next = nullptr;
}

// Match count and task counter to zero (a kernel, not a memset, so that the
// pair can sit in a captured graph).
__global__ void batch_reset_kernel(unsigned long long *count, uint32_t *next_task) {
    *count = 0;
    *next_task = 0;
}

template <typename T>
int upload(const std::vector<T> &v, T **dst, hipStream_t s) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return set_error(AC_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    *dst = static_cast<T *>(p);
    if (!v.empty()) {
        e = hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return set_error(AC_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    }
    return AC_OK;
}

int launch(ac_batch *b, const uint8_t *text, uint64_t *out, uint64_t cap, uint64_t *count,
           hipStream_t s) {
    std::string err;
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, s,
                       reinterpret_cast<unsigned long long *>(count), b->d_next);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(AC_ERR_HIP, std::string("batch reset launch: ") + hipGetErrorString(e));
    if (b->n_tasks == 0) return AC_OK;
    acm::dfa::BatchArgs args{};
    args.text = text;
    args.items = b->d_items;
    args.tasks = b->d_tasks;
    args.n_tasks = b->n_tasks;
    args.autos = b->d_autos;
    args.out = out;
    args.cap = cap;
    args.count = reinterpret_cast<unsigned long long *>(count);
    args.next_task = b->d_next;
    const int rc = acm::launch_kernel(b->kernel, b->grid, b->block, b->lds, s, args, err);
    return rc == AC_OK ? AC_OK : set_error(rc, err);
}

}  // namespace

extern "C" {

int ac_batch_create(const ac_automaton *const *autos, uint32_t n_autos, const uint64_t *text_off,
                    const uint64_t *text_len, const uint32_t *text_auto, uint32_t n_texts,
                    const ac_batch_tune *tune, void *stream, ac_batch **out) {
    if (!out) return set_error(AC_ERR_INVALID, "ac_batch_create: out is NULL");
    *out = nullptr;
    if (!autos || n_autos == 0) return set_error(AC_ERR_INVALID, "ac_batch_create: no automata");
    if (n_texts > 0 && (!text_off || !text_len || !text_auto))
        return set_error(AC_ERR_INVALID, "ac_batch_create: NULL text arrays");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(AC_ERR_HIP, "ac_batch_create: hipGetDevice failed");
    bool all_images = true;
    for (uint32_t i = 0; i < n_autos; ++i) {
        const ac_automaton *a = autos[i];
        if (!a || !a->on_device || a->device != dev || a->m.goto_only)
            return set_error(AC_ERR_INVALID, "ac_batch_create: automaton " + std::to_string(i) +
                                                 " is NULL, host-only, goto-only or on another device");
        if (a->m.hashed != autos[0]->m.hashed ||
            (a->m.hashed && a->m.log2_cols != autos[0]->m.log2_cols))
            return set_error(AC_ERR_INVALID,
                             "ac_batch_create: automata must share one byte-class scheme (same "
                             "alphabet layout); split the batch by alphabet");
        all_images &= a->m.hot_states > 0;
    }
    const uint32_t want_place = tune ? tune->placement : AC_PLACE_AUTO;
    uint32_t place = want_place == AC_PLACE_AUTO ? (all_images ? AC_PLACE_LDS_HOT : AC_PLACE_GLOBAL) : want_place;
    if (place != AC_PLACE_LDS_HOT && place != AC_PLACE_GLOBAL)
        return set_error(AC_ERR_INVALID, "ac_batch_create: placement must be AUTO, GLOBAL or LDS_HOT");
    if (place == AC_PLACE_LDS_HOT && !all_images)
        return set_error(AC_ERR_INVALID, "ac_batch_create: LDS_HOT needs every automaton built with an "
                                         "LDS image (ac_build with AC_PLACE_LDS_HOT)");
    const uint32_t K = tune && tune->walkers ? tune->walkers : (place == AC_PLACE_LDS_HOT ? 2u : 1u);
    if (K < 1 || K > 4) return set_error(AC_ERR_INVALID, "ac_batch_create: walkers must be 1, 2, 3 or 4");
    const uint32_t bb = K >= 3 ? 64u : 128u;
    const bool hashed = autos[0]->m.hashed;
    const int l2 = hashed ? int(autos[0]->m.log2_cols) : -1;

    ac_batch *b = new (std::nothrow) ac_batch();
    if (!b) return set_error(AC_ERR_NOMEM, "ac_batch_create: out of host memory");
    b->device = dev;
    b->placement = place;
    b->walkers = K;
    b->block_bytes = bb;
    b->n_texts = n_texts;
    b->n_autos = n_autos;
    b->kernel = place == AC_PLACE_LDS_HOT ? acm::dfa::select_batch_hot(hashed, l2, K, bb)
                                          : acm::dfa::select_batch_global(hashed, l2, K, bb);
    b->block = place == AC_PLACE_LDS_HOT ? (K == 4 ? 768u : 1024u) : 256u;
    if (!b->kernel) {
        delete b;
        return set_error(AC_ERR_INVALID, "ac_batch_create: no batch kernel for this class scheme");
    }
    uint32_t image = 0;
    if (place == AC_PLACE_LDS_HOT)
        for (uint32_t i = 0; i < n_autos; ++i)
            image = std::max<uint32_t>(image, ((autos[i]->m.hot_states * autos[i]->m.n_cols * 2u) + 15u) & ~15u);
    b->lds = (b->block / 64) * acm::kQueueBytesPerWave + 256 + image;
    if (b->lds > acm::kLdsPerWorkgroup) {
        delete b;
        return set_error(AC_ERR_INVALID, "ac_batch_create: an LDS image does not fit beside the match queues");
    }
    if (acm::allow_lds(reinterpret_cast<const void *>(b->kernel), b->lds) != hipSuccess) {
        delete b;
        return set_error(AC_ERR_HIP, "ac_batch_create: hipFuncSetAttribute failed");
    }
    const int occ = acm::occupancy(reinterpret_cast<const void *>(b->kernel), b->block, b->lds);
    const uint64_t grid_max = uint64_t(acm::compute_units(dev)) * uint64_t(occ);

    // texts: validate, total bytes, then order by automaton (stable)
    uint64_t total = 0;
    uint32_t m_max = 1;
    for (uint32_t i = 0; i < n_autos; ++i) m_max = std::max(m_max, autos[i]->m.m_max);
    for (uint32_t t = 0; t < n_texts; ++t) {
        if (text_auto[t] >= n_autos) {
            delete b;
            return set_error(AC_ERR_INVALID, "ac_batch_create: text " + std::to_string(t) + " names automaton " +
                                                 std::to_string(text_auto[t]) + " of " + std::to_string(n_autos));
        }
        if (text_len[t] && (text_off[t] & 15u)) {
            delete b;
            return set_error(AC_ERR_INVALID, "ac_batch_create: text offsets must be multiples of 16");
        }
        if (text_off[t] + text_len[t] >= (1ull << 32) || text_len[t] >= (1ull << 32)) {
            delete b;
            return set_error(AC_ERR_TOO_LARGE, "ac_batch_create: the batch buffer must stay below 2^32 bytes");
        }
        total += text_len[t];
    }
    b->text_bytes = total;
    uint64_t chunk = tune && tune->chunk ? tune->chunk : 0;
    if (chunk == 0) {
        // about kRounds tasks per workgroup slot, so the dynamic hand-out can
        // even out automata of different cost per byte
        constexpr uint64_t kRounds = 4;
        const uint64_t walkers = grid_max * b->block * K * kRounds;
        chunk = std::max<uint64_t>(1, (total + walkers - 1) / walkers);
        chunk = std::max<uint64_t>(chunk, 4ull * m_max);
    }
    chunk = std::max<uint64_t>(bb, (chunk + bb - 1) & ~uint64_t(bb - 1));
    if (chunk > (1u << 30)) chunk = 1u << 30;
    b->chunk = uint32_t(chunk);
    std::vector<uint32_t> order(n_texts);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return text_auto[x] < text_auto[y]; });
    std::vector<acm::dfa::BatchItem> items;
    std::vector<uint32_t> item_auto;
    try {
        for (uint32_t t : order) {
            const uint64_t lo = text_off[t], hi = text_off[t] + text_len[t];
            for (uint64_t p = lo; p < hi; p += chunk) {
                items.push_back({uint32_t(p), uint32_t(std::min(hi, p + chunk)), uint32_t(lo), 0u});
                item_auto.push_back(text_auto[t]);
            }
        }
    } catch (const std::bad_alloc &) {
        delete b;
        return set_error(AC_ERR_NOMEM, "ac_batch_create: out of host memory");
    }
    b->n_items = uint32_t(items.size());
    // tasks: runs of at most one item per walker (block x walkers), all of one
    // automaton
    const uint64_t per_task = uint64_t(b->block) * K;
    std::vector<acm::dfa::BatchTask> tasks;
    for (size_t i = 0; i < items.size();) {
        size_t j = i;
        while (j < items.size() && item_auto[j] == item_auto[i] && j - i < per_task) ++j;
        tasks.push_back({uint32_t(i), uint32_t(j), item_auto[i], 0u});
        i = j;
    }
    b->n_tasks = uint32_t(tasks.size());
    b->grid = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(grid_max, tasks.size())));
    std::vector<acm::dfa::DfaArgs> dargs(n_autos);
    for (uint32_t i = 0; i < n_autos; ++i) acm::dfa::fill_machine_args(autos[i]->dm, dargs[i]);

    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc;
    const std::vector<uint32_t> next(1, 0u);
    if ((rc = upload(items, &b->d_items, s)) || (rc = upload(tasks, &b->d_tasks, s)) ||
        (rc = upload(dargs, &b->d_autos, s)) || (rc = upload(next, &b->d_next, s))) {
        (void)hipStreamSynchronize(s);
        release(b);
        delete b;
        return rc;
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        release(b);
        delete b;
        return set_error(AC_ERR_HIP, std::string("ac_batch_create: ") + hipGetErrorString(e));
    }
    *out = b;
    return AC_OK;
}

int ac_batch_info(const ac_batch *b, ac_batch_info_t *info) {
    if (!b || !info) return set_error(AC_ERR_INVALID, "ac_batch_info: NULL argument");
    info->placement = b->placement;
    info->walkers = b->walkers;
    info->block_bytes = b->block_bytes;
    info->chunk = b->chunk;
    info->threads = b->block;
    info->grid = b->grid;
    info->n_items = b->n_items;
    info->n_tasks = b->n_tasks;
    info->text_bytes = b->text_bytes;
    return AC_OK;
}

int ac_batch_scan(ac_batch *b, const uint8_t *d_texts, uint64_t *d_matches, uint64_t capacity,
                  uint64_t *d_count, int use_graph, void *stream) {
    if (!b || !d_count) return set_error(AC_ERR_INVALID, "ac_batch_scan: NULL batch or count");
    if (b->n_items && !d_texts) return set_error(AC_ERR_INVALID, "ac_batch_scan: NULL texts");
    if (capacity && !d_matches) return set_error(AC_ERR_INVALID, "ac_batch_scan: NULL match buffer");
    if (reinterpret_cast<uintptr_t>(d_texts) & 15u)
        return set_error(AC_ERR_INVALID, "ac_batch_scan: the batch buffer must be 16-byte aligned");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return set_error(AC_ERR_INVALID, "ac_batch_scan: batch planned for another device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!use_graph) return launch(b, d_texts, d_matches, capacity, d_count, s);
    if (!b->exec || b->g_text != d_texts || b->g_out != d_matches || b->g_cap != capacity ||
        b->g_count != d_count) {
        // an earlier replay of the old graph may still run on the stream
        if (b->exec) (void)hipStreamSynchronize(s);
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        hipError_t e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return set_error(AC_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
        const int rc = launch(b, d_texts, d_matches, capacity, d_count, b->capture);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->capture, &g);
        if (rc != AC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return set_error(AC_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        b->graph = g;
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            b->exec = nullptr;
            return set_error(AC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        b->g_text = d_texts;
        b->g_out = d_matches;
        b->g_cap = capacity;
        b->g_count = d_count;
    }
    hipError_t e = hipGraphLaunch(b->exec, s);
    return e == hipSuccess ? AC_OK : set_error(AC_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
}

void ac_batch_free(ac_batch *b) {
    if (!b) return;
    release(b);
    delete b;
}

int ac_scan_batch(const ac_automaton *const *autos, uint32_t n_autos, const uint8_t *d_texts,
                  const uint64_t *text_off, const uint32_t *text_auto, uint32_t n_texts, uint64_t *d_matches,
                  uint64_t capacity, uint64_t *d_count, const ac_batch_tune *tune, void *stream) {
    if (n_texts > 0 && !text_off) return set_error(AC_ERR_INVALID, "ac_scan_batch: NULL text offsets");
    std::vector<uint64_t> off, len;
    try {
        off.resize(n_texts);
        len.resize(n_texts);
    } catch (const std::bad_alloc &) {
        return set_error(AC_ERR_NOMEM, "ac_scan_batch: out of host memory");
    }
    for (uint32_t t = 0; t < n_texts; ++t) {
        if (text_off[t + 1] < text_off[t]) return set_error(AC_ERR_INVALID, "ac_scan_batch: decreasing text offsets");
        off[t] = text_off[t];
        len[t] = text_off[t + 1] - text_off[t];
    }
    ac_batch *b = nullptr;
    int rc = ac_batch_create(autos, n_autos, off.data(), len.data(), text_auto, n_texts, tune, stream, &b);
    if (rc != AC_OK) return rc;
    rc = ac_batch_scan(b, d_texts, d_matches, capacity, d_count, 0, stream);
    // the plan's device arrays must outlive the launch
    const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    ac_batch_free(b);
    if (rc != AC_OK) return rc;
    return e == hipSuccess ? AC_OK : set_error(AC_ERR_HIP, std::string("ac_scan_batch: ") + hipGetErrorString(e));
}

}  // extern "C"
