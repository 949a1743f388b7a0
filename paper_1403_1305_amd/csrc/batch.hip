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

#include <memory>
#include <mutex>

#include "automaton.h"
#include "dfa_kernel.h"

struct ac_batch {
    int device = -1;
    bool gated = false;  // the gated plan (tasks of tiles) rather than the DFA's items
    acm::GateTask *d_gtasks = nullptr;
    bool gate_dense = false;  // some automaton stages its matches in registers
    void *d_gautos = nullptr;  // per automaton: the gated scan's argument block
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
    if (b->d_gtasks) (void)hipFree(b->d_gtasks);
    if (b->d_gautos) (void)hipFree(b->d_gautos);
    b->d_gtasks = nullptr;
    b->d_gautos = nullptr;
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
    if (b->gated) {
        const int rc = acm::launch_gate_batch(text, b->d_gtasks, b->n_tasks, b->d_gautos, out, cap, count, b->d_next,
                                              b->grid, b->gate_dense, s, err);
        return rc == AC_OK ? AC_OK : set_error(rc, err);
    }
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

// ------------------------------------------------------------ one-shot batches
// ac_scan_batch and ac_scan_batch_noalloc take the texts' offsets and
// automata in device memory, so the work items are planned on the device, in
// a scratch buffer: a one-workgroup kernel validates the texts, picks the
// chunk length from their total, counts each automaton's items and tasks and
// gives every text its run of items (texts of one automaton in one block of
// items); a kernel with a workgroup per text then writes its items; then the
// persistent batch kernel runs the tasks, reading their count from the
// scratch. The chunk is chosen so that the items never outnumber
// kPlanMaxItems.

// The scratch header (64 bytes).
struct PlanHeader {
    uint32_t n_tasks;    // tasks of the plan (0 when the texts were rejected)
    uint32_t next_task;  // the persistent launch's task counter
    uint32_t error;      // kPlan* code
    uint32_t n_items;
    uint32_t chunk;
    uint32_t pad[11];
};
static_assert(sizeof(PlanHeader) == 64, "plan header");
enum : uint32_t { kPlanOk = 0, kPlanBadOffsets = 1, kPlanMisaligned = 2, kPlanBadAutomaton = 3, kPlanTooLarge = 4 };

constexpr uint32_t kPlanMaxItems = 1u << 20;
constexpr uint32_t kPlanMaxTexts = kPlanMaxItems / 2;  // each text may end in a partial item
constexpr uint32_t kBatchMaxAutos = 256;
constexpr uint32_t kPlanThreads = 1024;

// Byte offsets of the scratch parts for n_texts texts.
struct PlanLayout {
    size_t autos = 0, text_item = 0, tasks = 0, items = 0, bytes = 0;
    uint32_t max_tasks = 0;
};
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr PlanLayout plan_layout(uint32_t n_texts) {
    PlanLayout l{};
    l.autos = align256(sizeof(PlanHeader));
    l.text_item = l.autos + align256(size_t(kBatchMaxAutos) * sizeof(acm::dfa::DfaArgs));
    // a task holds at least 256 items (one per walker), each automaton ends one
    l.max_tasks = kPlanMaxItems / 256 + kBatchMaxAutos + 1;
    l.tasks = l.text_item + align256(size_t(n_texts) * 4);
    l.items = l.tasks + align256(size_t(l.max_tasks) * sizeof(acm::dfa::BatchTask));
    l.bytes = l.items + size_t(kPlanMaxItems) * sizeof(acm::dfa::BatchItem);
    return l;
}

struct PlanParams {
    const uint64_t *text_off;   // n_texts + 1 offsets into the batch buffer
    const uint32_t *text_auto;  // n_texts automaton indices
    uint32_t n_texts, n_autos, m_max, block_bytes, per_task;
    uint64_t walkers;           // walkers of the persistent launch (chunk choice)
    uint32_t tune_chunk;        // 0 = chosen from the total
    PlanHeader *hdr;
    uint32_t *text_item;        // first item of each text
    acm::dfa::BatchTask *tasks;
    unsigned long long *count;  // the caller's match count, zeroed here
};

__global__ void __launch_bounds__(kPlanThreads) batch_plan_kernel(PlanParams p) {
    __shared__ unsigned long long s_total;
    __shared__ uint32_t s_err;
    __shared__ uint32_t s_items[kBatchMaxAutos], s_cursor[kBatchMaxAutos];
    __shared__ uint32_t s_task_base[kBatchMaxAutos + 1], s_item_base[kBatchMaxAutos + 1];
    const uint32_t tid = threadIdx.x;
    if (tid == 0) {
        s_total = 0;
        s_err = kPlanOk;
        *p.count = 0;
    }
    for (uint32_t a = tid; a < kBatchMaxAutos; a += kPlanThreads) s_items[a] = 0;
    __syncthreads();
    // every text: non-decreasing offsets, 16-byte aligned starts, an automaton
    // of the batch, a buffer below 2^32 bytes
    unsigned long long local = 0;
    uint32_t err = kPlanOk;
    for (uint32_t t = tid; t < p.n_texts; t += kPlanThreads) {
        const uint64_t lo = p.text_off[t], hi = p.text_off[t + 1];
        if (hi < lo) {
            err = kPlanBadOffsets;
            continue;
        }
        if (hi > lo && (lo & 15u)) err = kPlanMisaligned;
        if (p.text_auto[t] >= p.n_autos) err = kPlanBadAutomaton;
        if (hi >= (1ull << 32)) err = kPlanTooLarge;
        local += hi - lo;
    }
    atomicAdd(&s_total, local);
    if (err) atomicMax(&s_err, err);
    __syncthreads();
    if (s_err) {
        if (tid == 0) {
            p.hdr->error = s_err;
            p.hdr->n_tasks = 0;
            p.hdr->n_items = 0;
        }
        return;
    }
    // chunk: about four walks per walker of the launch, at least 4 m_max, in
    // whole text blocks, and few enough items for the scratch
    const uint64_t total = s_total, bb = p.block_bytes;
    uint64_t c = p.tune_chunk ? p.tune_chunk
                              : max((total + p.walkers * 4 - 1) / (p.walkers * 4), 4ull * p.m_max);
    c = max(bb, (c + bb - 1) / bb * bb);
    const uint64_t room = kPlanMaxItems - p.n_texts;  // each text may end in a partial item
    if (total / c > room) c = ((total + room - 1) / room + bb - 1) / bb * bb;
    c = min<uint64_t>(c, 1u << 30);
    for (uint32_t t = tid; t < p.n_texts; t += kPlanThreads) {
        const uint64_t len = p.text_off[t + 1] - p.text_off[t];
        atomicAdd(&s_items[p.text_auto[t]], uint32_t((len + c - 1) / c));
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t base = 0, tbase = 0;
        for (uint32_t a = 0; a < p.n_autos; ++a) {
            s_item_base[a] = base;
            s_cursor[a] = base;
            s_task_base[a] = tbase;
            base += s_items[a];
            tbase += (s_items[a] + p.per_task - 1) / p.per_task;
        }
        s_item_base[p.n_autos] = base;
        s_task_base[p.n_autos] = tbase;
        p.hdr->n_items = base;
        p.hdr->n_tasks = tbase;
        p.hdr->chunk = uint32_t(c);
        p.hdr->next_task = 0;
        p.hdr->error = kPlanOk;
    }
    __syncthreads();
    // tasks: runs of at most per_task items of one automaton
    for (uint32_t k = tid; k < s_task_base[p.n_autos]; k += kPlanThreads) {
        uint32_t a = 0;
        while (s_task_base[a + 1] <= k) ++a;
        const uint32_t b = s_item_base[a] + (k - s_task_base[a]) * p.per_task;
        p.tasks[k] = acm::dfa::BatchTask{b, min(b + p.per_task, s_item_base[a + 1]), a, 0u};
    }
    // each text's run of items within its automaton's block (any order)
    for (uint32_t t = tid; t < p.n_texts; t += kPlanThreads) {
        const uint64_t len = p.text_off[t + 1] - p.text_off[t];
        p.text_item[t] = atomicAdd(&s_cursor[p.text_auto[t]], uint32_t((len + c - 1) / c));
    }
}

// The items of text blockIdx.x.
__global__ void __launch_bounds__(256) batch_fill_kernel(const uint64_t *text_off, const PlanHeader *hdr,
                                                         const uint32_t *text_item, acm::dfa::BatchItem *items) {
    if (hdr->error) return;
    const uint32_t t = blockIdx.x;
    const uint64_t lo = text_off[t], hi = text_off[t + 1], c = hdr->chunk;
    const uint32_t first = text_item[t], n = uint32_t((hi - lo + c - 1) / c);
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
        const uint64_t b = lo + uint64_t(j) * c;
        items[first + j] = acm::dfa::BatchItem{uint32_t(b), uint32_t(min(hi, b + c)), uint32_t(lo), t};
    }
}

// The text of each match: the last text whose offset is at or before the
// match's end position.
__global__ void match_text_kernel(const uint64_t *keys, const unsigned long long *count, uint64_t cap,
                                  const uint64_t *text_off, uint32_t n_texts, uint32_t *match_text) {
    const uint64_t n = min(uint64_t(*count), cap);
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t pos = keys[i] >> 32;
        uint32_t lo = 0, hi = n_texts;  // largest t with text_off[t] <= pos lies in [lo, hi)
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (text_off[mid] <= pos)
                lo = mid;
            else
                hi = mid;
        }
        match_text[i] = lo;
    }
}

// Everything of a one-shot batch that does not depend on the texts: the
// kernel, its shape and the automata's arguments (host side).
struct OneShot {
    acm::dfa::BatchKernel kernel = nullptr;
    uint32_t block = 0, lds = 0, grid = 0, walkers_per_lane = 1, bb = 128, m_max = 1;
    acm::dfa::DfaArgs args[kBatchMaxAutos];
};

int prepare_one_shot(const char *fn, const ac_automaton *const *autos, uint32_t n_autos,
                     const ac_batch_tune *tune, OneShot &o) {
    auto f = [fn] { return std::string(fn); };  // built only for an error message
    if (!autos || n_autos == 0 || n_autos > kBatchMaxAutos)
        return set_error(AC_ERR_INVALID, f() + ": need 1 to 256 automata");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(AC_ERR_HIP, f() + ": hipGetDevice failed");
    bool all_images = true;
    for (uint32_t i = 0; i < n_autos; ++i) {
        const ac_automaton *a = autos[i];
        if (!a || !a->on_device || a->device != dev || a->m.goto_only)
            return set_error(AC_ERR_INVALID, f() + ": automaton " + std::to_string(i) +
                                                 " is NULL, host-only, goto-only or on another device");
        if (a->m.hashed != autos[0]->m.hashed || (a->m.hashed && a->m.log2_cols != autos[0]->m.log2_cols))
            return set_error(AC_ERR_INVALID, f() + ": automata must share one byte-class scheme");
        all_images &= a->m.hot_states > 0;
        o.m_max = std::max(o.m_max, a->m.m_max);
        o.args[i] = acm::dfa::DfaArgs{};
        acm::dfa::fill_machine_args(a->dm, o.args[i]);
    }
    const uint32_t want = tune ? tune->placement : AC_PLACE_AUTO;
    const uint32_t place = want == AC_PLACE_AUTO ? (all_images ? AC_PLACE_LDS_HOT : AC_PLACE_GLOBAL) : want;
    if ((place != AC_PLACE_LDS_HOT && place != AC_PLACE_GLOBAL) || (place == AC_PLACE_LDS_HOT && !all_images))
        return set_error(AC_ERR_INVALID, f() + ": placement must be AUTO, GLOBAL, or LDS_HOT with an image in every automaton");
    const uint32_t K = tune && tune->walkers ? tune->walkers : (place == AC_PLACE_LDS_HOT ? 2u : 1u);
    if (K < 1 || K > 4) return set_error(AC_ERR_INVALID, f() + ": walkers must be 1, 2, 3 or 4");
    if (tune && tune->chunk % 16) return set_error(AC_ERR_INVALID, f() + ": chunk must be a multiple of 16");
    if (tune && tune->algo != AC_ALGO_AUTO && tune->algo != AC_ALGO_DFA)
        return set_error(AC_ERR_INVALID, f() + ": the one-shot batch scans with the DFA (algo AUTO or DFA)");
    o.walkers_per_lane = K;
    o.bb = K >= 3 ? 64u : 128u;
    const bool hashed = autos[0]->m.hashed;
    const int l2 = hashed ? int(autos[0]->m.log2_cols) : -1;
    o.kernel = place == AC_PLACE_LDS_HOT ? acm::dfa::select_batch_hot(hashed, l2, K, o.bb)
                                         : acm::dfa::select_batch_global(hashed, l2, K, o.bb);
    if (!o.kernel) return set_error(AC_ERR_INVALID, f() + ": no batch kernel for this class scheme");
    o.block = place == AC_PLACE_LDS_HOT ? (K == 4 ? 768u : 1024u) : 256u;
    uint32_t image = 0;
    if (place == AC_PLACE_LDS_HOT)
        for (uint32_t i = 0; i < n_autos; ++i)
            image = std::max<uint32_t>(image, ((autos[i]->m.hot_states * autos[i]->m.n_cols * 2u) + 15u) & ~15u);
    o.lds = (o.block / 64) * acm::kQueueBytesPerWave + 256 + image;
    if (o.lds > acm::kLdsPerWorkgroup) return set_error(AC_ERR_INVALID, f() + ": an LDS image does not fit");
    if (acm::allow_lds(reinterpret_cast<const void *>(o.kernel), o.lds) != hipSuccess)
        return set_error(AC_ERR_HIP, f() + ": hipFuncSetAttribute failed");
    const int occ = acm::occupancy(reinterpret_cast<const void *>(o.kernel), o.block, o.lds);
    o.grid = uint32_t(std::max<int64_t>(1, int64_t(acm::compute_units(dev)) * occ));
    return AC_OK;
}

// Plan and scan a one-shot batch in `scratch` (at least plan_layout(n_texts)
// bytes of device memory), then wait for `stream` and report a rejected plan.
int run_one_shot(const char *fn, const OneShot &o, uint32_t n_autos, const uint8_t *d_texts, const uint64_t *d_text_off,
                 const uint32_t *d_text_auto, uint32_t n_texts, uint32_t *d_match_text, uint64_t *d_matches,
                 uint64_t capacity, uint64_t *d_count, const ac_batch_tune *tune, uint8_t *scratch, hipStream_t s) {
    auto f = [fn] { return std::string(fn); };  // built only for an error message
    const PlanLayout L = plan_layout(n_texts);
    PlanHeader *hdr = reinterpret_cast<PlanHeader *>(scratch);
    auto *d_autos = reinterpret_cast<acm::dfa::DfaArgs *>(scratch + L.autos);
    hipError_t e = hipMemcpyAsync(d_autos, o.args, size_t(n_autos) * sizeof(acm::dfa::DfaArgs), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return set_error(AC_ERR_HIP, f() + ": " + hipGetErrorString(e));
    PlanParams pp{};
    pp.text_off = d_text_off;
    pp.text_auto = d_text_auto;
    pp.n_texts = n_texts;
    pp.n_autos = n_autos;
    pp.m_max = o.m_max;
    pp.block_bytes = o.bb;
    pp.per_task = o.block * o.walkers_per_lane;
    pp.walkers = uint64_t(o.grid) * o.block * o.walkers_per_lane;
    pp.tune_chunk = tune ? tune->chunk : 0u;
    pp.hdr = hdr;
    pp.text_item = reinterpret_cast<uint32_t *>(scratch + L.text_item);
    pp.tasks = reinterpret_cast<acm::dfa::BatchTask *>(scratch + L.tasks);
    pp.count = reinterpret_cast<unsigned long long *>(d_count);
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, pp);
    auto *items = reinterpret_cast<acm::dfa::BatchItem *>(scratch + L.items);
    if (n_texts) hipLaunchKernelGGL(batch_fill_kernel, dim3(n_texts), dim3(256), 0, s, d_text_off, hdr, pp.text_item, items);
    e = hipGetLastError();
    if (e != hipSuccess) return set_error(AC_ERR_HIP, f() + ": plan launch: " + hipGetErrorString(e));
    acm::dfa::BatchArgs args{};
    args.text = d_texts;
    args.items = items;
    args.tasks = pp.tasks;
    args.n_tasks = 0;
    args.n_tasks_dev = &hdr->n_tasks;
    args.autos = d_autos;
    args.out = d_matches;
    args.cap = capacity;
    args.count = reinterpret_cast<unsigned long long *>(d_count);
    args.next_task = &hdr->next_task;
    hipError_t le = acm::allow_lds(reinterpret_cast<const void *>(o.kernel), o.lds);
    if (le == hipSuccess) {
        hipLaunchKernelGGL(o.kernel, dim3(o.grid), dim3(o.block), o.lds, s, args);
        le = hipGetLastError();
    }
    if (le != hipSuccess) return set_error(AC_ERR_HIP, f() + ": batch launch: " + hipGetErrorString(le));
    if (d_match_text && capacity) {
        hipLaunchKernelGGL(match_text_kernel, dim3(1024), dim3(256), 0, s, d_matches,
                           reinterpret_cast<const unsigned long long *>(d_count), capacity, d_text_off, n_texts,
                           d_match_text);
        e = hipGetLastError();
        if (e != hipSuccess) return set_error(AC_ERR_HIP, f() + ": match text launch: " + hipGetErrorString(e));
    }
    PlanHeader h{};
    e = hipMemcpyAsync(&h, hdr, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(AC_ERR_HIP, f() + ": " + hipGetErrorString(e));
    switch (h.error) {
        case kPlanOk: return AC_OK;
        case kPlanBadOffsets: return set_error(AC_ERR_INVALID, f() + ": decreasing text offsets");
        case kPlanMisaligned: return set_error(AC_ERR_INVALID, f() + ": text starts must be multiples of 16");
        case kPlanBadAutomaton: return set_error(AC_ERR_INVALID, f() + ": a text names an automaton past n_autos");
        default: return set_error(AC_ERR_TOO_LARGE, f() + ": the batch buffer must stay below 2^32 bytes");
    }
}

int check_one_shot_args(const char *fn, const uint8_t *d_texts, const uint64_t *d_text_off,
                        const uint32_t *d_text_auto, uint32_t n_texts, uint64_t *d_matches, uint64_t capacity,
                        uint64_t *d_count) {
    auto f = [fn] { return std::string(fn); };  // built only for an error message
    if (!d_count || !d_text_off) return set_error(AC_ERR_INVALID, f() + ": NULL count or text offsets");
    if (n_texts && (!d_texts || !d_text_auto)) return set_error(AC_ERR_INVALID, f() + ": NULL texts or automaton indices");
    if (capacity && !d_matches) return set_error(AC_ERR_INVALID, f() + ": NULL match buffer");
    if (reinterpret_cast<uintptr_t>(d_texts) & 15u) return set_error(AC_ERR_INVALID, f() + ": the batch buffer must be 16-byte aligned");
    return AC_OK;
}

// The no-allocation form's scratch: one array per GPU, for up to
// kNoAllocMaxTexts texts. Host code reaches it only through the address that
// hipGetSymbolAddress gives on each device.
constexpr uint32_t kNoAllocMaxTexts = 1u << 16;
constexpr size_t kNoAllocScratchBytes = plan_layout(kNoAllocMaxTexts).bytes;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[64] = {};

// This device's copy of `scratch` (looked up once per device, current).
int scratch_address(int dev, uint8_t **out) {
    if (dev < 0 || dev >= 64) return set_error(AC_ERR_INVALID, "ac_scan_batch_noalloc: device index past 63");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(AC_ERR_HIP, std::string("ac_scan_batch_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return AC_OK;
}

// The gated plan: every text cut into tasks of whole tiles (at most `per`
// tiles each), ordered by automaton; one per-automaton argument block.
int create_gated(const ac_automaton *const *autos, uint32_t n_autos, const uint64_t *text_off,
                 const uint64_t *text_len, const uint32_t *text_auto, uint32_t n_texts, const ac_batch_tune *tune,
                 void *stream, int dev, ac_batch **out) {
    const uint64_t tile = acm::gate_batch_tile_bytes();
    uint64_t total = 0, tiles = 0;
    for (uint32_t t = 0; t < n_texts; ++t) {
        if (text_auto[t] >= n_autos)
            return set_error(AC_ERR_INVALID, "ac_batch_create: text " + std::to_string(t) + " names automaton " +
                                                 std::to_string(text_auto[t]) + " of " + std::to_string(n_autos));
        if (text_len[t] && (text_off[t] & 15u))
            return set_error(AC_ERR_INVALID, "ac_batch_create: text offsets must be multiples of 16");
        if (text_off[t] + text_len[t] >= (1ull << 32) || text_len[t] >= (1ull << 32))
            return set_error(AC_ERR_TOO_LARGE, "ac_batch_create: the batch buffer must stay below 2^32 bytes");
        total += text_len[t];
        tiles += (text_len[t] + tile - 1) / tile;
    }
    const uint32_t grid_max = uint32_t(acm::compute_units(dev));  // one workgroup per CU (the bitmaps fill the LDS)
    uint64_t per = tune && tune->chunk ? (tune->chunk + tile - 1) / tile : 0;
    if (per == 0) {
        // about kRounds tasks per workgroup, so that the hand-out evens out
        // texts and automata of different cost
        constexpr uint64_t kRounds = 8;
        per = std::max<uint64_t>(16, (tiles + grid_max * kRounds - 1) / (grid_max * kRounds));
    }
    std::unique_ptr<ac_batch> b(new (std::nothrow) ac_batch());
    if (!b) return set_error(AC_ERR_NOMEM, "ac_batch_create: out of host memory");
    b->device = dev;
    b->gated = true;
    b->placement = 0;
    b->walkers = 0;
    b->block_bytes = 0;
    b->chunk = uint32_t(std::min<uint64_t>(per * tile, 1u << 30));
    b->block = 1024;
    b->n_texts = n_texts;
    b->n_autos = n_autos;
    b->text_bytes = total;
    std::vector<uint32_t> order(n_texts);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return text_auto[x] < text_auto[y]; });
    std::vector<acm::GateTask> tasks;
    std::vector<uint8_t> blob;
    try {
        for (uint32_t t : order) {
            const uint64_t nt = (text_len[t] + tile - 1) / tile;
            for (uint64_t t0 = 0; t0 < nt; t0 += per) {
                acm::GateTask g{};
                g.off = text_off[t];
                g.len = uint32_t(text_len[t]);
                g.pos_base = uint32_t(text_off[t]);  // end positions in the batch buffer
                g.t0 = uint32_t(t0);
                g.t1 = uint32_t(std::min(nt, t0 + per));
                g.automaton = text_auto[t];
                tasks.push_back(g);
            }
        }
        blob.resize(size_t(n_autos) * acm::gate_batch_auto_bytes());
    } catch (const std::bad_alloc &) {
        return set_error(AC_ERR_NOMEM, "ac_batch_create: out of host memory");
    }
    for (uint32_t i = 0; i < n_autos; ++i) {
        acm::fill_gate_batch_auto(autos[i]->dm, blob.data() + size_t(i) * acm::gate_batch_auto_bytes());
        b->gate_dense |= autos[i]->dm.dense;
    }
    b->n_items = b->n_tasks = uint32_t(tasks.size());
    b->grid = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(grid_max, tasks.size())));
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc;
    const std::vector<uint32_t> next(1, 0u);
    uint8_t *d_blob = nullptr;
    if ((rc = upload(tasks, &b->d_gtasks, s)) || (rc = upload(blob, &d_blob, s)) || (rc = upload(next, &b->d_next, s))) {
        b->d_gautos = d_blob;
        (void)hipStreamSynchronize(s);
        release(b.get());
        return rc;
    }
    b->d_gautos = d_blob;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        release(b.get());
        return set_error(AC_ERR_HIP, std::string("ac_batch_create: ") + hipGetErrorString(e));
    }
    *out = b.release();
    return AC_OK;
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
    const uint32_t algo = tune ? tune->algo : AC_ALGO_AUTO;
    if (algo != AC_ALGO_AUTO && algo != AC_ALGO_DFA && algo != AC_ALGO_GATED)
        return set_error(AC_ERR_INVALID, "ac_batch_create: algo must be AUTO, DFA or GATED");
    bool all_gates = true, all_auto_gated = true;
    for (uint32_t i = 0; i < n_autos; ++i) {
        all_gates &= autos[i]->dm.gate_bits != nullptr;
        all_auto_gated &= autos[i]->dm.gate_bits != nullptr && acm::auto_algo(autos[i]) == AC_ALGO_GATED;
    }
    if (algo == AC_ALGO_GATED && !all_gates)
        return set_error(AC_ERR_INVALID, "ac_batch_create: AC_ALGO_GATED needs the class gate in every automaton");
    if (algo == AC_ALGO_GATED || (algo == AC_ALGO_AUTO && all_auto_gated))
        return create_gated(autos, n_autos, text_off, text_len, text_auto, n_texts, tune, stream, dev, out);
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
    info->algo = b->gated ? AC_ALGO_GATED : AC_ALGO_DFA;
    info->pad = 0;
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
                  const uint64_t *d_text_off, const uint32_t *d_text_auto, uint32_t n_texts, uint32_t *d_match_text,
                  uint64_t *d_matches, uint64_t capacity, uint64_t *d_count, const ac_batch_tune *tune, void *stream) {
    static const char *fn = "ac_scan_batch";
    int rc = check_one_shot_args(fn, d_texts, d_text_off, d_text_auto, n_texts, d_matches, capacity, d_count);
    if (rc != AC_OK) return rc;
    if (n_texts > kPlanMaxTexts)
        return set_error(AC_ERR_TOO_LARGE, "ac_scan_batch: at most 2^19 texts (the plan holds 2^20 work items)");
    std::unique_ptr<OneShot> o(new (std::nothrow) OneShot());
    if (!o) return set_error(AC_ERR_NOMEM, "ac_scan_batch: out of host memory");
    if ((rc = prepare_one_shot(fn, autos, n_autos, tune, *o)) != AC_OK) return rc;
    void *scr = nullptr;
    hipError_t e = hipMalloc(&scr, plan_layout(n_texts).bytes);
    if (e != hipSuccess) return set_error(AC_ERR_NOMEM, std::string("ac_scan_batch: scratch: ") + hipGetErrorString(e));
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = run_one_shot(fn, *o, n_autos, d_texts, d_text_off, d_text_auto, n_texts, d_match_text, d_matches, capacity,
                      d_count, tune, static_cast<uint8_t *>(scr), s);
    // the plan in the scratch must outlive the launches
    (void)hipStreamSynchronize(s);
    (void)hipFree(scr);
    return rc;
}

int ac_scan_batch_noalloc(const ac_automaton *const *autos, uint32_t n_autos, const uint8_t *d_texts,
                          const uint64_t *d_text_off, const uint32_t *d_text_auto, uint32_t n_texts,
                          uint32_t *d_match_text, uint64_t *d_matches, uint64_t capacity, uint64_t *d_count,
                          const ac_batch_tune *tune, void *stream) {
    static const char *fn = "ac_scan_batch_noalloc";
    int rc = check_one_shot_args(fn, d_texts, d_text_off, d_text_auto, n_texts, d_matches, capacity, d_count);
    if (rc != AC_OK) return rc;
    if (n_texts > kNoAllocMaxTexts)
        return set_error(AC_ERR_TOO_LARGE, "ac_scan_batch_noalloc: at most 65536 texts (its scratch array is fixed)");
    // the host-side plan in static storage (no allocation); calls that
    // overlap on one GPU race on the scratch anyway, so they take turns here
    static OneShot o;
    static std::mutex mu;
    std::lock_guard<std::mutex> g(mu);
    if ((rc = prepare_one_shot(fn, autos, n_autos, tune, o)) != AC_OK) return rc;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(AC_ERR_HIP, "ac_scan_batch_noalloc: hipGetDevice failed");
    uint8_t *scr = nullptr;
    if ((rc = scratch_address(dev, &scr)) != AC_OK) return rc;
    return run_one_shot(fn, o, n_autos, d_texts, d_text_off, d_text_auto, n_texts, d_match_text, d_matches, capacity,
                        d_count, tune, scr, static_cast<hipStream_t>(stream));
}

}  // extern "C"
