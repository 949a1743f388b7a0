// device_common.h -- match compaction and launch helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <type_traits>
#include <utility>

#include "../../include/ac.h"

namespace acm {

// Rank of this lane among the set lanes of `mask` below it (mbcnt prefix).
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

// Per-wave match staging. Each wave owns kQueueKeys key slots and one count
// word of LDS; matches are appended with a ballot and an mbcnt rank, and a
// full queue is flushed to the global list with one atomic on the global
// counter and coalesced writes. Only the owning wave touches its slots, so no
// barrier is involved. The count lives in LDS (not in a register) because
// callers may run with only some lanes active.
constexpr uint32_t kQueueKeys = 64;
constexpr uint32_t kQueueBytesPerWave = kQueueKeys * 8 + 16;

struct Emitter {
    uint64_t *q;   // this wave's LDS key slots
    uint32_t *qn;  // this wave's LDS count word
    uint64_t *out;
    uint64_t cap;
    unsigned long long *count;

    // Point at the wave's region of `lds` (kQueueBytesPerWave per wave) and
    // clear its count. Call once per wave before any emit.
    __device__ __forceinline__ void init(uint8_t *lds, uint64_t *out_, uint64_t cap_,
                                         unsigned long long *count_) {
        const uint32_t wave = threadIdx.x / 64;
        q = reinterpret_cast<uint64_t *>(lds + wave * kQueueBytesPerWave);
        qn = reinterpret_cast<uint32_t *>(lds + wave * kQueueBytesPerWave + kQueueKeys * 8);
        out = out_;
        cap = cap_;
        count = count_;
        if (__lane_id() == 0) *qn = 0;
    }

    // Copy the n staged keys out with the active lanes.
    __device__ __forceinline__ void drain(uint32_t n) {
        const uint64_t act = __ballot(true);
        const uint32_t r = lane_rank(act), w = uint32_t(__popcll(act));
        unsigned long long base = 0;
        if (r == 0) base = atomicAdd(count, (unsigned long long)n);
        base = __shfl(base, __ffsll((unsigned long long)act) - 1);
        for (uint32_t i = r; i < n; i += w) {
            const uint64_t idx = base + i;
            if (idx < cap) out[idx] = q[i];
        }
    }

    // Append `key` for every active lane with `has`.
    __device__ __forceinline__ void emit(bool has, uint64_t key) {
        const uint64_t mask = __ballot(has);
        if (mask == 0) return;
        const uint32_t c = uint32_t(__popcll(mask));
        uint32_t n = *qn;
        if (n + c > kQueueKeys) {
            drain(n);
            n = 0;
        }
        if (has) q[n + lane_rank(mask)] = key;
        if (lane_rank(__ballot(true)) == 0) *qn = n + c;
    }

    // Flush what is staged (at the end of the kernel).
    __device__ __forceinline__ void flush() {
        const uint32_t n = *qn;
        if (n) drain(n);
        if (lane_rank(__ballot(true)) == 0) *qn = 0;
    }

    // flush() for every wave of the workgroup at once, with one atomic for all
    // of them (called by every thread, every wave having called init; s: LDS,
    // waves + 2 words): the waves' counts become offsets in s, and thread 0
    // reserves their total.
    __device__ __forceinline__ void flush_group(uint32_t *s) {
        const uint32_t lane = __lane_id(), wave = threadIdx.x / 64u, waves = blockDim.x / 64u;
        const uint32_t n = *qn;
        __syncthreads();  // s may alias memory the waves used until now
        if (lane == 0) s[wave] = n;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t total = 0;
            for (uint32_t w = 0; w < waves; ++w) {
                const uint32_t c = s[w];
                s[w] = total;
                total += c;
            }
            const unsigned long long base = total ? atomicAdd(count, (unsigned long long)total) : 0ull;
            s[waves] = uint32_t(base);
            s[waves + 1] = uint32_t(base >> 32);
        }
        __syncthreads();
        const uint64_t base = (uint64_t(s[waves + 1]) << 32 | s[waves]) + s[wave];
        for (uint32_t i = lane; i < n; i += 64u)
            if (base + i < cap) out[base + i] = q[i];
        if (lane == 0) *qn = 0;
        __syncthreads();  // s may be reused
    }
};

// Per-wave match staging in registers, for kernels that call emit with every
// lane of the wave active: lane l holds queue entries l, l + 64, ..., K of
// them, so a wave reserves room in the global list (one atomic on its
// counter, the step whose cost grows with the number of flushes, as every
// workgroup of the grid updates the same word) once per up to 64 K matches.
// A call moves the new keys to their queue lanes with one forward permute
// (a bijection: the keys to lanes n .. n + c - 1, the other lanes' values to
// the rest).
template <uint32_t K>
struct RegEmitter {
    // The low and high words of the lane's entries. They are updated with
    // byte permutes: a select written as one, over j, would be turned into a
    // store at a computed index, which puts the arrays in scratch memory.
    uint32_t lo_[K], hi_[K];
    uint32_t n;  // queued keys (the same in every lane)
    uint64_t *out;
    uint64_t cap;
    unsigned long long *count;

    __device__ __forceinline__ void init(uint64_t *out_, uint64_t cap_, unsigned long long *count_) {
        n = 0;
        out = out_;
        cap = cap_;
        count = count_;
#pragma unroll
        for (uint32_t j = 0; j < K; ++j) lo_[j] = hi_[j] = 0;
    }

    // Write the queued keys to the list and empty the queue.
    __device__ __forceinline__ void flush() {
        if (n == 0) return;
        const uint32_t lane = __lane_id();
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(count, (unsigned long long)n);
        base = (unsigned long long)__builtin_amdgcn_readfirstlane(uint32_t(base)) |
               (unsigned long long)__builtin_amdgcn_readfirstlane(uint32_t(base >> 32)) << 32;
#pragma unroll
        for (uint32_t j = 0; j < K; ++j) {
            const uint32_t e = j * 64u + lane;
            if (e < n && base + e < cap) out[base + e] = uint64_t(hi_[j]) << 32 | lo_[j];
        }
        n = 0;
    }

    // flush() for every wave of the workgroup at once, with one atomic for all
    // of them (called by every thread; s: LDS, waves + 2 words): the waves'
    // counts become offsets in s, and thread 0 reserves their total.
    __device__ __forceinline__ void flush_group(uint32_t *s) {
        const uint32_t lane = __lane_id(), wave = threadIdx.x / 64u, waves = blockDim.x / 64u;
        __syncthreads();  // s may alias memory the waves used until now
        if (lane == 0) s[wave] = n;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t total = 0;
            for (uint32_t w = 0; w < waves; ++w) {
                const uint32_t c = s[w];
                s[w] = total;
                total += c;
            }
            const unsigned long long base = total ? atomicAdd(count, (unsigned long long)total) : 0ull;
            s[waves] = uint32_t(base);
            s[waves + 1] = uint32_t(base >> 32);
        }
        __syncthreads();
        const uint64_t base = (uint64_t(s[waves + 1]) << 32 | s[waves]) + s[wave];
#pragma unroll
        for (uint32_t j = 0; j < K; ++j) {
            const uint32_t e = j * 64u + lane;
            if (e < n && base + e < cap) out[base + e] = uint64_t(hi_[j]) << 32 | lo_[j];
        }
        n = 0;
        __syncthreads();  // s may be reused
    }

    // Append `key` for every lane with `has`.
    __device__ __forceinline__ void emit(bool has, uint64_t key) {
        const uint64_t mask = __ballot(has);
        if (mask == 0) return;
        const uint32_t c = uint32_t(__popcll(mask));
        if (n + c > 64u * K) flush();
        const uint32_t lane = __lane_id();
        const uint32_t r = has ? lane_rank(mask) : c + lane_rank(~mask);
        const int to = int(((n + r) & 63u) << 2);
        const uint32_t lo = uint32_t(__builtin_amdgcn_ds_permute(to, int(uint32_t(key))));
        const uint32_t hi = uint32_t(__builtin_amdgcn_ds_permute(to, int(uint32_t(key >> 32))));
        // this lane received entry n + k when k < c
        const uint32_t k = (lane - n) & 63u;
        // its slot: (n + k) >> 6, or none (K) for a lane that received no key
        const uint32_t s = k < c ? (n + k) >> 6 : K;
#pragma unroll
        for (uint32_t j = 0; j < K; ++j) {
            // perm(x, y, 0x07060504) is x, perm(x, y, 0x03020100) is y
            const uint32_t sel = s == j ? 0x07060504u : 0x03020100u;
            lo_[j] = __builtin_amdgcn_perm(lo, lo_[j], sel);
            hi_[j] = __builtin_amdgcn_perm(hi, hi_[j], sel);
        }
        n += c;
    }
};

// Workgroup LDS an emitter type needs (for `waves` wavefronts), and its set-up.
template <class Em>
struct EmitterLds {
    static constexpr uint32_t bytes(uint32_t) { return 16; }
};
template <>
struct EmitterLds<Emitter> {
    static constexpr uint32_t bytes(uint32_t waves) { return waves * kQueueBytesPerWave; }
};
__device__ __forceinline__ void init_emitter(Emitter &em, uint8_t *lds, uint64_t *out, uint64_t cap,
                                             unsigned long long *count) {
    em.init(lds, out, cap, count);
}
template <uint32_t K>
__device__ __forceinline__ void init_emitter(RegEmitter<K> &em, uint8_t *, uint64_t *out, uint64_t cap,
                                             unsigned long long *count) {
    em.init(out, cap, count);
}

// f(integral_constant<K>) for K = 0, 1, ... while it returns true: a loop
// unrolled whatever the size of its body.
template <class F, uint32_t... K>
__device__ __forceinline__ bool for_each_while(F &&f, std::integer_sequence<uint32_t, K...>) {
    return (f(std::integral_constant<uint32_t, K>{}) && ...);
}

// Every pattern id of the set ids[off[s] .. off[s+1]) as a match ending at pos.
template <class Em>
__device__ __forceinline__ void emit_set(Em &em, bool has, uint32_t s, uint64_t pos,
                                         const uint32_t *off, const uint32_t *ids) {
    uint32_t k = 0, kend = 0;
    if (has) {
        k = off[s];
        kend = off[s + 1];
    }
    while (__any(k < kend)) {
        const bool h = k < kend;
        const uint32_t id = h ? ids[k] : 0u;
        em.emit(h, (pos << 32) | id);
        k += h ? 1u : 0u;
    }
}

// A launch that reports its own completion (the served form): the last
// workgroup to finish writes the match total and the run's sequence number to
// a completion word in host memory (total, then the sequence with release
// order at system scope) and clears the count and the finish counter for the
// next launch on the same stream. finished == NULL: no completion word.
struct Completion {
    unsigned int *finished;  // device: workgroups done so far (0 before the launch)
    uint64_t *word;          // host-visible: {total, sequence}
    uint64_t seq;
};

// Called by every thread of every workgroup at the end of the kernel, after
// its last match is written.
__device__ __forceinline__ void complete_launch(const Completion &c, unsigned long long *count) {
    if (!c.finished) return;
    __syncthreads();
    if (threadIdx.x != 0) return;
    __threadfence();  // this workgroup's matches and count updates first
    if (atomicAdd(c.finished, 1u) != gridDim.x - 1) return;
    __threadfence();  // every other workgroup's, seen through the counter
    const uint64_t total = __hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(count, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(c.finished, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(c.word, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(c.word + 1, c.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

inline int hip_fail(hipError_t e, const char *what, std::string &err) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return AC_ERR_HIP;
}

// Raise `kernel`'s dynamic-LDS limit to at least `lds` bytes on the current
// device (a no-op up to 64 KiB, and once granted; defined in scan.hip).
hipError_t allow_lds(const void *kernel, uint32_t lds);
// Workgroups of `block` threads and `lds` bytes that one CU holds at once
// (at least 1), cached per device, kernel and shape.
int occupancy(const void *kernel, uint32_t block, uint32_t lds);

// Launch with `lds` bytes of dynamic LDS and report launch errors.
template <typename K, typename A>
int launch_kernel(K kernel, uint32_t grid, uint32_t block, uint32_t lds, hipStream_t stream,
                  const A &args, std::string &err) {
    hipError_t le = allow_lds(reinterpret_cast<const void *>(kernel), lds);
    if (le != hipSuccess) return hip_fail(le, "hipFuncSetAttribute", err);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, stream, args);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch", err);
    return AC_OK;
}

}  // namespace acm
