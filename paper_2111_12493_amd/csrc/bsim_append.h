// bsim_append.h -- appends to a global list whose counter many waves share.
//
// A device-scope atomic on one address is serialized across the whole
// chip, so a list that every wave appends to with its own atomic (one per
// 64 candidates) spends most of its time on the counter once it holds
// millions of entries.  Both helpers here reserve space for many entries
// with one atomic:
//   - block_reserve: kernels whose blocks step through their items
//     together (one item per thread per step): one atomic per block step;
//   - WaveAppender: kernels whose waves take items on their own (grid-stride
//     over waves): each wave gathers entries in its own LDS buffer and
//     writes them out with one atomic per kAppendBuf - 63 entries.
// List order is not kept; the lists here are sets.
#pragma once

#include "bsim_device.h"

namespace bsim {

constexpr uint32_t kAppendBuf = 512;  // entries of a wave's LDS buffer

// Memory order among the lanes of one wave (LDS written by some lanes, read
// by others).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The list position of every taking thread's entry, reserved with one
// atomic per block.  Every thread of the block calls it (it synchronizes
// the block); s_wave needs kBlock / 64 + 1 entries.  Threads that do not
// take get ~0u.
__device__ __forceinline__ uint32_t block_reserve(bool take, uint32_t* count, uint32_t* s_wave) {
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
    const uint64_t b = __ballot(take);
    if (lane == 0) s_wave[wid] = static_cast<uint32_t>(__popcll(b));
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t w = 0; w < kBlock / 64; w++) {
            const uint32_t c = s_wave[w];
            s_wave[w] = run;
            run += c;
        }
        s_wave[kBlock / 64] = run ? atomicAdd(count, run) : 0u;
    }
    __syncthreads();
    const uint32_t pos = s_wave[kBlock / 64] + s_wave[wid] + static_cast<uint32_t>(__popcll(b & ((1ull << lane) - 1)));
    __syncthreads();  // s_wave is free again for the next call
    return take ? pos : ~0u;
}

// A wave's appends to (list, count) through its LDS buffer `buf`
// (kAppendBuf entries).  All lanes of the wave call push() and flush()
// together; flush() must run once more after the wave's last push().
struct WaveAppender {
    volatile uint32_t* buf;
    uint32_t* list;
    uint32_t* count;
    uint32_t n;  // entries held (the same in every lane)

    __device__ void push(bool take, uint32_t v) {
        const uint64_t b = __ballot(take);
        if (take) buf[n + static_cast<uint32_t>(__popcll(b & ((1ull << lane_id()) - 1)))] = v;
        n += static_cast<uint32_t>(__popcll(b));
        if (n > kAppendBuf - 64) flush();
    }

    __device__ void flush() {
        wave_sync();
        uint32_t pos = 0;
        if (lane_id() == 0 && n) pos = atomicAdd(count, n);
        pos = static_cast<uint32_t>(__shfl(static_cast<int>(pos), 0, 64));
        for (uint32_t j = lane_id(); j < n; j += 64) list[pos + j] = buf[j];
        wave_sync();
        n = 0;
    }
};

}  // namespace bsim
