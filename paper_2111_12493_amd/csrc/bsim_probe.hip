// bsim_probe.hip -- measurement probes for the refinement's roofline.
//
// bsim_probe_gather times the memory pattern that bounds a refinement
// iteration and nothing else: stream every edge target once and gather one
// 8-byte value per edge from an n-entry array (the neighbour-hash gather of
// a refinement step, without labels, de-duplication or classes).  Its rate
// is the ceiling a refinement launch can reach on that graph's targets.
// bsim_probe_copy is a STREAM-style copy (read + write of a byte range),
// the practical HBM bandwidth of the device.
#include "bsim_api_internal.h"

namespace bsim {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbePerThread = 8;

__global__ void __launch_bounds__(kProbeBlock) k_probe_gather(const uint32_t* __restrict__ tgt, uint64_t m,
                                                              const uint64_t* __restrict__ h, uint32_t n,
                                                              uint64_t* __restrict__ sink) {
    const uint64_t base = (static_cast<uint64_t>(blockIdx.x) * kProbePerThread) * kProbeBlock + threadIdx.x;
    uint32_t w[kProbePerThread];
#pragma unroll
    for (int r = 0; r < kProbePerThread; r++) {
        const uint64_t e = base + static_cast<uint64_t>(r) * kProbeBlock;
        w[r] = e < m ? __builtin_nontemporal_load(&tgt[e]) : 0xFFFFFFFFu;
    }
    uint64_t acc = 0;
#pragma unroll
    for (int r = 0; r < kProbePerThread; r++)
        if (w[r] < n) acc += h[w[r]];
    // one store per thread that nothing reads: the gathers cannot be dropped
    if (acc == 0x5EEDull) sink[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(kProbeBlock) k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                            uint64_t n16) {
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kProbeBlock + threadIdx.x; i < n16;
         i += static_cast<uint64_t>(gridDim.x) * kProbeBlock)
        dst[i] = src[i];
}

}  // namespace
}  // namespace bsim

using namespace bsim;

extern "C" {

int bsim_probe_gather(bsim_ctx* ctx, const uint32_t* tgt, uint64_t m, const uint64_t* h, uint32_t n,
                      uint32_t reps, float* ms_per_pass) {
    if (!ctx || !ms_per_pass || (m && (!tgt || !h)) || reps == 0) return BSIM_E_INVALID;
    try {
        hip_check(hipSetDevice(ctx->device), "set device");
        hipStream_t s = ctx->stream;
        const uint64_t per_block = static_cast<uint64_t>(kProbeBlock) * kProbePerThread;
        const uint64_t blocks = std::max<uint64_t>((m + per_block - 1) / per_block, 1);
        if (blocks > 0x7FFFFFFFull) throw DeviceError{BSIM_E_UNSUPPORTED, "graph too large for the probe"};
        // gather from a copy of h in the ctx's work memory, where the
        // refinement keeps its hash arrays
        Arena arena(s);
        ctx_back_arena(ctx, arena, static_cast<size_t>(n) * 8 + blocks * 8 + 1024);
        uint64_t* hc = arena.alloc<uint64_t>(n);
        uint64_t* sink = arena.alloc<uint64_t>(blocks);
        if (n) hip_check(hipMemcpyAsync(hc, h, static_cast<size_t>(n) * 8, hipMemcpyDeviceToDevice, s), "probe copy");
        h = hc;
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        k_probe_gather<<<static_cast<uint32_t>(blocks), kProbeBlock, 0, s>>>(tgt, m, h, n, sink);  // warm-up
        hip_check(hipEventRecord(e0, s), "event");
        for (uint32_t r = 0; r < reps; r++)
            k_probe_gather<<<static_cast<uint32_t>(blocks), kProbeBlock, 0, s>>>(tgt, m, h, n, sink);
        hip_check(hipEventRecord(e1, s), "event");
        hip_check(hipEventSynchronize(e1), "probe sync");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "probe time");
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *ms_per_pass = ms / reps;
        return BSIM_OK;
    } catch (const DeviceError& e) {
        ctx->err = e.msg;
        return e.status;
    }
}

int bsim_probe_copy(bsim_ctx* ctx, uint64_t bytes, uint32_t reps, float* ms_per_pass) {
    if (!ctx || !ms_per_pass || reps == 0 || bytes < 16) return BSIM_E_INVALID;
    try {
        hip_check(hipSetDevice(ctx->device), "set device");
        hipStream_t s = ctx->stream;
        const uint64_t n16 = bytes / 16;
        Arena arena(s);
        uint4* a = arena.alloc<uint4>(n16);
        uint4* b = arena.alloc<uint4>(n16);
        hip_check(hipMemsetAsync(a, 1, n16 * 16, s), "probe fill");
        int cus = 0;
        hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device), "CU count");
        const uint32_t grid = static_cast<uint32_t>(std::max(cus, 1)) * 16;
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        k_probe_copy<<<grid, kProbeBlock, 0, s>>>(a, b, n16);
        hip_check(hipEventRecord(e0, s), "event");
        for (uint32_t r = 0; r < reps; r++) k_probe_copy<<<grid, kProbeBlock, 0, s>>>(a, b, n16);
        hip_check(hipEventRecord(e1, s), "event");
        hip_check(hipEventSynchronize(e1), "probe sync");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "probe time");
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *ms_per_pass = ms / reps;
        return BSIM_OK;
    } catch (const DeviceError& e) {
        ctx->err = e.msg;
        return e.status;
    }
}

}  // extern "C"
