// Source-label payload of a summary (Sec. 3.3: a payload function may
// memorize the source label of each vertex, and merging two vertices of one
// block joins their source lists).  For a result's block ids and one source
// label per vertex: the distinct (block, source label) pairs over the alive
// vertices, sorted by (block, label).  One 64-bit key per vertex, the
// library's LSD radix sort, a first-of-run flag, a scan and a compaction.
#include <cstring>

#include "bsim_api_internal.h"

namespace bsim {
namespace {

constexpr uint64_t kDeadKey = ~0ull;

__global__ void __launch_bounds__(kBlock) k_payload_keys(const uint32_t* __restrict__ block_ids,
                                                         const uint32_t* __restrict__ labels, uint32_t n,
                                                         uint64_t* __restrict__ keys) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    const uint32_t b = block_ids[v];
    keys[v] = b == 0xFFFFFFFFu ? kDeadKey : (static_cast<uint64_t>(b) << 32) | labels[v];
}

__global__ void __launch_bounds__(kBlock) k_payload_flags(const uint64_t* __restrict__ sorted, uint32_t n,
                                                          uint32_t* __restrict__ flag) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = sorted[i];
    flag[i] = (k != kDeadKey && (i == 0 || sorted[i - 1] != k)) ? 1u : 0u;
}

__global__ void __launch_bounds__(kBlock) k_payload_unpack(const uint64_t* __restrict__ sorted, uint32_t n,
                                                           const uint32_t* __restrict__ flag,
                                                           const uint32_t* __restrict__ pos,
                                                           uint32_t* __restrict__ out_block,
                                                           uint32_t* __restrict__ out_label) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n || !flag[i]) return;
    out_block[pos[i]] = static_cast<uint32_t>(sorted[i] >> 32);
    out_label[pos[i]] = static_cast<uint32_t>(sorted[i]);
}

void source_payload(bsim_ctx* ctx, const bsim_result* r, const uint32_t* labels, uint32_t mem_kind,
                    uint32_t* out_block, uint32_t* out_label, uint64_t* n_pairs) {
    hipStream_t s = ctx->stream;
    Arena arena(s);
    const uint32_t n = r->n_vertices;
    *n_pairs = 0;
    if (n == 0) return;
    const uint32_t* bid = r->block_ids;
    if (r->mem_kind == BSIM_MEM_HOST) {
        uint32_t* d = arena.alloc<uint32_t>(n);
        hip_check(hipMemcpyAsync(d, bid, static_cast<size_t>(n) * 4, hipMemcpyHostToDevice, s), "block ids");
        bid = d;
    }
    const uint32_t* lab = labels;
    if (mem_kind == BSIM_MEM_HOST) {
        uint32_t* d = arena.alloc<uint32_t>(n);
        hip_check(hipMemcpyAsync(d, labels, static_cast<size_t>(n) * 4, hipMemcpyHostToDevice, s), "labels");
        lab = d;
    }
    uint64_t* ka = arena.alloc<uint64_t>(n);
    uint64_t* kb = arena.alloc<uint64_t>(n);
    const uint32_t grid = ceil_div(n, kBlock);
    k_payload_keys<<<grid, kBlock, 0, s>>>(bid, lab, n, ka);
    // dead vertices carry all-ones keys, so every key bit takes part
    const uint64_t* sorted = radix_sort(ka, kb, n, 64, arena, s);
    uint32_t* flag = arena.alloc<uint32_t>(n);
    uint32_t* pos = arena.alloc<uint32_t>(n);
    uint32_t* total = arena.alloc<uint32_t>(1);
    k_payload_flags<<<grid, kBlock, 0, s>>>(sorted, n, flag);
    scan_exclusive(flag, pos, n, total, arena, s);
    uint32_t np = 0;
    hip_check(hipMemcpyAsync(&np, total, 4, hipMemcpyDeviceToHost, s), "pair count");
    hip_check(hipStreamSynchronize(s), "pair count");
    uint32_t* ob = out_block;
    uint32_t* ol = out_label;
    if (mem_kind == BSIM_MEM_HOST) {
        ob = arena.alloc<uint32_t>(np + 1);
        ol = arena.alloc<uint32_t>(np + 1);
    }
    k_payload_unpack<<<grid, kBlock, 0, s>>>(sorted, n, flag, pos, ob, ol);
    hip_check(hipGetLastError(), "payload launch");
    if (mem_kind == BSIM_MEM_HOST && np) {
        hip_check(hipMemcpyAsync(out_block, ob, static_cast<size_t>(np) * 4, hipMemcpyDeviceToHost, s), "pairs");
        hip_check(hipMemcpyAsync(out_label, ol, static_cast<size_t>(np) * 4, hipMemcpyDeviceToHost, s), "pairs");
    }
    hip_check(hipStreamSynchronize(s), "payload sync");
    *n_pairs = np;
}

}  // namespace
}  // namespace bsim

using namespace bsim;

int bsim_source_payload(bsim_ctx* ctx, const bsim_result* result, const uint32_t* source_labels, uint32_t mem_kind,
                        uint32_t* out_block, uint32_t* out_label, uint64_t* n_pairs) {
    if (n_pairs) *n_pairs = 0;
    if (!ctx || !result || !n_pairs || (mem_kind != BSIM_MEM_HOST && mem_kind != BSIM_MEM_DEVICE))
        return BSIM_E_INVALID;
    if (result->n_vertices && (!source_labels || !out_block || !out_label || !result->block_ids))
        return BSIM_E_INVALID;
    try {
        hip_check(hipSetDevice(ctx->device), "set device");
        source_payload(ctx, result, source_labels, mem_kind, out_block, out_label, n_pairs);
        return BSIM_OK;
    } catch (const DeviceError& e) {
        ctx->err = e.msg;
        (void)hipStreamSynchronize(ctx->stream);
        return e.status;
    } catch (const std::bad_alloc&) {
        ctx->err = "host allocation failed";
        return BSIM_E_NOMEM;
    }
}
