// Streaming-read probe: the practical HBM read roof that the scans are
// measured against.  A workgroup reads a contiguous range of 16-byte chunks
// with non-temporal loads, U chunks in flight per lane, and XOR-folds them
// into one 16-byte word (so the loads cannot be dropped), written to
// sink[workgroup].  No other memory traffic.
#include <hip/hip_runtime.h>

#include "pir_internal.h"
#include "pir_runtime.h"

namespace pir {

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kProbeThreads = 256;

template <int U>
__global__ void __launch_bounds__(kProbeThreads)
k_read_probe(const u32x4* __restrict__ src, uint64_t n_chunks, uint64_t chunks_per_wg, u32x4* __restrict__ sink) {
    __shared__ u32x4 red[kProbeThreads / 64];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t begin = (uint64_t)blockIdx.x * chunks_per_wg;
    const uint64_t end = begin + chunks_per_wg < n_chunks ? begin + chunks_per_wg : n_chunks;
    u32x4 acc = {0, 0, 0, 0};
    // wave w reads rows of 64 chunks w*U .. w*U + U-1, then skips the other waves' rows
    uint64_t c = begin + (uint64_t)wave * 64 * U + lane;
    for (; c + 64 * (U - 1) < end; c += (uint64_t)kProbeThreads * U) {
        u32x4 d[U];
#pragma unroll
        for (int k = 0; k < U; ++k) d[k] = __builtin_nontemporal_load(src + c + 64 * k);
#pragma unroll
        for (int k = 0; k < U; ++k) acc ^= d[k];
    }
    for (int k = 0; k < U; ++k)
        if (c + 64 * k < end) acc ^= __builtin_nontemporal_load(src + c + 64 * k);
    // fold the lanes, then the waves
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        acc.x ^= (uint32_t)__shfl_xor((int)acc.x, m);
        acc.y ^= (uint32_t)__shfl_xor((int)acc.y, m);
        acc.z ^= (uint32_t)__shfl_xor((int)acc.z, m);
        acc.w ^= (uint32_t)__shfl_xor((int)acc.w, m);
    }
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32x4 t = red[0];
        for (int w = 1; w < kProbeThreads / 64; ++w) t ^= red[w];
        sink[blockIdx.x] = t;
    }
}

}  // namespace

}  // namespace pir

using namespace pir;

extern "C" int pir_read_probe_async(pir_ctx* c, const void* d_src, uint64_t bytes, uint32_t unroll,
                                    uint32_t workgroups, void* d_sink, void* hip_stream) {
    clear_error();
    if (!c || !d_src || !d_sink) return fail(PIR_E_INVAL, "pir_read_probe_async: NULL argument");
    if (bytes == 0 || bytes % 16 != 0) return fail(PIR_E_INVAL, "pir_read_probe_async: bytes must be a positive multiple of 16");
    if ((reinterpret_cast<uintptr_t>(d_src) & 15) || (reinterpret_cast<uintptr_t>(d_sink) & 15))
        return fail(PIR_E_INVAL, "pir_read_probe_async: buffers must be 16-byte aligned");
    if (workgroups == 0 || workgroups > (1u << 20)) return fail(PIR_E_INVAL, "pir_read_probe_async: workgroups outside [1, 2^20]");
    Ctx* ctx = reinterpret_cast<Ctx*>(c);
    int rc = ctx->bind();
    if (rc) return rc;
    const uint64_t n_chunks = bytes / 16;
    const uint64_t per = (n_chunks + workgroups - 1) / workgroups;
    const uint32_t grid = (uint32_t)((n_chunks + per - 1) / per);
    hipStream_t s = (hipStream_t)hip_stream;
    const u32x4* src = (const u32x4*)d_src;
    u32x4* sink = (u32x4*)d_sink;
    switch (unroll) {
        case 4: hipLaunchKernelGGL(k_read_probe<4>, dim3(grid), dim3(kProbeThreads), 0, s, src, n_chunks, per, sink); break;
        case 8: hipLaunchKernelGGL(k_read_probe<8>, dim3(grid), dim3(kProbeThreads), 0, s, src, n_chunks, per, sink); break;
        case 16: hipLaunchKernelGGL(k_read_probe<16>, dim3(grid), dim3(kProbeThreads), 0, s, src, n_chunks, per, sink); break;
        default: return fail(PIR_E_INVAL, "pir_read_probe_async: unroll must be 4, 8 or 16");
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "read probe launch");
    return PIR_OK;
}
