// Device-side pieces of the stage-1 scan kernels: launch parameters, the
// XCD-aware block decode, the fp4 operand spreads of the GF(2) contraction
// and the wait / barrier helpers of the LDS rings.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pir_internal.h"

namespace pir {
namespace scan {

constexpr int kThreads = 256;  // 4 waves of 64
constexpr int kWaves = kThreads / 64;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
struct Stage1Params {
    uint64_t n_units;
    uint64_t units_per_group;
    uint64_t stride_words;  // selection row pitch in 32-bit words
    uint64_t nb;            // blocks holding records (selection words per row)
    uint32_t q_total;
    uint32_t groups;
    uint32_t n_ct;
    uint32_t n_qt;
    uint32_t cpb;         // chunks per block
    uint32_t bpw;         // blocks per unit
    uint32_t lpb;         // lanes per block
    uint32_t tile_bytes;  // record bytes per column tile
    uint32_t R;
    uint32_t rpad;
};

// Workgroup -> (record group, column tile, query tile).  Workgroups are
// dispatched round-robin over the 8 XCDs; consecutive workgroups on one XCD
// get the column/query tiles of the same record group, so the selection
// words and database chunks they share meet in that XCD's L2.
__device__ __forceinline__ bool decode_block(uint32_t groups, uint32_t n_ct, uint32_t n_qt,
                                             uint32_t& group, uint32_t& ct, uint32_t& qt) {
    const uint32_t total = groups * n_ct * n_qt;
    const uint32_t per_xcd = (total + 7) / 8;
    const uint32_t v = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (v >= total) return false;
    const uint32_t co = n_ct * n_qt;
    group = v / co;
    const uint32_t rem = v - group * co;
    ct = rem / n_qt;
    qt = rem - ct * n_qt;
    return true;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x8 __attribute__((ext_vector_type(8)));

constexpr uint32_t kMfmaBlocksPerStep = 16;

// s_waitcnt with vmcnt <= N and no wait on the other counters (gfx9
// encoding: vmcnt[3:0] bits 3:0, vmcnt[5:4] bits 15:14, expcnt 6:4,
// lgkmcnt 11:8).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Workgroup barrier without the memory fences of __syncthreads (which would
// wait for every load in flight); the clobber keeps LDS accesses on their
// side of it.
__device__ __forceinline__ void wg_barrier() { asm volatile("s_barrier" ::: "memory"); }

// 32 records of one word -> 32 E2M1 values, element (dword t, nibble n) =
// record 4n + t.  The selection side (A, record order) and the database side
// (B, stored order) use reciprocal values so that every product of two set
// bits is exactly 1.0:
//   t:    0     1     2     3
//   A:   0.5   1.0   2.0   2.0     (E2M1 0b0001, 0b0010, 0b0100, 0b0100)
//   B:   2.0   1.0   0.5   0.5
// Each record is taken where it already sits in its nibble when that position
// carries the wanted value (a mask only); nibble bit 3 would be the sign, so
// record 4n+3 is shifted down on both sides.
__device__ __forceinline__ i32x8 spread_fp4_a(uint32_t w) {  // w in record order
    i32x8 r;
    r[0] = (int32_t)(w & 0x11111111u);          // record 4n   at bit 0: 0.5
    r[1] = (int32_t)(w & 0x22222222u);          // record 4n+1 at bit 1: 1.0
    r[2] = (int32_t)(w & 0x44444444u);          // record 4n+2 at bit 2: 2.0
    r[3] = (int32_t)((w >> 1) & 0x44444444u);   // record 4n+3 to bit 2: 2.0
    r[4] = 0;
    r[5] = 0;
    r[6] = 0;
    r[7] = 0;
    return r;
}
__device__ __forceinline__ i32x8 spread_fp4_b(uint32_t w) {  // w in stored order
    i32x8 r;
    r[0] = (int32_t)(w & 0x44444444u);          // record 4n   stored at bit 2: 2.0
    r[1] = (int32_t)(w & 0x22222222u);          // record 4n+1 at bit 1: 1.0
    r[2] = (int32_t)(w & 0x11111111u);          // record 4n+2 stored at bit 0: 0.5
    r[3] = (int32_t)((w >> 3) & 0x11111111u);   // record 4n+3 to bit 0: 0.5
    r[4] = 0;
    r[5] = 0;
    r[6] = 0;
    r[7] = 0;
    return r;
}

// One 16x16x128 product on E2M1 operands (the low four dwords of each i32x8;
// the spreads above leave the high four zero).  Zero block-scale operands
// make the compiler emit the unscaled instruction,
// v_mfma_f32_16x16x128_f8f6f4 with four-register fp4 sources.
__device__ __forceinline__ f32x4 mfma_fp4(const i32x8& a, const i32x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 4, 4, 0, 0, 0, 0);
}

constexpr uint32_t kStageDbBytes = 16 * 256 * 4;

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// A wave-uniform pointer re-read through v_readfirstlane.  The loads below
// add a 32-bit lane offset to it; without this the compiler folds base and
// offset into one 64-bit pointer per lane and load, kept in vector registers
// and advanced with vector adds every step (12 of them per step instead of
// the 8 that forming each address from the scalar base takes).
__device__ __forceinline__ const uint8_t* uniform_ptr(const uint8_t* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const uint8_t*>(((uint64_t)hi << 32) | lo);
}

}  // namespace scan
}  // namespace pir
