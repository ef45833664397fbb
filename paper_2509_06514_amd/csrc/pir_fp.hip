// Inner products over F_p on the matrix cores: the server answer in the form
// the paper states it for a database over F_p (IM-PIR Sec. 2, D in
// F_p^{N x L}; the linear operations of Sec. 3.3), of which the XOR scan is
// the case p = 2 on bits:
//
//     r_q[l] = ( sum_j v_q[j] * D[j][l] ) mod p
//
// For Q queries this is the product of a Q x N matrix of query bytes with
// the N x L database, a dense contraction over the records: it runs on the
// int8 MFMA (v_mfma_i32_16x16x64_i8) with exact int32 sums, reduced mod p
// once per record group.
//
// Layout in HBM: records in tiles of 64 (one K-step); inside a tile the
// elements are column-major -- element c of records 64t .. 64t+63 are 64
// consecutive bytes at t * 64 * lpad + c * 64 -- so the B operand of a lane
// (16 consecutive records of one column) is one 16-byte load and a wave's
// 64 lanes read 1 KiB contiguously.  lpad = L rounded up to 16 (one MFMA
// column tile); padded columns and records past N are zero.
#include <hip/hip_runtime.h>

#include "pir_internal.h"

namespace pir {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

constexpr int kFpThreads = 256;  // 4 waves; the waves of a workgroup split its K-steps

// Operand source for query rows and column tiles that fall outside the
// problem: every load of the main loop is unconditional (so the compiler can
// count the loads in flight), and masked operands read zeros from here.
__device__ uint8_t g_zero64[64];

__device__ __forceinline__ u32x4 ld16(const uint8_t* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
}

// x mod p for x < 2^32, with m = floor(2^32 / p): q = mulhi(x, m) is
// floor(x / p) or one less, so one correction step suffices.
__device__ __forceinline__ uint32_t mod_p(uint32_t x, uint32_t p, uint32_t m) {
    const uint32_t q = __umulhi(x, m);
    uint32_t r = x - q * p;
    return r >= p ? r - p : r;
}

// Stage 1: workgroup = (record group g, query tile qt, column group cg).
// RT row tiles of 16 queries, CT column tiles of 16 elements.  A wave step
// covers KT consecutive tiles (KT * 64 contiguous bytes of every query row);
// the waves of a workgroup take the steps of its range in turn.  The four
// waves' sums (each reduced mod p) meet in LDS; one byte per (group, query,
// element) is written: partials[(g * q_total + q) * L + c].
template <int RT, int CT, int KT>
__global__ void __launch_bounds__(kFpThreads)
k_fp_stage1(const uint8_t* __restrict__ db, const uint8_t* __restrict__ v, uint8_t* __restrict__ partials,
            FpParams a) {
    __shared__ uint32_t red[RT * CT * 4 * 64];
    for (uint32_t i = threadIdx.x; i < RT * CT * 4 * 64; i += kFpThreads) red[i] = 0;

    const uint32_t g = blockIdx.x % a.groups;
    const uint32_t rest = blockIdx.x / a.groups;
    const uint32_t qt = rest % a.n_qt, cg = rest / a.n_qt;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t row = lane & 15, kq = lane >> 4;

    const uint64_t t0 = (uint64_t)g * a.tiles_per_group;
    const uint64_t t1 = t0 + a.tiles_per_group < a.tiles ? t0 + a.tiles_per_group : a.tiles;

    // A operand: query row q0 + 16 rt + row, record bytes 16 kq .. 16 kq + 15
    // of a tile; B operand: column 16 c + row of the tile, records
    // 16 kq .. 16 kq + 15.  Masked rows / column tiles read zeros (step 0).
    const uint8_t* abase[RT];
    uint64_t astep[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const uint32_t q = qt * 16 * RT + 16 * rt + row;
        const bool ok = q < a.q_total;
        abase[rt] = ok ? v + (uint64_t)q * a.v_stride + 16 * kq : g_zero64 + 16 * kq;
        astep[rt] = ok ? 64 : 0;
    }
    const uint64_t tile_bytes = 64ull * a.lpad;
    const uint8_t* bbase[CT];
    uint64_t bstep[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const uint32_t c = cg * CT + ct;
        const bool ok = c < a.n_ct;
        bbase[ct] = ok ? db + c * 1024 + row * 64 + 16 * kq : g_zero64 + 16 * kq;
        bstep[ct] = ok ? tile_bytes : 0;
    }

    i32x4 acc[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = i32x4{0, 0, 0, 0};

    // every load is unconditional: tiles past the range are clamped to the
    // last one (their products are skipped below)
    u32x4 A[KT][RT], B[KT][CT], An[KT][RT], Bn[KT][CT];
    auto load = [&](uint64_t t, u32x4(&ra)[KT][RT], u32x4(&rb)[KT][CT]) {
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            const uint64_t tk = t + k < t1 ? t + k : t1 - 1;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) ra[k][rt] = ld16(abase[rt] + tk * astep[rt]);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) rb[k][ct] = ld16(bbase[ct] + tk * bstep[ct]);
        }
    };
    auto compute = [&](uint64_t t, const u32x4(&ra)[KT][RT], const u32x4(&rb)[KT][CT]) {
        // keep the loads issued before this point ahead of the matrix work
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            if (k > 0 && t + k >= t1) break;  // uniform: the range ends inside this step
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
                    acc[rt][ct] =
                        __builtin_amdgcn_mfma_i32_16x16x64_i8((i32x4)ra[k][rt], (i32x4)rb[k][ct], acc[rt][ct], 0, 0, 0);
        }
    };

    // Two register sets in turn: the next step's loads are in flight while a
    // step runs on the matrix cores.  Wave w takes the steps starting at
    // t0 + KT (w + 4 i); the step after the last reloads it (unconditional).
    constexpr uint64_t kStride = 4 * KT;
    uint64_t t = t0 + KT * wave;
    if (t < t1) {
        load(t, A, B);
        for (;;) {
            const uint64_t t2 = t + kStride;
            load(t2 < t1 ? t2 : t, An, Bn);
            compute(t, A, B);
            if (t2 >= t1) break;
            const uint64_t t3 = t2 + kStride;
            load(t3 < t1 ? t3 : t2, A, B);
            compute(t2, An, Bn);
            if (t3 >= t1) break;
            t = t3;
        }
    }

    // 16x16 MFMA tile: lane holds column lane % 16 and rows 4 (lane / 16) + r
    __syncthreads();  // red[] cleared
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                atomicAdd(&red[((rt * CT + ct) * 4 + r) * 64 + lane], mod_p((uint32_t)acc[rt][ct][r], a.p, a.magic));
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < RT * CT * 4 * 64; i += kFpThreads) {
        const uint32_t ln = i & 63, r = (i >> 6) & 3, tc = i >> 8;
        const uint32_t rt = tc / CT, ct = tc % CT;
        const uint32_t q = qt * 16 * RT + 16 * rt + 4 * (ln >> 4) + r;
        const uint32_t c = (cg * CT + ct) * 16 + (ln & 15);
        if (q < a.q_total && c < a.L)
            partials[((uint64_t)g * a.q_total + q) * a.L + c] = (uint8_t)mod_p(red[i], a.p, a.magic);
    }
}

// Stage 2, in two levels so that no thread walks all groups (with few
// outputs that walk is a long chain of dependent byte loads):
//  1. block (x, y) sums groups [64 y, 64 y + 64) for 64 outputs -- 16 loads
//     per thread, all independent -- into tmp[y][o];
//  2. one thread per output adds the slices and reduces mod p.
constexpr uint32_t kFpSliceGroups = 64;

__global__ void __launch_bounds__(kFpThreads)
k_fp_reduce_slices(const uint8_t* __restrict__ partials, uint32_t groups, uint64_t outputs,
                   uint32_t* __restrict__ tmp) {
    __shared__ uint32_t part[4][64];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t o = (uint64_t)blockIdx.x * 64 + lane;
    const uint32_t g0 = blockIdx.y * kFpSliceGroups;
    uint32_t s = 0;
    if (o < outputs) {
#pragma unroll
        for (uint32_t i = 0; i < kFpSliceGroups / 4; ++i) {
            const uint32_t g = g0 + w + 4 * i;
            if (g < groups) s += partials[(uint64_t)g * outputs + o];
        }
    }
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && o < outputs)
        tmp[(uint64_t)blockIdx.y * outputs + o] = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
}

__global__ void __launch_bounds__(kFpThreads)
k_fp_finish(const uint32_t* __restrict__ tmp, uint32_t slices, uint64_t outputs, uint32_t p, uint32_t magic,
            uint8_t* __restrict__ out) {
    const uint64_t o = (uint64_t)blockIdx.x * kFpThreads + threadIdx.x;
    if (o >= outputs) return;
    uint32_t s = 0;  // < groups * 126 < 2^32
    for (uint32_t k = 0; k < slices; ++k) s += tmp[(uint64_t)k * outputs + o];
    out[o] = (uint8_t)mod_p(s, p, magic);
}

// Row-major records [0, nrec) of a chunk -> tiles at dst (the chunk starts
// on a tile boundary); one thread per 16-byte piece (tile, column, quarter).
__global__ void __launch_bounds__(kFpThreads)
k_fp_tile(const uint8_t* __restrict__ src, uint64_t nrec, uint32_t L, uint32_t lpad, uint64_t ntiles,
          uint8_t* __restrict__ dst) {
    const uint64_t i = (uint64_t)blockIdx.x * kFpThreads + threadIdx.x;
    if (i >= ntiles * lpad * 4) return;
    const uint32_t k = (uint32_t)(i & 3);
    const uint64_t tc = i >> 2;
    const uint32_t c = (uint32_t)(tc % lpad);
    const uint64_t t = tc / lpad;
    uint32_t w[4] = {0, 0, 0, 0};
    for (int b = 0; b < 16; ++b) {
        const uint64_t j = 64 * t + 16 * k + b;
        const uint32_t x = (j < nrec && c < L) ? src[j * L + c] : 0u;
        w[b >> 2] |= x << (8 * (b & 3));
    }
    *reinterpret_cast<u32x4*>(dst + t * 64ull * lpad + c * 64ull + 16 * k) = u32x4{w[0], w[1], w[2], w[3]};
}

// Tiles -> row-major records [0, nrec) of a chunk starting at tile 0 of src.
__global__ void __launch_bounds__(kFpThreads)
k_fp_untile(const uint8_t* __restrict__ src, uint64_t nrec, uint32_t L, uint32_t lpad, uint8_t* __restrict__ dst) {
    const uint64_t i = (uint64_t)blockIdx.x * kFpThreads + threadIdx.x;
    if (i >= nrec * L) return;
    const uint64_t j = i / L;
    const uint32_t c = (uint32_t)(i % L);
    dst[i] = src[(j / 64) * 64ull * lpad + c * 64ull + (j % 64)];
}

template <int RT, int CT, int KT>
hipError_t launch_rt_ct(const uint8_t* db, const uint8_t* v, uint8_t* partials, const FpParams& a, uint32_t grid,
                        hipStream_t s) {
    hipLaunchKernelGGL((k_fp_stage1<RT, CT, KT>), dim3(grid), dim3(kFpThreads), 0, s, db, v, partials, a);
    return hipGetLastError();
}

}  // namespace

bool fp_supported(uint32_t rt, uint32_t ct, uint32_t kt) {
    return (rt == 1 || rt == 2 || rt == 4) && (ct == 1 || ct == 2 || ct == 4) && (kt == 1 || kt == 2);
}

hipError_t launch_fp_stage1(const uint8_t* db, const uint8_t* v, uint8_t* partials, const FpParams& a, uint32_t rt,
                            uint32_t ct, uint32_t kt, hipStream_t s) {
    const uint32_t grid = a.groups * a.n_qt * a.n_cg;
#define PIR_FP_CASE(R_, C_, K_) \
    if (rt == R_ && ct == C_ && kt == K_) return launch_rt_ct<R_, C_, K_>(db, v, partials, a, grid, s);
#define PIR_FP_CASES(K_) \
    PIR_FP_CASE(1, 1, K_) PIR_FP_CASE(1, 2, K_) PIR_FP_CASE(1, 4, K_) \
    PIR_FP_CASE(2, 1, K_) PIR_FP_CASE(2, 2, K_) PIR_FP_CASE(2, 4, K_) \
    PIR_FP_CASE(4, 1, K_) PIR_FP_CASE(4, 2, K_) PIR_FP_CASE(4, 4, K_)
    PIR_FP_CASES(1)
    PIR_FP_CASES(2)
#undef PIR_FP_CASES
#undef PIR_FP_CASE
    return hipErrorInvalidValue;
}

size_t fp_stage2_tmp_bytes(uint32_t groups, uint64_t outputs) {
    return (size_t)((groups + kFpSliceGroups - 1) / kFpSliceGroups) * outputs * 4;
}

hipError_t launch_fp_stage2(const uint8_t* partials, uint32_t groups, uint64_t outputs, uint32_t p, uint32_t magic,
                            uint32_t* tmp, uint8_t* out, hipStream_t s) {
    const uint32_t slices = (groups + kFpSliceGroups - 1) / kFpSliceGroups;
    hipLaunchKernelGGL(k_fp_reduce_slices, dim3((uint32_t)((outputs + 63) / 64), slices), dim3(kFpThreads), 0, s,
                       partials, groups, outputs, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fp_finish, dim3((uint32_t)((outputs + kFpThreads - 1) / kFpThreads)), dim3(kFpThreads), 0,
                       s, tmp, slices, outputs, p, magic, out);
    return hipGetLastError();
}

hipError_t launch_fp_tile(const uint8_t* src, uint64_t nrec, uint32_t L, uint32_t lpad, uint8_t* dst, hipStream_t s) {
    const uint64_t ntiles = (nrec + 63) / 64;
    const uint64_t threads = ntiles * lpad * 4;
    hipLaunchKernelGGL(k_fp_tile, dim3((uint32_t)((threads + kFpThreads - 1) / kFpThreads)), dim3(kFpThreads), 0, s,
                       src, nrec, L, lpad, ntiles, dst);
    return hipGetLastError();
}

hipError_t launch_fp_untile(const uint8_t* src, uint64_t nrec, uint32_t L, uint32_t lpad, uint8_t* dst,
                            hipStream_t s) {
    const uint64_t threads = nrec * L;
    hipLaunchKernelGGL(k_fp_untile, dim3((uint32_t)((threads + kFpThreads - 1) / kFpThreads)), dim3(kFpThreads), 0,
                       s, src, nrec, L, lpad, dst);
    return hipGetLastError();
}

}  // namespace pir
