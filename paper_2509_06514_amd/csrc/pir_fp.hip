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

// Operand source for column tiles that fall outside the problem (and, at
// g_zero128, for query rows past the last one): the main loop's loads are
// unconditional, masked operands read zeros from here.
__device__ uint8_t g_zero64[64];
__device__ __attribute__((aligned(16))) uint8_t g_zero128[128];

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
    // 8 independent loads in flight: few workgroups, so the walk over the
    // slices is latency-bound
    uint32_t a[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // sums < groups * 126 < 2^32
    uint32_t k = 0;
    for (; k + 8 <= slices; k += 8) {
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) a[u] += tmp[(uint64_t)(k + u) * outputs + o];
    }
    for (; k < slices; ++k) a[0] += tmp[(uint64_t)k * outputs + o];
    const uint32_t s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
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

// s_waitcnt vmcnt(<= N), other counters not waited for (gfx9 encoding).
template <int N>
__device__ __forceinline__ void fp_wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Stage 1: workgroup = (record group g, query tile qt, column group cg), RT
// row tiles of 16 queries, CT column tiles of 16 elements.  A wave step
// covers two tiles (128 records: one whole 128-byte line of every query row
// of the tile); the four waves of a workgroup take the steps of its range in
// turn, and their sums (each reduced mod p) meet in LDS.  One byte per
// (group, query, element) is written: partials[(g * q_total + q) * L + c].
//
// The query rows go through LDS.  Read straight into the MFMA layout, a
// lane's A operand is 16 bytes of one row and a load instruction would touch
// 64 bytes of each of 16 rows: half of every line, the other half going to
// another instruction.  Here each direct-to-LDS load (global_load_lds_dwordx4)
// moves 8 rows x 128 bytes into a wave-private LDS buffer, and the operands
// are read from there.  Two buffers per wave: the next step's lines are in
// flight while a step runs.  Row 8i + r, 16-byte chunk c of the line sits at
// i * 1 KiB + 128 * (c ^ (i & 1)) + 16 r: the XOR spreads the 16 rows that
// one operand read touches over all LDS banks.  The database operand (whole
// lines in the tile layout) is loaded into registers.
//
// Workgroups are numbered XCD-major, as in the XOR scan: the query tiles and
// column groups of one record group run on one XCD, close together in time,
// and share its L2 copy of the record tiles.
template <int RT, int CT>
__host__ __device__ constexpr uint32_t fp_lds_bytes() {
    return 4u * 2u * (16u * RT * 128u) + RT * CT * 4u * 64u * 4u;
}

template <int RT, int CT>
__global__ void __launch_bounds__(kFpThreads)
k_fp_stage1_lds(const uint8_t* __restrict__ db, const uint8_t* __restrict__ v, uint8_t* __restrict__ partials,
                FpParams a) {
    constexpr int kRows = 16 * RT;
    constexpr int kAInstr = kRows / 8;  // direct-to-LDS loads per step (8 rows x 128 B each)
    constexpr int kLoadsPerStep = kAInstr + 2 * CT;
    constexpr uint32_t kBuf = kRows * 128;
    extern __shared__ __attribute__((aligned(16))) uint8_t fp_lds[];
    uint32_t* const red = reinterpret_cast<uint32_t*>(fp_lds + 4 * 2 * kBuf);

    const uint32_t total = a.groups * a.n_qt * a.n_cg;
    const uint32_t per_xcd = (total + 7) / 8;
    const uint32_t vb = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (vb >= total) return;  // grid padding (whole workgroup)
    const uint32_t qt = vb % a.n_qt;
    const uint32_t cg = (vb / a.n_qt) % a.n_cg;
    const uint32_t g = vb / (a.n_qt * a.n_cg);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t row = lane & 15, kq = lane >> 4;
    uint8_t* const bufs = fp_lds + wave * 2 * kBuf;
    for (uint32_t i = threadIdx.x; i < RT * CT * 4 * 64; i += kFpThreads) red[i] = 0;

    const uint64_t t0 = (uint64_t)g * a.tiles_per_group;
    const uint64_t t1 = t0 + a.tiles_per_group < a.tiles ? t0 + a.tiles_per_group : a.tiles;

    // loader: instruction i, lane l -> row 8i + (l & 7), chunk (l >> 3) ^ (i & 1)
    const uint8_t* abase[kAInstr];
    uint32_t astep[kAInstr], achunk[kAInstr];
#pragma unroll
    for (int i = 0; i < kAInstr; ++i) {
        const uint32_t q = qt * kRows + 8 * i + (lane & 7);
        const bool ok = q < a.q_total;
        abase[i] = ok ? v + (uint64_t)q * a.v_stride : g_zero128;
        astep[i] = ok ? 64 : 0;
        achunk[i] = (lane >> 3) ^ (i & 1);
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
    // this lane's A operand of half h, row tile rt: row 16 rt + row, chunk 4h + kq
    uint32_t rd[2][RT];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const uint32_t i = 2 * rt + (row >> 3);
            rd[h][rt] = i * 1024 + 128 * ((4 * h + kq) ^ (i & 1)) + 16 * (row & 7);
        }

    i32x4 acc[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = i32x4{0, 0, 0, 0};

    // a step at tile t covers t and t + 1 (when t + 1 < t1; otherwise the
    // second half re-reads the first, in bounds, and its products are skipped)
    auto issue = [&](uint64_t t, uint32_t b, u32x4(&rb)[2][CT]) {
        const bool two = t + 1 < t1;
        uint8_t* dst = bufs + b * kBuf;
#pragma unroll
        for (int i = 0; i < kAInstr; ++i) {
            const uint32_t ch = (two || achunk[i] < 4) ? achunk[i] : achunk[i] - 4;
            __builtin_amdgcn_global_load_lds(
                reinterpret_cast<const uint32_t*>(abase[i] + t * astep[i] + 16 * ch), dst + i * 1024, 16, 0, 0);
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            rb[0][ct] = ld16(bbase[ct] + t * bstep[ct]);
            rb[1][ct] = ld16(bbase[ct] + (two ? t + 1 : t) * bstep[ct]);
        }
    };
    auto compute = [&](uint64_t t, uint32_t b, const u32x4(&rb)[2][CT]) {
        const uint8_t* src = bufs + b * kBuf;
        const int halves = t + 1 < t1 ? 2 : 1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h >= halves) break;  // uniform
            u32x4 ra[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) ra[rt] = *reinterpret_cast<const u32x4*>(src + rd[h][rt]);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
                    acc[rt][ct] =
                        __builtin_amdgcn_mfma_i32_16x16x64_i8((i32x4)ra[rt], (i32x4)rb[h][ct], acc[rt][ct], 0, 0, 0);
        }
    };

    // Wave w takes the steps at t0 + 2 (w + 4 i).  Each step waits for its own
    // loads (vmcnt) with the next step's in flight; a buffer is refilled only
    // after the step that read it has finished its LDS reads.
    constexpr uint64_t kStride = 8;
    uint64_t t = t0 + 2 * wave;
    if (t < t1) {
        u32x4 B0[2][CT], B1[2][CT];
        issue(t, 0, B0);
        for (;;) {
            uint64_t t2 = t + kStride;
            if (t2 >= t1) {
                fp_wait_vmcnt<0>();
                compute(t, 0, B0);
                break;
            }
            issue(t2, 1, B1);
            fp_wait_vmcnt<kLoadsPerStep>();
            compute(t, 0, B0);
            __builtin_amdgcn_sched_barrier(0);
            const uint64_t t3 = t2 + kStride;
            if (t3 >= t1) {
                fp_wait_vmcnt<0>();
                compute(t2, 1, B1);
                break;
            }
            issue(t3, 0, B0);
            fp_wait_vmcnt<kLoadsPerStep>();
            compute(t2, 1, B1);
            __builtin_amdgcn_sched_barrier(0);
            t = t3;
        }
    }

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
        const uint32_t q = qt * kRows + 16 * rt + 4 * (ln >> 4) + r;
        const uint32_t c = (cg * CT + ct) * 16 + (ln & 15);
        if (q < a.q_total && c < a.L)
            partials[((uint64_t)g * a.q_total + q) * a.L + c] = (uint8_t)mod_p(red[i], a.p, a.magic);
    }
}

template <int RT, int CT>
hipError_t launch_lds_rt_ct(const uint8_t* db, const uint8_t* v, uint8_t* partials, const FpParams& a,
                            uint32_t grid, hipStream_t s) {
    constexpr uint32_t bytes = fp_lds_bytes<RT, CT>();
    const hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_fp_stage1_lds<RT, CT>), (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fp_stage1_lds<RT, CT>), dim3(grid), dim3(kFpThreads), bytes, s, db, v, partials, a);
    return hipGetLastError();
}


}  // namespace

bool fp_supported(uint32_t rt, uint32_t ct) {
    return (rt == 1 || rt == 2 || rt == 4) && (ct == 1 || ct == 2 || ct == 4);
}

hipError_t launch_fp_stage1(const uint8_t* db, const uint8_t* v, uint8_t* partials, const FpParams& a, uint32_t rt,
                            uint32_t ct, hipStream_t s) {
    const uint32_t total = a.groups * a.n_qt * a.n_cg;
    const uint32_t grid = (total + 7) / 8 * 8;
#define PIR_FP_CASE(R_, C_) \
    if (rt == R_ && ct == C_) return launch_lds_rt_ct<R_, C_>(db, v, partials, a, grid, s);
    PIR_FP_CASE(1, 1) PIR_FP_CASE(1, 2) PIR_FP_CASE(1, 4)
    PIR_FP_CASE(2, 1) PIR_FP_CASE(2, 2) PIR_FP_CASE(2, 4)
    PIR_FP_CASE(4, 1) PIR_FP_CASE(4, 2) PIR_FP_CASE(4, 4)
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
