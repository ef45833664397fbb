// dpXOR kernels for gfx950 (CDNA4): bit-slicing transpose, the stage-1
// database scan (select + XOR + in-workgroup reduction) and the stage-2
// cross-workgroup reduction.
//
// The computation is r = XOR_j v[j] * D[j] (IM-PIR Sec. 3.3, "Inner products
// and XORing operations").  Over the bit-sliced layout (see pir_internal.h)
// bit b of r is the parity of  XOR over blocks of (W[blk][b] AND S[blk]),
// where W[blk][b] is word b of the block and S[blk] the 32 selection bits of
// the block's records.  Each lane keeps 32-bit XOR accumulators per bit
// column; parities are taken once, at the end of a workgroup's range.  This
// is the paper's two-stage parallel reduction (per-tasklet partials, then a
// master XOR per DPU, then host aggregation), mapped to lanes, waves,
// workgroups and a second kernel.
#include <hip/hip_runtime.h>

#include "pir_internal.h"
#include "pir_scan_common.h"

namespace pir {

namespace {

using namespace scan;


// One 16-byte chunk per lane (global_load_dwordx4); NT marks it streaming.
template <bool NT>
__device__ __forceinline__ u32x4 load16(const u32x4* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}


__device__ __forceinline__ uint32_t parity4(const u32x4& a) {
    return (__builtin_popcount(a.x) & 1u) | ((__builtin_popcount(a.y) & 1u) << 1) |
           ((__builtin_popcount(a.z) & 1u) << 2) | ((__builtin_popcount(a.w) & 1u) << 3);
}

// acc ^= d & s on four words, one v_bitop3_b32 each.  The truth-table index
// of v_bitop3 is (S0 << 2) | (S1 << 1) | S2, so S0 ^ (S1 & S2) is 0x78.
__device__ __forceinline__ uint32_t xor_and(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x78);
}
__device__ __forceinline__ void sel_xor(u32x4& acc, const u32x4& d, uint32_t s) {
    acc.x = xor_and(acc.x, d.x, s);
    acc.y = xor_and(acc.y, d.y, s);
    acc.z = xor_and(acc.z, d.z, s);
    acc.w = xor_and(acc.w, d.w, s);
}


// Stage 1, vector-ALU variant.  QT queries per workgroup, U units per wave
// iteration (U independent 16-byte loads in flight per lane).
template <int QT, int U, bool NARROW>
__global__ void __launch_bounds__(kThreads)
k_stage1_valu(const u32x4* __restrict__ db, const uint32_t* __restrict__ sel,
              uint8_t* __restrict__ partials, Stage1Params p) {
    __shared__ uint8_t nib[kWaves][QT][64];

    uint32_t group, ct, qt;
    if (!decode_block(p.groups, p.n_ct, p.n_qt, group, ct, qt)) return;

    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t q0 = qt * QT;

    // lane -> (block within unit, chunk within block); idle lanes read chunk 0
    // of a valid block and their accumulators are never reported.
    uint32_t bi = 0, cc;
    if (NARROW) {
        bi = lane / p.lpb;
        cc = lane - bi * p.lpb;
        if (bi >= p.bpw) { bi = 0; cc = 0; }
    } else {
        cc = ct * 64 + lane;
        if (cc >= p.cpb) cc = 0;
    }
    const uint64_t unit_chunks = (uint64_t)p.bpw * p.cpb;
    const u32x4* dl = db + (uint64_t)bi * p.cpb + cc;

    const uint32_t* srow[QT];
#pragma unroll
    for (int q = 0; q < QT; ++q) {
        const uint32_t qq = (q0 + q < p.q_total) ? q0 + q : q0;
        srow[q] = sel + (uint64_t)qq * p.stride_words;
    }

    u32x4 acc[QT];
#pragma unroll
    for (int q = 0; q < QT; ++q) acc[q] = u32x4{0, 0, 0, 0};

    const uint64_t u_begin = (uint64_t)group * p.units_per_group;
    const uint64_t u_end = (u_begin + p.units_per_group < p.n_units) ? u_begin + p.units_per_group
                                                                     : p.n_units;
    uint64_t u = u_begin + (uint64_t)wave * U;
    for (; u + U <= u_end; u += (uint64_t)kWaves * U) {
        u32x4 d[U];
#pragma unroll
        for (int k = 0; k < U; ++k) d[k] = load16<true>(dl + (u + k) * unit_chunks);
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (NARROW) {
                uint64_t blk = (u + k) * p.bpw + bi;
                blk = blk < p.nb ? blk : p.nb - 1;  // padding blocks are zero: any word will do
#pragma unroll
                for (int q = 0; q < QT; ++q) sel_xor(acc[q], d[k], nib_swap02(srow[q][blk]));
            } else {
#pragma unroll
                for (int q = 0; q < QT; ++q) sel_xor(acc[q], d[k], nib_swap02(srow[q][u + k]));
            }
        }
    }
    // this wave's last, partial iteration
    for (uint32_t k = 0; k < (uint32_t)U && u + k < u_end; ++k) {
        const u32x4 dk = load16<true>(dl + (u + k) * unit_chunks);
        if (NARROW) {
            uint64_t blk = (u + k) * p.bpw + bi;
            blk = blk < p.nb ? blk : p.nb - 1;
#pragma unroll
            for (int q = 0; q < QT; ++q) sel_xor(acc[q], dk, nib_swap02(srow[q][blk]));
        } else {
#pragma unroll
            for (int q = 0; q < QT; ++q) sel_xor(acc[q], dk, nib_swap02(srow[q][u + k]));
        }
    }

    // Per-lane parity of each accumulated bit column, then XOR across waves
    // (and, for narrow records, across the blocks of a unit).
#pragma unroll
    for (int q = 0; q < QT; ++q) nib[wave][q][lane] = (uint8_t)parity4(acc[q]);
    __syncthreads();

    const uint32_t tb = p.tile_bytes;
    for (uint32_t t = threadIdx.x; t < QT * tb; t += kThreads) {
        const uint32_t q = t / tb, m = t - q * tb;
        const uint32_t byte_pos = (NARROW ? 0 : ct * 32) + m;
        if (q0 + q >= p.q_total || byte_pos >= p.R) continue;
        uint32_t x = 0;
        for (int w = 0; w < kWaves; ++w)
            for (uint32_t b = 0; b < p.bpw; ++b) {
                const uint32_t c = b * p.lpb + 2 * m;
                x ^= (uint32_t)nib[w][q][c] | ((uint32_t)nib[w][q][c + 1] << 4);
            }
        partials[((uint64_t)group * p.q_total + q0 + q) * p.rpad + byte_pos] = (uint8_t)x;
    }
}

// ---------------------------------------------------------------------------
// Stage 1, matrix-core variants (many queries).
//
// Over F_2, answer bit b of query q is the parity of
//     C[q][b] = sum_j S[q][j] * Dbit[j][b],
// an integer matrix product with 0/1 entries.  The matrix cores compute it
// exactly: products are 0 or 1 and the sums are record counts (below 2^24
// per workgroup, so exact in fp32; int32 in the int8 form), and the parity
// of the count is the answer bit.  Nothing is approximated.
//
// Operands come straight from the bit-sliced layout: in one MFMA a lane holds
// 32 k-elements (fp4) or 16 (int8) for one row or column.  Taking those k to
// be the 32 records of one block makes a lane's A operand one selection word
// of its query and its B operand one bit-sliced database word of its bit
// column; each is spread to one element per bit.  Any fixed order of the 32
// records inside a lane is fine as long as A and B use the same one.
//
// Work split: a workgroup owns (record group, column tile of 256 bit columns,
// query tile of 16*MT queries); wave w owns bit columns [64w, 64w+64) of the
// tile as 4 MFMA column tiles, and all MT row tiles.  A K-step covers 16
// blocks: lane group g = lane/16 reads blocks kb+4g .. kb+4g+3, one per
// sub-step s.  Column tile t of lane j is bit column 64w + 4j + t, so a lane
// reads its 4 columns with one 16-byte load.



// 32 records -> 32 int8 0/1 values in two 16-element halves: dword t, byte
// m holds record 8m + t (half 0: t = 0..3, half 1: t = 4..7).  Record
// 8m + t sits at bit 8m + t of a selection word; in a stored database word
// records 8m, 8m+2 (and 8m+4, 8m+6) trade places.
__device__ __forceinline__ void spread_i8(uint32_t w, i32x4& lo, i32x4& hi) {  // record order
    lo[0] = (int32_t)(w & 0x01010101u);
    lo[1] = (int32_t)((w >> 1) & 0x01010101u);
    lo[2] = (int32_t)((w >> 2) & 0x01010101u);
    lo[3] = (int32_t)((w >> 3) & 0x01010101u);
    hi[0] = (int32_t)((w >> 4) & 0x01010101u);
    hi[1] = (int32_t)((w >> 5) & 0x01010101u);
    hi[2] = (int32_t)((w >> 6) & 0x01010101u);
    hi[3] = (int32_t)((w >> 7) & 0x01010101u);
}
__device__ __forceinline__ void spread_i8_stored(uint32_t w, i32x4& lo, i32x4& hi) {  // stored order
    lo[0] = (int32_t)((w >> 2) & 0x01010101u);
    lo[1] = (int32_t)((w >> 1) & 0x01010101u);
    lo[2] = (int32_t)(w & 0x01010101u);
    lo[3] = (int32_t)((w >> 3) & 0x01010101u);
    hi[0] = (int32_t)((w >> 6) & 0x01010101u);
    hi[1] = (int32_t)((w >> 5) & 0x01010101u);
    hi[2] = (int32_t)((w >> 4) & 0x01010101u);
    hi[3] = (int32_t)((w >> 7) & 0x01010101u);
}

template <bool F4>
struct MfmaAcc;
template <>
struct MfmaAcc<true> {
    typedef f32x4 type;
};
template <>
struct MfmaAcc<false> {
    typedef i32x4 type;
};

// Operand reads of one K-step from an LDS stage: four database chunks at
// `b` + 0/1/2/3 KiB and MT selection quads at `a` + rt KiB.  The reads and
// their lgkmcnt wait sit in one asm block, so the values are complete when
// the block ends; the stage is known to be filled by the caller's vmcnt wait
// and barrier.
template <int MT>
__device__ __forceinline__ void lds_read_step(uint32_t b, uint32_t a, u32x4 (&bw)[4], u32x4 (&aw)[MT]) {
    if constexpr (MT == 1) {
        asm volatile(
            "ds_read_b128 %0, %5\n\t"
            "ds_read_b128 %1, %5 offset:1024\n\t"
            "ds_read_b128 %2, %5 offset:2048\n\t"
            "ds_read_b128 %3, %5 offset:3072\n\t"
            "ds_read_b128 %4, %6\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(bw[0]), "=&v"(bw[1]), "=&v"(bw[2]), "=&v"(bw[3]), "=&v"(aw[0])
            : "v"(b), "v"(a));
    } else if constexpr (MT == 2) {
        asm volatile(
            "ds_read_b128 %0, %6\n\t"
            "ds_read_b128 %1, %6 offset:1024\n\t"
            "ds_read_b128 %2, %6 offset:2048\n\t"
            "ds_read_b128 %3, %6 offset:3072\n\t"
            "ds_read_b128 %4, %7\n\t"
            "ds_read_b128 %5, %7 offset:1024\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(bw[0]), "=&v"(bw[1]), "=&v"(bw[2]), "=&v"(bw[3]), "=&v"(aw[0]), "=&v"(aw[1])
            : "v"(b), "v"(a));
    } else {
        static_assert(MT == 4, "row tiles");
        asm volatile(
            "ds_read_b128 %0, %8\n\t"
            "ds_read_b128 %1, %8 offset:1024\n\t"
            "ds_read_b128 %2, %8 offset:2048\n\t"
            "ds_read_b128 %3, %8 offset:3072\n\t"
            "ds_read_b128 %4, %9\n\t"
            "ds_read_b128 %5, %9 offset:1024\n\t"
            "ds_read_b128 %6, %9 offset:2048\n\t"
            "ds_read_b128 %7, %9 offset:3072\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(bw[0]), "=&v"(bw[1]), "=&v"(bw[2]), "=&v"(bw[3]), "=&v"(aw[0]), "=&v"(aw[1]),
              "=&v"(aw[2]), "=&v"(aw[3])
            : "v"(b), "v"(a));
    }
}

// Matrix-core scan with a multi-stage LDS ring.  Direct-to-LDS loads
// (global_load_lds_dwordx4 / _dword) stream the next S-1 K-steps of database
// chunks and selection words into LDS while the current K-step runs on the
// matrix cores, so the bytes in flight do not cost registers.  Per K-step a
// stage holds the workgroup's 16 blocks x 256 bit columns (16 KiB) and its
// 16*MT query rows x 16 selection words; the ring lives in dynamic LDS
// (up to 160 KiB on gfx950).  Each wave waits for its own loads of the step
// (vmcnt) and a barrier makes every wave's part visible; the same barrier
// tells the wave that refills a stage that everyone has read it.  Stage
// operands are read by lds_read_step, whose own lgkmcnt wait completes them.

template <int MT>
__host__ __device__ constexpr uint32_t ring_bytes(int stages) {
    return (uint32_t)stages * (kStageDbBytes + 16u * MT * 16u * 4u);
}

template <int MT, bool F4, int S>
__global__ void __launch_bounds__(kThreads)
k_stage1_mfma_lds(const uint32_t* __restrict__ db, const uint32_t* __restrict__ sel,
                  uint8_t* __restrict__ partials, Stage1Params p) {
    typedef typename MfmaAcc<F4>::type acc_t;
    constexpr int QT = 16 * MT;
    constexpr int kLoadsPerStep = 4 + MT;  // per wave: 4 database chunks + MT selection rows-of-4
    constexpr uint32_t kStageSelBytes = QT * 16 * 4;
    static_assert(S >= 2 && S <= 8, "ring stages");
    extern __shared__ __attribute__((aligned(16))) uint8_t pir_ring[];
    uint8_t* const ring_db = pir_ring;                        // S x [16 blocks][256 words]
    uint8_t* const ring_sel = pir_ring + S * kStageDbBytes;  // S x [QT rows][16 words]

    uint32_t group, ct, qt;
    if (!decode_block(p.groups, p.n_ct, p.n_qt, group, ct, qt)) return;

    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t j = lane & 15, g = lane >> 4;
    const uint32_t q0 = qt * QT;
    const uint64_t block_words = 8ull * p.R;

    // Query rows past q_total read row q0 (a valid row) and are never
    // written out, so the scan needs no per-step masking.
    //
    // loader geometry: database chunk of lane l = words 4l..4l+3 of the tile
    // (wave w loads blocks w, w+4, w+8, w+12 of the step); selection row
    // 4*(w + 4i) + l/16, word l%16 of the step
    const uint32_t* db_tile = db + ct * 256;  // wave-uniform base; lanes add 16 B each
    const uint32_t* sel_src[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        const uint32_t row = 4 * (wave + 4 * i) + lane / 16;  // 0 .. QT-1
        const uint32_t q = q0 + row < p.q_total ? q0 + row : q0;
        sel_src[i] = sel + (uint64_t)q * p.stride_words + (lane & 15);
    }
    auto issue = [&](uint64_t kb, uint32_t slot) {
        uint8_t* dst_db = ring_db + slot * kStageDbBytes;
        uint8_t* dst_sel = ring_sel + slot * kStageSelBytes;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t b = 4 * i + wave;
            const uint32_t* base = db_tile + (kb + b) * block_words;  // uniform
            // database chunks are read once: nontemporal (cache policy NT = 2)
            __builtin_amdgcn_global_load_lds(base + 4 * lane, dst_db + b * 1024, 16, 0, 2);
        }
#pragma unroll
        for (int i = 0; i < MT; ++i)
            __builtin_amdgcn_global_load_lds(sel_src[i] + kb, dst_sel + (wave + 4 * i) * 256, 4, 0, 0);
    };

    acc_t acc[MT][4];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[rt][t] = acc_t{0, 0, 0, 0};

    auto mma = [&](const u32x4 bw[4], const u32x4 aw4[MT]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (F4) {
                i32x8 bx[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) bx[t] = spread_fp4_b(bw[s][t]);
#pragma unroll
                for (int rt = 0; rt < MT; ++rt) {
                    const i32x8 ax = spread_fp4_a(aw4[rt][s]);
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        acc[rt][t] = (acc_t)mfma_fp4(ax, bx[t], (f32x4)acc[rt][t]);
                }
            } else {
                i32x4 blo[4], bhi[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) spread_i8_stored(bw[s][t], blo[t], bhi[t]);
#pragma unroll
                for (int rt = 0; rt < MT; ++rt) {
                    i32x4 alo, ahi;
                    spread_i8(aw4[rt][s], alo, ahi);
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        acc[rt][t] = (acc_t)__builtin_amdgcn_mfma_i32_16x16x64_i8(alo, blo[t], (i32x4)acc[rt][t], 0, 0, 0);
                        acc[rt][t] = (acc_t)__builtin_amdgcn_mfma_i32_16x16x64_i8(ahi, bhi[t], (i32x4)acc[rt][t], 0, 0, 0);
                    }
                }
            }
        }
    };
    // this lane's operand addresses inside stage 0; stage k adds k * stage size
    const uint32_t rd_db = (uint32_t)(uintptr_t)(ring_db + (4 * g) * 1024 + (64 * wave + 4 * j) * 4);
    const uint32_t rd_sel = (uint32_t)(uintptr_t)(ring_sel + j * 64 + (4 * g) * 4);
    auto compute_slot = [&](uint32_t slot) {
        u32x4 bw[4];
        u32x4 aw4[MT];
        lds_read_step<MT>(rd_db + slot * kStageDbBytes, rd_sel + slot * kStageSelBytes, bw, aw4);
        mma(bw, aw4);
    };

    const uint64_t b_begin = (uint64_t)group * p.units_per_group;
    const uint64_t b_end = (b_begin + p.units_per_group < p.n_units) ? b_begin + p.units_per_group : p.n_units;
    const uint64_t nsteps = (b_end - b_begin) / kMfmaBlocksPerStep;

    // prologue: steps 0 .. S-2 in flight
#pragma unroll
    for (int k = 0; k < S - 1; ++k)
        if ((uint64_t)k < nsteps) issue(b_begin + k * kMfmaBlocksPerStep, k);

    uint64_t k = 0;
    uint32_t slot = 0, fill = S - 1;  // stage of step k, stage that step k+S-1 loads into
    // Steady state: every step issues the load of step k+S-1; straight-line
    // body so the per-step scheduling barrier holds.
    for (; k + S - 1 < nsteps; ++k) {
        wait_vmcnt<(S - 2) * kLoadsPerStep>();  // own loads of step k have landed
        wg_barrier();                            // ... and everyone's; stage `fill` has been read
        issue(b_begin + (k + S - 1) * kMfmaBlocksPerStep, fill);
        compute_slot(slot);
        __builtin_amdgcn_sched_barrier(0);       // keep this step's matrix work here
        slot = slot + 1 == S ? 0 : slot + 1;
        fill = fill + 1 == S ? 0 : fill + 1;
    }
    // last S-1 steps: everything is already in flight
    wait_vmcnt<0>();
    wg_barrier();
    for (; k < nsteps; ++k) {
        compute_slot(slot);
        slot = slot + 1 == S ? 0 : slot + 1;
    }

    // ragged tail (fewer than 16 blocks) straight from memory
    const uint64_t kb = b_begin + nsteps * kMfmaBlocksPerStep;
    if (kb < b_end) {
        const u32x4* dl = reinterpret_cast<const u32x4*>(db + ct * 256 + wave * 64 + 4 * j);
        u32x4 bw[4], aw4[MT];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const uint64_t blk = kb + 4 * g + s;
            const bool ok = blk < b_end;
            bw[s] = ok ? dl[blk * (block_words / 4)] : u32x4{0, 0, 0, 0};
#pragma unroll
            for (int rt = 0; rt < MT; ++rt) {
                const uint32_t q = q0 + 16 * rt + j;
                aw4[rt][s] = (ok && q < p.q_total) ? sel[(uint64_t)q * p.stride_words + blk] : 0u;
            }
        }
        mma(bw, aw4);
    }

#pragma unroll
    for (int rt = 0; rt < MT; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            uint32_t nib = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t cnt = F4 ? (uint32_t)(float)acc[rt][t][r] : (uint32_t)acc[rt][t][r];
                nib |= (cnt & 1u) << t;
            }
            const uint32_t other = (uint32_t)__shfl_xor((int)nib, 1);
            const uint32_t q = q0 + 16 * rt + 4 * g + r;
            if ((j & 1) == 0 && q < p.q_total) {
                const uint32_t byte_pos = ct * 32 + wave * 8 + j / 2;
                partials[((uint64_t)group * p.q_total + q) * p.rpad + byte_pos] = (uint8_t)(nib | (other << 4));
            }
        }
}



// Operand reads of one K-step for the split-K kernel: two sub-steps of two
// database chunks (columns +0 and +64 words) at `b` and `b` + 1 KiB, and the
// two selection words of each of the four row tiles at `a` + rt KiB.
__device__ __forceinline__ void lds_read_ks(uint32_t b, uint32_t a, u32x4 (&bw)[4], u32x2 (&aw)[4]) {
    asm volatile(
        "ds_read_b128 %0, %8\n\t"
        "ds_read_b128 %1, %8 offset:256\n\t"
        "ds_read_b128 %2, %8 offset:1024\n\t"
        "ds_read_b128 %3, %8 offset:1280\n\t"
        "ds_read_b64 %4, %9\n\t"
        "ds_read_b64 %5, %9 offset:1024\n\t"
        "ds_read_b64 %6, %9 offset:2048\n\t"
        "ds_read_b64 %7, %9 offset:3072\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(bw[0]), "=&v"(bw[1]), "=&v"(bw[2]), "=&v"(bw[3]), "=&v"(aw[0]), "=&v"(aw[1]),
          "=&v"(aw[2]), "=&v"(aw[3])
        : "v"(b), "v"(a));
}

// ---- the contraction of one K-step of the split-K kernels, in issue order
//
// A wave's K-step is 64 products (2 sub-steps x 4 row tiles x 8 column
// tiles).  Each operand word is spread into E2M1 values by four "pieces"
// (spread_fp4_a/b: three masks and one shift-and-mask).  An in-order wave can
// issue vector-ALU work while the matrix core runs its previous product, but
// not ahead of a product it is waiting to issue, so the pieces are laid out
// between the products: the first sub-step's selection operands and its
// first database operand come first; then, column tile by column tile, each
// product is followed by one or two pieces of the operands the later
// products need (the next column tile of this sub-step, then the second
// sub-step's operands).  Scheduling barriers keep the compiler to this order.

// Spread operands of one K-step: a[sl][rt] (selection, row tile rt) and
// b[sl][t] (database, column tile t) for sub-step sl, E2M1 in four dwords.
struct KswOps {
    i32x4 a[2][4];
    i32x4 b[2][8];
};

__device__ __forceinline__ i32x8 widen(const i32x4& x) { return i32x8{x[0], x[1], x[2], x[3], 0, 0, 0, 0}; }

// piece P of spread_fp4_a / spread_fp4_b
template <int P>
__device__ __forceinline__ int32_t piece_a(uint32_t w) {
    if constexpr (P == 0) return (int32_t)(w & 0x11111111u);
    else if constexpr (P == 1) return (int32_t)(w & 0x22222222u);
    else if constexpr (P == 2) return (int32_t)(w & 0x44444444u);
    else return (int32_t)((w >> 1) & 0x44444444u);
}
template <int P>
__device__ __forceinline__ int32_t piece_b(uint32_t w) {
    if constexpr (P == 0) return (int32_t)(w & 0x44444444u);
    else if constexpr (P == 1) return (int32_t)(w & 0x22222222u);
    else if constexpr (P == 2) return (int32_t)(w & 0x11111111u);
    else return (int32_t)((w >> 3) & 0x11111111u);
}

// piece I (0..19) of sub-step SL's first operands: the selection operand of
// row tile I / 4 (I < 16), else the database operand of column tile 0
template <int SL, int I>
__device__ __forceinline__ void pro_piece(KswOps& o, const u32x4 (&bw)[4], const u32x2 (&aw)[4]) {
    if constexpr (I < 16) o.a[SL][I / 4][I % 4] = piece_a<I % 4>(aw[I / 4][SL]);
    else o.b[SL][0][I % 4] = piece_b<I % 4>(bw[2 * SL][0]);
}
// piece P of the database operand of sub-step SL, column tile T
template <int SL, int T, int P>
__device__ __forceinline__ void b_piece(KswOps& o, const u32x4 (&bw)[4]) {
    o.b[SL][T][P] = piece_b<P>(bw[2 * SL + (T >> 2)][T & 3]);
}
template <int SL, int I>
__device__ __forceinline__ void pro_all(KswOps& o, const u32x4 (&bw)[4], const u32x2 (&aw)[4]) {
    if constexpr (I < 20) {
        pro_piece<SL, I>(o, bw, aw);
        pro_all<SL, I + 1>(o, bw, aw);
    }
}
// piece K (0..5) issued among the first sub-step's products of column tile
// T: the next database operand (K < 4, T < 7), else the second sub-step's
// first operands
template <int T, int K>
__device__ __forceinline__ void group_piece(KswOps& o, const u32x4 (&bw)[4], const u32x2 (&aw)[4]) {
    if constexpr (T < 7 && K < 4) b_piece<0, T + 1, K>(o, bw);
    else if constexpr (T < 7) pro_piece<1, 2 * T + (K - 4)>(o, bw, aw);
    else pro_piece<1, 14 + K>(o, bw, aw);
}

// product M (sub-step M / 32, column tile M % 32 / 4, row tile M % 4), then
// its pieces: 2, 1, 2, 1 per column tile in the first sub-step, one (the next
// database operand's) in the second
template <int M>
__device__ __forceinline__ void ksw_sched(f32x4 (&acc)[4][8], KswOps& o, const u32x4 (&bw)[4], const u32x2 (&aw)[4]) {
    if constexpr (M < 64) {
        constexpr int sl = M / 32, t = (M % 32) / 4, rt = M % 4;
        acc[rt][t] = mfma_fp4(widen(o.a[sl][rt]), widen(o.b[sl][t]), acc[rt][t]);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (sl == 0) {
            constexpr int k0 = rt == 0 ? 0 : rt == 1 ? 2 : rt == 2 ? 3 : 5;
            group_piece<t, k0>(o, bw, aw);
            if constexpr (rt == 0 || rt == 2) group_piece<t, k0 + 1>(o, bw, aw);
        } else if constexpr (t < 7) {
            b_piece<1, t + 1, rt>(o, bw);
        }
        __builtin_amdgcn_sched_barrier(0);
        ksw_sched<M + 1>(acc, o, bw, aw);
    }
}

// acc[rt][t] += the K-step whose words are bw (database: bw[2*sl + half] for
// sub-step sl, columns 64*half + 4j ..) and aw (selection: aw[rt][sl])
__device__ __forceinline__ void ksw_step_sched(f32x4 (&acc)[4][8], const u32x4 (&bw)[4], const u32x2 (&aw)[4]) {
    KswOps o;
    pro_all<0, 0>(o, bw, aw);
    __builtin_amdgcn_sched_barrier(0);
    ksw_sched<0>(acc, o, bw, aw);
}

// The same K-step with `mid` issued between the first operands' spread and
// the first product (k_stage1_mfma_ksv issues its next loads there).
template <class F>
__device__ __forceinline__ void ksw_step_sched_mid(f32x4 (&acc)[4][8], const u32x4 (&bw)[4], const u32x2 (&aw)[4],
                                                   F&& mid) {
    KswOps o;
    pro_all<0, 0>(o, bw, aw);
    __builtin_amdgcn_sched_barrier(0);
    mid();
    __builtin_amdgcn_sched_barrier(0);
    ksw_sched<0>(acc, o, bw, aw);
}

// Split-K matrix-core scan (fp4, 64-query tiles).  The spread of an operand
// word costs vector-ALU issue slots that the matrix cores then lose, and a
// wave spreads (row tiles + column tiles) words per sub-step for
// (row tiles x column tiles) MFMAs.  Here a wave owns 128 bit columns
// (8 column tiles) instead of 64 and half of each K-step's blocks: wave w
// takes column half c = w & 1 and sub-steps 2h, 2h+1 with h = w >> 1.  Per
// K-step a wave spreads 2 x (8 + 4) words for 64 MFMAs instead of
// 4 x (4 + 4).  The two K halves of a column are combined at the end: the
// parity of a sum of counts is the XOR of their parities.
//
// Loads and the LDS ring are those of k_stage1_mfma_lds.  Each load's
// address is a wave-uniform base plus a fixed 32-bit lane offset; the
// selection offsets span three rows, which bounds the selection pitch
// (checked by the launcher).
template <int S, int DBP>
__global__ void __launch_bounds__(kThreads)
k_stage1_mfma_ks(const uint32_t* __restrict__ db, const uint32_t* __restrict__ sel,
                 uint8_t* __restrict__ partials, Stage1Params p) {
    constexpr int MT = 4, NT = 8, QT = 64;
    constexpr int kLoadsPerStep = 4 + MT;
    constexpr uint32_t kStageSelBytes = QT * 16 * 4;
    static_assert(S >= 2 && S <= 8, "ring stages");
    extern __shared__ __attribute__((aligned(16))) uint8_t pir_ring[];
    uint8_t* const ring_db = pir_ring;
    uint8_t* const ring_sel = pir_ring + S * kStageDbBytes;

    uint32_t group, ct, qt;
    if (!decode_block(p.groups, p.n_ct, p.n_qt, group, ct, qt)) return;

    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t c = wave & 1, h = wave >> 1;
    const uint32_t j = lane & 15, g = lane >> 4;
    const uint32_t q0 = qt * QT;
    const uint64_t block_words = 8ull * p.R;

    // loader geometry as in k_stage1_mfma_lds: wave w loads blocks w, w+4,
    // w+8, w+12 of a step (lane l: words 4l..4l+3) and selection rows
    // 4*(w + 4i) + l/16, word l%16.  A row past q_total reads the first row
    // of its group of four (or row q0), a valid row never written out.
    const uint8_t* db_tile = reinterpret_cast<const uint8_t*>(db + ct * 256);
    const uint32_t db_off = 16 * lane;
    const uint8_t* sel_base[MT];
    uint32_t sel_off[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        uint32_t r0 = q0 + 4 * (wave + 4 * i);
        const bool any = r0 < p.q_total;
        if (!any) r0 = q0;
        const uint32_t rl = (any && r0 + lane / 16 < p.q_total) ? lane / 16 : 0;
        sel_base[i] = reinterpret_cast<const uint8_t*>(sel + (uint64_t)r0 * p.stride_words);
        sel_off[i] = rl * (uint32_t)(p.stride_words * 4) + 4 * (lane & 15);
    }
    auto issue = [&](uint64_t kb, uint32_t slot) {
        uint8_t* dst_db = ring_db + slot * kStageDbBytes;
        uint8_t* dst_sel = ring_sel + slot * kStageSelBytes;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t b = 4 * i + wave;
            const uint8_t* base = uniform_ptr(db_tile + (kb + b) * block_words * 4);
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint32_t*>(base + db_off),
                                             dst_db + b * 1024, 16, 0, DBP);
        }
#pragma unroll
        for (int i = 0; i < MT; ++i)
            __builtin_amdgcn_global_load_lds(
                reinterpret_cast<const uint32_t*>(uniform_ptr(sel_base[i] + kb * 4) + sel_off[i]),
                dst_sel + (wave + 4 * i) * 256, 4, 0, 0);
    };

    f32x4 acc[MT][NT];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[rt][t] = f32x4{0, 0, 0, 0};

    // bw[2*sl + half]: sub-step 2h + sl, columns 128c + 64*half + 4j .. +3;
    // aw[rt][sl]: selection word of row 16rt + j for that sub-step
    auto mma = [&](const u32x4 (&bw)[4], const u32x2 (&aw)[MT]) { ksw_step_sched(acc, bw, aw); };
    const uint32_t rd_db =
        (uint32_t)(uintptr_t)(ring_db + (4 * g + 2 * h) * 1024 + (128 * c + 4 * j) * 4);
    const uint32_t rd_sel = (uint32_t)(uintptr_t)(ring_sel + j * 64 + (4 * g + 2 * h) * 4);
    auto compute_slot = [&](uint32_t slot) {
        u32x4 bw[4];
        u32x2 aw[MT];
        lds_read_ks(rd_db + slot * kStageDbBytes, rd_sel + slot * kStageSelBytes, bw, aw);
        mma(bw, aw);
    };
    const uint64_t b_begin = (uint64_t)group * p.units_per_group;
    const uint64_t b_end = (b_begin + p.units_per_group < p.n_units) ? b_begin + p.units_per_group : p.n_units;
    const uint64_t nsteps = (b_end - b_begin) / kMfmaBlocksPerStep;

#pragma unroll
    for (int k = 0; k < S - 1; ++k)
        if ((uint64_t)k < nsteps) issue(b_begin + k * kMfmaBlocksPerStep, k);

    uint64_t k = 0;
    uint32_t slot = 0, fill = S - 1;
    for (; k + S - 1 < nsteps; ++k) {
        wait_vmcnt<(S - 2) * kLoadsPerStep>();
        wg_barrier();
        issue(b_begin + (k + S - 1) * kMfmaBlocksPerStep, fill);
        compute_slot(slot);
        __builtin_amdgcn_sched_barrier(0);
        slot = slot + 1 == S ? 0 : slot + 1;
        fill = fill + 1 == S ? 0 : fill + 1;
    }
    wait_vmcnt<0>();
    wg_barrier();
    for (; k < nsteps; ++k) {
        compute_slot(slot);
        slot = slot + 1 == S ? 0 : slot + 1;
    }

    // ragged tail (fewer than 16 blocks) straight from memory
    const uint64_t kb = b_begin + nsteps * kMfmaBlocksPerStep;
    if (kb < b_end) {
        const u32x4* dl = reinterpret_cast<const u32x4*>(db + ct * 256 + 128 * c + 4 * j);
        u32x4 bw[4];
        u32x2 aw[MT];
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
            const uint64_t blk = kb + 4 * g + 2 * h + sl;
            const bool ok = blk < b_end;
            bw[2 * sl] = ok ? dl[blk * (block_words / 4)] : u32x4{0, 0, 0, 0};
            bw[2 * sl + 1] = ok ? dl[blk * (block_words / 4) + 16] : u32x4{0, 0, 0, 0};
#pragma unroll
            for (int rt = 0; rt < MT; ++rt) {
                const uint32_t q = q0 + 16 * rt + j;
                aw[rt][sl] = (ok && q < p.q_total) ? sel[(uint64_t)q * p.stride_words + blk] : 0u;
            }
        }
        mma(bw, aw);
    }

    // answer bits: lane holds columns 128c + 64*half + 4j + t' of rows
    // 16rt + 4g + r; bit 8r + 4*half + t' of par[rt]
    uint32_t par[MT];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt) {
        par[rt] = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < NT; ++t) par[rt] |= (((uint32_t)acc[rt][t][r]) & 1u) << (8 * r + t);
    }
    // fold the K halves through LDS (the ring is idle: every load has landed
    // and, after this barrier, every wave has read its last stage)
    __syncthreads();
    u32x4* fold = reinterpret_cast<u32x4*>(pir_ring) + c * 64 + lane;
    if (h == 1) *fold = u32x4{par[0], par[1], par[2], par[3]};
    __syncthreads();  // the fold writes are complete and visible
    if (h == 1) return;
    const u32x4 o = *fold;
    par[0] ^= o[0];
    par[1] ^= o[1];
    par[2] ^= o[2];
    par[3] ^= o[3];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt) {
        const uint32_t other = (uint32_t)__shfl_xor((int)par[rt], 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t q = q0 + 16 * rt + 4 * g + r;
            const uint32_t mine = par[rt] >> (8 * r), theirs = other >> (8 * r);
            if ((j & 1) == 0 && q < p.q_total) {
                uint8_t* dst = partials + ((uint64_t)group * p.q_total + q) * p.rpad + ct * 32 + 16 * c + j / 2;
                dst[0] = (uint8_t)((mine & 0xF) | ((theirs & 0xF) << 4));
                dst[8] = (uint8_t)(((mine >> 4) & 0xF) | (theirs & 0xF0));
            }
        }
    }
}

// Split-K kernel with wide selection reads: the database ring is that of
// k_stage1_mfma_ks (2 stages of 16 blocks), while the selection words move
// in stages of 4 K-steps, 256 contiguous bytes per query row (two whole
// 128-byte lines instead of half a line per row and step), double-buffered.
// A selection stage holds rows 4i .. 4i+3 at i * kWsRowGroup (one 1 KiB
// load, 64 bytes of padding after it), row r's 16-byte chunk c at
// (r & 3) * 256 + 16 * (c ^ (r & 3)) within its group.
constexpr uint32_t kWsRowGroup = 1024 + 64;
constexpr uint32_t kWsStageSelBytes = 16 * kWsRowGroup;
constexpr uint32_t kWsLdsBytes = 2 * kStageDbBytes + 2 * kWsStageSelBytes;

// Largest selection pitch (32-bit words) for which the wide loads' lane
// offsets, up to three rows plus 256 bytes, fit in 32 bits.
constexpr uint64_t kWsMaxStrideWords = ((1ull << 32) - 256) / 12;

// Operand reads of one K-step for k_stage1_mfma_ksw: the database chunks as
// in lds_read_ks, and both sub-steps' selection words of each row tile at
// `a` + rt * 4 * kWsRowGroup.
__device__ __forceinline__ void lds_read_ksw(uint32_t b, uint32_t a, u32x4 (&bw)[4], u32x2 (&aw)[4]) {
    asm volatile(
        "ds_read_b128 %0, %8\n\t"
        "ds_read_b128 %1, %8 offset:256\n\t"
        "ds_read_b128 %2, %8 offset:1024\n\t"
        "ds_read_b128 %3, %8 offset:1280\n\t"
        "ds_read_b64 %4, %9\n\t"
        "ds_read_b64 %5, %9 offset:4352\n\t"
        "ds_read_b64 %6, %9 offset:8704\n\t"
        "ds_read_b64 %7, %9 offset:13056\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(bw[0]), "=&v"(bw[1]), "=&v"(bw[2]), "=&v"(bw[3]), "=&v"(aw[0]), "=&v"(aw[1]),
          "=&v"(aw[2]), "=&v"(aw[3])
        : "v"(b), "v"(a));
}
static_assert(4 * kWsRowGroup == 4352, "row-tile offset in lds_read_ksw");

// The database loads and the K-half fold are those of k_stage1_mfma_ks<2>;
// the contraction is ksw_step_sched.  Selection stage 0 is loaded before the
// first step and stage m + 1 during the steps of stage m, one 1 KiB load per
// wave and step (load 4s + w in step s by wave w); the steps of the last
// stage load no selection words.  Each step waits for all of its wave's
// earlier loads and then meets the others at a barrier, as in the 2-stage
// ring.
template <int DBP>
__global__ void __launch_bounds__(kThreads)
k_stage1_mfma_ksw(const uint32_t* __restrict__ db, const uint32_t* __restrict__ sel,
                  uint8_t* __restrict__ partials, Stage1Params p) {
    constexpr int MT = 4, NT = 8, QT = 64;
    constexpr uint32_t RG = kWsRowGroup, kSelStage = kWsStageSelBytes;
    extern __shared__ __attribute__((aligned(16))) uint8_t pir_ring[];
    uint8_t* const ring_db = pir_ring;
    uint8_t* const ring_sel = pir_ring + 2 * kStageDbBytes;

    uint32_t group, ct, qt;
    if (!decode_block(p.groups, p.n_ct, p.n_qt, group, ct, qt)) return;

    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t c = wave & 1, h = wave >> 1;
    const uint32_t j = lane & 15, g = lane >> 4;
    const uint32_t q0 = qt * QT;
    const uint64_t block_words = 8ull * p.R;
    const uint64_t b_begin = (uint64_t)group * p.units_per_group;
    const uint64_t b_end = (b_begin + p.units_per_group < p.n_units) ? b_begin + p.units_per_group : p.n_units;
    const uint32_t nsteps = (uint32_t)((b_end - b_begin) / kMfmaBlocksPerStep);

    // database: wave w loads blocks w, w+4, w+8, w+12 of a step (lane l:
    // words 4l..4l+3 of the tile)
    const uint8_t* db_tile = reinterpret_cast<const uint8_t*>(db + ct * 256);
    const uint32_t db_off = 16 * lane;
    auto issue_db = [&](uint32_t k, uint32_t slot) {
        uint8_t* dst = ring_db + slot * kStageDbBytes;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t b = 4 * i + wave;
            const uint8_t* base =
                uniform_ptr(db_tile + (b_begin + (uint64_t)k * kMfmaBlocksPerStep + b) * block_words * 4);
            // cache policy DBP: nontemporal (2) when one query tile reads each
            // database chunk once, default (0) when several tiles' workgroups
            // read it in turn through L2
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint32_t*>(base + db_off), dst + b * 1024, 16,
                                             0, DBP);
        }
    };

    // selection load 4s + w covers rows r0 = q0 + 4(4s + w) .. +3; lane l
    // reads row r0 + l/16, chunk (l & 15) ^ (l >> 4).  A row past q_total
    // reads the first row of its load (or row q0), a valid row never
    // written out.
    const uint32_t ch = (lane & 15) ^ (lane >> 4);
    const uint8_t* sel_row[4];
    uint32_t sel_off[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        uint32_t r0 = q0 + 4 * (4 * st + wave);
        const bool any = r0 < p.q_total;
        if (!any) r0 = q0;
        const uint32_t rl = (any && r0 + lane / 16 < p.q_total) ? lane / 16 : 0;
        sel_row[st] = reinterpret_cast<const uint8_t*>(sel + (uint64_t)r0 * p.stride_words + b_begin);
        sel_off[st] = rl * (uint32_t)(p.stride_words * 4) + 16 * ch;
    }
    // a chunk of a K-step past the group's last full step re-reads the same
    // position of the stage's first step (valid, never used)
    auto issue_sel = [&](uint32_t m, int st) {
        uint32_t off = sel_off[st];
        if (4 * m + 3 >= nsteps && 4 * m + (ch >> 2) >= nsteps) off -= 16 * (ch & ~3u);
        // whole lines of each row, read once: nontemporal (the 4-byte loads
        // of the ring kernels take half a line per step and keep the default)
        __builtin_amdgcn_global_load_lds(
            reinterpret_cast<const uint32_t*>(uniform_ptr(sel_row[st] + (uint64_t)m * 256) + off),
            ring_sel + (m & 1) * kSelStage + (4 * st + wave) * RG, 16, 0, 2);
    };

    f32x4 acc[MT][NT];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[rt][t] = f32x4{0, 0, 0, 0};

    // bw[2*sl + half]: sub-step 2h + sl, columns 128c + 64*half + 4j .. +3;
    // aw[rt][sl]: selection word of row 16rt + j for that sub-step
    auto mma = [&](const u32x4 (&bw)[4], const u32x2 (&aw)[MT]) { ksw_step_sched(acc, bw, aw); };
    const uint32_t rd_db =
        (uint32_t)(uintptr_t)(ring_db + (4 * g + 2 * h) * 1024 + (128 * c + 4 * j) * 4);
    // row 16rt + j, word 16s + 4g + 2h (chunk 4s + g) of stage buffer m & 1
    const uint32_t rd_sel = (uint32_t)(uintptr_t)(ring_sel + (j >> 2) * RG + (j & 3) * 256 +
                                                  16 * (g ^ (j & 3)) + 8 * h);

    if (nsteps > 0) {
#pragma unroll
        for (int st = 0; st < 4; ++st) issue_sel(0, st);
        issue_db(0, 0);
    }
    for (uint32_t m = 0; 4 * m < nsteps; ++m) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const uint32_t k = 4 * m + st;
            if (k >= nsteps) break;
            wait_vmcnt<0>();  // this wave's loads of step k (and of stage m) have landed
            wg_barrier();     // ... and everyone's; step k - 1's stages have been read
            if (k + 1 < nsteps) issue_db(k + 1, (k + 1) & 1);
            if (4 * (m + 1) < nsteps) issue_sel(m + 1, st);
            u32x4 bw[4];
            u32x2 aw[MT];
            lds_read_ksw(rd_db + (k & 1) * kStageDbBytes, rd_sel + (m & 1) * kSelStage + 64 * st, bw, aw);
            mma(bw, aw);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    wait_vmcnt<0>();

    // ragged tail (fewer than 16 blocks) straight from memory
    const uint64_t kb = b_begin + (uint64_t)nsteps * kMfmaBlocksPerStep;
    if (kb < b_end) {
        const u32x4* dl = reinterpret_cast<const u32x4*>(db + ct * 256 + 128 * c + 4 * j);
        u32x4 bw[4];
        u32x2 aw[MT];
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
            const uint64_t blk = kb + 4 * g + 2 * h + sl;
            const bool ok = blk < b_end;
            bw[2 * sl] = ok ? dl[blk * (block_words / 4)] : u32x4{0, 0, 0, 0};
            bw[2 * sl + 1] = ok ? dl[blk * (block_words / 4) + 16] : u32x4{0, 0, 0, 0};
#pragma unroll
            for (int rt = 0; rt < MT; ++rt) {
                const uint32_t q = q0 + 16 * rt + j;
                aw[rt][sl] = (ok && q < p.q_total) ? sel[(uint64_t)q * p.stride_words + blk] : 0u;
            }
        }
        mma(bw, aw);
    }

    // answer bits: lane holds columns 128c + 64*half + 4j + t' of rows
    // 16rt + 4g + r; bit 8r + 4*half + t' of par[rt]
    uint32_t par[MT];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt) {
        par[rt] = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < NT; ++t) par[rt] |= (((uint32_t)acc[rt][t][r]) & 1u) << (8 * r + t);
    }
    // fold the K halves through LDS (every load has landed and, after this
    // barrier, every wave has read its last stage)
    __syncthreads();
    u32x4* fold = reinterpret_cast<u32x4*>(pir_ring) + c * 64 + lane;
    if (h == 1) *fold = u32x4{par[0], par[1], par[2], par[3]};
    __syncthreads();  // the fold writes are complete and visible
    if (h == 1) return;
    const u32x4 o = *fold;
    par[0] ^= o[0];
    par[1] ^= o[1];
    par[2] ^= o[2];
    par[3] ^= o[3];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt) {
        const uint32_t other = (uint32_t)__shfl_xor((int)par[rt], 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t q = q0 + 16 * rt + 4 * g + r;
            const uint32_t mine = par[rt] >> (8 * r), theirs = other >> (8 * r);
            if ((j & 1) == 0 && q < p.q_total) {
                uint8_t* dst = partials + ((uint64_t)group * p.q_total + q) * p.rpad + ct * 32 + 16 * c + j / 2;
                dst[0] = (uint8_t)((mine & 0xF) | ((theirs & 0xF) << 4));
                dst[8] = (uint8_t)(((mine >> 4) & 0xF) | (theirs & 0xF0));
            }
        }
    }
}

// Split-K kernel with wave-private database stages: each wave's quarter of a
// K-step's database words (its K half: blocks 4g + 2h + sl; its 128 columns)
// is read by that wave alone, so each wave streams it into its own two-slot
// LDS ring, one K-step ahead, and waits only for its own loads: no barrier
// per K-step.  The selection words, shared by the two waves of a K
// half, move in the stages of k_stage1_mfma_ksw (4 K-steps, double-buffered),
// issued at the first step of the stage before; the waves meet at a barrier
// once per stage.
constexpr uint32_t kSpLdsBytes = 2 * kWsStageSelBytes + 4 * 2 * 4096;

template <int DBP>
__global__ void __launch_bounds__(kThreads)
k_stage1_mfma_ksp(const uint32_t* __restrict__ db, const uint32_t* __restrict__ sel,
                  uint8_t* __restrict__ partials, Stage1Params p) {
    constexpr int MT = 4, NT = 8, QT = 64;
    constexpr uint32_t RG = kWsRowGroup, kSelStage = kWsStageSelBytes;
    extern __shared__ __attribute__((aligned(16))) uint8_t pir_ring[];
    uint8_t* const ring_sel = pir_ring;

    uint32_t group, ct, qt;
    if (!decode_block(p.groups, p.n_ct, p.n_qt, group, ct, qt)) return;

    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t c = wave & 1, h = wave >> 1;
    const uint32_t j = lane & 15, g = lane >> 4;
    const uint32_t q0 = qt * QT;
    const uint64_t block_words = 8ull * p.R;
    const uint64_t b_begin = (uint64_t)group * p.units_per_group;
    const uint64_t b_end = (b_begin + p.units_per_group < p.n_units) ? b_begin + p.units_per_group : p.n_units;
    const uint32_t nsteps = (uint32_t)((b_end - b_begin) / kMfmaBlocksPerStep);

    // this wave's ring: slot s at ring_db + s * 4096; load i of a step puts
    // block 4i + 2h + sl (sl = lane / 32), words 128c + 4(lane % 32) .. +3,
    // at i * 1024 + 16 * lane
    uint8_t* const ring_db = pir_ring + 2 * kSelStage + wave * (2 * 4096);
    const uint8_t* db_wave = reinterpret_cast<const uint8_t*>(db + ct * 256 + (b_begin + 2 * h) * block_words + 128 * c);
    const uint32_t db_lane = (uint32_t)((lane >> 5) * block_words * 4 + 16 * (lane & 31));
    auto issue_db = [&](uint32_t k, uint32_t slot) {
        uint8_t* dst = ring_db + slot * 4096;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint8_t* base =
                uniform_ptr(db_wave + ((uint64_t)k * kMfmaBlocksPerStep + 4 * i) * block_words * 4);
            // cache policy DBP, as in k_stage1_mfma_ksw
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint32_t*>(base + db_lane), dst + i * 1024, 16,
                                             0, DBP);
        }
    };

    // selection loads as in k_stage1_mfma_ksw: load 4s + w of a stage covers
    // rows q0 + 4(4s + w) .. +3; stage m goes to buffer m & 1
    const uint32_t ch = (lane & 15) ^ (lane >> 4);
    const uint8_t* sel_row[4];
    uint32_t sel_off[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        uint32_t r0 = q0 + 4 * (4 * st + wave);
        const bool any = r0 < p.q_total;
        if (!any) r0 = q0;
        const uint32_t rl = (any && r0 + lane / 16 < p.q_total) ? lane / 16 : 0;
        sel_row[st] = reinterpret_cast<const uint8_t*>(sel + (uint64_t)r0 * p.stride_words + b_begin);
        sel_off[st] = rl * (uint32_t)(p.stride_words * 4) + 16 * ch;
    }
    // a chunk of a K-step past the group's last full step re-reads the same
    // position of the stage's first step (valid, never used)
    auto issue_sel = [&](uint32_t m) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            uint32_t off = sel_off[st];
            if (4 * m + 3 >= nsteps && 4 * m + (ch >> 2) >= nsteps) off -= 16 * (ch & ~3u);
            // whole lines of each row, read once: nontemporal
            __builtin_amdgcn_global_load_lds(
                reinterpret_cast<const uint32_t*>(uniform_ptr(sel_row[st] + (uint64_t)m * 256) + off),
                ring_sel + (m & 1) * kSelStage + (4 * st + wave) * RG, 16, 0, 2);
        }
    };

    f32x4 acc[MT][NT];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[rt][t] = f32x4{0, 0, 0, 0};

    auto mma = [&](const u32x4 (&bw)[4], const u32x2 (&aw)[MT]) { ksw_step_sched(acc, bw, aw); };
    // bw[2*sl + half] (block 4g + 2h + sl, words 128c + 64*half + 4j) at
    // g * 1024 + sl * 512 + half * 256 + 16j of a slot
    const uint32_t rd_db = (uint32_t)(uintptr_t)(ring_db + g * 1024 + 16 * j);
    // row 16rt + j, word 16s + 4g + 2h (chunk 4s + g) of stage buffer m & 1
    const uint32_t rd_sel = (uint32_t)(uintptr_t)(ring_sel + (j >> 2) * RG + (j & 3) * 256 +
                                                  16 * (g ^ (j & 3)) + 8 * h);
    auto read_ops = [&](uint32_t b, uint32_t a, u32x4 (&bw)[4], u32x2 (&aw)[MT]) {
        asm volatile(
            "ds_read_b128 %0, %8\n\t"
            "ds_read_b128 %1, %8 offset:256\n\t"
            "ds_read_b128 %2, %8 offset:512\n\t"
            "ds_read_b128 %3, %8 offset:768\n\t"
            "ds_read_b64 %4, %9\n\t"
            "ds_read_b64 %5, %9 offset:4352\n\t"
            "ds_read_b64 %6, %9 offset:8704\n\t"
            "ds_read_b64 %7, %9 offset:13056\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(bw[0]), "=&v"(bw[1]), "=&v"(bw[2]), "=&v"(bw[3]), "=&v"(aw[0]), "=&v"(aw[1]),
              "=&v"(aw[2]), "=&v"(aw[3])
            : "v"(b), "v"(a));
    };

    if (nsteps > 0) {
        issue_sel(0);
        issue_db(0, 0);
    }
    for (uint32_t m = 0; 4 * m < nsteps; ++m) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const uint32_t k = 4 * m + st;
            if (k >= nsteps) break;
            // this wave's database loads of step k were its last: all of its
            // loads have landed (the selection loads of stage m with them)
            wait_vmcnt<0>();
            if (st == 0) {
                // ... for every wave; stage m - 1's buffer has been read
                wg_barrier();
                if (4 * (m + 1) < nsteps) issue_sel(m + 1);
            }
            if (k + 1 < nsteps) issue_db(k + 1, (k + 1) & 1);
            u32x4 bw[4];
            u32x2 aw[MT];
            read_ops(rd_db + (k & 1) * 4096, rd_sel + (m & 1) * kSelStage + 64 * st, bw, aw);
            mma(bw, aw);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    wait_vmcnt<0>();

    // ragged tail (fewer than 16 blocks) straight from memory
    const uint64_t kb = b_begin + (uint64_t)nsteps * kMfmaBlocksPerStep;
    if (kb < b_end) {
        const u32x4* dl = reinterpret_cast<const u32x4*>(db + ct * 256 + 128 * c + 4 * j);
        u32x4 bw[4];
        u32x2 aw[MT];
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
            const uint64_t blk = kb + 4 * g + 2 * h + sl;
            const bool ok = blk < b_end;
            bw[2 * sl] = ok ? dl[blk * (block_words / 4)] : u32x4{0, 0, 0, 0};
            bw[2 * sl + 1] = ok ? dl[blk * (block_words / 4) + 16] : u32x4{0, 0, 0, 0};
#pragma unroll
            for (int rt = 0; rt < MT; ++rt) {
                const uint32_t q = q0 + 16 * rt + j;
                aw[rt][sl] = (ok && q < p.q_total) ? sel[(uint64_t)q * p.stride_words + blk] : 0u;
            }
        }
        mma(bw, aw);
    }

    // answer bits: lane holds columns 128c + 64*half + 4j + t' of rows
    // 16rt + 4g + r; bit 8r + 4*half + t' of par[rt]
    uint32_t par[MT];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt) {
        par[rt] = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < NT; ++t) par[rt] |= (((uint32_t)acc[rt][t][r]) & 1u) << (8 * r + t);
    }
    // fold the K halves through LDS (every load has landed and, after this
    // barrier, every wave has read its last stage)
    __syncthreads();
    u32x4* fold = reinterpret_cast<u32x4*>(pir_ring) + c * 64 + lane;
    if (h == 1) *fold = u32x4{par[0], par[1], par[2], par[3]};
    __syncthreads();  // the fold writes are complete and visible
    if (h == 1) return;
    const u32x4 o = *fold;
    par[0] ^= o[0];
    par[1] ^= o[1];
    par[2] ^= o[2];
    par[3] ^= o[3];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt) {
        const uint32_t other = (uint32_t)__shfl_xor((int)par[rt], 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t q = q0 + 16 * rt + 4 * g + r;
            const uint32_t mine = par[rt] >> (8 * r), theirs = other >> (8 * r);
            if ((j & 1) == 0 && q < p.q_total) {
                uint8_t* dst = partials + ((uint64_t)group * p.q_total + q) * p.rpad + ct * 32 + 16 * c + j / 2;
                dst[0] = (uint8_t)((mine & 0xF) | ((theirs & 0xF) << 4));
                dst[8] = (uint8_t)(((mine >> 4) & 0xF) | (theirs & 0xF0));
            }
        }
    }
}

// Split-K kernel with the database words loaded straight into registers.
// Each wave's database words (its K half, its 128 columns) are used by that
// wave alone, so instead of staging them through LDS (k_stage1_mfma_ksp) it
// loads them into the registers the products read, one K-step ahead: no LDS
// write and read-back per word.  The selection stages stay shared (four
// K-steps, 256 bytes per row, double-buffered), but they too arrive through
// registers (the same 16-byte chunks, then written to the stage buffer at
// the end of the stage before): with no direct-to-LDS load in flight the
// compiler counts the outstanding loads in order and waits only for the one
// an operand needs.  The next step's loads are issued after the first
// operands' spread, behind the compiler's wait for this step's words, and
// unconditionally: the group's last step is peeled off the loop.
constexpr uint32_t kSvLdsBytes = 2 * kWsStageSelBytes;

// Word 3 of a buffer resource for raw 32-bit loads on gfx950: DATA_FORMAT
// (bits 15-18) = 4, the 32-bit format; no swizzle, no index stride.
constexpr int kRawBufferWord3 = 0x00020000;

template <int DBP>
__global__ void __launch_bounds__(kThreads)
k_stage1_mfma_ksv(const uint32_t* __restrict__ db, const uint32_t* __restrict__ sel,
                  uint8_t* __restrict__ partials, Stage1Params p) {
    constexpr int MT = 4, NT = 8, QT = 64;
    constexpr uint32_t RG = kWsRowGroup, kSelStage = kWsStageSelBytes;
    extern __shared__ __attribute__((aligned(16))) uint8_t pir_ring[];
    uint8_t* const ring_sel = pir_ring;

    uint32_t group, ct, qt;
    if (!decode_block(p.groups, p.n_ct, p.n_qt, group, ct, qt)) return;

    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t c = wave & 1, h = wave >> 1;
    const uint32_t j = lane & 15, g = lane >> 4;
    const uint32_t q0 = qt * QT;
    const uint64_t block_words = 8ull * p.R;
    const uint64_t b_begin = (uint64_t)group * p.units_per_group;
    const uint64_t b_end = (b_begin + p.units_per_group < p.n_units) ? b_begin + p.units_per_group : p.n_units;
    const uint32_t nsteps = (uint32_t)((b_end - b_begin) / kMfmaBlocksPerStep);

    // database: lane (j, g) takes bw[2*sl + half] = block 4g + 2h + sl of the
    // step, words 128c + 64*half + 4j .. +3 (the operand layout of
    // ksw_step_sched).  Buffer loads: the record group's range of this column
    // tile is one buffer (base in scalar registers; launch_ksv keeps it under
    // 4 GiB), a lane's offset one 32-bit register, the second block of a pair
    // a scalar offset and the second half an immediate one, so a K-step's
    // addresses cost one 32-bit add (global loads take 64-bit adds).  Cache
    // policy DBP: 2 (non-temporal) for one query tile, 0 for several.
    const __amdgpu_buffer_rsrc_t db_rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(db + ct * 256 + b_begin * block_words), (short)0,
        (int)(uint32_t)((b_end - b_begin) * block_words * 4), kRawBufferWord3);
    const uint32_t db_lane = (uint32_t)(((4 * g + 2 * h) * block_words + 128 * c + 4 * j) * 4);
    const uint32_t db_step = (uint32_t)(kMfmaBlocksPerStep * block_words * 4);
    const uint32_t db_blk = (uint32_t)(block_words * 4);
    auto load_db = [&](uint32_t k, u32x4 (&w)[4]) {
        const uint32_t vo = db_lane + k * db_step;
        w[0] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(db_rsrc, vo, 0, DBP));
        w[1] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(db_rsrc, vo + 256, 0, DBP));
        w[2] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(db_rsrc, vo, db_blk, DBP));
        w[3] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(db_rsrc, vo + 256, db_blk, DBP));
    };

    // selection chunks as in k_stage1_mfma_ksw: chunk 4s + w of a stage is
    // rows q0 + 4(4s + w) .. +3; lane l takes chunk (l & 15) ^ (l >> 4) of
    // row l >> 4 and stores it at position l & 15 of that row
    const uint32_t ch = (lane & 15) ^ (lane >> 4);
    const uint8_t* sel_row[4];
    uint32_t sel_off[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        uint32_t r0 = q0 + 4 * (4 * st + wave);
        const bool any = r0 < p.q_total;
        if (!any) r0 = q0;
        const uint32_t rl = (any && r0 + lane / 16 < p.q_total) ? lane / 16 : 0;
        sel_row[st] = reinterpret_cast<const uint8_t*>(sel + (uint64_t)r0 * p.stride_words + b_begin);
        sel_off[st] = rl * (uint32_t)(p.stride_words * 4) + 16 * ch;
    }
    // a chunk of a K-step past the group's last full step re-reads the same
    // position of the stage's first step (valid, never used); whole lines of
    // each row, read once: nontemporal
    auto load_sel = [&](uint32_t m, u32x4 (&sv)[4]) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            uint32_t off = sel_off[st];
            if (4 * m + 3 >= nsteps && 4 * m + (ch >> 2) >= nsteps) off -= 16 * (ch & ~3u);
            sv[st] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(sel_row[st] + (uint64_t)m * 256 + off));
        }
    };
    auto store_sel = [&](uint32_t m, const u32x4 (&sv)[4]) {
#pragma unroll
        for (int st = 0; st < 4; ++st)
            *reinterpret_cast<u32x4*>(ring_sel + (m & 1) * kSelStage + (4 * st + wave) * RG + 16 * lane) = sv[st];
    };

    f32x4 acc[MT][NT];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[rt][t] = f32x4{0, 0, 0, 0};

    auto mma = [&](const u32x4 (&bw)[4], const u32x2 (&aw)[MT]) { ksw_step_sched(acc, bw, aw); };
    // row 16rt + j, word 16s + 4g + 2h (chunk 4s + g) of stage buffer m & 1
    const uint32_t rd_sel = (uint32_t)(uintptr_t)(ring_sel + (j >> 2) * RG + (j & 3) * 256 +
                                                  16 * (g ^ (j & 3)) + 8 * h);
    auto read_sel = [&](uint32_t a, u32x2 (&aw)[MT]) {
        asm volatile(
            "ds_read_b64 %0, %4\n\t"
            "ds_read_b64 %1, %4 offset:4352\n\t"
            "ds_read_b64 %2, %4 offset:8704\n\t"
            "ds_read_b64 %3, %4 offset:13056\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(aw[0]), "=&v"(aw[1]), "=&v"(aw[2]), "=&v"(aw[3])
            : "v"(a));
    };

    u32x4 bwc[4], svn[4];
    if (nsteps > 0) {
        u32x4 sv0[4];
        load_sel(0, sv0);
        store_sel(0, sv0);
        load_db(0, bwc);
        if (4 < nsteps) load_sel(1, svn);
    }
    // every step but the group's last loads the next step's database words;
    // the last one runs after the loop and loads nothing
    for (uint32_t m = 0; 4 * m < nsteps; ++m) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const uint32_t k = 4 * m + st;
            if (k + 1 >= nsteps) break;
            if (st == 0) {
                // this wave's stores of stage m are done ...
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
                // ... and every wave's; stage m - 1's buffer has been read
                wg_barrier();
            }
            u32x2 aw[MT];
            read_sel(rd_sel + (m & 1) * kSelStage + 64 * st, aw);
            u32x4 bwn[4];
            ksw_step_sched_mid(acc, bwc, aw, [&] { load_db(k + 1, bwn); });
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 4; ++i) bwc[i] = bwn[i];
            if (st == 3 && 4 * (m + 1) < nsteps) {
                // stage m + 1 into the buffer of stage m - 1, which every
                // wave has read (all passed this stage's barrier)
                store_sel(m + 1, svn);
                if (4 * (m + 2) < nsteps) load_sel(m + 2, svn);
            }
        }
    }
    if (nsteps > 0) {
        const uint32_t k = nsteps - 1, m = k / 4, st = k % 4;
        if (st == 0) {
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            wg_barrier();
        }
        u32x2 aw[MT];
        read_sel(rd_sel + (m & 1) * kSelStage + 64 * st, aw);
        mma(bwc, aw);
        __builtin_amdgcn_sched_barrier(0);
    }
    wait_vmcnt<0>();

    // ragged tail (fewer than 16 blocks) straight from memory
    const uint64_t kb = b_begin + (uint64_t)nsteps * kMfmaBlocksPerStep;
    if (kb < b_end) {
        const u32x4* dl = reinterpret_cast<const u32x4*>(db + ct * 256 + 128 * c + 4 * j);
        u32x4 bw[4];
        u32x2 aw[MT];
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
            const uint64_t blk = kb + 4 * g + 2 * h + sl;
            const bool ok = blk < b_end;
            bw[2 * sl] = ok ? dl[blk * (block_words / 4)] : u32x4{0, 0, 0, 0};
            bw[2 * sl + 1] = ok ? dl[blk * (block_words / 4) + 16] : u32x4{0, 0, 0, 0};
#pragma unroll
            for (int rt = 0; rt < MT; ++rt) {
                const uint32_t q = q0 + 16 * rt + j;
                aw[rt][sl] = (ok && q < p.q_total) ? sel[(uint64_t)q * p.stride_words + blk] : 0u;
            }
        }
        mma(bw, aw);
    }

    // answer bits: lane holds columns 128c + 64*half + 4j + t' of rows
    // 16rt + 4g + r; bit 8r + 4*half + t' of par[rt]
    uint32_t par[MT];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt) {
        par[rt] = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < NT; ++t) par[rt] |= (((uint32_t)acc[rt][t][r]) & 1u) << (8 * r + t);
    }
    // fold the K halves through LDS (every load has landed and, after this
    // barrier, every wave has read its last stage)
    __syncthreads();
    u32x4* fold = reinterpret_cast<u32x4*>(pir_ring) + c * 64 + lane;
    if (h == 1) *fold = u32x4{par[0], par[1], par[2], par[3]};
    __syncthreads();  // the fold writes are complete and visible
    if (h == 1) return;
    const u32x4 o = *fold;
    par[0] ^= o[0];
    par[1] ^= o[1];
    par[2] ^= o[2];
    par[3] ^= o[3];
#pragma unroll
    for (int rt = 0; rt < MT; ++rt) {
        const uint32_t other = (uint32_t)__shfl_xor((int)par[rt], 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t q = q0 + 16 * rt + 4 * g + r;
            const uint32_t mine = par[rt] >> (8 * r), theirs = other >> (8 * r);
            if ((j & 1) == 0 && q < p.q_total) {
                uint8_t* dst = partials + ((uint64_t)group * p.q_total + q) * p.rpad + ct * 32 + 16 * c + j / 2;
                dst[0] = (uint8_t)((mine & 0xF) | ((theirs & 0xF) << 4));
                dst[8] = (uint8_t)(((mine >> 4) & 0xF) | (theirs & 0xF0));
            }
        }
    }
}

// Stage 2: out[q][m] = XOR over groups of partials[g][q][m].  Each workgroup
// owns `wpb` consecutive 32-bit words of the [q][rpad] result (wpb a power of
// two) and splits the groups over 256 / wpb slices, then folds the slices
// through LDS.  A launch covers `words` words from the start of `partials`
// and `out` (whole rows); consecutive groups' partials are gstride words apart.
__global__ void __launch_bounds__(kThreads)
k_stage2(const uint32_t* __restrict__ partials, uint8_t* __restrict__ out, uint32_t groups,
         uint32_t words, uint64_t gstride, uint32_t wpb, uint32_t rpad, uint32_t R) {
    __shared__ uint32_t red[kThreads];
    const uint32_t nsl = kThreads / wpb;
    const uint32_t wl = threadIdx.x % wpb, sl = threadIdx.x / wpb;
    const uint32_t w = blockIdx.x * wpb + wl;
    uint32_t acc = 0;
    if (w < words && sl < nsl) {
        // 16 independent loads in flight per thread: the walk over the
        // groups is latency-bound (few workgroups), not bandwidth-bound
        constexpr uint32_t U = 16;
        uint32_t a[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) a[u] = 0;
        uint32_t g = sl;
        for (; g + (U - 1) * nsl < groups; g += U * nsl) {
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) a[u] ^= partials[(uint64_t)(g + u * nsl) * gstride + w];
        }
        for (; g < groups; g += nsl) a[0] ^= partials[(uint64_t)g * gstride + w];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) acc ^= a[u];
    }
    // fold the slices pairwise (nsl is a power of two)
    red[threadIdx.x] = acc;
    for (uint32_t half = nsl / 2; half > 0; half /= 2) {
        __syncthreads();
        if (sl < half) red[threadIdx.x] ^= red[threadIdx.x + half * wpb];
    }
    __syncthreads();
    if (sl == 0 && w < words) {
        acc = red[wl];
        const uint32_t q = (4 * w) / rpad, m0 = (4 * w) - q * rpad;
        for (uint32_t b = 0; b < 4; ++b) {
            const uint32_t m = m0 + b;
            if (m < R) out[(uint64_t)q * R + m] = (uint8_t)(acc >> (8 * b));
        }
    }
}

// Natural -> bit-sliced, one wave per 32-record block.  Lanes 0-31 hold byte
// c of records 0-31 of the block, lanes 32-63 byte c+1; each ballot over bit
// t yields the two words of columns 8c+t and 8(c+1)+t.
__global__ void __launch_bounds__(kThreads)
k_slice(const uint8_t* __restrict__ src, uint64_t nrec, uint32_t R, uint32_t* __restrict__ dst,
        uint64_t nblk) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t blk = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (blk >= nblk) return;
    const uint32_t i = lane & 31, h = lane >> 5;
    const uint64_t rec = blk * 32 + i;
    const bool valid = rec < nrec;
    const uint8_t* rp = src + (valid ? rec : 0) * R;
    uint32_t* out = dst + blk * 8ull * R;
    for (uint32_t c = 0; c < R; c += 2) {
        const uint32_t cb = c + h;
        const uint32_t byte = (valid && cb < R) ? rp[cb] : 0u;
        uint32_t w = 0;
#pragma unroll
        for (uint32_t t = 0; t < 8; ++t) {
            const unsigned long long m = __ballot((byte >> t) & 1u);
            if ((lane & 7) == t) w = (lane & 8) ? (uint32_t)(m >> 32) : (uint32_t)m;
        }
        const uint32_t col = 8 * c + (lane & 15);
        if (lane < 16 && col < 8 * R) out[col] = nib_swap02(w);  // stored order
    }
}

// Bit-sliced -> natural: lane i < 32 rebuilds record 32*blk + i.
__global__ void __launch_bounds__(kThreads)
k_unslice(const uint32_t* __restrict__ src, uint64_t nblk, uint32_t R, uint8_t* __restrict__ dst,
          uint64_t nrec) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t blk = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (blk >= nblk || lane >= 32) return;
    const uint64_t rec = blk * 32 + lane;
    if (rec >= nrec) return;
    const uint32_t* in = src + blk * 8ull * R;
    uint8_t* rp = dst + rec * R;
    for (uint32_t c = 0; c < R; ++c) {
        uint32_t byte = 0;
        for (uint32_t t = 0; t < 8; ++t) byte |= ((nib_swap02(in[8 * c + t]) >> lane) & 1u) << t;
        rp[c] = (uint8_t)byte;
    }
}

template <int QT, int U>
hipError_t launch_valu_t(const Geometry& g, const Plan& pl, const void* db, const uint32_t* sel,
                         uint64_t stride_words, uint32_t q, uint8_t* partials, hipStream_t s) {
    Stage1Params p;
    p.n_units = g.n_units;
    p.units_per_group = pl.units_per_group;
    p.stride_words = stride_words;
    p.nb = g.nb;
    p.q_total = q;
    p.groups = pl.groups;
    p.n_ct = g.n_ct;
    p.n_qt = pl.n_qt;
    p.cpb = g.cpb;
    p.bpw = g.bpw;
    p.lpb = g.lpb;
    p.tile_bytes = g.tile_bytes;
    p.R = g.R;
    p.rpad = g.rpad;
    const uint32_t total = pl.groups * g.n_ct * pl.n_qt;
    const uint32_t grid = (total + 7) / 8 * 8;
    if (g.narrow)
        hipLaunchKernelGGL((k_stage1_valu<QT, U, true>), dim3(grid), dim3(kThreads), 0, s,
                           (const u32x4*)db, sel, partials, p);
    else
        hipLaunchKernelGGL((k_stage1_valu<QT, U, false>), dim3(grid), dim3(kThreads), 0, s,
                           (const u32x4*)db, sel, partials, p);
    return hipGetLastError();
}

}  // namespace

// (QT, U) pairs compiled for the vector-ALU scan.
#define PIR_VALU_TABLE(X) \
    X(1, 4) X(1, 8) X(1, 16) \
    X(2, 4) X(2, 8) \
    X(4, 2) X(4, 4) X(4, 8) \
    X(8, 1) X(8, 2) X(8, 4) \
    X(16, 1) X(16, 2) X(16, 4) \
    X(32, 1) X(32, 2)

bool valu_supported(uint32_t qt, uint32_t unroll) {
#define X(a, b) if (qt == a && unroll == b) return true;
    PIR_VALU_TABLE(X)
#undef X
    return false;
}

hipError_t launch_stage1_valu(const Geometry& g, const Plan& p, const void* db, const uint32_t* sel,
                              uint64_t stride_words, uint32_t q, uint8_t* partials, hipStream_t s) {
#define X(a, b) \
    if (p.qt == a && p.unroll == b) return launch_valu_t<a, b>(g, p, db, sel, stride_words, q, partials, s);
    PIR_VALU_TABLE(X)
#undef X
    return hipErrorInvalidValue;
}

// SplitMix64's output function over a counter (Steele, Lea and Flood, 2014)
__global__ void __launch_bounds__(kThreads) k_fill_hash(uint32_t* __restrict__ dst, uint64_t words, uint64_t seed) {
    const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += step) {
        uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        dst[i] = (uint32_t)(z ^ (z >> 31));
    }
}

hipError_t launch_fill_hash(uint32_t* dst, uint64_t words, uint64_t seed, hipStream_t s) {
    if (words == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((words + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_fill_hash, dim3((uint32_t)blocks), dim3(kThreads), 0, s, dst, words, seed);
    return hipGetLastError();
}

hipError_t launch_stage2(const Geometry& g, uint32_t groups, uint32_t q, const uint8_t* partials,
                         uint8_t* out, hipStream_t s) {
    // partials[group] holds q rows of rpad bytes: gstride words per group
    const uint64_t row_words = g.rpad / 4, gstride = (uint64_t)q * row_words;
    // one launch covers whole answer rows, at most 2^22 workgroups of
    // kThreads work-items (a launch dimension holds fewer than 2^32)
    const uint64_t rows_per_launch = std::max<uint64_t>(1, (4ull << 22) / row_words);
    for (uint64_t r0 = 0; r0 < q; r0 += rows_per_launch) {
        const uint32_t words = (uint32_t)(std::min<uint64_t>(rows_per_launch, q - r0) * row_words);
        // at least ~128 workgroups where the result allows: the walk over
        // the groups is latency-bound, and narrower word tiles give more
        // workgroups and fewer groups per thread (4 words = 16 contiguous
        // bytes per group)
        const uint32_t wpb = words >= 16 * 128 ? 16 : (words >= 8 * 128 ? 8 : 4);
        const uint32_t grid = (words + wpb - 1) / wpb;
        hipLaunchKernelGGL(k_stage2, dim3(grid), dim3(kThreads), 0, s,
                           (const uint32_t*)partials + r0 * row_words, out + r0 * g.R, groups, words, gstride, wpb,
                           g.rpad, g.R);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_slice(const Geometry& g, const uint8_t* src, uint64_t nrec, uint32_t* dst_block0,
                        uint64_t nblk, hipStream_t s) {
    if (nblk == 0) return hipSuccess;
    const uint64_t grid = (nblk + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(k_slice, dim3((uint32_t)grid), dim3(kThreads), 0, s, src, nrec, g.R,
                       dst_block0, nblk);
    return hipGetLastError();
}

hipError_t launch_unslice(const Geometry& g, const uint32_t* src_block0, uint64_t nblk, uint8_t* dst,
                          uint64_t nrec, hipStream_t s) {
    if (nblk == 0) return hipSuccess;
    const uint64_t grid = (nblk + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(k_unslice, dim3((uint32_t)grid), dim3(kThreads), 0, s, src_block0, nblk, g.R,
                       dst, nrec);
    return hipGetLastError();
}

bool mfma_supported(uint32_t variant, const Geometry& g, uint32_t qt, uint32_t unroll) {
    if (variant != PIR_VARIANT_MFMA_F4 && variant != PIR_VARIANT_MFMA_I8) return false;
    if (g.R % 32 != 0) return false;  // whole 256-column tiles
    // unroll selects the pipeline: 2, 3, 4 = an LDS ring of that many stages
    // (that many minus one K-steps in flight); 12 = the split-K kernel on a
    // 2-stage ring (fp4, 64-query tiles); 15 = the split-K kernel whose
    // selection words arrive four K-steps at a time, 16 = the same with
    // wave-private database stages (both fp4, 64-query tiles)
    if (unroll == 12 || unroll == 15 || unroll == 16 || unroll == 17) return variant == PIR_VARIANT_MFMA_F4 && qt == 64;
    if (unroll != 2 && unroll != 3 && unroll != 4) return false;
    return qt == 16 || qt == 32 || qt == 64;
}

template <int MT, bool F4, int S>
static hipError_t launch_ring(dim3 grid, hipStream_t s, const uint32_t* db, const uint32_t* sel, uint8_t* partials,
                              const Stage1Params& p) {
    constexpr uint32_t bytes = ring_bytes<MT>(S);
    const hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_lds<MT, F4, S>), (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_stage1_mfma_lds<MT, F4, S>), grid, dim3(kThreads), bytes, s, db, sel, partials, p);
    return hipGetLastError();
}

// Largest selection pitch (32-bit words) for which the split-K kernel's lane
// offsets, up to three rows plus 60 bytes, fit in 32 bits.
constexpr uint64_t kKsMaxStrideWords = ((1ull << 32) - 64) / 12;

// Database cache policy of the split-K kernels: nontemporal (2) when the
// launch has one query tile, so that each database chunk is read once;
// default (0) when several query tiles' workgroups read each chunk in turn
// (they run on one XCD and meet in its L2: at Q = 512 on 8 GiB the
// nontemporal policy fetched 1.32x the algorithmic bytes, the default 1.00x)
static bool db_shared_by_tiles(const Stage1Params& p) { return p.n_qt > 1; }

template <int S, int DBP>
static hipError_t launch_ks_p(dim3 grid, hipStream_t s, const uint32_t* db, const uint32_t* sel, uint8_t* partials,
                              const Stage1Params& p) {
    constexpr uint32_t bytes = ring_bytes<4>(S);
    const hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_ks<S, DBP>), (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_stage1_mfma_ks<S, DBP>), grid, dim3(kThreads), bytes, s, db, sel, partials, p);
    return hipGetLastError();
}

template <int S>
static hipError_t launch_ks(dim3 grid, hipStream_t s, const uint32_t* db, const uint32_t* sel, uint8_t* partials,
                            const Stage1Params& p) {
    if (p.stride_words > kKsMaxStrideWords) return launch_ring<4, true, S>(grid, s, db, sel, partials, p);
    return db_shared_by_tiles(p) ? launch_ks_p<S, 0>(grid, s, db, sel, partials, p)
                                 : launch_ks_p<S, 2>(grid, s, db, sel, partials, p);
}

// The split-K kernels with wide selection loads move 16 bytes per lane: rows
// must start on 16-byte boundaries; other pitches take the 4-byte loads of
// the split-K ring kernel
static bool wide_sel_ok(const uint32_t* sel, const Stage1Params& p) {
    return p.stride_words <= kWsMaxStrideWords && p.stride_words % 4 == 0 &&
           (reinterpret_cast<uintptr_t>(sel) & 15) == 0;
}

template <int DBP>
static hipError_t launch_ksw_p(dim3 grid, hipStream_t s, const uint32_t* db, const uint32_t* sel, uint8_t* partials,
                               const Stage1Params& p) {
    const hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_ksw<DBP>), (int)kWsLdsBytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stage1_mfma_ksw<DBP>, grid, dim3(kThreads), kWsLdsBytes, s, db, sel, partials, p);
    return hipGetLastError();
}

static hipError_t launch_ksw(dim3 grid, hipStream_t s, const uint32_t* db, const uint32_t* sel, uint8_t* partials,
                             const Stage1Params& p) {
    if (!wide_sel_ok(sel, p)) return launch_ks<2>(grid, s, db, sel, partials, p);
    return db_shared_by_tiles(p) ? launch_ksw_p<0>(grid, s, db, sel, partials, p)
                                 : launch_ksw_p<2>(grid, s, db, sel, partials, p);
}

template <int DBP>
static hipError_t launch_ksp_p(dim3 grid, hipStream_t s, const uint32_t* db, const uint32_t* sel, uint8_t* partials,
                               const Stage1Params& p) {
    const hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_ksp<DBP>), (int)kSpLdsBytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stage1_mfma_ksp<DBP>, grid, dim3(kThreads), kSpLdsBytes, s, db, sel, partials, p);
    return hipGetLastError();
}

static hipError_t launch_ksp(dim3 grid, hipStream_t s, const uint32_t* db, const uint32_t* sel, uint8_t* partials,
                             const Stage1Params& p) {
    if (!wide_sel_ok(sel, p)) return launch_ks<2>(grid, s, db, sel, partials, p);
    return db_shared_by_tiles(p) ? launch_ksp_p<0>(grid, s, db, sel, partials, p)
                                 : launch_ksp_p<2>(grid, s, db, sel, partials, p);
}

template <int DBP>
static hipError_t launch_ksv_p(dim3 grid, hipStream_t s, const uint32_t* db, const uint32_t* sel, uint8_t* partials,
                               const Stage1Params& p) {
    const hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_ksv<DBP>), (int)kSvLdsBytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stage1_mfma_ksv<DBP>, grid, dim3(kThreads), kSvLdsBytes, s, db, sel, partials, p);
    return hipGetLastError();
}

static hipError_t launch_ksv(dim3 grid, hipStream_t s, const uint32_t* db, const uint32_t* sel, uint8_t* partials,
                             const Stage1Params& p) {
    if (!wide_sel_ok(sel, p)) return launch_ks<2>(grid, s, db, sel, partials, p);
    // a record group's database range is one buffer of 32-bit size
    if (p.units_per_group * 32ull * p.R >= (1ull << 32)) return launch_ksp(grid, s, db, sel, partials, p);
    return db_shared_by_tiles(p) ? launch_ksv_p<0>(grid, s, db, sel, partials, p)
                                 : launch_ksv_p<2>(grid, s, db, sel, partials, p);
}

template <int MT, bool F4>
static hipError_t launch_mfma_t(const Geometry& g, const Plan& pl, const void* db, const uint32_t* sel,
                                uint64_t stride_words, uint32_t q, uint8_t* partials, hipStream_t s) {
    Stage1Params p;
    p.n_units = g.n_units;
    p.units_per_group = pl.units_per_group;
    p.stride_words = stride_words;
    p.nb = g.nb;
    p.q_total = q;
    p.groups = pl.groups;
    p.n_ct = g.n_ct;
    p.n_qt = pl.n_qt;
    p.cpb = g.cpb;
    p.bpw = g.bpw;
    p.lpb = g.lpb;
    p.tile_bytes = g.tile_bytes;
    p.R = g.R;
    p.rpad = g.rpad;
    const uint32_t total = pl.groups * g.n_ct * pl.n_qt;
    const dim3 grid((total + 7) / 8 * 8);
    const uint32_t* d = (const uint32_t*)db;
    switch (pl.unroll) {
        case 2: return launch_ring<MT, F4, 2>(grid, s, d, sel, partials, p);
        case 3: return launch_ring<MT, F4, 3>(grid, s, d, sel, partials, p);
        case 4: return launch_ring<MT, F4, 4>(grid, s, d, sel, partials, p);
        case 12:
            if constexpr (MT == 4 && F4) return launch_ks<2>(grid, s, d, sel, partials, p);
            return hipErrorInvalidValue;
        case 15:
            if constexpr (MT == 4 && F4) return launch_ksw(grid, s, d, sel, partials, p);
            return hipErrorInvalidValue;
        case 16:
            if constexpr (MT == 4 && F4) return launch_ksp(grid, s, d, sel, partials, p);
            return hipErrorInvalidValue;
        case 17:
            if constexpr (MT == 4 && F4) return launch_ksv(grid, s, d, sel, partials, p);
            return hipErrorInvalidValue;
        default:
            return hipErrorInvalidValue;
    }
}

template <int MT, bool F4>
static hipError_t prepare_rings() {
    hipError_t e = hipSuccess;
    if ((e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_lds<MT, F4, 2>), (int)ring_bytes<MT>(2))) ||
        (e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_lds<MT, F4, 3>), (int)ring_bytes<MT>(3))) ||
        (e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_lds<MT, F4, 4>), (int)ring_bytes<MT>(4))))
        return e;
    return hipSuccess;
}

hipError_t prepare_scan_kernels() {
    hipError_t e = hipSuccess;
    if ((e = prepare_rings<1, true>()) || (e = prepare_rings<2, true>()) || (e = prepare_rings<4, true>()) ||
        (e = prepare_rings<1, false>()) || (e = prepare_rings<2, false>()) || (e = prepare_rings<4, false>()))
        return e;
    if ((e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_ks<2, 0>), (int)ring_bytes<4>(2))) ||
        (e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_ks<2, 2>), (int)ring_bytes<4>(2))) ||
        (e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_ksw<0>), (int)kWsLdsBytes)) ||
        (e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_ksw<2>), (int)kWsLdsBytes)) ||
        (e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_ksp<0>), (int)kSpLdsBytes)) ||
        (e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_ksp<2>), (int)kSpLdsBytes)) ||
        (e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_ksv<0>), (int)kSvLdsBytes)) ||
        (e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_stage1_mfma_ksv<2>), (int)kSvLdsBytes)))
        return e;
    return hipSuccess;
}

hipError_t launch_stage1_mfma(const Geometry& g, const Plan& p, const void* db, const uint32_t* sel,
                              uint64_t stride_words, uint32_t q, uint8_t* partials, hipStream_t s) {
    if (!mfma_supported(p.variant, g, p.qt, p.unroll)) return hipErrorInvalidValue;
    const bool f4 = p.variant == PIR_VARIANT_MFMA_F4;
    if (p.qt == 16) return f4 ? launch_mfma_t<1, true>(g, p, db, sel, stride_words, q, partials, s)
                              : launch_mfma_t<1, false>(g, p, db, sel, stride_words, q, partials, s);
    if (p.qt == 32) return f4 ? launch_mfma_t<2, true>(g, p, db, sel, stride_words, q, partials, s)
                              : launch_mfma_t<2, false>(g, p, db, sel, stride_words, q, partials, s);
    return f4 ? launch_mfma_t<4, true>(g, p, db, sel, stride_words, q, partials, s)
              : launch_mfma_t<4, false>(g, p, db, sel, stride_words, q, partials, s);
}

Geometry make_geometry(uint64_t n, uint32_t R) {
    Geometry g;
    g.n = n;
    g.R = R;
    g.rpad = (R + 3) / 4 * 4;
    g.nb = (n + 31) / 32;
    g.cpb = 2 * R;
    g.narrow = R < 32;
    if (g.narrow) {
        g.lpb = g.cpb;
        g.bpw = 64 / g.cpb;
        g.n_ct = 1;
        g.tile_bytes = R;
    } else {
        g.lpb = 64;
        g.bpw = 1;
        g.n_ct = (g.cpb + 63) / 64;
        g.tile_bytes = 32;
    }
    g.n_units = (g.nb + g.bpw - 1) / g.bpw;
    g.nb_alloc = g.n_units * g.bpw;
    return g;
}

}  // namespace pir
