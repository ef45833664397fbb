// Internal declarations shared by the runtime, the kernels and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pir.h"

namespace pir {

// Raise a kernel's dynamic-LDS limit to `bytes` on the current device, once
// per (kernel, device); safe to call from several host threads.
hipError_t ensure_dynamic_lds(const void* kernel, int bytes);

// Stored word order.  Inside every nibble of a bit-sliced word the records
// 4n and 4n+2 trade places (an involution): stored bit 4n+2 is record 4n and
// stored bit 4n is record 4n+2.  This lets the matrix-core spread of a
// database word use masks for three of its four parts.  A selection word,
// which arrives in record order, is brought to stored order with the same
// swap before it meets a stored word bit for bit.
__host__ __device__ inline uint32_t nib_swap02(uint32_t x) {
    return (x & 0xAAAAAAAAu) | ((x & 0x11111111u) << 2) | ((x >> 2) & 0x11111111u);
}

// Geometry of a bit-sliced database.
//
// Records are grouped in blocks of 32.  Block blk is 8*R 32-bit words; word b
// holds bit b of the 32 records (bit b of a record = bit (b & 7) of byte
// b >> 3; record 32*blk + i sits at bit i of the word, except that inside each
// 4-bit group records 4n and 4n+2 trade places; see nib_swap02).  A block is 32*R
// bytes = 2*R 16-byte chunks.  Scans read whole chunks, one per lane.
//
//  - R >= 32 ("wide"): a wave covers 64 chunks (1 KiB, 256 bit columns) of one
//    block per load; a block spans n_ct = ceil(2R/64) column tiles.  The
//    query's selection word for the block is the same for the whole wave.
//  - R < 32 ("narrow"): a wave covers bpw = floor(32/R) whole blocks per load
//    (lpb = 2R lanes each); lanes past bpw*lpb idle.
//
// A "unit" is what one wave reads per load: 1 block (wide) or bpw blocks
// (narrow).  The device allocation is rounded up to whole units; padding
// blocks hold zero records.
struct Geometry {
    uint64_t n = 0;         // records
    uint32_t R = 0;         // record bytes
    uint32_t rpad = 0;      // R rounded up to 4 (partial-result row pitch)
    uint64_t nb = 0;        // blocks holding records: ceil(n / 32)
    uint32_t cpb = 0;       // 16-byte chunks per block = 2R
    bool narrow = false;    // R < 32
    uint32_t bpw = 1;       // blocks per unit
    uint32_t lpb = 64;      // lanes per block (narrow: 2R)
    uint32_t n_ct = 1;      // column tiles per block
    uint32_t tile_bytes = 32;  // record bytes per column tile (narrow: R)
    uint64_t n_units = 0;   // ceil(nb / bpw)
    uint64_t nb_alloc = 0;  // n_units * bpw
    uint64_t bytes() const { return nb_alloc * 32ull * R; }
};

Geometry make_geometry(uint64_t n, uint32_t R);

// One launch of the stage-1 scan.
// Fields left 0 are filled in by finish_plan.
struct Plan {
    uint32_t variant = PIR_VARIANT_VALU;
    uint32_t qt = 0;        // queries per tile
    uint32_t unroll = 0;    // units per wave iteration
    uint32_t groups = 0;    // record groups (contiguous unit ranges)
    uint32_t n_qt = 1;      // query tiles
    uint64_t units_per_group = 0;
    uint32_t grid = 0;      // workgroups launched
};

// Kernel launchers (pir_kernels.hip).  All enqueue on `stream` and return the
// launch status.
bool valu_supported(uint32_t qt, uint32_t unroll);
hipError_t launch_stage1_valu(const Geometry& g, const Plan& p, const void* db, const uint32_t* sel,
                              uint64_t stride_words, uint32_t q, uint8_t* partials, hipStream_t s);
bool mfma_supported(uint32_t variant, const Geometry& g, uint32_t qt, uint32_t unroll);
hipError_t launch_stage1_mfma(const Geometry& g, const Plan& p, const void* db, const uint32_t* sel,
                              uint64_t stride_words, uint32_t q, uint8_t* partials, hipStream_t s);
// Raise the dynamic-LDS limit of every stage-1 ring kernel on the current
// device (done when a context is created, so that no scan call needs to)
hipError_t prepare_scan_kernels();
hipError_t launch_stage2(const Geometry& g, uint32_t groups, uint32_t q, const uint8_t* partials,
                         uint8_t* out, hipStream_t s);
// words[i] = a 32-bit hash of (seed, i): stand-in selection bits for the
// autotuner's timing runs (a scan's duration depends on how many of its
// operand bits toggle, so a constant fill times it too fast)
hipError_t launch_fill_hash(uint32_t* dst, uint64_t words, uint64_t seed, hipStream_t s);
// natural row-major records [rec0, rec0 + nrec) -> bit-sliced blocks starting at rec0 / 32
hipError_t launch_slice(const Geometry& g, const uint8_t* src, uint64_t nrec, uint32_t* dst_block0,
                        uint64_t nblk, hipStream_t s);
// bit-sliced blocks -> natural records (nrec valid records from block 0)
hipError_t launch_unslice(const Geometry& g, const uint32_t* src_block0, uint64_t nblk, uint8_t* dst,
                          uint64_t nrec, hipStream_t s);

// DPF (pir_dpf.hip).
constexpr uint64_t kDpfBigLaunch = 256 * 1024;  // threads from which DPF launches use 1024-thread workgroups
uint64_t dpf_key_bytes(uint32_t n);
// nodes per key in each of the two scratch buffers of an evaluation
uint64_t dpf_scratch_nodes(uint32_t n, uint64_t n_leaves);
// top of the tree in one workgroup per key: up to this many levels, by
// kDpfTopThreads threads (2^(levels - 1) <= kDpfTopThreads)
constexpr uint32_t kDpfTopLevels = 10;
constexpr int kDpfTopThreads = 1024;
uint32_t dpf_top_levels(uint32_t n);
// launch chain from level a0 as (first level, levels expanded); returns the number of launches
int dpf_plan(uint32_t n, uint64_t n_leaves, uint32_t n_keys, uint32_t a0, uint32_t steps[][2]);
// full-domain evaluation of n_keys keys (device, dpf_key_bytes(n) apart):
// selection words [0, ceil(n_leaves / 32)) of row q at d_sel + q * stride_words;
// scratch holds 2 * n_keys * scratch_nodes 16-byte nodes
hipError_t launch_dpf_eval(int device, const uint8_t* d_keys, uint32_t n, uint32_t n_keys, uint64_t n_leaves,
                           uint32_t* d_sel, uint64_t stride_words, void* scratch, uint64_t scratch_nodes,
                           hipStream_t s);
void dpf_gen_host(uint64_t alpha, uint32_t n, const uint8_t root0[16], const uint8_t root1[16], uint8_t* key0,
                  uint8_t* key1);
void aes128_encrypt_host(const uint8_t key[16], const uint8_t in[16], uint8_t out[16]);

// Inner products over F_p (pir_fp.hip).  Records in 64-record tiles,
// column-major inside a tile; lpad = elements per record rounded up to 16.
struct FpParams {
    uint64_t tiles = 0;            // 64-record tiles holding records
    uint64_t tiles_per_group = 0;  // <= kFpMaxTilesPerGroup (int32 sums stay exact)
    uint64_t v_stride = 0;         // query row pitch (bytes)
    uint32_t L = 0, lpad = 0, n_ct = 0;
    uint32_t groups = 0, n_qt = 0, n_cg = 0;
    uint32_t q_total = 0, p = 0, magic = 0;  // magic = floor(2^32 / p)
};
// A wave sums a quarter of its group's tiles (two of every eight):
// 2^31 / (64 * 127 * 126) > 2048 tiles per wave, so 8192 tiles per group keep
// every int32 sum exact.
constexpr uint64_t kFpMaxTilesPerGroup = 8192;
bool fp_supported(uint32_t rt, uint32_t ct);
// rt row tiles (16 queries each), ct column tiles (16 elements each)
hipError_t launch_fp_stage1(const uint8_t* db, const uint8_t* v, uint8_t* partials, const FpParams& a, uint32_t rt,
                            uint32_t ct, hipStream_t s);
// cross-group reduction: tmp holds fp_stage2_tmp_bytes(groups, outputs)
size_t fp_stage2_tmp_bytes(uint32_t groups, uint64_t outputs);
hipError_t launch_fp_stage2(const uint8_t* partials, uint32_t groups, uint64_t outputs, uint32_t p, uint32_t magic,
                            uint32_t* tmp, uint8_t* out, hipStream_t s);
hipError_t launch_fp_tile(const uint8_t* src, uint64_t nrec, uint32_t L, uint32_t lpad, uint8_t* dst, hipStream_t s);
hipError_t launch_fp_untile(const uint8_t* src, uint64_t nrec, uint32_t L, uint32_t lpad, uint8_t* dst,
                            hipStream_t s);

}  // namespace pir
