// Full-domain DPF evaluation on gfx950 -- the step that turns a query key into
// the selection bits the scan consumes (IM-PIR Sec. 3.2, eq. 1-3) -- and the
// client-side key generation (Sec. 3.1).
//
//   Eval(k, j) = R(n, j);  R(0, 0) = C0[0, 0];
//   R(d, j) = PRF_{R(d-1, j/2)}(j mod 2) XOR C_{R(d-1, j/2) mod 2}[j mod 2, d]
//
// Node values are 128-bit blocks (16 bytes, byte 0 first); "mod 2" is bit 0 of
// byte 0; PRF_s(x) is AES-128 (FIPS-197) under key s of the block whose byte 0
// is x and whose other bytes are 0; the selection bit of leaf j is bit 0 of
// Eval(k, j).  A key is two codewords C0, C1 of 2 x (n+1) blocks each, block
// [x][d] at index x*(n+1) + d; codeword C1 follows C0.
//
// Work layout.  Every internal node of the tree is expanded exactly once
// (one AES key schedule, two encryptions that share it).  A launch takes the
// nodes of level a (from HBM, or the root from the key when a = 0) and each
// thread expands its node E <= 5 levels further in a depth-first walk held in
// registers, writing either the 2^E nodes of level a+E back to HBM or, on the
// last launch (E = 5), the 32 leaf bits as one selection word.  The host
// chains launches with small E near the root (few nodes: latency) and E = 5
// below (many nodes: throughput, little HBM traffic).
//
// AES on the VALU: T-tables Te0 (the MixColumns column of each S-box output)
// and Te2 (Te0 rotated by 16 bits); Te1 and Te3 are rotations, and
// Te1[b] ^ Te3[d] = rotr(Te0[b] ^ Te2[d], 24) costs one rotation per column.
// The S-box itself is byte 1 of Te0.  LDS serves a wave's 32-bit reads in
// two halves of 32 lanes, so 32 copies of each table keep every lookup of a
// half-wave in its own bank: row i of the 64 KiB table holds Te0[i] for lanes
// 0..31 (mod 32) and then Te2[i] for the same lanes, and a lookup address is
// one v_perm_b32 of the state word and a per-lane offset register.  (One
// 64-copy Te0 table plus three rotations per column measured 9 % slower; a
// 128 KiB layout halves the waves per CU and measured slower still.)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "pir_internal.h"

namespace pir {

// ------------------------------------------------------------ AES tables

static uint8_t gmul(uint8_t a, uint8_t b) {
    uint8_t p = 0;
    for (int i = 0; i < 8; ++i) {
        if (b & 1) p ^= a;
        const bool hi = a & 0x80;
        a = (uint8_t)(a << 1);
        if (hi) a ^= 0x1b;  // x^8 = x^4 + x^3 + x + 1
        b >>= 1;
    }
    return p;
}

// S-box from its definition (FIPS-197 Sec. 5.1.1): the inverse in GF(2^8)
// (0 maps to 0), then the affine map b ^ rotl(b,1..4) ^ 0x63.
struct AesTables {
    uint8_t sbox[256];
    uint32_t te0[256];  // bytes (2s, s, s, 3s), byte 0 least significant
    AesTables() {
        uint8_t inv[256] = {0};
        for (int a = 1; a < 256; ++a)
            for (int b = 1; b < 256; ++b)
                if (gmul((uint8_t)a, (uint8_t)b) == 1) {
                    inv[a] = (uint8_t)b;
                    break;
                }
        for (int x = 0; x < 256; ++x) {
            const uint8_t b = inv[x];
            uint8_t s = b;
            for (int r = 1; r <= 4; ++r) s ^= (uint8_t)((b << r) | (b >> (8 - r)));
            sbox[x] = (uint8_t)(s ^ 0x63);
        }
        for (int x = 0; x < 256; ++x) {
            const uint8_t s = sbox[x];
            te0[x] = (uint32_t)gmul(s, 2) | ((uint32_t)s << 8) | ((uint32_t)s << 16) | ((uint32_t)gmul(s, 3) << 24);
        }
    }
};

static const AesTables& tables() {
    static const AesTables t;
    return t;
}

__constant__ uint32_t c_te0[256];

// ------------------------------------------------------------ host AES (Gen)

namespace host_aes {

static inline uint32_t rotr(uint32_t x, int s) { return (x >> s) | (x << (32 - s)); }

static inline uint32_t sub_word(const AesTables& T, uint32_t w) {
    return (uint32_t)T.sbox[w & 0xff] | ((uint32_t)T.sbox[(w >> 8) & 0xff] << 8) |
           ((uint32_t)T.sbox[(w >> 16) & 0xff] << 16) | ((uint32_t)T.sbox[w >> 24] << 24);
}

// FIPS-197 Sec. 5.2 / 5.1 in the 32-bit T-table form; words little-endian.
static void encrypt(const uint8_t key[16], const uint8_t in[16], uint8_t out[16]) {
    const AesTables& T = tables();
    uint32_t rk[44];
    memcpy(rk, key, 16);
    uint8_t rc = 1;
    for (int i = 4; i < 44; ++i) {
        uint32_t t = rk[i - 1];
        if (i % 4 == 0) {
            t = sub_word(T, rotr(t, 8)) ^ rc;
            rc = gmul(rc, 2);
        }
        rk[i] = rk[i - 4] ^ t;
    }
    uint32_t s[4], t[4];
    memcpy(s, in, 16);
    for (int c = 0; c < 4; ++c) s[c] ^= rk[c];
    for (int r = 1; r < 10; ++r) {
        for (int c = 0; c < 4; ++c)
            t[c] = T.te0[s[c] & 0xff] ^ rotr(T.te0[(s[(c + 1) & 3] >> 8) & 0xff], 24) ^
                   rotr(T.te0[(s[(c + 2) & 3] >> 16) & 0xff], 16) ^ rotr(T.te0[s[(c + 3) & 3] >> 24], 8) ^
                   rk[4 * r + c];
        memcpy(s, t, sizeof s);
    }
    for (int c = 0; c < 4; ++c)
        t[c] = ((uint32_t)T.sbox[s[c] & 0xff] | ((uint32_t)T.sbox[(s[(c + 1) & 3] >> 8) & 0xff] << 8) |
                ((uint32_t)T.sbox[(s[(c + 2) & 3] >> 16) & 0xff] << 16) |
                ((uint32_t)T.sbox[s[(c + 3) & 3] >> 24] << 24)) ^
               rk[40 + c];
    memcpy(out, t, 16);
}

static void prf(const uint8_t s[16], int x, uint8_t out[16]) {
    uint8_t blk[16] = {0};
    blk[0] = (uint8_t)x;
    encrypt(s, blk, out);
}

}  // namespace host_aes

void aes128_encrypt_host(const uint8_t key[16], const uint8_t in[16], uint8_t out[16]) {
    host_aes::encrypt(key, in, out);
}

// ------------------------------------------------------------ device side

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kTabBytes = 256 * 64 * 4;  // 64 KiB: 32 copies of Te0 and of Te2

// AES round constants x^(i-1) in GF(2^8), i = 1..10.
__host__ __device__ constexpr uint32_t rcon(int i) {
    uint32_t r = 1;
    for (int k = 1; k < i; ++k) r = (r << 1) ^ ((r & 0x80) ? 0x11b : 0);
    return r;
}

struct Lut {
    const uint32_t* tab;  // LDS table: row i = 32 copies of Te0[i], then 32 of Te2[i]
    uint32_t lane4;       // 4 * (lane % 32)
    uint32_t lane4b;      // 128 + 4 * (lane % 32)

    template <int K>
    __device__ __forceinline__ uint32_t t(uint32_t s) const {
        const uint32_t addr = __builtin_amdgcn_perm(s, lane4, 0x0c0c0400u + (K << 8));
        return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(tab) + addr);
    }
    template <int K>
    __device__ __forceinline__ uint32_t u(uint32_t s) const {
        const uint32_t addr = __builtin_amdgcn_perm(s, lane4b, 0x0c0c0400u + (K << 8));
        return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(tab) + addr);
    }
};

__device__ __forceinline__ uint32_t rotr(uint32_t x, uint32_t s) { return __builtin_amdgcn_alignbit(x, x, s); }

// Bytes (S(a), S(b), S(c), S(d)) from four T-table entries (S = byte 1).
__device__ __forceinline__ uint32_t sbox4(uint32_t ta, uint32_t tb, uint32_t tc, uint32_t td) {
    return __builtin_amdgcn_perm(tb, ta, 0x0c0c0501u) ^ __builtin_amdgcn_perm(td, tc, 0x05010c0cu);
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// One column of SubBytes + ShiftRows + MixColumns + AddRoundKey.
__device__ __forceinline__ uint32_t mix_col(const Lut& L, uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                            uint32_t k) {
    return xor3(L.t<0>(a), L.u<2>(c), k) ^ rotr(L.t<1>(b) ^ L.u<3>(d), 24);
}

// Last-round column (no MixColumns).
__device__ __forceinline__ uint32_t last_col(const Lut& L, uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                             uint32_t k) {
    const uint32_t ta = L.t<0>(a), tb = L.t<1>(b), tc = L.t<2>(c), td = L.t<3>(d);
    return xor3(__builtin_amdgcn_perm(tb, ta, 0x0c0c0501u), __builtin_amdgcn_perm(td, tc, 0x05010c0cu), k);
}

// Next round key (KeyExpansion for one round, words in place).
template <int R>
__device__ __forceinline__ void key_step(const Lut& L, uint32_t& w0, uint32_t& w1, uint32_t& w2, uint32_t& w3) {
    // RotWord then SubWord: bytes (S(w3.1), S(w3.2), S(w3.3), S(w3.0))
    w0 ^= sbox4(L.t<1>(w3), L.t<2>(w3), L.t<3>(w3), L.t<0>(w3)) ^ rcon(R);
    w1 ^= w0;
    w2 ^= w1;
    w3 ^= w2;
}

// AES-128 under key k of the blocks (0, 0, ..) and (1, 0, ..): the two
// children PRF_k(0), PRF_k(1).  The round keys are produced on the fly and
// shared; after the first AddRoundKey the blocks differ only in byte 0, so
// round 1 changes only column 0 of the second block.
//
// FULL = false computes only bit 0 of each output (what a leaf contributes):
// byte 0 of the last round reads only byte 0 of column 0 of round 9, and
// needs only byte 0 of the last round key; o0.x, o1.x then hold that bit in
// bit 0 and nothing else is defined.
template <bool FULL>
__device__ __forceinline__ void prf_pair(const Lut& L, u32x4 k, u32x4& o0, u32x4& o1) {
    uint32_t w0 = k.x, w1 = k.y, w2 = k.z, w3 = k.w;
    uint32_t a0 = w0, a1 = w1, a2 = w2, a3 = w3;
    uint32_t b0 = w0 ^ 1u;
    key_step<1>(L, w0, w1, w2, w3);
    uint32_t n0 = mix_col(L, a0, a1, a2, a3, w0);
    uint32_t n1 = mix_col(L, a1, a2, a3, a0, w1);
    uint32_t n2 = mix_col(L, a2, a3, a0, a1, w2);
    uint32_t n3 = mix_col(L, a3, a0, a1, a2, w3);
    uint32_t m0 = mix_col(L, b0, a1, a2, a3, w0);
    a0 = n0, a1 = n1, a2 = n2, a3 = n3;
    b0 = m0;
    uint32_t b1 = n1, b2 = n2, b3 = n3;
#define PIR_AES_ROUND(R)                                    \
    key_step<R>(L, w0, w1, w2, w3);                         \
    n0 = mix_col(L, a0, a1, a2, a3, w0);                    \
    n1 = mix_col(L, a1, a2, a3, a0, w1);                    \
    n2 = mix_col(L, a2, a3, a0, a1, w2);                    \
    n3 = mix_col(L, a3, a0, a1, a2, w3);                    \
    m0 = mix_col(L, b0, b1, b2, b3, w0);                    \
    {                                                       \
        const uint32_t m1 = mix_col(L, b1, b2, b3, b0, w1); \
        const uint32_t m2 = mix_col(L, b2, b3, b0, b1, w2); \
        const uint32_t m3 = mix_col(L, b3, b0, b1, b2, w3); \
        b1 = m1, b2 = m2, b3 = m3;                          \
    }                                                       \
    a0 = n0, a1 = n1, a2 = n2, a3 = n3, b0 = m0;
    PIR_AES_ROUND(2)
    PIR_AES_ROUND(3)
    PIR_AES_ROUND(4)
    PIR_AES_ROUND(5)
    PIR_AES_ROUND(6)
    PIR_AES_ROUND(7)
    PIR_AES_ROUND(8)
    if (!FULL) {
        key_step<9>(L, w0, w1, w2, w3);
        const uint32_t s0 = mix_col(L, a0, a1, a2, a3, w0), r0 = mix_col(L, b0, b1, b2, b3, w0);
        // last round, byte 0 of column 0: S(s0.0) ^ w0.0 ^ S(w3.1) ^ rcon(10); S(x) is byte 1 of a
        // table entry, so bit 0 of the result sits at bit 8 below
        const uint32_t kx = L.t<1>(w3) ^ (w0 << 8) ^ (rcon(10) << 8);
        o0.x = (L.t<0>(s0) ^ kx) >> 8;
        o1.x = (L.t<0>(r0) ^ kx) >> 8;
        return;
    }
    PIR_AES_ROUND(9)
#undef PIR_AES_ROUND
    key_step<10>(L, w0, w1, w2, w3);
    o0 = u32x4{last_col(L, a0, a1, a2, a3, w0), last_col(L, a1, a2, a3, a0, w1), last_col(L, a2, a3, a0, a1, w2),
               last_col(L, a3, a0, a1, a2, w3)};
    o1 = u32x4{last_col(L, b0, b1, b2, b3, w0), last_col(L, b1, b2, b3, b0, w1), last_col(L, b2, b3, b0, b1, w2),
               last_col(L, b3, b0, b1, b2, w3)};
}

// eq. 3 for both children of node r at child level d: PRF_r(x) XOR C_t[x][d],
// t = r mod 2.  kq points at the key's blocks (C0 rows, then C1 rows).
__device__ __forceinline__ void expand(const Lut& L, const u32x4* __restrict__ kq, uint32_t n1, uint32_t d, u32x4 r,
                                       u32x4& c0, u32x4& c1) {
    u32x4 g0, g1;
    prf_pair<true>(L, r, g0, g1);
    const u32x4 z0 = kq[d], z1 = kq[n1 + d];               // C0[0][d], C0[1][d]
    const u32x4 o0 = kq[2 * n1 + d], o1 = kq[3 * n1 + d];  // C1[0][d], C1[1][d]
    const uint32_t m = 0u - (r.x & 1u);
    const u32x4 mm = u32x4{m, m, m, m};
    c0 = g0 ^ z0 ^ (mm & (z0 ^ o0));
    c1 = g1 ^ z1 ^ (mm & (z1 ^ o1));
}

// Bit 0 of both children of node r at the leaf level d = n (eq. 3 on bit 0).
__device__ __forceinline__ uint32_t expand_leaf_bits(const Lut& L, const u32x4* __restrict__ kq, uint32_t n1,
                                                     uint32_t d, u32x4 r) {
    u32x4 g0, g1;
    prf_pair<false>(L, r, g0, g1);
    const uint32_t t = r.x & 1u;
    const uint32_t z0 = t ? kq[2 * n1 + d].x : kq[d].x;       // C_t[0][d]
    const uint32_t z1 = t ? kq[3 * n1 + d].x : kq[n1 + d].x;  // C_t[1][d]
    return ((g0.x ^ z0) & 1u) | (((g1.x ^ z1) & 1u) << 1);
}

// Depth-first walk of E levels below node `cur` of level a (0 <= E <= 5),
// right children held in registers.  BITS: returns the 2^E leaf bits (leaf
// p at bit p; E = 0 returns the node's own bit).  Otherwise writes the 2^E
// nodes of level a+E to orow[0 .. 2^E) and returns 0.
template <bool BITS>
__device__ __forceinline__ uint32_t dfs_expand(const Lut& L, const u32x4* __restrict__ kq, uint32_t n1, uint32_t a,
                                               uint32_t E, u32x4 cur, u32x4* __restrict__ orow) {
    uint32_t word = (E == 0) ? (cur.x & 1u) : 0u;
    u32x4 st1 = cur, st2 = cur, st3 = cur, st4 = cur;  // right children still to visit
    uint32_t depth = 0, p = 0;
    const uint32_t total = (1u << E) - 1u;
    for (uint32_t k = 0; k < total; ++k) {
        const bool last = depth + 1 == E;  // the children are outputs
        u32x4 c0, c1;
        if (BITS && last)
            word |= expand_leaf_bits(L, kq, n1, a + E, cur) << (2 * p);
        else
            expand(L, kq, n1, a + depth + 1, cur, c0, c1);
        if (last) {
            if (!BITS) {
                orow[2 * p] = c0;
                orow[2 * p + 1] = c1;
            }
            ++p;
            depth = E - 1 - __builtin_ctz(p);  // the next node is the right child stored at this depth
            cur = depth == 1 ? st1 : depth == 2 ? st2 : depth == 3 ? st3 : st4;
        } else {
            ++depth;
            if (depth == 1)
                st1 = c1;
            else if (depth == 2)
                st2 = c1;
            else if (depth == 3)
                st3 = c1;
            else
                st4 = c1;
            cur = c0;
        }
    }
    return word;
}

// The LDS lookup table, staged by every thread of the workgroup; it is the
// kernel's only LDS object, at address 0, so a lookup's LDS address is the
// v_perm_b32 result itself.
template <int BS>
__device__ __forceinline__ void stage_table(uint32_t* s_tab) {
    for (uint32_t m = threadIdx.x; m < kTabBytes / 16; m += BS) {
        const uint32_t v0 = c_te0[m >> 4];
        const uint32_t v = (m & 8) ? rotr(v0, 16) : v0;  // second half of the row: Te2
        reinterpret_cast<u32x4*>(s_tab)[m] = u32x4{v, v, v, v};
    }
    __syncthreads();
}

// Expand node i of level a (key blockIdx.y) by E levels (0 <= E <= 5).
// BITS: write the 2^E leaf bits (E = 5, or a = 0 for domains of at most 32
// leaves) as word i of the key's selection row.  Otherwise write the 2^E
// nodes of level a+E at positions (i << E) .. of the key's output row.
template <int BS, bool BITS>
__global__ void __launch_bounds__(BS)
k_dpf_expand(const uint8_t* __restrict__ keys, uint32_t key_bytes, uint32_t n, uint32_t a, uint32_t E,
             uint64_t count, const u32x4* __restrict__ in, uint64_t in_stride, u32x4* __restrict__ out_nodes,
             uint64_t out_stride, uint32_t* __restrict__ out_bits, uint64_t bits_stride) {
    __shared__ uint32_t s_tab[kTabBytes / 4];
    stage_table<BS>(s_tab);
    const uint64_t i = (uint64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= count) return;
    const uint32_t q = blockIdx.y;
    const u32x4* kq = reinterpret_cast<const u32x4*>(keys + (uint64_t)q * key_bytes);
    const Lut L{s_tab, (threadIdx.x & 31u) * 4u, 128u + (threadIdx.x & 31u) * 4u};
    const u32x4 cur = (a == 0) ? kq[0] : in[q * in_stride + i];  // eq. 2 at the root
    u32x4* orow = BITS ? nullptr : out_nodes + q * out_stride + (i << E);
    const uint32_t word = dfs_expand<BITS>(L, kq, n + 1, a, E, cur, orow);
    if (BITS) out_bits[q * bits_stride + i] = word;
}

// The top T levels of every key's tree in one workgroup per key (blockIdx.x),
// breadth-first: at level a each of the first count(a) threads expands one
// node (eq. 3) into an LDS buffer, a barrier, the next level.  count(a) =
// ceil(n_leaves / 2^(n - a)) nodes lead to leaves below n_leaves.  The
// children of level T - 1 go to out_nodes (row q), where the launch chain
// continues.  This replaces T single-level launches near the root, whose
// cost is launch latency, not work.  Dynamic LDS: the lookup table at
// address 0 (the kernel has no static LDS), then two node buffers of BS.
template <int BS>
__global__ void __launch_bounds__(BS)
k_dpf_top(const uint8_t* __restrict__ keys, uint32_t key_bytes, uint32_t n, uint64_t n_leaves, uint32_t T,
          u32x4* __restrict__ out_nodes, uint64_t out_stride) {
    extern __shared__ __attribute__((aligned(16))) uint32_t dpf_dyn[];
    uint32_t* const s_tab = dpf_dyn;
    u32x4* const nodes = reinterpret_cast<u32x4*>(dpf_dyn + kTabBytes / 4);
    for (uint32_t m = threadIdx.x; m < kTabBytes / 16; m += BS) {
        const uint32_t v0 = c_te0[m >> 4];
        const uint32_t v = (m & 8) ? rotr(v0, 16) : v0;  // second half of the row: Te2
        reinterpret_cast<u32x4*>(s_tab)[m] = u32x4{v, v, v, v};
    }
    const uint32_t q = blockIdx.x;
    const u32x4* kq = reinterpret_cast<const u32x4*>(keys + (uint64_t)q * key_bytes);
    const uint32_t n1 = n + 1;
    const Lut L{s_tab, (threadIdx.x & 31u) * 4u, 128u + (threadIdx.x & 31u) * 4u};
    if (threadIdx.x == 0) nodes[0] = kq[0];  // eq. 2 at the root
    __syncthreads();
    for (uint32_t a = 0; a < T; ++a) {
        const uint32_t sh = n - a;
        const uint64_t cnt = (n_leaves + (1ull << sh) - 1) >> sh;
        const u32x4* src = nodes + (a & 1) * BS;
        u32x4* dst = nodes + ((a + 1) & 1) * BS;
        const bool last = a + 1 == T;
        for (uint32_t i = threadIdx.x; i < cnt; i += BS) {
            u32x4 c0, c1;
            expand(L, kq, n1, a + 1, src[i], c0, c1);
            if (last) {
                out_nodes[q * out_stride + 2 * i] = c0;
                out_nodes[q * out_stride + 2 * i + 1] = c1;
            } else {
                dst[2 * i] = c0;
                dst[2 * i + 1] = c1;
            }
        }
        __syncthreads();
    }
}

}  // namespace

// ------------------------------------------------------------ host side

static std::once_flag g_setup_once[64];
static hipError_t g_setup_err[64];

static hipError_t setup_device(int device) {
    std::call_once(g_setup_once[device & 63], [device] {
        g_setup_err[device & 63] = hipMemcpyToSymbol(HIP_SYMBOL(c_te0), tables().te0, sizeof(uint32_t) * 256);
    });
    return g_setup_err[device & 63];
}

uint64_t dpf_key_bytes(uint32_t n) { return 64ull * (n + 1); }

static inline uint64_t ceil_shift(uint64_t x, uint32_t s) { return (x + (1ull << s) - 1) >> s; }

// Levels the top kernel expands for a 2^n domain (0: none).  Level T must
// still be at most n - 5 (the chain's last launch expands five levels, or
// the whole tree for n <= 5), and 2^(T-1) nodes fit in a node buffer.
uint32_t dpf_top_levels(uint32_t n) { return n > 5 ? std::min<uint32_t>(kDpfTopLevels, n - 5) : 0; }

// The chain of launches from level a0 for a 2^n domain as (a, E) pairs; the
// last one writes bits.  Near the root, where a level has few nodes, a launch
// expands one to three levels (its latency is E sequential expansions per
// thread); below, five.
int dpf_plan(uint32_t n, uint64_t n_leaves, uint32_t n_keys, uint32_t a0, uint32_t steps[][2]) {
    int ns = 0;
    uint32_t a = a0;
    while (n > a + 5) {
        const uint64_t threads = ceil_shift(n_leaves, n - a) * n_keys;
        uint32_t E = threads < 4096 ? 1 : threads < 65536 ? 2 : threads < (1u << 19) ? 3 : 5;
        if (E > n - 5 - a) E = n - 5 - a;
        steps[ns][0] = a;
        steps[ns][1] = E;
        ++ns;
        a += E;
    }
    steps[ns][0] = a;
    steps[ns][1] = n - a;
    return ns + 1;
}

uint64_t dpf_scratch_nodes(uint32_t n, uint64_t n_leaves) {
    // the widest level written to HBM is n - 5; a launch writes all 2^E
    // children of each of its nodes, so round up by one group
    if (n <= 5) return 0;
    return ceil_shift(n_leaves, 5) + 32;
}

template <int BS>
static void launch_step(bool bits, dim3 grid, hipStream_t s, const uint8_t* d_keys, uint32_t kb, uint32_t n,
                        uint32_t a, uint32_t E, uint64_t count, const u32x4* in, uint64_t in_stride, u32x4* out,
                        uint64_t out_stride, uint32_t* d_sel, uint64_t stride_words) {
    if (bits)
        hipLaunchKernelGGL((k_dpf_expand<BS, true>), grid, dim3(BS), 0, s, d_keys, kb, n, a, E, count, in, in_stride,
                           nullptr, 0, d_sel, stride_words);
    else
        hipLaunchKernelGGL((k_dpf_expand<BS, false>), grid, dim3(BS), 0, s, d_keys, kb, n, a, E, count, in,
                           in_stride, out, out_stride, nullptr, 0);
}

// Threads per workgroup of a chain launch over `count` nodes per key: large
// launches use 1024-thread workgroups, one per CU, sharing one table copy
// between 16 waves; small ones 256 threads, spread over more CUs.
static int launch_threads(uint64_t count, uint32_t n_keys) { return count * n_keys >= kDpfBigLaunch ? 1024 : 256; }

hipError_t launch_dpf_eval(int device, const uint8_t* d_keys, uint32_t n, uint32_t n_keys, uint64_t n_leaves,
                           uint32_t* d_sel, uint64_t stride_words, void* scratch, uint64_t scratch_nodes,
                           hipStream_t s) {
    hipError_t e = setup_device(device);
    if (e != hipSuccess) return e;
    uint32_t steps[64][2];
    const uint32_t T = dpf_top_levels(n);
    const int ns = dpf_plan(n, n_leaves, n_keys, T, steps);
    const uint32_t kb = (uint32_t)dpf_key_bytes(n);
    u32x4* buf[2] = {reinterpret_cast<u32x4*>(scratch),
                     reinterpret_cast<u32x4*>(scratch) + (uint64_t)n_keys * scratch_nodes};
    // `in` always points into the scratch (the a = 0 launch reads the root
    // from the key instead, but a valid pointer keeps any load in bounds)
    const u32x4* in = buf[1];
    int slot = 0;  // buffer the next launch writes
    if (T > 0) {
        constexpr uint32_t bytes = kTabBytes + 2 * kDpfTopThreads * 16;
        e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_dpf_top<kDpfTopThreads>), (int)bytes);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_dpf_top<kDpfTopThreads>), dim3(n_keys), dim3(kDpfTopThreads), bytes, s, d_keys, kb, n,
                           n_leaves, T, buf[0], scratch_nodes);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        in = buf[0];
        slot = 1;
    }
    for (int k = 0; k < ns; ++k) {
        const uint32_t a = steps[k][0], E = steps[k][1];
        const uint64_t count = ceil_shift(n_leaves, n - a);
        const bool bits = k + 1 == ns;
        u32x4* out = bits ? nullptr : buf[slot];
        slot ^= 1;
        if (launch_threads(count, n_keys) == 1024)
            launch_step<1024>(bits, dim3((uint32_t)((count + 1023) / 1024), n_keys), s, d_keys, kb, n, a, E, count, in,
                              scratch_nodes, out, scratch_nodes, d_sel, stride_words);
        else
            launch_step<256>(bits, dim3((uint32_t)((count + 255) / 256), n_keys), s, d_keys, kb, n, a, E, count, in,
                             scratch_nodes, out, scratch_nodes, d_sel, stride_words);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (!bits) in = out;
    }
    return hipSuccess;
}

// Client-side key generation for the point function that is 1 at alpha (the
// tree DPF of Boyle, Gilboa and Ishai, CCS 2016, written as the codewords of
// eq. 3): C0[0][0] is the party's root (its bit 0 is the party index), every
// other C0 block is zero; C1[x][d] is the level-d correction word for child
// x, the same in both keys; C1[x][0] is zero.
void dpf_gen_host(uint64_t alpha, uint32_t n, const uint8_t root0[16], const uint8_t root1[16], uint8_t* key0,
                  uint8_t* key1) {
    const size_t kb = dpf_key_bytes(n);
    memset(key0, 0, kb);
    memset(key1, 0, kb);
    const uint32_t n1 = n + 1;
    auto blk = [n1](uint8_t* k, int cw, int x, uint32_t d) { return k + ((size_t)cw * 2 * n1 + x * n1 + d) * 16; };
    uint8_t r[2][16];
    memcpy(r[0], root0, 16);
    memcpy(r[1], root1, 16);
    r[0][0] = (uint8_t)(r[0][0] & 0xFE);
    r[1][0] = (uint8_t)((r[1][0] & 0xFE) | 1);
    memcpy(blk(key0, 0, 0, 0), r[0], 16);
    memcpy(blk(key1, 0, 0, 0), r[1], 16);
    for (uint32_t d = 1; d <= n; ++d) {
        const int on = (int)((alpha >> (n - d)) & 1), off = on ^ 1;
        uint8_t g[2][2][16];  // [party][child]
        for (int b = 0; b < 2; ++b)
            for (int x = 0; x < 2; ++x) host_aes::prf(r[b], x, g[b][x]);
        uint8_t c[2][16];
        for (int x = 0; x < 2; ++x) {
            // seed part: the parties' off-path children must coincide
            for (int i = 0; i < 16; ++i) c[x][i] = g[0][off][i] ^ g[1][off][i];
            // control bit: equal off the path, different on it
            const int tc = (g[0][x][0] & 1) ^ (g[1][x][0] & 1) ^ (x == on ? 1 : 0);
            c[x][0] = (uint8_t)((c[x][0] & 0xFE) | tc);
            memcpy(blk(key0, 1, x, d), c[x], 16);
            memcpy(blk(key1, 1, x, d), c[x], 16);
        }
        for (int b = 0; b < 2; ++b) {
            const bool t = r[b][0] & 1;
            for (int i = 0; i < 16; ++i) r[b][i] = (uint8_t)(g[b][on][i] ^ (t ? c[on][i] : 0));
        }
    }
}

}  // namespace pir
