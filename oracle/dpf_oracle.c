/*
 * ORACLE for the DPF step before dpXOR -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded C.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the HIP library shares no
 * code with it.
 *
 * 1. AES-128 as specified in FIPS-197 (Sec. 5.1 Cipher, Sec. 5.2
 *    KeyExpansion).  The S-box is computed from its definition (Sec. 5.1.1:
 *    multiplicative inverse in GF(2^8) modulo x^8+x^4+x^3+x+1, then the
 *    affine map), not copied from a table.
 *
 * 2. DPF evaluation exactly as IM-PIR Sec. 3.2 writes it (eq. 1-3):
 *        Eval(k, j) = R(n, j),  n = log2 N                          (1)
 *        R(0, 0)    = C0[0, 0]                                       (2)
 *        R(d, j)    = PRF_{R(d-1, j/2)}(j mod 2)
 *                     + C_{R(d-1, j/2) mod 2}[j mod 2, d]            (3)
 *    Readings: node values are 128-bit blocks (lambda = 128); "+" in
 *    F_{2^lambda} is XOR; "mod 2" is the low bit (bit 0 of byte 0); PRF_s(x)
 *    is AES-128 under key s of the block whose byte 0 is x and whose other
 *    bytes are 0; the selection bit of leaf j is the low bit of Eval(k, j).
 *
 * 3. Key generation for a point function P_{alpha,1} (Sec. 3.1: Gen(1^lambda,
 *    i) -> (k1, k2), each key two codewords C0, C1 of 2 x (n+1) blocks).  The
 *    paper takes its construction from prior work without restating it; this
 *    oracle uses the tree-based construction of Boyle, Gilboa and Ishai
 *    ("Function Secret Sharing: Improvements and Extensions", CCS 2016, the
 *    DPF of its Fig. 1) in the codeword form of eq. 3:
 *      - C0[0][0] is the party's root (party b's root has low bit b), all
 *        other C0 entries are zero;
 *      - C1[x][d] (d = 1..n) is the level-d correction word for child x,
 *        identical in both keys; C1[x][0] is zero.
 *    The two root seeds are inputs (the caller draws them).
 *    Byte compatibility of these keys with the construction the paper cites
 *    is parity unpinned (that work's code is not available here); what the
 *    tests pin is the point-function identity for every key this produces,
 *    and eq. 1-3 for arbitrary codewords (AESAVS known answers).
 *
 * Built with: gcc -O2 -std=c11 -fPIC -shared.
 */
#include <stdint.h>
#include <string.h>

/* ------------------------------------------------------------------ AES */

static uint8_t SBOX[256];
static int sbox_ready = 0;

static uint8_t gf_mul(uint8_t a, uint8_t b) {
    uint8_t p = 0;
    while (b) {
        if (b & 1) p ^= a;
        uint8_t hi = a & 0x80;
        a <<= 1;
        if (hi) a ^= 0x1b; /* reduce modulo x^8 + x^4 + x^3 + x + 1 */
        b >>= 1;
    }
    return p;
}

static uint8_t gf_inv(uint8_t a) {
    if (a == 0) return 0; /* {00} maps to itself */
    for (int c = 1; c < 256; ++c)
        if (gf_mul(a, (uint8_t)c) == 1) return (uint8_t)c;
    return 0;
}

static uint8_t rotl8(uint8_t x, int s) { return (uint8_t)((x << s) | (x >> (8 - s))); }

static void build_sbox(void) {
    if (sbox_ready) return;
    for (int x = 0; x < 256; ++x) {
        uint8_t b = gf_inv((uint8_t)x);
        SBOX[x] = b ^ rotl8(b, 1) ^ rotl8(b, 2) ^ rotl8(b, 3) ^ rotl8(b, 4) ^ 0x63;
    }
    sbox_ready = 1;
}

uint8_t oracle_aes_sbox(uint8_t x) {
    build_sbox();
    return SBOX[x];
}

/* FIPS-197 Sec. 5.2: 44 words w[0..43]; word i = bytes 4i..4i+3 of rk. */
static void key_expansion(const uint8_t key[16], uint8_t rk[176]) {
    build_sbox();
    memcpy(rk, key, 16);
    uint8_t rcon = 0x01;
    for (int i = 4; i < 44; ++i) {
        uint8_t t[4];
        memcpy(t, rk + 4 * (i - 1), 4);
        if (i % 4 == 0) {
            uint8_t t0 = t[0]; /* RotWord, SubWord, Rcon */
            t[0] = SBOX[t[1]] ^ rcon;
            t[1] = SBOX[t[2]];
            t[2] = SBOX[t[3]];
            t[3] = SBOX[t0];
            rcon = gf_mul(rcon, 0x02);
        }
        for (int b = 0; b < 4; ++b) rk[4 * i + b] = rk[4 * (i - 4) + b] ^ t[b];
    }
}

/* FIPS-197 Sec. 5.1; the state is column-major: s[r + 4c] = in[r + 4c]. */
void oracle_aes128_encrypt(const uint8_t key[16], const uint8_t in[16], uint8_t out[16]) {
    uint8_t rk[176], s[16], t[16];
    key_expansion(key, rk);
    for (int i = 0; i < 16; ++i) s[i] = in[i] ^ rk[i];
    for (int round = 1; round <= 10; ++round) {
        for (int i = 0; i < 16; ++i) s[i] = SBOX[s[i]];                  /* SubBytes */
        for (int r = 0; r < 4; ++r)                                       /* ShiftRows */
            for (int c = 0; c < 4; ++c) t[r + 4 * c] = s[r + 4 * ((c + r) % 4)];
        memcpy(s, t, 16);
        if (round != 10) {                                                /* MixColumns */
            for (int c = 0; c < 4; ++c) {
                uint8_t a0 = s[4 * c], a1 = s[4 * c + 1], a2 = s[4 * c + 2], a3 = s[4 * c + 3];
                s[4 * c + 0] = gf_mul(a0, 2) ^ gf_mul(a1, 3) ^ a2 ^ a3;
                s[4 * c + 1] = a0 ^ gf_mul(a1, 2) ^ gf_mul(a2, 3) ^ a3;
                s[4 * c + 2] = a0 ^ a1 ^ gf_mul(a2, 2) ^ gf_mul(a3, 3);
                s[4 * c + 3] = gf_mul(a0, 3) ^ a1 ^ a2 ^ gf_mul(a3, 2);
            }
        }
        for (int i = 0; i < 16; ++i) s[i] ^= rk[16 * round + i];        /* AddRoundKey */
    }
    memcpy(out, s, 16);
}

/* ------------------------------------------------------------------ DPF */

/* Key layout (one party): C0 then C1, each 2 x (n+1) blocks of 16 bytes,
 * block [x][d] at offset ((x * (n+1)) + d) * 16 within its codeword. */
static uint8_t* cw(uint8_t* key, int n, int which, int x, int d) {
    return key + ((size_t)which * 2 * (n + 1) + (size_t)x * (n + 1) + d) * 16;
}
static const uint8_t* ccw(const uint8_t* key, int n, int which, int x, int d) {
    return key + ((size_t)which * 2 * (n + 1) + (size_t)x * (n + 1) + d) * 16;
}

uint64_t oracle_dpf_key_bytes(int n) { return (uint64_t)2 * 2 * (n + 1) * 16; }

static void prf(const uint8_t s[16], int x, uint8_t out[16]) {
    uint8_t blk[16] = {0};
    blk[0] = (uint8_t)x;
    oracle_aes128_encrypt(s, blk, out);
}

/* Eval(k, j): the full 128-bit leaf value R(n, j) by eq. (1)-(3). */
void oracle_dpf_eval_block(const uint8_t* key, int n, uint64_t j, uint8_t out[16]) {
    uint8_t r[16], g[16];
    memcpy(r, ccw(key, n, 0, 0, 0), 16); /* (2) */
    for (int d = 1; d <= n; ++d) {
        const int x = (int)((j >> (n - d)) & 1); /* j mod 2 at depth d; the parent is j / 2 */
        const int t = r[0] & 1;                  /* R(d-1, j/2) mod 2 */
        prf(r, x, g);
        const uint8_t* c = ccw(key, n, t, x, d);
        for (int i = 0; i < 16; ++i) r[i] = g[i] ^ c[i]; /* (3) */
    }
    memcpy(out, r, 16);
}

int oracle_dpf_eval_bit(const uint8_t* key, int n, uint64_t j) {
    uint8_t r[16];
    oracle_dpf_eval_block(key, n, j, r);
    return r[0] & 1;
}

/* All 2^n selection bits, packed LSB first: bit j at (out[j>>3] >> (j&7)). */
void oracle_dpf_eval_full(const uint8_t* key, int n, uint8_t* out) {
    const uint64_t N = (uint64_t)1 << n;
    memset(out, 0, (N + 7) / 8);
    for (uint64_t j = 0; j < N; ++j)
        if (oracle_dpf_eval_bit(key, n, j)) out[j >> 3] |= (uint8_t)(1u << (j & 7));
}

/* Gen for P_{alpha,1} over a 2^n domain (BGI16 Fig. 1, codeword form).
 * root0/root1: 16 random bytes each (their low bits are overwritten with the
 * party index).  key0/key1: oracle_dpf_key_bytes(n) bytes each. */
void oracle_dpf_gen(uint64_t alpha, int n, const uint8_t root0[16], const uint8_t root1[16],
                    uint8_t* key0, uint8_t* key1) {
    const size_t kb = (size_t)oracle_dpf_key_bytes(n);
    memset(key0, 0, kb);
    memset(key1, 0, kb);
    uint8_t r0[16], r1[16];
    memcpy(r0, root0, 16);
    memcpy(r1, root1, 16);
    r0[0] = (uint8_t)(r0[0] & 0xFE);        /* t = 0 */
    r1[0] = (uint8_t)((r1[0] & 0xFE) | 1);  /* t = 1 */
    memcpy(cw(key0, n, 0, 0, 0), r0, 16);
    memcpy(cw(key1, n, 0, 0, 0), r1, 16);
    for (int d = 1; d <= n; ++d) {
        const int keep = (int)((alpha >> (n - d)) & 1), lose = 1 - keep;
        uint8_t g0[2][16], g1[2][16];
        prf(r0, 0, g0[0]);
        prf(r0, 1, g0[1]);
        prf(r1, 0, g1[0]);
        prf(r1, 1, g1[1]);
        uint8_t c[2][16];
        for (int x = 0; x < 2; ++x) {
            for (int i = 0; i < 16; ++i) c[x][i] = g0[lose][i] ^ g1[lose][i]; /* seed part */
            /* control bit: off the path the two parties end equal (XOR 0),
             * on the path they differ (XOR 1) */
            const int tcw = (g0[x][0] & 1) ^ (g1[x][0] & 1) ^ (x == keep ? 1 : 0);
            c[x][0] = (uint8_t)((c[x][0] & 0xFE) | tcw);
            memcpy(cw(key0, n, 1, x, d), c[x], 16);
            memcpy(cw(key1, n, 1, x, d), c[x], 16);
        }
        const int t0 = r0[0] & 1, t1 = r1[0] & 1;
        for (int i = 0; i < 16; ++i) {
            r0[i] = g0[keep][i] ^ (t0 ? c[keep][i] : 0);
            r1[i] = g1[keep][i] ^ (t1 ? c[keep][i] : 0);
        }
    }
}
