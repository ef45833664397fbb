/*
 * ORACLE for dpXOR -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded, obviously correct CPU code.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path (the HIP library and its Python binding) never calls it and
 * shares no code with it.
 *
 * What it computes (IM-PIR, Sec. 2 "Multi-Server PIR", the display equation
 * for the server subresult r, and Sec. 3.3 "Inner products and XORing
 * operations"):
 *
 *     r = XOR over j = 0 .. N-1 of  v[j] * D[j]
 *
 * where D[j] is record j (R bytes), v[j] in {0,1} is bit j of the selection
 * vector (the expanded DPF key share Eval(k, j)), and v[j] * D[j] is D[j] when
 * the bit is set and the all-zero record otherwise.  Over F_2 this is exact;
 * every tiling or reduction order gives the same bytes.
 *
 * Layout readings (the paper leaves these open):
 *  - record j occupies bytes [j*R, (j+1)*R) of the database buffer;
 *  - bit j of a selection vector is (sel[j >> 3] >> (j & 7)) & 1 (LSB first);
 *  - bits at positions >= N are ignored;
 *  - the empty sum is the all-zero record (the zero initialisation of the
 *    per-tasklet, per-DPU and host accumulators in the paper's Algorithm 1).
 *
 * Built with: gcc -O2 -std=c11 -fPIC -shared (no intrinsics, no threads).
 */
#include <stdint.h>
#include <string.h>

/* r = XOR_{j<n} v[j] * D[j] for one selection vector. */
void oracle_dpxor(const uint8_t* db, uint64_t n_records, uint32_t record_bytes,
                  const uint8_t* sel, uint8_t* out) {
    memset(out, 0, record_bytes);
    for (uint64_t j = 0; j < n_records; ++j) {
        int bit = (sel[j >> 3] >> (j & 7)) & 1;
        if (bit) {
            const uint8_t* rec = db + j * (uint64_t)record_bytes;
            for (uint32_t b = 0; b < record_bytes; ++b) out[b] ^= rec[b];
        }
    }
}

/* Q independent queries: row q of out is oracle_dpxor of row q of sel. */
void oracle_dpxor_batch(const uint8_t* db, uint64_t n_records, uint32_t record_bytes,
                        const uint8_t* sel, uint64_t sel_stride, uint32_t q, uint8_t* out) {
    for (uint32_t i = 0; i < q; ++i)
        oracle_dpxor(db, n_records, record_bytes, sel + (uint64_t)i * sel_stride,
                     out + (uint64_t)i * record_bytes);
}

/* Client reconstruction of the two-server scheme: D[i] = r1 XOR r2. */
void oracle_reconstruct(const uint8_t* r1, const uint8_t* r2, uint32_t record_bytes, uint8_t* out) {
    for (uint32_t b = 0; b < record_bytes; ++b) out[b] = r1[b] ^ r2[b];
}
