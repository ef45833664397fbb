/*
 * ORACLE for the F_p inner-product form of the server's answer -- TEST
 * INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded C.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the HIP library shares no
 * code with it.
 *
 * IM-PIR Sec. 2 states the database as D in F_p^{N x L} and the server's
 * answer as an inner product of the query vector with the database (Sec. 2,
 * "Multi-Server PIR"; the linear operations of Sec. 3.3); the XOR form the
 * paper implements is the case p = 2 on bits.  This is the definition
 * written out for a prime p:
 *
 *     r[l] = ( sum over j = 0..N-1 of v[j] * D[j][l] ) mod p,   l = 0..L-1
 *
 * with D[j][l] the l-th element of record j (one byte each, row-major, record
 * j at byte j*L) and v[j] one byte per record.  Sums are exact in 64 bits
 * (N * 255 * 255 < 2^64 for any N that fits in memory) and reduced once.
 * Reading: the elements and query values are the integers the bytes hold;
 * the answer elements are in [0, p).
 *
 * Built with: gcc -O2 -std=c11 -fPIC -shared.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Returns 0, or -1 if the accumulator array cannot be allocated. */
int oracle_fp_inner(const uint8_t* db, uint64_t n, uint32_t L, const uint8_t* v, uint32_t p, uint8_t* out) {
    uint64_t* acc = (uint64_t*)calloc(L ? L : 1, sizeof(uint64_t));
    if (!acc) return -1;
    for (uint64_t j = 0; j < n; ++j)
        for (uint32_t l = 0; l < L; ++l) acc[l] += (uint64_t)v[j] * db[j * L + l];
    for (uint32_t l = 0; l < L; ++l) out[l] = (uint8_t)(acc[l] % p);
    free(acc);
    return 0;
}
