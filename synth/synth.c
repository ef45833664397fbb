/*
 * Seeded synthetic inputs for dpXOR: database records and selection
 * bitvectors.  This module holds no part of the retrieval arithmetic; it only
 * produces bytes.  Both the CPU oracle tests and the GPU path draw their
 * inputs from here.
 *
 * Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), used in its counter form: output word k
 * (k = 0, 1, ...) of the stream with seed s is mix64(s + (k+1)*GAMMA).  Byte o
 * of a stream is byte (o mod 8), little-endian, of word floor(o/8).  This is
 * the same sequence the sequential generator emits, so its published test
 * vectors apply.
 *
 * The paper's workload is a database of uniformly random 32-byte hash records
 * (evaluation, "PIR database"); selection vectors of a two-server scheme are
 * uniformly random bit vectors (multi-server PIR background).  Bytes of the
 * stream are i.i.d. uniform, and so are the bits.
 */
#include <stdint.h>
#include <string.h>
#include <pthread.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

uint64_t synth_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t synth_word(uint64_t seed, uint64_t k) { return synth_mix64(seed + (k + 1) * GAMMA); }

static void fill_range(uint64_t seed, uint64_t off, uint8_t* out, uint64_t n) {
    uint64_t o = off, end = off + n;
    /* leading bytes up to a word boundary */
    while (o < end && (o & 7)) {
        uint64_t w = synth_word(seed, o >> 3);
        *out++ = (uint8_t)(w >> (8 * (o & 7)));
        ++o;
    }
    /* whole words (little-endian byte order) */
    while (o + 8 <= end) {
        uint64_t w = synth_word(seed, o >> 3);
        for (int b = 0; b < 8; ++b) out[b] = (uint8_t)(w >> (8 * b));
        out += 8;
        o += 8;
    }
    while (o < end) {
        uint64_t w = synth_word(seed, o >> 3);
        *out++ = (uint8_t)(w >> (8 * (o & 7)));
        ++o;
    }
}

typedef struct { uint64_t seed, off, n; uint8_t* out; } fill_job;

static void* fill_thread(void* p) {
    fill_job* j = (fill_job*)p;
    fill_range(j->seed, j->off, j->out, j->n);
    return 0;
}

/* Bytes [off, off+n) of stream `seed` into out, using up to `threads` threads. */
void synth_fill_bytes(uint64_t seed, uint64_t off, uint8_t* out, uint64_t n, int threads) {
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    if (n < (1u << 22) || threads == 1) { fill_range(seed, off, out, n); return; }
    pthread_t tid[64];
    fill_job job[64];
    /* ceil(n / threads) rounded up to whole words, so the pieces cover all n bytes */
    uint64_t per = ((n + threads - 1) / threads + 7) & ~7ULL;
    int used = 0;
    for (int t = 0; t < threads; ++t) {
        uint64_t s = per * t;
        if (s >= n) break;
        uint64_t len = (s + per > n) ? n - s : per;
        job[t].seed = seed; job[t].off = off + s; job[t].n = len; job[t].out = out + s;
        if (pthread_create(&tid[t], 0, fill_thread, &job[t]) != 0) { fill_range(seed, off + s, out + s, len); job[t].n = 0; tid[t] = 0; }
        used = t + 1;
    }
    for (int t = 0; t < used; ++t) if (job[t].n && tid[t]) pthread_join(tid[t], 0);
}

/* Seed of query q's selection stream: mix64(sel_seed + q). */
uint64_t synth_sel_seed(uint64_t sel_seed, uint64_t q) { return synth_mix64(sel_seed + q); }

/*
 * Q selection bitvectors over n_records records into rows `stride` bytes
 * apart.  Bit j of row q is bit (j mod 8) of byte floor(j/8) (LSB first) and
 * equals bit (j mod 64) of word floor(j/64) of query q's stream.  Bits at
 * positions >= n_records within the row are cleared when tail_junk == 0 and
 * left as stream bits otherwise; bytes of the row past ceil(n/8) are zero
 * (tail_junk == 0) or 0xA5 (tail_junk != 0).
 */
void synth_selections(uint64_t sel_seed, uint64_t q0, uint32_t nq, uint64_t n_records,
                      uint8_t* out, uint64_t stride, int tail_junk, int threads) {
    uint64_t nbytes = (n_records + 7) / 8;
    for (uint32_t i = 0; i < nq; ++i) {
        uint8_t* row = out + (uint64_t)i * stride;
        synth_fill_bytes(synth_sel_seed(sel_seed, q0 + i), 0, row, nbytes, threads);
        if (!tail_junk && (n_records & 7)) row[nbytes - 1] &= (uint8_t)((1u << (n_records & 7)) - 1);
        if (stride > nbytes) memset(row + nbytes, tail_junk ? 0xA5 : 0, stride - nbytes);
    }
}
