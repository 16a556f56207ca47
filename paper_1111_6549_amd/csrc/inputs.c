/*
 * Seeded synthetic inputs: bit-packed GF(2) matrices.
 *
 * This file only draws random bits.  It contains no elimination, no table
 * and no product: the PLE decomposition and everything that checks it live
 * elsewhere.  Both the HIP library's tests and the CPU oracle's tests get
 * their inputs from here.
 *
 * Packed format: row-major, `ldw` 64-bit words per row; column j of row i is
 * bit (j & 63) of word i*ldw + (j >> 6).  Bits at columns >= n are zero.
 *
 * Generator: every row has its own xoshiro256** stream, seeded through
 * splitmix64 from (seed, stream id).  The stream id of row i is i + id_base,
 * so a matrix can be regenerated one row at a time.
 *   density 1/2 : each word is one raw 64-bit output (last word masked);
 *   density p   : one output per bit, bit = (out >> 32) < thresh,
 *                 thresh = round(p * 2^32).
 */
#include <stdint.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += GOLDEN);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

typedef struct { uint64_t s[4]; } xoshiro;

static inline void xo_seed(xoshiro *g, uint64_t seed, uint64_t id) {
    uint64_t x = seed ^ (GOLDEN * (id + 1));
    for (int i = 0; i < 4; i++) g->s[i] = splitmix64(&x);
}

static inline uint64_t xo_next(xoshiro *g) {
    uint64_t *s = g->s;
    uint64_t res = rotl64(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return res;
}

/* Fill an m x n packed matrix (row stride ldw words).  thresh == 0 selects
 * density 1/2 (raw words); otherwise bit = (out >> 32) < thresh. */
void gf2in_bernoulli(uint64_t *out, int64_t m, int64_t n, int64_t ldw,
                     uint64_t seed, uint64_t id_base, uint64_t thresh) {
    int64_t nw = (n + 63) / 64;
    uint64_t lastmask = (n % 64) ? ((1ULL << (n % 64)) - 1) : ~0ULL;
#pragma omp parallel for schedule(static) if (m * nw > (1 << 16))
    for (int64_t i = 0; i < m; i++) {
        xoshiro g;
        xo_seed(&g, seed, id_base + (uint64_t)i);
        uint64_t *row = out + i * ldw;
        if (thresh == 0) {
            for (int64_t w = 0; w < nw; w++) row[w] = xo_next(&g);
        } else {
            for (int64_t w = 0; w < nw; w++) {
                uint64_t word = 0;
                int64_t nb = (w == nw - 1 && (n % 64)) ? (n % 64) : 64;
                for (int64_t b = 0; b < nb; b++)
                    if ((xo_next(&g) >> 32) < thresh) word |= 1ULL << b;
                row[w] = word;
            }
        }
        if (nw > 0) row[nw - 1] &= lastmask;
        for (int64_t w = nw; w < ldw; w++) row[w] = 0;
    }
}

/* Raw stream outputs (used by the Python side for derived draws). */
void gf2in_raw(uint64_t *out, int64_t count, uint64_t seed, uint64_t id) {
    xoshiro g;
    xo_seed(&g, seed, id);
    for (int64_t i = 0; i < count; i++) out[i] = xo_next(&g);
}
