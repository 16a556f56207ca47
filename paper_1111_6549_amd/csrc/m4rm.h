// The Four-Russians trailing update (Section 3.2 with MakeTable and
// AddRowsFromTable of Appendix A), templated on its schedule:
//   TW  words per column tile (the row segment one block streams),
//   NT  threads per block,
//   U   rows in flight per thread (independent loads before the lookups).
// For every row i of the block's row chunk and every word w of its tile:
//   C[i][w] ^= T_0[c_i byte 0][w] ^ ... ^ T_7[c_i byte 7][w],
// where T_b holds all 256 sums of the rows 8b..8b+7 of B (restricted to the
// tile) and c_i = coef[i * coef_ld] (bit t = "add row t of B").
#pragma once
#include "dev.h"

namespace gf2 {

template <int TW>
struct M4Lds {
    uint64_t T[8][256][TW];
    uint64_t lo[8][16][TW];
    uint64_t hi[8][16][TW];
    uint64_t Bt[KW][TW];
};

// Tables for one tile: T[b][x] = lo[b][x & 15] ^ hi[b][x >> 4], where lo/hi
// are the 16 sums of rows 8b..8b+3 and 8b+4..8b+7.
template <int TW, int NT>
__device__ __forceinline__ void m4_build_tables(M4Lds<TW> &L, const uint64_t *__restrict__ B, int64_t ldb, int nbits,
                                                int64_t wt0, int64_t w_begin, int64_t w_end, int tid) {
    for (int e = tid; e < KW * TW; e += NT) {
        const int k = e / TW, wl = e % TW;
        const int64_t w = wt0 + wl;
        L.Bt[k][wl] = (k < nbits && w >= w_begin && w < w_end) ? B[(int64_t)k * ldb + w] : 0ull;
    }
    __syncthreads();
    for (int e = tid; e < 8 * 16 * TW * 2; e += NT) {
        const int wl = e % TW;
        const int x = (e / TW) & 15;
        const int b = (e / (TW * 16)) & 7;
        const int half = e / (TW * 16 * 8);
        uint64_t acc = 0;
#pragma unroll
        for (int t = 0; t < 4; t++)
            if ((x >> t) & 1) acc ^= L.Bt[8 * b + 4 * half + t][wl];
        if (half) L.hi[b][x][wl] = acc;
        else L.lo[b][x][wl] = acc;
    }
    __syncthreads();
    const int nbytes = (nbits + 7) >> 3;
    for (int e = tid; e < 8 * 256 * TW; e += NT) {
        const int wl = e % TW;
        const int x = (e / TW) & 255;
        const int b = e / (TW * 256);
        L.T[b][x][wl] = b < nbytes ? (L.lo[b][x & 15][wl] ^ L.hi[b][x >> 4][wl]) : 0ull;
    }
    __syncthreads();
}

template <int TW, int NT, int U>
__device__ __forceinline__ void m4_rows(const M4Lds<TW> &L, uint64_t *__restrict__ C, int64_t ldc,
                                        const uint64_t *__restrict__ coef, int64_t coef_ld, int nbits, int64_t rb,
                                        int64_t re, int64_t wt0, int64_t w_begin, int64_t w_end, int tid) {
    constexpr int RS = NT / TW;
    constexpr int64_t STEP = (int64_t)RS * U;
    const int wl = tid % TW;
    const int rs = tid / TW;
    const int64_t w = wt0 + wl;
    const bool wok = w >= w_begin && w < w_end;
    const int nbytes = (nbits + 7) >> 3;
    // rows i0, i0 + RS, ..., i0 + (U-1) RS; the next batch is loaded while
    // the current one is looked up
    auto load = [&](uint64_t(&cw)[U], uint64_t(&x)[U], int64_t i0) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = i0 + (int64_t)u * RS;
            cw[u] = i < re ? coef[i * coef_ld] : 0ull;
            x[u] = (i < re && wok) ? C[i * ldc + w] : 0ull;
        }
    };
    auto work = [&](const uint64_t(&cw)[U], uint64_t(&x)[U], int64_t i0) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            uint64_t acc = 0;
#pragma unroll
            for (int b = 0; b < 8; b++)
                if (b < nbytes) acc ^= L.T[b][(cw[u] >> (8 * b)) & 255][wl];
            x[u] ^= acc;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = i0 + (int64_t)u * RS;
            if (i < re && wok && cw[u]) C[i * ldc + w] = x[u];
        }
    };
    uint64_t ca[U], xa[U], cb[U], xb[U];
    int64_t i0 = rb + rs;
    if (i0 < re) load(ca, xa, i0);
    for (; i0 < re; i0 += 2 * STEP) {
        const int64_t i1 = i0 + STEP;
        if (i1 < re) load(cb, xb, i1);
        work(ca, xa, i0);
        if (i1 >= re) break;
        if (i1 + STEP < re) load(ca, xa, i1 + STEP);
        work(cb, xb, i1);
    }
}

// Block -> (tile, chunk), tiles fastest.  Blocks are handed to the 8 XCDs
// round-robin, so the logical index is remapped to give each XCD a
// contiguous range: neighbouring tiles of the same rows then share that
// XCD's L2.
__device__ __forceinline__ int xcd_logical(int bid, int G) {
    const int xcd = bid & 7, jx = bid >> 3;
    const int g8 = G >> 3, rem = G & 7;
    return xcd * g8 + (xcd < rem ? xcd : rem) + jx;
}

}  // namespace gf2

namespace gf2 {

// Wave-per-row schedule: a block's column tile is 64 words (512 B of each
// row, one word per lane), the coefficient word of a row is wave-uniform and
// is split on the scalar unit into sixteen 4-bit indices; the tables are
// sixteen 16-entry tables T_t[x] = sum of B rows 4t..4t+3 selected by x, each
// entry 64 words (all lanes of a lookup read one contiguous 512-byte entry).
constexpr int WR_TW = 64;

template <int NT>
__device__ __forceinline__ void m4w_build_tables(uint64_t *__restrict__ T, const uint64_t *__restrict__ B, int64_t ldb,
                                                 int nbits, int64_t wt0, int64_t w_begin, int64_t w_end, int tid) {
    // single-row entries and the zero entry
    for (int e = tid; e < KW * WR_TW; e += NT) {
        const int k = e / WR_TW, wl = e % WR_TW;
        const int64_t w = wt0 + wl;
        const int t = k >> 2, b = k & 3;
        T[(t * 16 + (1 << b)) * WR_TW + wl] = (k < nbits && w >= w_begin && w < w_end) ? B[(int64_t)k * ldb + w] : 0ull;
        if (b == 0) T[(t * 16) * WR_TW + wl] = 0ull;
    }
    __syncthreads();
    // entries with two or more bits, from the single-row entries
    for (int e = tid; e < 16 * 16 * WR_TW; e += NT) {
        const int wl = e % WR_TW;
        const int x = (e / WR_TW) & 15;
        const int t = e / (WR_TW * 16);
        if (__popc(x) < 2) continue;
        uint64_t acc = 0;
#pragma unroll
        for (int b = 0; b < 4; b++)
            if ((x >> b) & 1) acc ^= T[(t * 16 + (1 << b)) * WR_TW + wl];
        T[(t * 16 + x) * WR_TW + wl] = acc;
    }
    __syncthreads();
}

template <int NT, int U>
__device__ __forceinline__ void m4w_rows(const uint64_t *__restrict__ T, uint64_t *__restrict__ C, int64_t ldc,
                                         const uint64_t *__restrict__ coef, int64_t coef_ld, int nbits, int64_t rb,
                                         int64_t re, int64_t wt0, int64_t w_begin, int64_t w_end, int tid) {
    constexpr int NWAVE = NT / 64;
    constexpr int64_t STEP = (int64_t)NWAVE * U;
    const int wave = uni(tid >> 6);
    const int lane = tid & 63;
    const int64_t w = wt0 + lane;
    const bool wok = w >= w_begin && w < w_end;
    const int ntab = (nbits + 3) >> 2;
    auto load = [&](uint64_t(&cw)[U], uint64_t(&x)[U], int64_t i0) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = i0 + (int64_t)u * NWAVE;
            cw[u] = i < re ? coef[i * coef_ld] : 0ull;
            x[u] = (i < re && wok) ? C[i * ldc + w] : 0ull;
        }
    };
    auto work = [&](const uint64_t(&cw)[U], uint64_t(&x)[U], int64_t i0) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            uint64_t acc = 0;
#pragma unroll
            for (int t = 0; t < 16; t++) {
                if (t < ntab) {
                    const int nib = (int)((cw[u] >> (4 * t)) & 15);
                    acc ^= T[(t * 16 + nib) * WR_TW + lane];
                }
            }
            x[u] ^= acc;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = i0 + (int64_t)u * NWAVE;
            if (i < re && wok && cw[u]) C[i * ldc + w] = x[u];
        }
    };
    uint64_t ca[U], xa[U], cb[U], xb[U];
    int64_t i0 = rb + wave;
    if (i0 < re) load(ca, xa, i0);
    for (; i0 < re; i0 += 2 * STEP) {
        const int64_t i1 = i0 + STEP;
        if (i1 < re) load(cb, xb, i1);
        work(ca, xa, i0);
        if (i1 >= re) break;
        if (i1 + STEP < re) load(ca, xa, i1 + STEP);
        work(cb, xb, i1);
    }
}

}  // namespace gf2

namespace gf2 {

// Nibble-table schedule for one block working alone (the batched kernel):
// sixteen 16-entry tables T_t[x] = sum of B rows 4t..4t+3 selected by x, over
// a tile of TW words; a thread owns one word of the tile and U rows in
// flight.  Tables are built from the tile's B rows staged in LDS.
template <int TW>
struct M4NLds {
    uint64_t T[16][16][TW];
    uint64_t Bt[KW][TW];
};

template <int TW, int NT>
__device__ __forceinline__ void m4n_build_tables(M4NLds<TW> &L, const uint64_t *__restrict__ B, int64_t ldb, int nbits,
                                                 int64_t wt0, int64_t w_begin, int64_t w_end, int tid) {
    for (int e = tid; e < KW * TW; e += NT) {
        const int k = e / TW, wl = e % TW;
        const int64_t w = wt0 + wl;
        L.Bt[k][wl] = (k < nbits && w >= w_begin && w < w_end) ? B[(int64_t)k * ldb + w] : 0ull;
    }
    __syncthreads();
    for (int e = tid; e < 16 * 16 * TW; e += NT) {
        const int wl = e % TW;
        const int x = (e / TW) & 15;
        const int t = e / (TW * 16);
        uint64_t acc = 0;
#pragma unroll
        for (int b = 0; b < 4; b++)
            if ((x >> b) & 1) acc ^= L.Bt[4 * t + b][wl];
        L.T[t][x][wl] = acc;
    }
    __syncthreads();
}

template <int TW, int NT, int U>
__device__ __forceinline__ void m4n_rows(const M4NLds<TW> &L, uint64_t *__restrict__ C, int64_t ldc,
                                         const uint64_t *__restrict__ coef, int nbits, int64_t rb, int64_t re,
                                         int64_t wt0, int64_t w_begin, int64_t w_end, int tid) {
    constexpr int RS = NT / TW;
    const int wl = tid % TW;
    const int rs = tid / TW;
    const int64_t w = wt0 + wl;
    const bool wok = w >= w_begin && w < w_end;
    const int ntab = (nbits + 3) >> 2;
    for (int64_t i0 = rb + rs; i0 < re; i0 += (int64_t)RS * U) {
        uint64_t cw[U], x[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = i0 + (int64_t)u * RS;
            cw[u] = i < re ? coef[i] : 0ull;
            x[u] = (i < re && wok && cw[u]) ? C[i * ldc + w] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            uint64_t acc = 0;
#pragma unroll
            for (int t = 0; t < 16; t++)
                if (t < ntab) acc ^= L.T[t][(cw[u] >> (4 * t)) & 15][wl];
            const int64_t i = i0 + (int64_t)u * RS;
            if (i < re && wok && cw[u]) C[i * ldc + w] = x[u] ^ acc;
        }
    }
}

}  // namespace gf2
