// Block-recursive PLE (Algorithm 3, Section 3.3) on top of the
// block-iterative pass loop (Algorithm 2), for gf2_ple with update = 2
// (products on the fp4 matrix cores), 3 (products on the Four-Russians
// tables) or 4 (products on the int8 matrix cores).
//
// One level on the m x n block A, split at column n1 (a multiple of 64):
//   1. PLE of the left block [A0 A1]'s first n1 columns; its swaps move whole
//      rows, so the right block A1 ends up with its rows permuted (P1^T A1);
//   2. A01 <- L00^-1 A01 on the first r1 rows of A1 (triangular solve, in
//      blocks of 128 rows: each block's own forward substitution, then one
//      Four-Russians sweep that removes the block from every row below it;
//      with fp4 products, in diagonal blocks of 4096 rows solved that way,
//      each removed from the rows below by one product);
//   3. A11 <- A11 + L10 A01 (the product that Algorithm 3 hands to matrix
//      multiplication);
//   4. PLE of A11 (rows r1.., columns n1..), again moving whole rows, so the
//      L bits of A10 take its swaps too;
//   5. P, Q and the rank of the two blocks combined (P_{r1+i} = r1 + P2_i,
//      Q_{r1+i} = n1 + Q2_i), and the right block's L bits moved left from
//      column n1 to column r1 (Algorithm 3's closing column moves), which
//      gives the same clean L\E form as Algorithm 2.
// Both PLEs recurse while levels remain; the leaves are the pass loop.
#include <algorithm>

#include "alg3.h"
#include "dev.h"
#include "m4rm.h"

namespace gf2 {

hipError_t launch_m4rm(uint64_t *C, int64_t ldc, int64_t m, const uint64_t *coef, int64_t coef_ld, const uint64_t *B,
                       int64_t ldb, int nbits, int64_t w_begin, int64_t w_end, int m4_variant, int m4_target,
                       hipStream_t s);
hipError_t launch_transpose_bits(const uint64_t *B, int64_t ldb, int64_t k, int64_t n, uint64_t *Bt, int64_t ldbt,
                                 hipStream_t s);
hipError_t launch_mfma_gf2(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda, const uint64_t *Bt, int64_t ldbt,
                           int64_t m, int64_t k, int64_t n, hipStream_t s, int fmt);
int device_cu_count();

// X <- L^-1 X on one diagonal block of nb <= 128 rows (step 2): rows
// j0 .. j0 + nb - 1 of A, whose L bits left of the diagonal inside the block
// sit in words lw, lw + 1, and X = their words [xw0, xw1).  One wave per
// word of X, two rows per lane: row j0 + l (L bits: word lw, bits < l) and
// row j0 + 64 + l (all of word lw, then word lw + 1, bits < l).  Forward
// substitution: once row j is final its word goes by readlane to every lane
// whose row has L[.][j] = 1; the first 64 rows are final after 64 steps, and
// by then their words are folded into the second half too.
__global__ __launch_bounds__(256) void k_trsm128(uint64_t *__restrict__ A, int64_t ldw, int64_t j0, int nb, int64_t lw,
                                                 int64_t xw0, int64_t xw1) {
    const int lane = threadIdx.x & 63;
    const int64_t w = xw0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= xw1) return;  // w is the same for the whole wave
    const bool on0 = lane < nb, on1 = 64 + lane < nb;
    uint64_t *row0 = A + (j0 + (on0 ? lane : 0)) * ldw;
    uint64_t *row1 = A + (j0 + (on1 ? 64 + lane : 0)) * ldw;
    uint64_t x0 = on0 ? row0[w] : 0ull, x1 = on1 ? row1[w] : 0ull;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint64_t l0 = on0 ? (row0[lw] & below) : 0ull;
    const uint64_t l1a = on1 ? row1[lw] : 0ull;
    const uint64_t l1b = on1 ? (row1[lw + 1] & below) : 0ull;
    // every step runs (rows past nb are zero with zero L bits); with j a
    // constant, bit j of an L word becomes an all-ones or zero 32-bit mask in
    // one signed bit-field extract (the builtin's result type is unsigned:
    // the mask is applied to each half of the row word, never widened)
    auto bitmask = [](uint64_t l, int j) -> uint32_t {
        const uint32_t h = (uint32_t)(j < 32 ? l : (l >> 32));
        return __builtin_amdgcn_sbfe(h, (unsigned)(j & 31), 1u);
    };
    // x ^= xj & mask, one v_bitop3 per half: S1 ^ (S0 & S2) with S0 = xj,
    // S1 = x, S2 = mask (truth table 0x6C; the function is symmetric in S0
    // and S2, so the table does not depend on which operand is the high
    // index bit)
    auto apply = [](uint64_t x, uint64_t xj, uint32_t msk) -> uint64_t {
        const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)xj, (uint32_t)x, msk, 0x6C);
        const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(xj >> 32), (uint32_t)(x >> 32), msk, 0x6C);
        return ((uint64_t)hi << 32) | lo;
    };
#pragma unroll
    for (int j = 0; j < 64; j++) {
        const uint64_t xj = readlane64(x0, j);
        x0 = apply(x0, xj, bitmask(l0, j));
        x1 = apply(x1, xj, bitmask(l1a, j));
    }
#pragma unroll
    for (int j = 0; j < 63; j++) {
        const uint64_t xj = readlane64(x1, j);
        x1 = apply(x1, xj, bitmask(l1b, j));
    }
    if (on0) row0[w] = x0;
    if (on1) row1[w] = x1;
}

// One sweep of the blocked triangular solve: rows [rb_all, re_all) of
// X = A[.][xw0, xw1) lose the solved rows j0 .. j0 + nb - 1 (nb <= 128):
//   X[i] ^= sum_j L[i][j0 + j] X[j0 + j],
// the coefficient bits being row i's L bits in words lw, lw + 1 (all of them
// L bits, as every row below the block is past its columns).  Thirty-two
// 16-entry tables of 4-row sums per 32-word tile in LDS (rows past nb are
// zero, so every table is read and a row's 32 reads carry no branch); 16
// lanes per row, two words per lane, the next row's words loaded during
// this row's lookups.  Blocks: (tile, row chunk), tiles fastest.
constexpr int TP_TW = 32;
__global__ __launch_bounds__(1024) void k_trsm_pair(uint64_t *__restrict__ A, int64_t ldw, int64_t j0, int nb,
                                                    int64_t lw, int64_t rb_all, int64_t re_all, int64_t xw0,
                                                    int64_t xw1, int ntiles, int nchunks) {
    constexpr int NT = 1024, LPR = TP_TW / 2, RS = NT / LPR;
    __shared__ __align__(16) uint64_t T[32][16][TP_TW];
    const int tid = threadIdx.x;
    const int logical = xcd_logical(blockIdx.x, gridDim.x);
    const int tile = logical % ntiles, chunk = logical / ntiles;
    if (chunk >= nchunks) return;
    const int64_t per = (re_all - rb_all + nchunks - 1) / nchunks;
    const int64_t rb = rb_all + (int64_t)chunk * per;
    const int64_t re = rb + per < re_all ? rb + per : re_all;
    if (rb >= re) return;
    const int64_t wt0 = (xw0 & ~(int64_t)(TP_TW - 1)) + (int64_t)tile * TP_TW;
    // single-row entries and the zero entries
    for (int e = tid; e < 128 * TP_TW; e += NT) {
        const int k = e / TP_TW, wl = e % TP_TW;
        const int64_t w = wt0 + wl;
        const int q = k >> 2, b = k & 3;
        T[q][1 << b][wl] = (k < nb && w >= xw0 && w < xw1) ? A[(j0 + k) * ldw + w] : 0ull;
        if (b == 0) T[q][0][wl] = 0ull;
    }
    __syncthreads();
    for (int e = tid; e < 32 * 16 * TP_TW; e += NT) {
        const int wl = e % TP_TW;
        const int x = (e / TP_TW) & 15;
        const int q = e / (TP_TW * 16);
        if (__popc(x) < 2) continue;
        uint64_t acc = 0;
#pragma unroll
        for (int b = 0; b < 4; b++)
            if ((x >> b) & 1) acc ^= T[q][1 << b][wl];
        T[q][x][wl] = acc;
    }
    __syncthreads();
    const int wp = tid % LPR, rs = tid / LPR;
    const int64_t w2 = wt0 + 2 * wp;
    const bool ok0 = w2 >= xw0 && w2 < xw1, ok1 = w2 + 1 >= xw0 && w2 + 1 < xw1;
    const uint32_t tbase = (uint32_t)(2 * wp) * 8u;  // byte offset of this lane's pair of words
    // a lane's two words move as one 16-byte access when the row stride is
    // even and the base 16-byte aligned (tiles start at even words)
    const bool wide = (ldw & 1) == 0 && ((uintptr_t)A & 15) == 0 && ok0 && ok1;
    auto load = [&](int64_t i, uint64_t &c0, uint64_t &c1, uint64_t &v0, uint64_t &v1) {
        if (i < re) {
            const uint64_t *row = A + i * ldw;
            c0 = row[lw];
            c1 = row[lw + 1];
            if (wide) {
                const ulonglong2 v = *(const ulonglong2 *)(row + w2);
                v0 = v.x;
                v1 = v.y;
            } else {
                v0 = ok0 ? row[w2] : 0ull;
                v1 = ok1 ? row[w2 + 1] : 0ull;
            }
        } else {
            c0 = c1 = v0 = v1 = 0ull;
        }
    };
    int64_t i = rb + rs;
    uint64_t nc0, nc1, nv0, nv1;
    load(i, nc0, nc1, nv0, nv1);
    for (; i < re; i += RS) {
        const uint64_t c0 = nc0, c1 = nc1, x0 = nv0, x1 = nv1;
        load(i + RS, nc0, nc1, nv0, nv1);
        const uint32_t h[4] = {(uint32_t)c0, (uint32_t)(c0 >> 32), (uint32_t)c1, (uint32_t)(c1 >> 32)};
        uint64_t a0 = 0, a1 = 0;
#pragma unroll
        for (int g = 0; g < 32; g += 2) {
            ulonglong2 t[2];
#pragma unroll
            for (int j = 0; j < 2; j++) {
                const int q = g + j;
                const uint32_t nib = (h[q >> 3] >> (4 * (q & 7))) & 15u;
                t[j] = *(const ulonglong2 *)((const char *)&T[0][0][0] + tbase +
                                             ((uint32_t)q * 16u + nib) * (uint32_t)(TP_TW * 8));
            }
            a0 = xor3_64(a0, t[0].x, t[1].x);
            a1 = xor3_64(a1, t[0].y, t[1].y);
        }
        if (c0 | c1) {
            uint64_t *row = A + i * ldw;
            if (wide) {
                ulonglong2 v;
                v.x = x0 ^ a0;
                v.y = x1 ^ a1;
                *(ulonglong2 *)(row + w2) = v;
            } else {
                if (ok0) row[w2] = x0 ^ a0;
                if (ok1) row[w2 + 1] = x1 ^ a1;
            }
        }
    }
}

// Step 5, the permutation and rank: the right block's P and Q entries
// (relative to its own rows and columns) become the matrix's, Q past the
// combined rank is -1, and rank = r1 + r2.  q_right = min(m - r1, n - n1)
// entries of Q were written by the right block's PLE.
__global__ void k_alg3_fix(int64_t *P, int64_t m, int64_t *Q, int64_t mn, int64_t *rank, const int64_t *rank2,
                           int64_t r1, int64_t n1, int64_t q_right) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t top = m > mn ? m : mn;
    for (int64_t i = r1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < top; i += stride) {
        if (i < m) P[i] += r1;
        if (i < mn) {
            if (i < r1 + q_right) {
                const int64_t q = Q[i];
                if (q >= 0) Q[i] = q + n1;
            } else {
                Q[i] = -1;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *rank = r1 + *rank2;
}

// bits of the column range [a, b) that fall in word w
__device__ __forceinline__ uint64_t range_bits(int64_t a, int64_t b, int64_t w) {
    const int64_t lo = w * 64;
    const int64_t x0 = a > lo ? a : lo, x1 = b < lo + 64 ? b : lo + 64;
    if (x0 >= x1) return 0ull;
    const int len = (int)(x1 - x0);
    return (len == 64 ? ~0ull : ((1ull << len) - 1ull)) << (x0 - lo);
}

// Step 5, the L bits (only when the left block's rank r1 is below n1): in
// each row i >= r1 the right block's L bits, columns [n1, n1 + nL) with
// nL = min(i - r1, r2), move to columns [r1, r1 + nL); the columns they
// leave become zero.  One thread per row walks its words left to right: a
// word's new value takes source bits from its own and later words only,
// which are still unchanged when it is written.
__global__ void k_alg3_shift(uint64_t *__restrict__ A, int64_t m, int64_t ldw, int64_t r1, int64_t n1,
                             const int64_t *rank2) {
    const int64_t r2 = *rank2;
    const int64_t d = n1 - r1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = r1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const int64_t nL = (i - r1) < r2 ? (i - r1) : r2;
        if (nL <= 0) continue;
        uint64_t *row = A + i * ldw;
        const int64_t s1 = n1 + nL;
        const int64_t wlast = (s1 - 1) >> 6;  // last source word
        for (int64_t w = r1 >> 6; w <= wlast; w++) {
            const uint64_t md = range_bits(r1, r1 + nL, w), ms = range_bits(n1, s1, w);
            uint64_t v = row[w] & ~ms & ~md;
            if (md) {
                const int64_t sc = w * 64 + d;  // source column of the word's bit 0
                const int64_t sw = sc >> 6;
                const int sh = (int)(sc & 63);
                const uint64_t a = row[sw];
                const uint64_t b = (sh && sw + 1 <= wlast) ? row[sw + 1] : 0ull;
                const uint64_t sv = sh ? ((a >> sh) | (b << (64 - sh))) : a;
                v |= sv & md;
            }
            row[w] = v;
        }
    }
}

namespace {

constexpr int MAX_DEPTH = 32;          // rank slots (one per recursion depth)
constexpr int64_t MFMA_MIN_K = 512;    // products with fewer inner bits use the tables

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Ctx {
    int64_t ldw;
    void *ws;  // the pass loop's workspace
    const gf2_ple_opts *opts;
    hipStream_t s;
    bool mfma;
    int fmt;              // matrix-core operands: 0 fp4, 1 int8
    int64_t *rank_slots;  // device, MAX_DEPTH
    uint64_t *bt;         // bit transpose of a product's right operand
    size_t bt_bytes;
    int64_t split;        // 0: halves; > 0: left strips of this many columns
};

// the left block's columns of a split of n columns
int64_t split_cols(int64_t n, int64_t split) {
    return split > 0 ? (split < n ? split : n) : ((n / 2 + 63) & ~(int64_t)63);
}

// A[crow0 .. crow0 + M)[xw0, xw1) ^= (bits [64 kw0, 64 kw0 + K) of those rows)
//                                    x A[brow0 .. brow0 + K)[xw0, xw1)
hipError_t product(Ctx &c, uint64_t *A, int64_t crow0, int64_t M, int64_t kw0, int64_t K, int64_t brow0, int64_t xw0,
                   int64_t xw1, int64_t N) {
    if (M <= 0 || K <= 0 || N <= 0) return hipSuccess;
    const int64_t ldw = c.ldw;
    if (c.mfma && K >= MFMA_MIN_K) {
        const int64_t ldbt = words_for(K);
        if ((size_t)words_for(N) * 64 * (size_t)ldbt * 8 > c.bt_bytes) return hipErrorInvalidValue;
        hipError_t e = launch_transpose_bits(A + brow0 * ldw + xw0, ldw, K, N, c.bt, ldbt, c.s);
        if (e != hipSuccess) return e;
        return launch_mfma_gf2(A + crow0 * ldw + xw0, ldw, A + crow0 * ldw + kw0, ldw, c.bt, ldbt, M, K, N, c.s,
                               c.fmt);
    }
    for (int64_t kb = 0; kb * 64 < K; kb++) {
        const int nb = (int)(K - kb * 64 < 64 ? K - kb * 64 : 64);
        hipError_t e = launch_m4rm(A + crow0 * ldw, ldw, M, A + crow0 * ldw + kw0 + kb, ldw, A + (brow0 + kb * 64) * ldw,
                                   ldw, nb, xw0, xw1, 0, 0, c.s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t trsm128(Ctx &c, uint64_t *A, int64_t j0, int nb, int64_t xw0, int64_t xw1) {
    const int64_t blocks = (xw1 - xw0 + 3) / 4;
    if (blocks <= 0 || nb <= 0) return hipSuccess;
    ProfScope ps(KID_TRSM, c.s);
    hipLaunchKernelGGL(k_trsm128, dim3((unsigned)blocks), dim3(256), 0, c.s, A, c.ldw, j0, nb, j0 >> 6, xw0, xw1);
    return hipGetLastError();
}

// rows [rb, re) of X lose the solved rows j0 .. j0 + nb - 1; the grid is
// whole rounds of one block per CU (at least 256 rows per chunk)
hipError_t trsm_sweep(Ctx &c, uint64_t *A, int64_t j0, int nb, int64_t rb, int64_t re, int64_t xw0, int64_t xw1) {
    if (rb >= re || xw0 >= xw1) return hipSuccess;
    const int64_t base = xw0 & ~(int64_t)(TP_TW - 1);
    const int nt = (int)((xw1 - base + TP_TW - 1) / TP_TW);
    const int64_t slots = device_cu_count();
    int64_t maxc = (re - rb) / 256;
    if (maxc < 1) maxc = 1;
    if (maxc > 4 * slots) maxc = 4 * slots;
    int nchunks = 1;
    double best = -1.0;
    for (int64_t nc = 1; nc <= maxc; nc++) {
        const int64_t g = nt * nc;
        const int64_t rounds = (g + slots - 1) / slots;
        const double eff = (double)g / (double)(rounds * slots) - 0.02 * (double)(rounds - 1);
        if (eff > best + 1e-9) {
            best = eff;
            nchunks = (int)nc;
        }
    }
    ProfScope ps(KID_TRSM, c.s);
    hipLaunchKernelGGL(k_trsm_pair, dim3((unsigned)(nt * nchunks)), dim3(1024), 0, c.s, A, c.ldw, j0, nb, j0 >> 6, rb,
                       re, xw0, xw1, nt, nchunks);
    return hipGetLastError();
}

// rows [d0, d1) of X = A[.][xw0, xw1) <- L^-1 X, with L the unit lower
// triangle of A[d0 .. d1)[d0 .. d1) (d0 a multiple of 128): 128-row blocks
// in order, each solved on its own and then removed from the rows below it
// (up to d1) in one sweep
hipError_t trsm_diag(Ctx &c, uint64_t *A, int64_t d0, int64_t d1, int64_t xw0, int64_t xw1) {
    hipError_t e;
    for (int64_t b = d0; b < d1; b += 128) {
        const int nb = (int)(d1 - b < 128 ? d1 - b : 128);
        if ((e = trsm128(c, A, b, nb, xw0, xw1)) != hipSuccess) return e;
        if ((e = trsm_sweep(c, A, b, nb, b + nb, d1, xw0, xw1)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// With fp4 products, diagonal blocks of this many rows: each is solved by
// the sweeps above, then removed from every row below it by one product
// (inner size TRSM_BLOCK) instead of TRSM_BLOCK / 128 sweeps.  (The int8
// product is too slow at this inner size to gain from it.)
constexpr int64_t TRSM_BLOCK = 4096;

// rows [0, r) of X = A[.][xw0, xw1) <- L^-1 X, with L the unit lower
// triangle of A[0 .. r)[0 .. r)
hipError_t trsm(Ctx &c, uint64_t *A, int64_t r, int64_t xw0, int64_t xw1, int64_t N) {
    if (!c.mfma || c.fmt != 0) return trsm_diag(c, A, 0, r, xw0, xw1);
    hipError_t e;
    for (int64_t d0 = 0; d0 < r; d0 += TRSM_BLOCK) {
        const int64_t d1 = r - d0 < TRSM_BLOCK ? r : d0 + TRSM_BLOCK;
        if ((e = trsm_diag(c, A, d0, d1, xw0, xw1)) != hipSuccess) return e;
        if (d1 < r && (e = product(c, A, d1, r - d1, d0 >> 6, d1 - d0, d0, xw0, xw1, N)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t ple_rec(Ctx &c, uint64_t *A, int64_t m, int64_t n, int64_t *P, int64_t *Q, int64_t *rank, int levels,
                   int64_t wlo, int depth) {
    if (levels <= 0 || n <= 64 || m == 0 || depth >= MAX_DEPTH || (c.split > 0 && n <= c.split))
        return ple_block(A, m, n, c.ldw, P, Q, rank, c.ws, c.opts, c.s, wlo);
    const int64_t ldw = c.ldw;
    const int64_t n1 = split_cols(n, c.split);
    // a strip is a leaf; halves recurse on both sides
    hipError_t e = ple_rec(c, A, m, n1, P, Q, rank, c.split > 0 ? 0 : levels - 1, wlo, depth + 1);
    if (e != hipSuccess) return e;
    int64_t r1 = 0;
    if ((e = hipMemcpyAsync(&r1, rank, 8, hipMemcpyDeviceToHost, c.s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(c.s)) != hipSuccess) return e;
    const int64_t xw0 = n1 >> 6, xw1 = words_for(n), N = n - n1;
    if (r1 > 0) {
        if ((e = trsm(c, A, r1, xw0, xw1, N)) != hipSuccess) return e;
        if ((e = product(c, A, r1, m - r1, 0, r1, 0, xw0, xw1, N)) != hipSuccess) return e;
    }
    if (m <= r1) return hipSuccess;  // then min(m, n) = r1: P and Q are complete
    int64_t *r2 = c.rank_slots + depth;
    if ((e = ple_rec(c, A + r1 * ldw + xw0, m - r1, N, P + r1, Q + r1, r2, levels - 1, wlo - xw0, depth + 1)) !=
        hipSuccess)
        return e;
    const int64_t mn = m < n ? m : n;
    const int64_t q_right = (m - r1) < N ? (m - r1) : N;
    const int64_t top = m > mn ? m : mn;
    int blocks = (int)((top - r1 + 255) / 256);
    blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
    {
        ProfScope ps(KID_INIT, c.s);
        hipLaunchKernelGGL(k_alg3_fix, dim3(blocks), dim3(256), 0, c.s, P, m, Q, mn, rank, (const int64_t *)r2, r1, n1,
                           q_right);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (r1 < n1) {
        int sb = (int)((m - r1 + 255) / 256);
        sb = sb < 1 ? 1 : (sb > 4096 ? 4096 : sb);
        ProfScope ps(KID_INIT, c.s);
        hipLaunchKernelGGL(k_alg3_shift, dim3(sb), dim3(256), 0, c.s, A, m, ldw, r1, n1, (const int64_t *)r2);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

size_t alg3_extra_bytes(int64_t m, int64_t n, int64_t ldw, int levels, bool mfma, int64_t split) {
    (void)ldw;
    size_t b = al((size_t)MAX_DEPTH * 8);
    if (mfma && levels > 0 && n > 64 && !(split > 0 && n <= split)) {
        // the largest product is the first split's: inner size at most
        // min(m, n1), n - n1 columns
        const int64_t n1 = split_cols(n, split);
        const int64_t k = m < n1 ? m : n1;
        b += al((size_t)words_for(n - n1) * 64 * (size_t)words_for(k) * 8);
    }
    return b;
}

hipError_t ple_alg3(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank, void *ws,
                    const gf2_ple_opts *opts, hipStream_t s, int levels, int products, int64_t split) {
    const bool mfma = products != 0;
    Ctx c;
    c.ldw = ldw;
    c.ws = ws;
    c.opts = opts;
    c.s = s;
    c.mfma = mfma;
    c.fmt = products == 2 ? 1 : 0;
    char *extra = (char *)ws + al(ple_workspace_total(m, ldw));
    c.rank_slots = (int64_t *)extra;
    c.bt = (uint64_t *)(extra + al((size_t)MAX_DEPTH * 8));
    c.split = split;
    c.bt_bytes = alg3_extra_bytes(m, n, ldw, levels, mfma, split) - al((size_t)MAX_DEPTH * 8);
    return ple_rec(c, A, m, n, P, Q, rank, levels, 0, 0);
}

}  // namespace gf2
