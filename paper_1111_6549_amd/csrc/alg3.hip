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
//      with fp4 products and a rank above one diagonal block of TRSM_BLOCK
//      rows, the inverses of all diagonal blocks are computed that way at
//      once, then each block, in order, loses the solved blocks above it
//      and is multiplied by its inverse, both as products);
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
hipError_t launch_fp4_product2(uint64_t *C0, int64_t ldc0, int64_t rows0, int64_t words0, uint64_t *C1, int64_t ldc1,
                               int64_t rows1, int64_t words1, const uint64_t *A, int64_t lda, const uint64_t *Bt,
                               int64_t ldbt, int64_t m, int64_t k, int64_t n, hipStream_t s);
int device_cu_count();

// ---------------------------------------------------------------------------
// Strassen's split of a product (the paper's implementation multiplies by
// Strassen-Winograd, Section 3.3).  Over GF(2) every sign in Strassen's
// seven products is a plus:
//   P1 = (A11 + A22)(B11 + B22) -> C11, C22     P5 = (A11 + A12) B22 -> C11, C12
//   P2 = (A21 + A22) B11        -> C21, C22     P6 = (A21 + A11)(B11 + B12) -> C22
//   P3 = A11 (B12 + B22)        -> C12, C22     P7 = (A12 + A22)(B21 + B22) -> C11
//   P4 = A22 (B21 + B11)        -> C11, C21
// The blocks need not be equal: the second row / inner / column part may be
// smaller, and reads as zero where it is shorter (A12, A22 and B21, B22 have
// K2 < K1 inner bits; A21, A22 have m2 <= m1 rows; B12, B22 have N2 <= N1
// columns).  A product then runs over the sizes its outputs need: P4 over
// the m2 rows and K2 inner bits of A22 (so B21 + B11 is cut to K2 bits, the
// A row's bits past K2 meeting zeros), P5 and P7 over K2 bits, P6 over the
// m2 x N2 block of C22 only.
// ---------------------------------------------------------------------------
namespace {
gf2_plan_block pblk(int64_t buf, int64_t row0, int64_t word0, int64_t ld, int64_t rows, int64_t bits) {
    gf2_plan_block b;
    b.buf = buf;
    b.row0 = row0;
    b.word0 = word0;
    b.ld = ld;
    b.rows = rows;
    b.bits = bits;
    return b;
}
const gf2_plan_block NO_BLOCK = pblk(0, 0, 0, 0, 0, 0);
}  // namespace

int64_t product_plan(int64_t m, int64_t k, int64_t n, int split, int64_t lda, int64_t ldbt, int64_t ldc,
                     gf2_plan_step *st, int64_t max, int64_t *ws_words) {
    if (m < 0 || k < 0 || n < 0 || split < -1 || split > 1 || lda < 0 || ldbt < 0 || ldc < 0 || max < 0 ||
        (max > 0 && !st))
        return -1;
    const int64_t kw = words_for(k), nw = words_for(n);
    bool halve = n % 64 == 0 && m >= 2 && kw >= 4 && nw >= 2;
    if (split < 0 || (split == 0 && (m < GF2_PLAN_MIN_BITS || k < GF2_PLAN_MIN_BITS || n < GF2_PLAN_MIN_BITS)))
        halve = false;
    int64_t ns = 0, ws = 0;
    auto put = [&](int64_t kind, gf2_plan_block b0, gf2_plan_block b1, gf2_plan_block b2, gf2_plan_block b3) {
        if (ns < max) {
            st[ns].kind = kind;
            st[ns].b[0] = b0;
            st[ns].b[1] = b1;
            st[ns].b[2] = b2;
            st[ns].b[3] = b3;
        }
        ns++;
    };
    if (!halve) {
        put(1, pblk(0, 0, 0, lda, m, k), pblk(1, 0, 0, ldbt, n, k), pblk(2, 0, 0, ldc, m, n), NO_BLOCK);
        if (ws_words) *ws_words = 0;
        return ns;
    }
    // rows at a multiple of 256 (the product's block rows), the inner size at
    // an even number of words (16-byte operand loads), columns at a multiple
    // of 256 bits; each first part at least as large as the second
    int64_t m1 = (((m + 1) / 2) + 255) & ~(int64_t)255;
    if (m1 >= m) m1 = (m + 1) / 2;
    const int64_t m2 = m - m1;
    const int64_t kw1 = (((kw + 1) / 2) + 1) & ~(int64_t)1;
    const int64_t K1 = 64 * kw1, K2 = k - K1;
    int64_t nw1 = (((nw + 1) / 2) + 3) & ~(int64_t)3;
    if (nw1 >= nw) nw1 = (nw + 1) / 2;
    const int64_t N1 = 64 * nw1, N2 = n - N1;
    const gf2_plan_block A11 = pblk(0, 0, 0, lda, m1, K1), A12 = pblk(0, 0, kw1, lda, m1, K2),
                         A21 = pblk(0, m1, 0, lda, m2, K1), A22 = pblk(0, m1, kw1, lda, m2, K2);
    const gf2_plan_block B11 = pblk(1, 0, 0, ldbt, N1, K1), B12 = pblk(1, N1, 0, ldbt, N2, K1),
                         B21 = pblk(1, 0, kw1, ldbt, N1, K2), B22 = pblk(1, N1, kw1, ldbt, N2, K2);
    const gf2_plan_block C11 = pblk(2, 0, 0, ldc, m1, N1), C12 = pblk(2, 0, nw1, ldc, m1, N2),
                         C21 = pblk(2, m1, 0, ldc, m2, N1), C22 = pblk(2, m1, nw1, ldc, m2, N2);
    // a workspace block: even row stride, 256-byte aligned
    auto wsb = [&](int64_t rows, int64_t bits) {
        const int64_t ld = (words_for(bits) + 1) & ~(int64_t)1;
        const gf2_plan_block b = pblk(3, 0, ws, ld, rows, bits);
        ws += (rows * ld + 31) & ~(int64_t)31;
        return b;
    };
    const gf2_plan_block S1 = wsb(m1, K1), S2 = wsb(m2, K1), S5 = wsb(m1, K2), S6 = wsb(m2, K1), S7 = wsb(m1, K2);
    const gf2_plan_block T1 = wsb(N1, K1), T3 = wsb(N2, K1), T4 = wsb(N1, K2), T6 = wsb(N2, K1), T7 = wsb(N1, K2);
    put(0, S1, A11, A22, NO_BLOCK);
    put(0, S2, A21, A22, NO_BLOCK);
    put(0, S5, A11, A12, NO_BLOCK);
    put(0, S6, A21, A11, NO_BLOCK);
    put(0, S7, A12, A22, NO_BLOCK);
    put(0, T1, B11, B22, NO_BLOCK);
    put(0, T3, B12, B22, NO_BLOCK);
    put(0, T4, B21, B11, NO_BLOCK);
    put(0, T6, B11, B12, NO_BLOCK);
    put(0, T7, B21, B22, NO_BLOCK);
    put(1, S1, T1, C11, C22);
    put(1, S2, B11, C21, C22);
    put(1, A11, T3, C12, C22);
    put(1, A22, T4, C21, pblk(2, 0, 0, ldc, m2, N1));  // C11's first m2 rows
    put(1, S5, B22, C12, pblk(2, 0, 0, ldc, m1, N2));  // C11's first N2 columns
    put(1, S6, T6, C22, NO_BLOCK);
    put(1, S7, T7, C11, NO_BLOCK);
    if (ws_words) *ws_words = ws;
    return ns;
}

// A bound on product_plan's workspace for products of at most m x k x n
// bits: ten blocks of at most m / 2 + 256 rows (or n / 2 + 256) and
// kw / 2 + 3 words, each rounded to 32 words.
int64_t product_plan_ws_bound(int64_t m, int64_t k, int64_t n) {
    const int64_t kl = words_for(k) / 2 + 3;
    return 5 * ((m / 2 + 256) * kl + 32) + 5 * ((n / 2 + 256) * kl + 32);
}

namespace {

constexpr int PLAN_MAX_SUMS = 10;
struct PlanSum {
    uint64_t *d;
    const uint64_t *x, *y;
    int64_t ldd, ldx, ldy;
    int32_t rows, words, xrows, xwords, yrows, ywords;
    uint64_t dmask, xmask, ymask;  // the last word's valid bits of d, x, y
};
struct PlanSums {
    PlanSum s[PLAN_MAX_SUMS];
};

// sum blockIdx.y of the plan: d = x ^ y, element by element over d's rows and
// words; x and y read as zero outside their own rows and words, and each
// last word masked to its bits
__global__ __launch_bounds__(256) void k_plan_sums(PlanSums ps) {
    const PlanSum &q = ps.s[blockIdx.y];
    const uint32_t words = (uint32_t)q.words, total = (uint32_t)q.rows * words;
    for (uint32_t e = blockIdx.x * 256u + threadIdx.x; e < total; e += gridDim.x * 256u) {
        const uint32_t i = e / words, w = e - i * words;
        uint64_t x = 0, y = 0;
        if ((int32_t)i < q.xrows && (int32_t)w < q.xwords) {
            x = q.x[(int64_t)i * q.ldx + w];
            if ((int32_t)w == q.xwords - 1) x &= q.xmask;
        }
        if ((int32_t)i < q.yrows && (int32_t)w < q.ywords) {
            y = q.y[(int64_t)i * q.ldy + w];
            if ((int32_t)w == q.ywords - 1) y &= q.ymask;
        }
        uint64_t v = x ^ y;
        if (w == words - 1) v &= q.dmask;
        q.d[(int64_t)i * q.ldd + w] = v;
    }
}

uint64_t last_mask(int64_t bits) { return (bits & 63) ? (1ull << (bits & 63)) - 1 : ~0ull; }

}  // namespace

// X <- L^-1 X on one diagonal block of nb <= 128 rows (step 2): rows
// j0 .. j0 + nb - 1 of A, whose L bits left of the diagonal inside the block
// sit in words lw, lw + 1, and X = their words [xw0, xw1).  One wave per
// word of X, two rows per lane: row j0 + l (L bits: word lw, bits < l) and
// row j0 + 64 + l (all of word lw, then word lw + 1, bits < l).  Forward
// substitution: once row j is final its word goes by readlane to every lane
// whose row has L[.][j] = 1; the first 64 rows are final after 64 steps, and
// by then their words are folded into the second half too.
//
// The L bits are row i's words of L (row stride ldl), X row i is at X + i ldx
// (the same rows as L's when X = L, or another matrix with a row per L row).
// rblk > 0 (several diagonal blocks at once): blockIdx.y = y takes the block
// of rows [y rblk, min(rend, (y + 1) rblk)), j0 is relative to its start and
// the block's rows past its end are not there.
__global__ __launch_bounds__(256) void k_trsm128(const uint64_t *__restrict__ L, int64_t ldl, uint64_t *__restrict__ X,
                                                 int64_t ldx, int64_t j0, int nb, int64_t xw0, int64_t xw1,
                                                 int64_t rblk, int64_t rend) {
    const int lane = threadIdx.x & 63;
    const int64_t w = xw0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= xw1) return;  // w is the same for the whole wave
    if (rblk > 0) {
        const int64_t y0 = (int64_t)blockIdx.y * rblk, y1 = y0 + rblk < rend ? y0 + rblk : rend;
        j0 += y0;
        if (y1 - j0 < nb) nb = (int)(y1 - j0);
        if (nb <= 0) return;
    }
    const int64_t lw = j0 >> 6;
    const bool on0 = lane < nb, on1 = 64 + lane < nb;
    const uint64_t *lrow0 = L + (j0 + (on0 ? lane : 0)) * ldl;
    const uint64_t *lrow1 = L + (j0 + (on1 ? 64 + lane : 0)) * ldl;
    uint64_t *row0 = X + (j0 + (on0 ? lane : 0)) * ldx;
    uint64_t *row1 = X + (j0 + (on1 ? 64 + lane : 0)) * ldx;
    uint64_t x0 = on0 ? row0[w] : 0ull, x1 = on1 ? row1[w] : 0ull;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint64_t l0 = on0 ? (lrow0[lw] & below) : 0ull;
    const uint64_t l1a = on1 ? lrow1[lw] : 0ull;
    const uint64_t l1b = on1 ? (lrow1[lw + 1] & below) : 0ull;
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
// L, X, rblk and rend as for k_trsm128: with rblk > 0, j0, rb_all are
// relative to the start of block y's rows and re_all is its end.
__global__ __launch_bounds__(1024) void k_trsm_pair(const uint64_t *__restrict__ L, int64_t ldl,
                                                    uint64_t *__restrict__ X, int64_t ldx, int64_t j0, int nb,
                                                    int64_t rb_all, int64_t re_all, int64_t xw0, int64_t xw1,
                                                    int ntiles, int nchunks, int64_t rblk, int64_t rend) {
    constexpr int NT = 1024, LPR = TP_TW / 2, RS = NT / LPR;
    __shared__ __align__(16) uint64_t T[32][16][TP_TW];
    const int tid = threadIdx.x;
    const int logical = xcd_logical(blockIdx.x, gridDim.x);
    const int tile = logical % ntiles, chunk = logical / ntiles;
    if (chunk >= nchunks) return;
    if (rblk > 0) {
        const int64_t y0 = (int64_t)blockIdx.y * rblk;
        j0 += y0;
        rb_all += y0;
        re_all = y0 + rblk < rend ? y0 + rblk : rend;
        if (re_all - j0 < nb) nb = (int)(re_all - j0);
        if (nb <= 0) return;
    }
    const int64_t lw = j0 >> 6;
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
        T[q][1 << b][wl] = (k < nb && w >= xw0 && w < xw1) ? X[(j0 + k) * ldx + w] : 0ull;
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
    const bool wide = (ldx & 1) == 0 && ((uintptr_t)X & 15) == 0 && ok0 && ok1;
    auto load = [&](int64_t i, uint64_t &c0, uint64_t &c1, uint64_t &v0, uint64_t &v1) {
        if (i < re) {
            const uint64_t *lrow = L + i * ldl;
            c0 = lrow[lw];
            c1 = lrow[lw + 1];
            const uint64_t *row = X + i * ldx;
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
            uint64_t *row = X + i * ldx;
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

// The diagonal blocks' identities in Y (rows [0, r), ldy words, the block of
// row i starting at row i - i mod blk, columns relative to it): Y[i] = e_(i mod
// blk) (flip = 0, one thread per word) or Y[i] ^= e_(i mod blk) (flip = 1,
// one thread per row).
__global__ void k_block_ident(uint64_t *__restrict__ Y, int64_t ldy, int64_t r, int64_t blk, int flip) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (flip) {
        if (e >= r) return;
        const int64_t rel = e % blk;
        Y[e * ldy + (rel >> 6)] ^= 1ull << (rel & 63);
        return;
    }
    const int64_t i = e / ldy, w = e % ldy;
    if (i >= r) return;
    const int64_t rel = i % blk;
    Y[i * ldy + w] = w == (rel >> 6) ? 1ull << (rel & 63) : 0ull;
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
    int psplit;           // Strassen's split of the fp4 products (product_plan)
    uint64_t *plan_ws;    // the plan's sums
    size_t plan_bytes;
    uint64_t *tinv;       // the solve's diagonal-block inverses
    size_t tinv_bytes;
};

// the left block's columns of a split of n columns
int64_t split_cols(int64_t n, int64_t split) {
    return split > 0 ? (split < n ? split : n) : ((n / 2 + 63) & ~(int64_t)63);
}

// A[crow0 .. crow0 + M)[xw0, xw1) ^= (bits [64 kw0, 64 kw0 + K) of those rows)
//                                    x A[brow0 .. brow0 + K)[xw0, xw1)
// The fp4 product C ^= Aop * B (Bt its bit transpose), by product_plan's
// steps: the sums in one launch, then the products in order.
hipError_t run_plan(Ctx &c, uint64_t *C, int64_t ldc, const uint64_t *Aop, int64_t lda, const uint64_t *Bt,
                    int64_t ldbt, int64_t M, int64_t K, int64_t N) {
    gf2_plan_step st[GF2_PLAN_MAX_STEPS];
    int64_t wsw = 0;
    const int64_t ns = product_plan(M, K, N, c.psplit, lda, ldbt, ldc, st, GF2_PLAN_MAX_STEPS, &wsw);
    if (ns < 1 || ns > GF2_PLAN_MAX_STEPS || (size_t)wsw * 8 > c.plan_bytes) return hipErrorInvalidValue;
    auto addr = [&](const gf2_plan_block &b) -> uint64_t * {
        uint64_t *base = b.buf == 0 ? (uint64_t *)Aop : b.buf == 1 ? (uint64_t *)Bt : b.buf == 2 ? C : c.plan_ws;
        return base + b.row0 * b.ld + b.word0;
    };
    PlanSums sums;
    int nsum = 0;
    int64_t most = 0;
    for (int64_t i = 0; i < ns; i++) {
        if (st[i].kind != 0) continue;
        const gf2_plan_block &d = st[i].b[0], &x = st[i].b[1], &y = st[i].b[2];
        if (nsum >= PLAN_MAX_SUMS || d.rows * words_for(d.bits) >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
        PlanSum &q = sums.s[nsum++];
        q.d = addr(d);
        q.x = addr(x);
        q.y = addr(y);
        q.ldd = d.ld;
        q.ldx = x.ld;
        q.ldy = y.ld;
        q.rows = (int32_t)d.rows;
        q.words = (int32_t)words_for(d.bits);
        q.xrows = (int32_t)x.rows;
        q.xwords = (int32_t)words_for(x.bits);
        q.yrows = (int32_t)y.rows;
        q.ywords = (int32_t)words_for(y.bits);
        q.dmask = last_mask(d.bits);
        q.xmask = last_mask(x.bits);
        q.ymask = last_mask(y.bits);
        most = std::max(most, d.rows * words_for(d.bits));
    }
    hipError_t e;
    if (nsum > 0 && most > 0) {
        const int64_t bx = std::min<int64_t>((most + 255) / 256, 2048);
        ProfScope ps(KID_SUMS, c.s);
        hipLaunchKernelGGL(k_plan_sums, dim3((unsigned)bx, (unsigned)nsum), dim3(256), 0, c.s, sums);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (int64_t i = 0; i < ns; i++) {
        if (st[i].kind != 1) continue;
        const gf2_plan_block &a = st[i].b[0], &b = st[i].b[1], &o0 = st[i].b[2], &o1 = st[i].b[3];
        if ((e = launch_fp4_product2(addr(o0), o0.ld, o0.rows, words_for(o0.bits), o1.rows > 0 ? addr(o1) : nullptr,
                                     o1.ld, o1.rows, words_for(o1.bits), addr(a), a.ld, addr(b), b.ld, a.rows, a.bits,
                                     b.rows, c.s)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// bt_ready: c.bt already holds the right operand's bit transpose (words_for(K)
// words per row), as the solve leaves it.
hipError_t product(Ctx &c, uint64_t *A, int64_t crow0, int64_t M, int64_t kw0, int64_t K, int64_t brow0, int64_t xw0,
                   int64_t xw1, int64_t N, bool bt_ready = false) {
    if (M <= 0 || K <= 0 || N <= 0) return hipSuccess;
    const int64_t ldw = c.ldw;
    if (c.mfma && K >= MFMA_MIN_K) {
        const int64_t ldbt = words_for(K);
        if ((size_t)words_for(N) * 64 * (size_t)ldbt * 8 > c.bt_bytes) return hipErrorInvalidValue;
        hipError_t e = bt_ready ? hipSuccess : launch_transpose_bits(A + brow0 * ldw + xw0, ldw, K, N, c.bt, ldbt, c.s);
        if (e != hipSuccess) return e;
        // (the plan takes whole words of columns: Bt's rows past N are zero)
        if (c.fmt == 0)
            return run_plan(c, A + crow0 * ldw + xw0, ldw, A + crow0 * ldw + kw0, ldw, c.bt, ldbt, M, K,
                            64 * words_for(N));
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
    hipLaunchKernelGGL(k_trsm128, dim3((unsigned)blocks), dim3(256), 0, c.s, A, c.ldw, A, c.ldw, j0, nb, xw0, xw1,
                       (int64_t)0, (int64_t)0);
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
    hipLaunchKernelGGL(k_trsm_pair, dim3((unsigned)(nt * nchunks)), dim3(1024), 0, c.s, A, c.ldw, A, c.ldw, j0, nb, rb,
                       re, xw0, xw1, nt, nchunks, (int64_t)0, (int64_t)0);
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

// With fp4 products, the solve's diagonal blocks: of this many rows, their
// inverses computed at once by the sweeps above, then applied by products
// (trsm below).  Of 1024, 2048, 3072 and 4096 rows, 2048 was the fastest on
// the 65536^2 PLE.  (The int8 product is too slow at these inner sizes to
// gain from it.)
constexpr int64_t TRSM_BLOCK = 2048;

// The inverses of the diagonal blocks L_dd of L (rows [0, r), blocks of
// TRSM_BLOCK rows, d0 a multiple of it) into Y (row i: row i - d0 of L_dd^-1,
// TRSM_BLOCK / 64 words), all blocks at once: Y = I, then the blocked forward
// substitution of each block on its own identity, 128-row steps in order,
// each step one launch of the substitution and one of the sweep for every
// block.  Row i of L_dd^-1 has no bit past column i - d0, so a step's
// launches cover only the words up to its rows' columns.
hipError_t invert_diag_blocks(Ctx &c, const uint64_t *A, int64_t r, uint64_t *Y) {
    constexpr int64_t ldy = TRSM_BLOCK / 64;
    const int64_t nblk = (r + TRSM_BLOCK - 1) / TRSM_BLOCK;
    ProfScope ps(KID_TRSM, c.s);
    hipLaunchKernelGGL(k_block_ident, dim3((unsigned)((r * ldy + 255) / 256)), dim3(256), 0, c.s, Y, ldy, r,
                       TRSM_BLOCK, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t slots = device_cu_count();
    for (int64_t b = 0; b < TRSM_BLOCK && b < r; b += 128) {
        const int64_t xw = (b + 128) / 64 < ldy ? (b + 128) / 64 : ldy;
        hipLaunchKernelGGL(k_trsm128, dim3((unsigned)((xw + 3) / 4), (unsigned)nblk), dim3(256), 0, c.s, A, c.ldw,
                           Y, ldy, b, 128, (int64_t)0, xw, TRSM_BLOCK, r);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int64_t rows = TRSM_BLOCK - b - 128;  // below the step, in a whole block
        if (rows <= 0) continue;
        const int nt = (int)((xw + TP_TW - 1) / TP_TW);
        int64_t nc = (rows + 255) / 256;
        // about one round of the CUs over all blocks
        const int64_t cap = (slots + nt * nblk - 1) / (nt * nblk);
        if (nc > cap) nc = cap;
        if (nc < 1) nc = 1;
        hipLaunchKernelGGL(k_trsm_pair, dim3((unsigned)(nt * nc), (unsigned)nblk), dim3(1024), 0, c.s, A, c.ldw, Y,
                           ldy, b, 128, b + 128, (int64_t)0, (int64_t)0, xw, nt, (int)nc, TRSM_BLOCK, r);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

// rows [0, r) of X = A[.][xw0, xw1) <- L^-1 X, with L the unit lower
// triangle of A[0 .. r)[0 .. r)
// *bt_x: set when c.bt holds X's bit transpose afterwards (words_for(r) words
// per column of X), the right operand of the Schur product.
hipError_t trsm(Ctx &c, uint64_t *A, int64_t r, int64_t xw0, int64_t xw1, int64_t N, bool *bt_x) {
    *bt_x = false;
    if (!c.mfma || c.fmt != 0 || r <= TRSM_BLOCK) return trsm_diag(c, A, 0, r, xw0, xw1);
    // With fp4 products and several diagonal blocks: their inverses at once
    // (Y, on identities TRSM_BLOCK / 64 words wide instead of the right
    // block's width), then for each block in order: X_d loses the solved
    // blocks above it, X_d^ = X_d + L[d][0, d0) X[0, d0), as one product with
    // inner size d0 (the solved blocks' bit transposes kept side by side in
    // Bs, one product's operand for every later block); then X_d <- L_dd^-1
    // X_d as X_d += (L_dd^-1 + I) X_d (the product reads X_d through its bit
    // transpose Bd, so it may add into X_d); then X_d's transpose joins Bs,
    // which in the end is X's, the Schur product's right operand.
    constexpr int64_t ldy = TRSM_BLOCK / 64;
    const int64_t Np = 64 * (xw1 - xw0);  // whole words of columns (Bt is zero past N)
    const int64_t ldbs = words_for(r);
    if (((size_t)r + (size_t)Np) * ldy * 8 > c.tinv_bytes || (size_t)Np * ldbs * 8 > c.bt_bytes)
        return hipErrorInvalidValue;
    uint64_t *Y = c.tinv, *Bd = c.tinv + r * ldy, *Bs = c.bt;
    hipError_t e;
    if ((e = invert_diag_blocks(c, A, r, Y)) != hipSuccess) return e;
    {
        ProfScope ps(KID_TRSM, c.s);
        hipLaunchKernelGGL(k_block_ident, dim3((unsigned)((r + 255) / 256)), dim3(256), 0, c.s, Y, ldy, r, TRSM_BLOCK,
                           1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (int64_t d0 = 0; d0 < r; d0 += TRSM_BLOCK) {
        const int64_t d1 = r - d0 < TRSM_BLOCK ? r : d0 + TRSM_BLOCK, K = d1 - d0;
        uint64_t *Xd = A + d0 * c.ldw + xw0;
        if (d0 > 0 && (e = run_plan(c, Xd, c.ldw, A + d0 * c.ldw, c.ldw, Bs, ldbs, K, d0, Np)) != hipSuccess) return e;
        if ((e = launch_transpose_bits(Xd, c.ldw, K, N, Bd, ldy, c.s)) != hipSuccess) return e;
        if ((e = run_plan(c, Xd, c.ldw, Y + d0 * ldy, ldy, Bd, ldy, K, K, Np)) != hipSuccess) return e;
        if ((e = launch_transpose_bits(Xd, c.ldw, K, N, Bs + (d0 >> 6), ldbs, c.s)) != hipSuccess) return e;
    }
    *bt_x = true;
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
        bool bt_x = false;
        if ((e = trsm(c, A, r1, xw0, xw1, N, &bt_x)) != hipSuccess) return e;
        if ((e = product(c, A, r1, m - r1, 0, r1, 0, xw0, xw1, N, bt_x)) != hipSuccess) return e;
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

namespace {
// the largest product is the first split's: at most m rows, inner size at
// most min(m, n1), n - n1 columns
size_t bt_bytes_for(int64_t m, int64_t n, int levels, bool mfma, int64_t split) {
    if (!(mfma && levels > 0 && n > 64 && !(split > 0 && n <= split))) return 0;
    const int64_t n1 = split_cols(n, split);
    const int64_t k = m < n1 ? m : n1;
    return al((size_t)words_for(n - n1) * 64 * (size_t)words_for(k) * 8);
}
size_t plan_bytes_for(int64_t m, int64_t n, int levels, bool mfma, int64_t split, int psplit) {
    if (psplit < 0 || !(mfma && levels > 0 && n > 64 && !(split > 0 && n <= split))) return 0;
    const int64_t n1 = split_cols(n, split);
    const int64_t k = m < n1 ? m : n1;
    return al((size_t)product_plan_ws_bound(m, k, n - n1) * 8);
}
// the solve's diagonal-block inverses, a row of TRSM_BLOCK bits per row of
// the largest solve (the first split's rank, at most min(m, n1)), then one
// block's bit transpose (a row of TRSM_BLOCK bits per column, n - n1 at most)
size_t tinv_bytes_for(int64_t m, int64_t n, int levels, bool mfma, int64_t split) {
    if (!(mfma && levels > 0 && n > 64 && !(split > 0 && n <= split))) return 0;
    const int64_t n1 = split_cols(n, split);
    const int64_t k = m < n1 ? m : n1;
    return al(((size_t)k + (size_t)words_for(n - n1) * 64) * (TRSM_BLOCK / 64) * 8);
}
}  // namespace

size_t alg3_extra_bytes(int64_t m, int64_t n, int64_t ldw, int levels, bool mfma, int64_t split, int psplit) {
    (void)ldw;
    return al((size_t)MAX_DEPTH * 8) + bt_bytes_for(m, n, levels, mfma, split) +
           plan_bytes_for(m, n, levels, mfma, split, psplit) + tinv_bytes_for(m, n, levels, mfma, split);
}

hipError_t ple_alg3(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank, void *ws,
                    const gf2_ple_opts *opts, hipStream_t s, int levels, int products, int64_t split, int psplit) {
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
    c.bt_bytes = bt_bytes_for(m, n, levels, mfma, split);
    c.psplit = products == 1 ? psplit : -1;
    c.plan_ws = (uint64_t *)((char *)c.bt + c.bt_bytes);
    c.plan_bytes = plan_bytes_for(m, n, levels, mfma, split, c.psplit);
    c.tinv = (uint64_t *)((char *)c.plan_ws + c.plan_bytes);
    c.tinv_bytes = tinv_bytes_for(m, n, levels, mfma, split);
    return ple_rec(c, A, m, n, P, Q, rank, levels, 0, 0);
}

}  // namespace gf2
