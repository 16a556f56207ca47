// Block-recursive PLE (Algorithm 3, Section 3.3) on top of the
// block-iterative pass loop (Algorithm 2), for gf2_ple with update = 2
// (products on the fp4 matrix cores), 3 (products on the Four-Russians
// tables) or 4 (products on the int8 matrix cores).
//
// One level on the m x n block A, split at column n1 (a multiple of 64):
//   1. PLE of the left block [A0 A1]'s first n1 columns; its swaps move whole
//      rows, so the right block A1 ends up with its rows permuted (P1^T A1);
//   2. A01 <- L00^-1 A01 on the first r1 rows of A1 (triangular solve, by
//      recursion on halves: each half's solve, then the product that removes
//      it from the other half);
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

namespace gf2 {

hipError_t launch_m4rm(uint64_t *C, int64_t ldc, int64_t m, const uint64_t *coef, int64_t coef_ld, const uint64_t *B,
                       int64_t ldb, int nbits, int64_t w_begin, int64_t w_end, int m4_variant, int m4_target,
                       hipStream_t s);
hipError_t launch_transpose_bits(const uint64_t *B, int64_t ldb, int64_t k, int64_t n, uint64_t *Bt, int64_t ldbt,
                                 hipStream_t s);
hipError_t launch_mfma_gf2(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda, const uint64_t *Bt, int64_t ldbt,
                           int64_t m, int64_t k, int64_t n, hipStream_t s, int fmt);

// X <- L^-1 X on one diagonal block of nb <= 64 rows (the leaves of step 2):
// rows j0 .. j0 + nb - 1 of A, whose L bits below the diagonal sit in word
// lw (row j0 + i: bits 0 .. i - 1), and X = their words [xw0, xw1).  One
// wave per word of X, lane i holding row j0 + i; once row j is final its
// word goes to every lane i > j with L[i][j] = 1 (forward substitution).
__global__ __launch_bounds__(256) void k_trsm64(uint64_t *__restrict__ A, int64_t ldw, int64_t j0, int nb, int64_t lw,
                                                int64_t xw0, int64_t xw1) {
    const int lane = threadIdx.x & 63;
    const int64_t w = xw0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= xw1) return;  // w is the same for the whole wave
    const bool on = lane < nb;
    uint64_t *row = A + (j0 + (on ? lane : 0)) * ldw;
    uint64_t x = on ? row[w] : 0ull;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint64_t l = on ? (row[lw] & below) : 0ull;
    for (int j = 0; j + 1 < nb; j++) {
        const uint64_t xj = readlane64(x, j);
        x ^= ((l >> j) & 1ull) ? xj : 0ull;
    }
    if (on) row[w] = x;
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
};

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

hipError_t trsm64(Ctx &c, uint64_t *A, int64_t j0, int nb, int64_t xw0, int64_t xw1) {
    const int64_t blocks = (xw1 - xw0 + 3) / 4;
    if (blocks <= 0 || nb <= 0) return hipSuccess;
    ProfScope ps(KID_M4RM, c.s);
    hipLaunchKernelGGL(k_trsm64, dim3((unsigned)blocks), dim3(256), 0, c.s, A, c.ldw, j0, nb, j0 >> 6, xw0, xw1);
    return hipGetLastError();
}

// rows [j0, j1) of X = A[.][xw0, xw1) <- L^-1 X, with L the unit lower
// triangle of A[j0 .. j1)[j0 .. j1) (j0 a multiple of 64)
hipError_t trsm(Ctx &c, uint64_t *A, int64_t j0, int64_t j1, int64_t xw0, int64_t xw1, int64_t N) {
    if (j1 - j0 <= 64) return trsm64(c, A, j0, (int)(j1 - j0), xw0, xw1);
    hipError_t e;
    if (!c.mfma) {
        // tables: one 64-row block at a time, each removed from the rows below
        for (int64_t b = j0; b < j1; b += 64) {
            const int nb = (int)(j1 - b < 64 ? j1 - b : 64);
            if ((e = trsm64(c, A, b, nb, xw0, xw1)) != hipSuccess) return e;
            if (b + 64 < j1 && (e = product(c, A, b + 64, j1 - b - 64, b >> 6, 64, b, xw0, xw1, N)) != hipSuccess)
                return e;
        }
        return hipSuccess;
    }
    const int64_t h = ((j1 - j0) / 2 + 63) & ~(int64_t)63;
    if ((e = trsm(c, A, j0, j0 + h, xw0, xw1, N)) != hipSuccess) return e;
    if ((e = product(c, A, j0 + h, j1 - j0 - h, j0 >> 6, h, j0, xw0, xw1, N)) != hipSuccess) return e;
    return trsm(c, A, j0 + h, j1, xw0, xw1, N);
}

hipError_t ple_rec(Ctx &c, uint64_t *A, int64_t m, int64_t n, int64_t *P, int64_t *Q, int64_t *rank, int levels,
                   int64_t wlo, int depth) {
    if (levels <= 0 || n <= 64 || m == 0 || depth >= MAX_DEPTH)
        return ple_block(A, m, n, c.ldw, P, Q, rank, c.ws, c.opts, c.s, wlo);
    const int64_t ldw = c.ldw;
    const int64_t n1 = (n / 2 + 63) & ~(int64_t)63;
    hipError_t e = ple_rec(c, A, m, n1, P, Q, rank, levels - 1, wlo, depth + 1);
    if (e != hipSuccess) return e;
    int64_t r1 = 0;
    if ((e = hipMemcpyAsync(&r1, rank, 8, hipMemcpyDeviceToHost, c.s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(c.s)) != hipSuccess) return e;
    const int64_t xw0 = n1 >> 6, xw1 = words_for(n), N = n - n1;
    if (r1 > 0) {
        if ((e = trsm(c, A, 0, r1, xw0, xw1, N)) != hipSuccess) return e;
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

size_t alg3_extra_bytes(int64_t m, int64_t n, int64_t ldw, int levels, bool mfma) {
    (void)ldw;
    size_t b = al((size_t)MAX_DEPTH * 8);
    if (mfma && levels > 0 && n > 64) {
        // the largest product: inner size at most min(m, n1), n - n1 columns
        const int64_t n1 = (n / 2 + 63) & ~(int64_t)63;
        const int64_t k = m < n1 ? m : n1;
        b += al((size_t)words_for(n - n1) * 64 * (size_t)words_for(k) * 8);
    }
    return b;
}

hipError_t ple_alg3(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank, void *ws,
                    const gf2_ple_opts *opts, hipStream_t s, int levels, int products) {
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
    c.bt_bytes = alg3_extra_bytes(m, n, ldw, levels, mfma) - al((size_t)MAX_DEPTH * 8);
    return ple_rec(c, A, m, n, P, Q, rank, levels, 0, 0);
}

}  // namespace gf2
