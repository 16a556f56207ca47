// GF(2) product on the int8 matrix cores: C ^= A B with A m x k, B k x n
// (Section 3.2's trailing update A22 <- L21 A12 + A22, done as a dense
// product, the way Algorithm 3 reduces its update to matrix multiplication).
//
// Bits are expanded to int8 0/1 operands of v_mfma_i32_32x32x32_i8, the
// int32 sums are reduced mod 2 (& 1) and packed back into words with
// ballots.  The matrix-core operands hold K-consecutive values per lane, so
// B is first bit-transposed (Bt, n x k bits) into scratch.  A and B use the
// same K order inside each operand, so only the accumulator layout matters:
// lane l holds column l % 32 of a 32 x 32 tile, register i its row
// 8 (i / 4) + 4 (l / 32) + i % 4.
#include "common.h"
#include "dev.h"
#include "m4rm.h"

namespace gf2 {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// 16 bits -> 16 bytes 0/1 (byte j = bit j).  For a 4-bit x, x * 0x204081
// puts bit t of x at bit 8t (the four shifted copies do not overlap); the
// mask keeps exactly those bits.
__device__ __forceinline__ v4i bits_to_bytes16(uint32_t b) {
    v4i r;
    r[0] = (int)(((b & 15u) * 0x204081u) & 0x01010101u);
    r[1] = (int)((((b >> 4) & 15u) * 0x204081u) & 0x01010101u);
    r[2] = (int)((((b >> 8) & 15u) * 0x204081u) & 0x01010101u);
    r[3] = (int)((((b >> 12) & 15u) * 0x204081u) & 0x01010101u);
    return r;
}

// Bt[j][.] = column j of B: one wave transposes a 64 x 64 bit block in
// registers (six butterfly stages: lanes l and l ^ s trade the s-bit halves
// of their s-aligned groups).  Rows of B at or past k and columns at or past
// n come out zero; Bt has words(n) * 64 rows of ldbt >= words(k) words.
__global__ __launch_bounds__(256) void k_transpose_bits(const uint64_t *__restrict__ B, int64_t ldb, int64_t k,
                                                        int64_t n, uint64_t *__restrict__ Bt, int64_t ldbt) {
    const int lane = threadIdx.x & 63;
    const int64_t kw = words_for(k), nw = words_for(n);
    const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (blk >= kw * nw) return;
    const int64_t kb = blk % kw, wb = blk / kw;
    const int64_t row = kb * 64 + lane;
    uint64_t x = row < k ? B[row * ldb + wb] : 0ull;
    const uint64_t masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                               0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int st = 0; st < 6; st++) {
        const int s = 32 >> st;
        const uint64_t M = masks[st];
        const uint32_t lo = __shfl_xor((int)(uint32_t)x, s, 64);
        const uint32_t hi = __shfl_xor((int)(uint32_t)(x >> 32), s, 64);
        const uint64_t y = ((uint64_t)hi << 32) | lo;
        x = (lane & s) ? (((y & ~M) >> s) | (x & ~M)) : ((x & M) | ((y & M) << s));
    }
    const int64_t col = wb * 64 + lane;
    Bt[col * ldbt + kb] = col < n ? x : 0ull;
}

// One wave computes a 64 x 64 block of C (64 rows, one output word): 2 x 2
// matrix-core tiles of 32 x 32, K consumed 32 bits per instruction.
template <int NWR, int NWC>
__global__ __launch_bounds__(NWR *NWC * 64) void k_mfma_gf2(uint64_t *__restrict__ C, int64_t ldc,
                                                           const uint64_t *__restrict__ A, int64_t lda,
                                                           const uint64_t *__restrict__ Bt, int64_t ldbt, int64_t m,
                                                           int64_t kw, int64_t nw, int64_t gcols) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t bid = blockIdx.x;
    const int64_t bc = bid % gcols, br = bid / gcols;  // column blocks fastest: neighbours share A rows
    const int64_t r0 = (br * NWR + wave / NWC) * 64;
    const int64_t w0 = bc * NWC + wave % NWC;
    if (r0 >= m || w0 >= nw) return;
    const int lr = lane & 31, kh = lane >> 5;
    const int64_t ra = r0 + lr, rb = r0 + 32 + lr;
    const uint64_t *pa = A + (ra < m ? ra : 0) * lda;
    const uint64_t *pb = A + (rb < m ? rb : 0) * lda;
    const uint64_t *qa = Bt + (w0 * 64 + lr) * ldbt;
    const uint64_t *qb = Bt + (w0 * 64 + 32 + lr) * ldbt;
    const bool va = ra < m, vb = rb < m;
    v16i c00 = {}, c01 = {}, c10 = {}, c11 = {};
    for (int64_t kk = 0; kk < kw; kk++) {
        const uint64_t xa = va ? pa[kk] : 0ull, xb = vb ? pb[kk] : 0ull;
        const uint64_t ya = qa[kk], yb = qb[kk];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int sh = 32 * h + 16 * kh;
            const v4i A0 = bits_to_bytes16((uint32_t)(xa >> sh) & 0xFFFFu);
            const v4i A1 = bits_to_bytes16((uint32_t)(xb >> sh) & 0xFFFFu);
            const v4i B0 = bits_to_bytes16((uint32_t)(ya >> sh) & 0xFFFFu);
            const v4i B1 = bits_to_bytes16((uint32_t)(yb >> sh) & 0xFFFFu);
            c00 = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0, B0, c00, 0, 0, 0);
            c01 = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0, B1, c01, 0, 0, 0);
            c10 = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1, B0, c10, 0, 0, 0);
            c11 = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1, B1, c11, 0, 0, 0);
        }
    }
    // sums mod 2 -> bits; lane L collects the output word of row r0 + L
    uint64_t out = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const int q = (i >> 2) * 8 + (i & 3);  // rows q (lanes < 32) and q + 4 (lanes >= 32) of a tile
        const uint64_t b00 = __ballot(c00[i] & 1), b01 = __ballot(c01[i] & 1);
        const uint64_t b10 = __ballot(c10[i] & 1), b11 = __ballot(c11[i] & 1);
        const uint64_t lo32 = 0xFFFFFFFFull;
        out = lane == q ? ((b00 & lo32) | (b01 << 32)) : out;
        out = lane == q + 4 ? ((b00 >> 32) | (b01 & ~lo32)) : out;
        out = lane == 32 + q ? ((b10 & lo32) | (b11 << 32)) : out;
        out = lane == 36 + q ? ((b10 >> 32) | (b11 & ~lo32)) : out;
    }
    const int64_t row = r0 + lane;
    if (row < m && out) C[row * ldc + w0] ^= out;
}

// One wave computes a (32 TR) x (32 TC) block of C with TR x TC matrix-core
// tiles (TC even: TC / 2 output words); the accumulators live in the AGPRs.
// Lane L finishes rows r0 + L + 64 p of the block.
template <int TR, int TC>
__global__ __launch_bounds__(256) void k_mfma_gf2t(uint64_t *__restrict__ C, int64_t ldc,
                                                  const uint64_t *__restrict__ A, int64_t lda,
                                                  const uint64_t *__restrict__ Bt, int64_t ldbt, int64_t m,
                                                  int64_t kw, int64_t nw, int64_t gcols) {
    constexpr int WPB = 4;  // waves per block, side by side in columns
    constexpr int NWD = TC / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t bid = blockIdx.x;
    const int64_t bc = bid % gcols, br = bid / gcols;
    const int64_t r0 = br * 32 * TR;
    const int64_t w0 = (bc * WPB + wave) * NWD;
    if (r0 >= m || w0 >= nw) return;
    const int lr = lane & 31, kh = lane >> 5;
    const uint64_t *pa[TR];
    bool va[TR];
#pragma unroll
    for (int i = 0; i < TR; i++) {
        const int64_t r = r0 + 32 * i + lr;
        va[i] = r < m;
        pa[i] = A + (va[i] ? r : 0) * lda;
    }
    const uint64_t *qb[TC];
#pragma unroll
    for (int j = 0; j < TC; j++) {
        const int64_t cidx = w0 * 64 + 32 * j + lr;
        qb[j] = Bt + (cidx < nw * 64 ? cidx : 0) * ldbt;
    }
    v16i acc[TR][TC];
#pragma unroll
    for (int i = 0; i < TR; i++)
#pragma unroll
        for (int j = 0; j < TC; j++) acc[i][j] = v16i{};
    for (int64_t kk = 0; kk < kw; kk++) {
        uint64_t x[TR], y[TC];
#pragma unroll
        for (int i = 0; i < TR; i++) x[i] = va[i] ? pa[i][kk] : 0ull;
#pragma unroll
        for (int j = 0; j < TC; j++) y[j] = qb[j][kk];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int sh = 32 * h + 16 * kh;
            v4i a[TR], b[TC];
#pragma unroll
            for (int i = 0; i < TR; i++) a[i] = bits_to_bytes16((uint32_t)(x[i] >> sh) & 0xFFFFu);
#pragma unroll
            for (int j = 0; j < TC; j++) b[j] = bits_to_bytes16((uint32_t)(y[j] >> sh) & 0xFFFFu);
#pragma unroll
            for (int i = 0; i < TR; i++)
#pragma unroll
                for (int j = 0; j < TC; j++) acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    constexpr int NP = (TR + 1) / 2;  // 64-row groups
    uint64_t out[NP][NWD];
#pragma unroll
    for (int p = 0; p < NP; p++)
#pragma unroll
        for (int d = 0; d < NWD; d++) out[p][d] = 0;
    const uint64_t lo32 = 0xFFFFFFFFull;
#pragma unroll
    for (int i = 0; i < TR; i++) {
#pragma unroll
        for (int e = 0; e < 16; e++) {
            const int q = 32 * i + (e >> 2) * 8 + (e & 3);  // rows q (lanes < 32) and q + 4 (lanes >= 32)
#pragma unroll
            for (int d = 0; d < NWD; d++) {
                const uint64_t b0 = __ballot(acc[i][2 * d][e] & 1), b1 = __ballot(acc[i][2 * d + 1][e] & 1);
                out[q >> 6][d] = lane == (q & 63) ? ((b0 & lo32) | (b1 << 32)) : out[q >> 6][d];
                out[(q + 4) >> 6][d] = lane == ((q + 4) & 63) ? ((b0 >> 32) | (b1 & ~lo32)) : out[(q + 4) >> 6][d];
            }
        }
    }
#pragma unroll
    for (int p = 0; p < NP; p++) {
        const int64_t row = r0 + 64 * p + lane;
#pragma unroll
        for (int d = 0; d < NWD; d++)
            if (row < m && w0 + d < nw && out[p][d]) C[row * ldc + w0 + d] ^= out[p][d];
    }
}

// ---------------------------------------------------------------------------
// The same product on the fp4 matrix cores (v_mfma_scale_f32_32x32x64_f8f6f4
// with e2m1 operands, unit scales): a clear bit becomes 0.0, a set bit a
// power of two whose product with the other operand's is exactly 1, so the
// fp32 sums are exact integers (at most k) and their low bit is the GF(2)
// sum.
//
// A block of eight waves (two per SIMD) computes 256 rows x 256 columns of C
// (4 output words); the waves sit 4 x 2, each 64 rows x 128 columns as 2 x 4
// tiles of 32 x 32 (128 fp32 accumulators per lane).  K advances F4_KS
// 64-bit words per barrier.  The block's 512 operand rows (256 rows of A,
// 256 rows of Bt) are loaded one row per thread, F4_KS words ahead, and
// stored into double-buffered LDS as raw 32-bit halves; each wave reads the
// halves of its own 2 + 4 operand tiles and expands them into fp4 in
// registers just before its matrix-core instructions.  LDS holds bits rather
// than fp4 nibbles, which cuts its traffic four-fold; the expansion (five or
// seven ALU instructions per operand and word) runs on one wave of a SIMD
// while the other's matrix-core instructions execute.
// ---------------------------------------------------------------------------
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// 32 bits -> 32 fp4 values in four dwords (the upper four operand dwords
// are unused by e2m1).  The K order inside an operand is free as long as A
// and B share it: bit 4s + d of v goes to nibble s of dword d.  The two
// operands use reciprocal values, so each product of two set bits is exactly
// 1 while each dword costs at most one shift and one mask:
//   half_to_fp4_x: a set bit is 0.5, 1, 2, 2 in dwords 0..3 (nibble bits
//                  0, 1, 2 -- a mask alone -- and bit 2 again for d = 3);
//   half_to_fp4_y: a set bit is 2, 1, 0.5, 0.5 (nibble bits 2, 1, 0, 0).
// (e2m1: 0b0001 = 0.5, 0b0010 = 1.0, 0b0100 = 2.0.)  Five and seven ALU
// instructions; the operand with more tiles per wave takes the cheaper one.
__device__ __forceinline__ v8i half_to_fp4_x(uint32_t v) {
    return v8i{(int)(v & 0x11111111u), (int)(v & 0x22222222u), (int)(v & 0x44444444u), (int)((v >> 1) & 0x44444444u),
               0, 0, 0, 0};
}
__device__ __forceinline__ v8i half_to_fp4_y(uint32_t v) {
    return v8i{(int)((v << 2) & 0x44444444u), (int)(v & 0x22222222u), (int)((v >> 2) & 0x11111111u),
               (int)((v >> 3) & 0x11111111u), 0, 0, 0, 0};
}

constexpr int F4_BM = 256, F4_BN = 256;  // block rows, block columns
struct F4Out {                            // a destination of the fp4 product
    uint64_t *C;
    int64_t ldc, rows, words;
};
constexpr int F4_KS = 8;                 // words of K per barrier

// One step's KS words of an operand row, zero past kw.  ld_full: the step
// lies inside [0, kw), loads without conditions (16-byte parts when VEC);
// ld_tail: word by word with bounds checks.
template <bool VEC>
__device__ __forceinline__ void f4_ld_full(const uint64_t *__restrict__ p, uint64_t *x) {
#pragma unroll
    for (int q = 0; q < F4_KS; q += (VEC ? 2 : 1)) {
        if constexpr (VEC) {
            const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(p + q);
            x[q] = v.x;
            x[q + 1] = v.y;
        } else {
            x[q] = p[q];
        }
    }
}
__device__ __forceinline__ void f4_ld_tail(const uint64_t *__restrict__ p, int64_t w0, int64_t kw, uint64_t *x) {
#pragma unroll
    for (int q = 0; q < F4_KS; q++) x[q] = w0 + q < kw ? p[q] : 0ull;
}

// VEC: rows are read in 16-byte parts (A and Bt 16-byte aligned, lda and
// ldbt even); otherwise word by word.
//
// Step kk, for each wave: store step kk + 1's words (loaded during step
// kk - 1) into LDS buffer (kk + 1) & 1; read the rest of step kk's operand
// halves from buffer kk & 1; issue the loads of step kk + 2; barrier; read
// the first operand halves of step kk + 1; then step kk's matrix-core
// instructions, which use registers only.  A buffer is rewritten only after
// the barrier that follows its last read, and the matrix-core work sits
// between barriers, where one wave's instructions overlap the other's loads,
// stores and expansion.
//
// The product (m x 64 nw bits) is added to o0 and, when o1.C is set, to o1,
// each over its own rows and words (at most the product's).
template <bool VEC>
__global__ __launch_bounds__(512) void k_mfma_gf2_fp4(F4Out o0, F4Out o1, const uint64_t *__restrict__ A,
                                                      int64_t lda, const uint64_t *__restrict__ Bt, int64_t ldbt,
                                                      int64_t m, int64_t kw, int64_t nw, int64_t gcols,
                                                      int64_t grows) {
    constexpr int KS = F4_KS, WC = 2, TI = 2, TJ = 4, CH = KS / 4;  // CH chunks of 4 words per step
    // [buffer][operand row: A rows, then Bt rows][low halves of the KS words, then high halves]
    __shared__ __align__(16) uint32_t sP[2][F4_BM + F4_BN][2 * KS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // blocks of one XCD take a contiguous range: neighbouring column blocks
    // of the same rows share that XCD's L2
    const int64_t logical = xcd_logical((int)blockIdx.x, (int)gridDim.x);
    const int64_t bc = logical % gcols, br = logical / gcols;
    if (br >= grows) return;  // (the grid is exactly gcols x grows)
    const int64_t r0 = br * F4_BM, w0 = bc * (F4_BN / 64);
    const int wr = wave / WC, wc = wave % WC;
    const int lr = lane & 31, kh = lane >> 5;
    // this thread's operand row (Bt has nw * 64 rows, zero past n); a row
    // past the end reads row 0 and stores zeros
    const int64_t g = tid < F4_BM ? r0 + tid : w0 * 64 + (tid - F4_BM);
    const bool valid = tid < F4_BM ? g < m : g < nw * 64;
    const uint64_t *src = tid < F4_BM ? A + (valid ? g : 0) * lda : Bt + (valid ? g : 0) * ldbt;
    const int64_t steps = (kw + KS - 1) / KS, full = kw / KS;
    auto ld = [&](int64_t kk, uint64_t *x) {
        if (kk < full)
            f4_ld_full<VEC>(src + kk * KS, x);
        else
            f4_ld_tail(src + kk * KS, kk * KS, kw, x);
    };
    auto put = [&](int buf, const uint64_t *x) {
        uint4 *d = reinterpret_cast<uint4 *>(&sP[buf][tid][0]);
        const uint64_t z = valid ? ~0ull : 0ull;
#pragma unroll
        for (int h = 0; h < KS / 4; h++) {
            const uint64_t a = x[4 * h] & z, b = x[4 * h + 1] & z, c = x[4 * h + 2] & z, e = x[4 * h + 3] & z;
            d[h] = uint4{(uint32_t)a, (uint32_t)b, (uint32_t)c, (uint32_t)e};
            d[KS / 4 + h] = uint4{(uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), (uint32_t)(e >> 32)};
        }
    };
    // the lane's raw operand halves (half kh of its rows) for chunk h of a step
    auto fetch = [&](int buf, int h, uint32_t (*ra)[4], uint32_t (*rb)[4]) {
#pragma unroll
        for (int i = 0; i < TI; i++) {
            const uint4 v = reinterpret_cast<const uint4 *>(&sP[buf][wr * TI * 32 + 32 * i + lr][kh * KS])[h];
            ra[i][0] = v.x, ra[i][1] = v.y, ra[i][2] = v.z, ra[i][3] = v.w;
        }
#pragma unroll
        for (int j = 0; j < TJ; j++) {
            const uint4 v = reinterpret_cast<const uint4 *>(&sP[buf][F4_BM + wc * TJ * 32 + 32 * j + lr][kh * KS])[h];
            rb[j][0] = v.x, rb[j][1] = v.y, rb[j][2] = v.z, rb[j][3] = v.w;
        }
    };
    v16f acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; i++)
#pragma unroll
        for (int j = 0; j < TJ; j++) acc[i][j] = v16f{};
    auto mma = [&](const uint32_t (*ra)[4], const uint32_t (*rb)[4]) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            v8i fa[TI], fb[TJ];
#pragma unroll
            for (int i = 0; i < TI; i++) fa[i] = half_to_fp4_y(ra[i][q]);
#pragma unroll
            for (int j = 0; j < TJ; j++) fb[j] = half_to_fp4_x(rb[j][q]);
#pragma unroll
            for (int i = 0; i < TI; i++)
#pragma unroll
                for (int j = 0; j < TJ; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[i], fb[j], acc[i][j], 4, 4, 0, 127,
                                                                               0, 127);
        }
    };
    uint64_t xs[KS];  // step kk + 1's words during step kk
    {
        uint64_t x0[KS];
        ld(0, x0);
        ld(1, xs);
        put(0, x0);
    }
    __syncthreads();
    uint32_t ca[TI][4], cb[TJ][4];  // chunk 0 of the current step
    fetch(0, 0, ca, cb);
    for (int64_t kk = 0; kk < steps; kk++) {
        const int cur = (int)(kk & 1), nxt = cur ^ 1;
        put(nxt, xs);
        uint32_t da[CH - 1][TI][4], db[CH - 1][TJ][4];  // chunks 1.. of the current step
#pragma unroll
        for (int h = 1; h < CH; h++) fetch(cur, h, da[h - 1], db[h - 1]);
        ld(kk + 2, xs);
        __syncthreads();
        uint32_t na[TI][4], nb[TJ][4];
        if (kk + 1 < steps) fetch(nxt, 0, na, nb);
        mma(ca, cb);
#pragma unroll
        for (int h = 1; h < CH; h++) mma(da[h - 1], db[h - 1]);
#pragma unroll
        for (int i = 0; i < TI; i++)
#pragma unroll
            for (int q = 0; q < 4; q++) ca[i][q] = na[i][q];
#pragma unroll
        for (int j = 0; j < TJ; j++)
#pragma unroll
            for (int q = 0; q < 4; q++) cb[j][q] = nb[j][q];
    }
    // sums mod 2 -> bits; lane L collects row L of the wave's 64, words
    // d = 0, 1 of its 128 columns
    uint64_t out[2] = {0, 0};
    const uint64_t lo32 = 0xFFFFFFFFull;
#pragma unroll
    for (int i = 0; i < TI; i++) {
#pragma unroll
        for (int e = 0; e < 16; e++) {
            const int q = 32 * i + (e >> 2) * 8 + (e & 3);  // rows q (lanes < 32) and q + 4 (lanes >= 32)
#pragma unroll
            for (int d = 0; d < 2; d++) {
                const uint64_t b0 = __ballot(((int)acc[i][2 * d][e]) & 1);
                const uint64_t b1 = __ballot(((int)acc[i][2 * d + 1][e]) & 1);
                out[d] = lane == q ? ((b0 & lo32) | (b1 << 32)) : out[d];
                out[d] = lane == q + 4 ? ((b0 >> 32) | (b1 & ~lo32)) : out[d];
            }
        }
    }
    const int64_t row = r0 + wr * TI * 32 + lane;
#pragma unroll
    for (int d = 0; d < 2; d++) {
        const int64_t w = w0 + wc * 2 + d;
        if (!out[d]) continue;
        if (row < o0.rows && w < o0.words) o0.C[row * o0.ldc + w] ^= out[d];
        if (o1.C && row < o1.rows && w < o1.words) o1.C[row * o1.ldc + w] ^= out[d];
    }
}

hipError_t launch_transpose_bits(const uint64_t *B, int64_t ldb, int64_t k, int64_t n, uint64_t *Bt, int64_t ldbt,
                                 hipStream_t s) {
    const int64_t blocks = (words_for(k) * words_for(n) + 3) / 4;
    if (blocks <= 0) return hipSuccess;
    ProfScope ps(KID_TRANSPOSE, s);
    hipLaunchKernelGGL(k_transpose_bits, dim3((unsigned)blocks), dim3(256), 0, s, B, ldb, k, n, Bt, ldbt);
    return hipGetLastError();
}

// C0 (rows0 x words0) ^= A (m x k) * B and, with C1, C1 (rows1 x words1) ^=
// the same product, on the fp4 matrix cores; Bt is B's bit transpose (n rows
// of ldbt words, zero past k).  rows0, rows1 <= m; words0, words1 <= the
// words of n.
hipError_t launch_fp4_product2(uint64_t *C0, int64_t ldc0, int64_t rows0, int64_t words0, uint64_t *C1, int64_t ldc1,
                               int64_t rows1, int64_t words1, const uint64_t *A, int64_t lda, const uint64_t *Bt,
                               int64_t ldbt, int64_t m, int64_t k, int64_t n, hipStream_t s) {
    const int64_t nw = words_for(n), kw = words_for(k);
    const int64_t gcols = (nw + F4_BN / 64 - 1) / (F4_BN / 64), grows = (m + F4_BM - 1) / F4_BM;
    if (gcols <= 0 || grows <= 0 || kw <= 0) return hipSuccess;
    if (rows0 > m || words0 > nw || (C1 && (rows1 > m || words1 > nw))) return hipErrorInvalidValue;
    const F4Out o0{C0, ldc0, rows0, words0}, o1{C1, ldc1, C1 ? rows1 : 0, C1 ? words1 : 0};
    const bool vec = (uintptr_t)A % 16 == 0 && (uintptr_t)Bt % 16 == 0 && lda % 2 == 0 && ldbt % 2 == 0;
    ProfScope ps(KID_MFMA, s);
    if (vec)
        hipLaunchKernelGGL(k_mfma_gf2_fp4<true>, dim3((unsigned)(gcols * grows)), dim3(512), 0, s, o0, o1, A, lda, Bt,
                           ldbt, m, kw, nw, gcols, grows);
    else
        hipLaunchKernelGGL(k_mfma_gf2_fp4<false>, dim3((unsigned)(gcols * grows)), dim3(512), 0, s, o0, o1, A, lda,
                           Bt, ldbt, m, kw, nw, gcols, grows);
    return hipGetLastError();
}

// fmt 0: fp4 matrix cores; 1: int8 matrix cores
hipError_t launch_mfma_gf2(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda, const uint64_t *Bt, int64_t ldbt,
                           int64_t m, int64_t k, int64_t n, hipStream_t s, int fmt) {
    if (fmt == 0) return launch_fp4_product2(C, ldc, m, words_for(n), nullptr, 0, 0, 0, A, lda, Bt, ldbt, m, k, n, s);
    if (k >= 128) {
        // 128 x 128 per wave, four waves side by side
        constexpr int TR = 4, TC = 4;
        const int64_t nw = words_for(n), kw = words_for(k);
        const int64_t gcols = (nw + 4 * (TC / 2) - 1) / (4 * (TC / 2)), grows = (m + 32 * TR - 1) / (32 * TR);
        if (gcols <= 0 || grows <= 0) return hipSuccess;
        ProfScope ps(KID_MFMA, s);
        hipLaunchKernelGGL((k_mfma_gf2t<TR, TC>), dim3((unsigned)(gcols * grows)), dim3(256), 0, s, C, ldc, A, lda, Bt,
                           ldbt, m, kw, nw, gcols);
        return hipGetLastError();
    }
    constexpr int NWR = 2, NWC = 2;
    const int64_t nw = words_for(n), kw = words_for(k);
    const int64_t gcols = (nw + NWC - 1) / NWC, grows = (m + 64 * NWR - 1) / (64 * NWR);
    if (gcols <= 0 || grows <= 0) return hipSuccess;
    ProfScope ps(KID_MFMA, s);
    hipLaunchKernelGGL((k_mfma_gf2<NWR, NWC>), dim3((unsigned)(gcols * grows)), dim3(NWR * NWC * 64), 0, s, C, ldc, A,
                       lda, Bt, ldbt, m, kw, nw, gcols);
    return hipGetLastError();
}

}  // namespace gf2
