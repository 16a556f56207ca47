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
// with e2m1 operands, unit scales): a bit becomes the fp4 value 0.0 or 1.0
// (nibble 0b0000 / 0b0010), the fp32 sums are exact integers (at most k),
// and their low bit is the GF(2) sum.
//
// A block computes 256 rows x 256 columns of C (4 output words) with four
// waves in 2 x 2, each 128 x 128 as 4 x 4 tiles of 32 x 32 (256 fp32
// accumulators per lane).  K advances one 64-bit word a step: each thread
// expands one word of A (its row) and one word of Bt (its column) into fp4
// in LDS -- once per block instead of once per wave, four shift-and-mask
// steps per 32 bits -- and the waves read their operands from there.  LDS is double-buffered, so the next step's
// expansion overlaps this step's matrix-core work; the words themselves are
// loaded four steps ahead.
// ---------------------------------------------------------------------------
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// 32 bits -> 32 fp4 values 0.0 / 1.0 (nibble 0b0010 = 1.0) in four dwords.
// The K order inside an operand is free as long as A and B share it, so
// bit 4s + d of v goes to nibble s of dword d: each dword is one shift and
// one mask of v.
__device__ __forceinline__ uint4 word_half_to_fp4(uint64_t w, int half) {
    const uint32_t v = (uint32_t)(w >> (32 * half));
    uint4 r;
    r.x = (v << 1) & 0x22222222u;
    r.y = v & 0x22222222u;
    r.z = (v >> 1) & 0x22222222u;
    r.w = (v >> 2) & 0x22222222u;
    return r;
}

constexpr int F4_BM = 256, F4_BN = 256, F4_AHEAD = 4;  // block rows, block columns, words loaded ahead

__global__ __launch_bounds__(256) void k_mfma_gf2_fp4(uint64_t *__restrict__ C, int64_t ldc,
                                                      const uint64_t *__restrict__ A, int64_t lda,
                                                      const uint64_t *__restrict__ Bt, int64_t ldbt, int64_t m,
                                                      int64_t kw, int64_t nw, int64_t gcols, int64_t grows) {
    // [buffer][K half][row or column]: 32 fp4 values (one K half of a word)
    __shared__ uint4 sA[2][2][F4_BM];
    __shared__ uint4 sB[2][2][F4_BN];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // blocks of one XCD take a contiguous range: neighbouring column blocks
    // of the same rows share that XCD's L2
    const int64_t logical = xcd_logical((int)blockIdx.x, (int)gridDim.x);
    const int64_t bc = logical % gcols, br = logical / gcols;
    if (br >= grows) return;  // (the grid is exactly gcols x grows)
    const int64_t r0 = br * F4_BM, w0 = bc * (F4_BN / 64);
    const int64_t ra = r0 + tid;
    const bool va = ra < m;
    const uint64_t *pa = A + (va ? ra : 0) * lda;
    const int64_t cb = w0 * 64 + tid;  // Bt has nw * 64 rows (zero past n)
    const bool vb = cb < nw * 64;
    const uint64_t *pb = Bt + (vb ? cb : 0) * ldbt;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 31, kh = lane >> 5;

    auto ldA = [&](int64_t kk) { return (va && kk < kw) ? pa[kk] : 0ull; };
    auto ldB = [&](int64_t kk) { return (vb && kk < kw) ? pb[kk] : 0ull; };
    auto store = [&](int buf, uint64_t x, uint64_t y) {
        sA[buf][0][tid] = word_half_to_fp4(x, 0);
        sA[buf][1][tid] = word_half_to_fp4(x, 1);
        sB[buf][0][tid] = word_half_to_fp4(y, 0);
        sB[buf][1][tid] = word_half_to_fp4(y, 1);
    };
    auto frag = [](const uint4 &t) { return v8i{(int)t.x, (int)t.y, (int)t.z, (int)t.w, 0, 0, 0, 0}; };
    // xa[i], xb[i]: the words of step kk + 1 + i, in flight
    uint64_t xa[F4_AHEAD], xb[F4_AHEAD];
#pragma unroll
    for (int i = 0; i < F4_AHEAD; i++) {
        xa[i] = ldA(1 + i);
        xb[i] = ldB(1 + i);
    }
    v16f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = v16f{};
    // step kk's operands come from buffer kk & 1: written (expanded) during
    // step kk - 1, read into registers right after the barrier that ends it,
    // so each step's matrix-core work overlaps the next step's expansion
    store(0, ldA(0), ldB(0));
    __syncthreads();
    v8i fa[4], fb[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        fa[i] = frag(sA[0][kh][wr * 128 + 32 * i + lr]);
        fb[i] = frag(sB[0][kh][wc * 128 + 32 * i + lr]);
    }
    for (int64_t kk = 0; kk < kw; kk++) {
        const int nxt = (int)((kk + 1) & 1);
        // buffer nxt was last read for step kk - 1, before the barrier that
        // ended it; past the last step this store is unused
        store(nxt, xa[0], xb[0]);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++)
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[i], fb[j], acc[i][j], 4, 4, 0, 127, 0,
                                                                           127);
#pragma unroll
        for (int i = 0; i + 1 < F4_AHEAD; i++) {
            xa[i] = xa[i + 1];
            xb[i] = xb[i + 1];
        }
        xa[F4_AHEAD - 1] = ldA(kk + 1 + F4_AHEAD);
        xb[F4_AHEAD - 1] = ldB(kk + 1 + F4_AHEAD);
        // issue order: the expansion's ALU work and LDS stores between the
        // matrix-core instructions (32 cycles each), and all of it before the
        // barrier
#pragma unroll
        for (int g = 0; g < 16; g++) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // two VALU
            if (g % 4 == 3) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // one LDS store
        }
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
        if (kk + 1 < kw) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                fa[i] = frag(sA[nxt][kh][wr * 128 + 32 * i + lr]);
                fb[i] = frag(sB[nxt][kh][wc * 128 + 32 * i + lr]);
            }
        }
    }
    // sums mod 2 -> bits; lane L collects rows L and 64 + L of the wave's
    // 128, words d = 0, 1 of its 128 columns
    uint64_t out[2][2] = {{0, 0}, {0, 0}};
    const uint64_t lo32 = 0xFFFFFFFFull;
#pragma unroll
    for (int i = 0; i < 4; i++) {
#pragma unroll
        for (int e = 0; e < 16; e++) {
            const int q = 32 * i + (e >> 2) * 8 + (e & 3);  // rows q (lanes < 32) and q + 4 (lanes >= 32)
#pragma unroll
            for (int d = 0; d < 2; d++) {
                const uint64_t b0 = __ballot(((int)acc[i][2 * d][e]) & 1);
                const uint64_t b1 = __ballot(((int)acc[i][2 * d + 1][e]) & 1);
                out[q >> 6][d] = lane == (q & 63) ? ((b0 & lo32) | (b1 << 32)) : out[q >> 6][d];
                out[(q + 4) >> 6][d] = lane == ((q + 4) & 63) ? ((b0 >> 32) | (b1 & ~lo32)) : out[(q + 4) >> 6][d];
            }
        }
    }
#pragma unroll
    for (int p = 0; p < 2; p++) {
        const int64_t row = r0 + wr * 128 + 64 * p + lane;
#pragma unroll
        for (int d = 0; d < 2; d++) {
            const int64_t w = w0 + wc * 2 + d;
            if (row < m && w < nw && out[p][d]) C[row * ldc + w] ^= out[p][d];
        }
    }
}

hipError_t launch_transpose_bits(const uint64_t *B, int64_t ldb, int64_t k, int64_t n, uint64_t *Bt, int64_t ldbt,
                                 hipStream_t s) {
    const int64_t blocks = (words_for(k) * words_for(n) + 3) / 4;
    if (blocks <= 0) return hipSuccess;
    ProfScope ps(KID_MFMA, s);
    hipLaunchKernelGGL(k_transpose_bits, dim3((unsigned)blocks), dim3(256), 0, s, B, ldb, k, n, Bt, ldbt);
    return hipGetLastError();
}

// fmt 0: fp4 matrix cores; 1: int8 matrix cores
hipError_t launch_mfma_gf2(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda, const uint64_t *Bt, int64_t ldbt,
                           int64_t m, int64_t k, int64_t n, hipStream_t s, int fmt) {
    if (fmt == 0) {
        const int64_t nw = words_for(n), kw = words_for(k);
        const int64_t gcols = (nw + F4_BN / 64 - 1) / (F4_BN / 64), grows = (m + F4_BM - 1) / F4_BM;
        if (gcols <= 0 || grows <= 0 || kw <= 0) return hipSuccess;
        ProfScope ps(KID_MFMA, s);
        hipLaunchKernelGGL(k_mfma_gf2_fp4, dim3((unsigned)(gcols * grows)), dim3(256), 0, s, C, ldc, A, lda, Bt, ldbt,
                           m, kw, nw, gcols, grows);
        return hipGetLastError();
    }
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
