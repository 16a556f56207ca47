// HIP kernels (gfx950) of block-iterative PLE over GF(2).
//
// One pass of Algorithm 2 ("Block-iterative PLE decomposition", Section 3.2)
// over the stripe of 64 columns starting at c is three launches:
//
//   k_panel    one wave.  Algorithm 1 (PartialPle) on the stripe: lazy
//              first-non-zero pivot search with ballots over a register window
//              of rows, whole-row swap bookkeeping, and the small dense algebra
//              that turns the pivot rows into linear maps (the T' of
//              Section 3.2): stripe word v -> w (coefficients on the pivot rows
//              as they were) and v -> u (the row's L bits).
//   k_permute  wide.  Applies the pass's row swaps to whole rows, stages the
//              pivot rows' trailing words, writes every row's coefficient word
//              w and its compressed L bits (the column swaps of "compress L",
//              Algorithm 4's effect, done as a bit placement per row).
//   k_m4rm     wide.  The trailing update A22 <- L21 A12 + A22 and
//              (A31, A32) <- (A31 E11^-1, A31 E11^-1 A12 + A32) as ONE
//              Four-Russians product: eight 256-entry tables (MakeTable) of the
//              staged pivot rows per 8-word column tile in LDS, one lookup per
//              byte of w per row word (AddRowsFromTable).  Pivot rows take the
//              same path with w = row of L11^-1, which is the TRSM of
//              Algorithm 2 folded into the lookup.
//
// The same k_m4rm kernel is the public GF(2) product gf2_addmul.
#include "common.h"

namespace gf2 {

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int readlane32(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        lo |= (uint32_t)__shfl_xor((int)lo, off, 64);
        hi |= (uint32_t)__shfl_xor((int)hi, off, 64);
    }
    return ((uint64_t)hi << 32) | lo;
}

// bits strictly above column j of a word
__device__ __forceinline__ uint64_t above(int j) { return j >= 63 ? 0ull : (~0ull << (j + 1)); }

// The part of the rbar-bit vector u (bit l = column r + l) that falls into word w.
__device__ __forceinline__ uint64_t place_bits(uint64_t u, int64_t w, int64_t wr0, int sh) {
    if (w == wr0) return u << sh;
    if (sh && w == wr0 + 1) return u >> (64 - sh);
    return 0;
}

// ---------------------------------------------------------------------------
// k_init: P = identity, Q = -1, rank = 0, empty pass record.
// ---------------------------------------------------------------------------
__global__ void k_init(int64_t *P, int64_t m, int64_t *Q, int64_t mn, int64_t *rank, PassRec *rec) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = i; t < m; t += stride) P[t] = t;
    for (int64_t t = i; t < mn; t += stride) Q[t] = -1;
    if (i == 0) {
        *rank = 0;
        rec->r = 0;
        rec->rbar = 0;
        rec->nspec = 0;
        rec->active = 0;
        rec->slow = 0;
    }
}

// ---------------------------------------------------------------------------
// k_panel: Algorithm 1 on the stripe word of rows r .. m-1 (one wave).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_panel(const uint64_t *__restrict__ A, int64_t m, int64_t n, int64_t ldw,
                                              int64_t c, PassRec *rec, int64_t *P, int64_t *Q, int64_t *rank_out,
                                              uint64_t *gsv, int32_t *gsid) {
    __shared__ uint64_t s_img_w[KW], s_img_u[KW];
    __shared__ int64_t s_dst[MAX_SPEC], s_src[MAX_SPEC];
    __shared__ uint64_t s_sv[SLOW_LDS_ROWS];
    __shared__ int32_t s_sid[SLOW_LDS_ROWS];

    const int lane = threadIdx.x;
    const int64_t r = rec->r + rec->rbar;  // rank after the previous pass
    __syncthreads();
    if (r >= m || c >= n) {
        if (lane == 0) {
            rec->r = r;
            rec->rbar = 0;
            rec->nspec = 0;
            rec->active = 0;
            rec->slow = 0;
            *rank_out = r;
        }
        return;
    }
    const int kp = (int)((n - c) < KW ? (n - c) : KW);
    const uint64_t kmask = kp == 64 ? ~0ull : ((1ull << kp) - 1);
    const int64_t sw = c >> 6;
    const int64_t rows = m - r;

    // lane l keeps pivot l: its stripe column, its reduced stripe word, and
    // the window position it was found at
    int my_q = 0;
    uint64_t my_fin = 0;
    int64_t my_p = 0;
    int npiv = 0;
    int nspec = 0;
    bool slow = false;

    // ---- fast path: rows r .. r + 64*WIN_Q - 1 in registers ------------------
    {
        uint64_t val[WIN_Q];
        int32_t id[WIN_Q];
        const int nload = (int)(rows < 64 * WIN_Q ? rows : 64 * WIN_Q);
#pragma unroll
        for (int q = 0; q < WIN_Q; q++) {
            int pos = 64 * q + lane;
            val[q] = pos < nload ? (A[(r + pos) * ldw + sw] & kmask) : 0ull;
            id[q] = pos;
        }
        for (int j = 0; j < kp; j++) {
            int found = -1;
#pragma unroll
            for (int q = 0; q < WIN_Q; q++) {
                if (found < 0 && 64 * q < nload && 64 * q + 64 > npiv) {
                    int pos = 64 * q + lane;
                    bool b = pos >= npiv && pos < nload && ((val[q] >> j) & 1ull);
                    uint64_t msk = __ballot(b);
                    if (msk) found = 64 * q + __builtin_ctzll(msk);
                }
            }
            if (found < 0) {
                if (nload < rows) {  // a row outside the window may hold the pivot
                    slow = true;
                    break;
                }
                continue;  // column j has no pivot
            }
            uint64_t pv = 0, vr = 0;
            int32_t idp = 0, idr = 0;
#pragma unroll
            for (int q = 0; q < WIN_Q; q++) {
                if (q == (found >> 6)) {
                    pv = readlane64(val[q], found & 63);
                    idp = readlane32(id[q], found & 63);
                }
                if (q == (npiv >> 6)) {
                    vr = readlane64(val[q], npiv & 63);
                    idr = readlane32(id[q], npiv & 63);
                }
            }
            const uint64_t pe = pv & above(j);
#pragma unroll
            for (int q = 0; q < WIN_Q; q++) {
                int pos = 64 * q + lane;
                if (pos == found) {
                    val[q] = vr;
                    id[q] = idr;
                }
                if (pos == npiv) {
                    val[q] = pv;
                    id[q] = idp;
                } else if (pos > npiv && pos < nload && ((val[q] >> j) & 1ull)) {
                    val[q] ^= pe;
                }
            }
            if (lane == npiv) {
                my_q = j;
                my_fin = pv;
                my_p = found;
            }
            npiv++;
            if (npiv == rows) break;
        }
        if (!slow) {
            int base = 0;
#pragma unroll
            for (int q = 0; q < WIN_Q; q++) {
                int pos = 64 * q + lane;
                bool f = pos < nload && (pos < npiv || id[q] != pos);
                uint64_t msk = __ballot(f);
                int idx = base + __popcll(msk & ((1ull << lane) - 1ull));
                if (f) {
                    s_dst[idx] = r + pos;
                    s_src[idx] = r + id[q];
                }
                base += __popcll(msk);
            }
            nspec = base;
        }
    }

    // ---- slow path: every remaining row, window in LDS or workspace ---------
    if (slow) {
        npiv = 0;
        my_q = 0;
        my_fin = 0;
        my_p = 0;
        volatile uint64_t *sv = rows <= SLOW_LDS_ROWS ? (volatile uint64_t *)s_sv : (volatile uint64_t *)gsv;
        volatile int32_t *sid = rows <= SLOW_LDS_ROWS ? (volatile int32_t *)s_sid : (volatile int32_t *)gsid;
        uint64_t orv = 0;
        for (int64_t pos = lane; pos < rows; pos += 64) {
            uint64_t v = A[(r + pos) * ldw + sw] & kmask;
            sv[pos] = v;
            sid[pos] = (int32_t)pos;
            orv |= v;
        }
        orv = wave_or64(orv);
        __syncthreads();
        for (int j = 0; j < kp && npiv < rows; j++) {
            if (!((orv >> j) & 1ull)) continue;  // no remaining row has a 1 here
            int64_t found = -1;
            for (int64_t base = npiv & ~(int64_t)63; base < rows; base += 64) {
                int64_t pos = base + lane;
                bool b = pos >= npiv && pos < rows && ((sv[pos] >> j) & 1ull);
                uint64_t msk = __ballot(b);
                if (msk) {
                    found = base + __builtin_ctzll(msk);
                    break;
                }
            }
            if (found < 0) continue;  // unreachable: orv says a row has bit j
            const uint64_t pv = sv[found];
            const int32_t idp = sid[found];
            const uint64_t vr = sv[npiv];
            const int32_t idr = sid[npiv];
            __syncthreads();
            if (lane == 0) {
                sv[found] = vr;
                sid[found] = idr;
                sv[npiv] = pv;
                sid[npiv] = idp;
            }
            if (lane == npiv) {
                my_q = j;
                my_fin = pv;
                my_p = found;
            }
            __syncthreads();
            const uint64_t pe = pv & above(j);
            orv = 0;
            for (int64_t pos = npiv + 1 + lane; pos < rows; pos += 64) {
                uint64_t v = sv[pos];
                if ((v >> j) & 1ull) {
                    v ^= pe;
                    sv[pos] = v;
                }
                orv |= v;
            }
            orv = wave_or64(orv);
            __syncthreads();
            npiv++;
        }
        int base = 0;
        for (int64_t pb = 0; pb < rows; pb += 64) {
            int64_t pos = pb + lane;
            bool f = pos < rows && (pos < npiv || sid[pos] != (int32_t)pos);
            uint64_t msk = __ballot(f);
            int idx = base + __popcll(msk & ((1ull << lane) - 1ull));
            if (f) {
                s_dst[idx] = r + pos;
                s_src[idx] = r + sid[pos];
            }
            base += __popcll(msk);
        }
        nspec = base;
    }
    __syncthreads();

    // ---- the pass's linear maps (Section 3.2, T and T') ---------------------
    // F = pivot row's reduced stripe at the pivot columns: strictly below the
    // diagonal the multipliers (L11), on and above it E11 restricted to the
    // pivot columns (unit upper triangular).
    const int rbar = npiv;
    uint64_t F = 0;
    for (int l2 = 0; l2 < rbar; l2++) {
        int q2 = readlane32(my_q, l2);
        F |= ((my_fin >> q2) & 1ull) << l2;
    }
    const uint64_t low = (1ull << lane) - 1ull;  // lane < 64
    const uint64_t Ls = F & low;
    const uint64_t Eu = F & ~low;
    // X = L11^-1 (forward substitution, column by column)
    uint64_t X = 1ull << lane;
    for (int l2 = 0; l2 < rbar; l2++) {
        uint64_t x2 = readlane64(X, l2);
        if (lane > l2 && ((Ls >> l2) & 1ull)) X ^= x2;
    }
    // Y = E11pc^-1 (backward substitution)
    uint64_t Y = 1ull << lane;
    for (int l2 = rbar - 1; l2 >= 0; l2--) {
        uint64_t y2 = readlane64(Y, l2);
        if (lane < l2 && ((Eu >> l2) & 1ull)) Y ^= y2;
    }
    // Z = Y X = (L11 E11pc)^-1 = (Orig rows at the pivot columns)^-1
    uint64_t Z = 0;
    for (int l2 = 0; l2 < rbar; l2++) {
        uint64_t x2 = readlane64(X, l2);
        if ((Y >> l2) & 1ull) Z ^= x2;
    }
    s_img_w[lane] = 0;
    s_img_u[lane] = 0;
    __syncthreads();
    if (lane < rbar) {
        s_img_w[my_q] = Z;  // stripe bit q_l -> w
        s_img_u[my_q] = Y;  // stripe bit q_l -> u
    }
    __syncthreads();
    rec->img_w[lane] = s_img_w[lane];
    rec->img_u[lane] = s_img_u[lane];

    // special rows: pivots first (position r + k), then displaced rows
    for (int k = lane; k < nspec; k += 64) {
        const int64_t dst = s_dst[k], src = s_src[k];
        rec->spec_dst[k] = dst;
        rec->spec_src[k] = src;
        if (k >= rbar) {
            const uint64_t v = A[src * ldw + sw] & kmask;
            uint64_t w = 0, u = 0;
            for (int j = 0; j < kp; j++) {
                if ((v >> j) & 1ull) {
                    w ^= s_img_w[j];
                    u ^= s_img_u[j];
                }
            }
            rec->spec_coef[k] = w;
            rec->spec_lbits[k] = u;
            rec->spec_stripe[k] = 0;
        }
    }
    if (lane < rbar) {
        rec->spec_coef[lane] = X ^ (1ull << lane);  // L11^-1 row without its diagonal
        rec->spec_lbits[lane] = Ls;                   // L11 row
        rec->spec_stripe[lane] = my_fin & ~((1ull << my_q) - 1ull);
        P[r + lane] = r + my_p;
        Q[r + lane] = c + my_q;
    }
    if (lane == 0) {
        rec->r = r;
        rec->rbar = rbar;
        rec->nspec = nspec;
        rec->active = rbar > 0;
        rec->slow = slow ? 1 : 0;
        *rank_out = r + rbar;
    }
}

// ---------------------------------------------------------------------------
// k_permute: swaps, pivot staging, coefficients, L bits.
//   blocks [0, nA): 64 word columns each, every special row (read all, then
//                   write all, so the permutation is applied in place);
//   blocks [nA, ..): grid-stride over the other rows r .. m-1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WIDE_THREADS) void k_permute(uint64_t *__restrict__ A, int64_t m, int64_t ldw, int64_t c,
                                                          const PassRec *__restrict__ rec, uint64_t *__restrict__ coef,
                                                          uint64_t *__restrict__ PB, int nA) {
    __shared__ uint64_t tw[8][256], tu[8][256];
    __shared__ uint64_t simg_w[KW], simg_u[KW];
    __shared__ int64_t sdisp[KW];
    __shared__ uint64_t sdcoef[KW];

    if (!rec->active) return;
    const int tid = threadIdx.x;
    const int64_t r = rec->r;
    const int rbar = rec->rbar;
    const int nspec = rec->nspec;
    const int64_t sw = c >> 6;
    const int64_t wr0 = r >> 6;
    const int sh = (int)(r & 63);

    if ((int)blockIdx.x < nA) {
        constexpr int SLOTS = WIDE_THREADS / 64;         // 16
        constexpr int PER = MAX_SPEC / SLOTS;            // 8
        const int64_t w = (int64_t)blockIdx.x * 64 + (tid & 63);
        const int slot = tid >> 6;
        uint64_t nv[PER];
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int k = slot + SLOTS * t;
            nv[t] = 0;
            if (k < nspec && w < ldw) {
                const int64_t src = rec->spec_src[k];
                const uint64_t old = A[src * ldw + w];
                uint64_t nw = old;
                if (w == sw)
                    nw = place_bits(rec->spec_lbits[k], w, wr0, sh) | rec->spec_stripe[k];
                else if (w >= wr0 && w < sw)
                    nw = old | place_bits(rec->spec_lbits[k], w, wr0, sh);
                if (k < rbar && w > sw) PB[(int64_t)k * ldw + w] = old;
                nv[t] = nw;
            }
        }
        __syncthreads();  // every read of these columns precedes every write
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int k = slot + SLOTS * t;
            if (k < nspec && w < ldw) {
                const int64_t src = rec->spec_src[k], dst = rec->spec_dst[k];
                if (dst != src || (w >= wr0 && w <= sw)) A[dst * ldw + w] = nv[t];
            }
        }
        return;
    }

    // ---- other rows ----
    const int ndisp = nspec - rbar;
    if (tid < KW) {
        simg_w[tid] = rec->img_w[tid];
        simg_u[tid] = rec->img_u[tid];
    }
    int64_t maxdisp = -1;
    if (tid < ndisp) {
        sdisp[tid] = rec->spec_dst[rbar + tid];
        sdcoef[tid] = rec->spec_coef[rbar + tid];
    }
    __syncthreads();
    for (int d = 0; d < ndisp; d++) maxdisp = sdisp[d] > maxdisp ? sdisp[d] : maxdisp;
    for (int e = tid; e < 8 * 256; e += WIDE_THREADS) {
        const int b = e >> 8, x = e & 255;
        uint64_t a = 0, bb = 0;
#pragma unroll
        for (int t = 0; t < 8; t++)
            if ((x >> t) & 1) {
                a ^= simg_w[8 * b + t];
                bb ^= simg_u[8 * b + t];
            }
        tw[b][x] = a;
        tu[b][x] = bb;
    }
    __syncthreads();
    const int64_t nB = (int64_t)gridDim.x - nA;
    for (int64_t i = r + ((int64_t)blockIdx.x - nA) * WIDE_THREADS + tid; i < m; i += nB * WIDE_THREADS) {
        if (i < r + rbar) {
            coef[i] = rec->spec_coef[i - r];
            continue;
        }
        if (i <= maxdisp) {
            bool disp = false;
            for (int d = 0; d < ndisp; d++)
                if (sdisp[d] == i) {
                    coef[i] = sdcoef[d];
                    disp = true;
                    break;
                }
            if (disp) continue;
        }
        uint64_t *row = A + i * ldw;
        const uint64_t v = row[sw];
        if (!v) {
            coef[i] = 0;
            continue;
        }
        uint64_t wv = 0, u = 0;
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const int x = (int)((v >> (8 * b)) & 255);
            wv ^= tw[b][x];
            u ^= tu[b][x];
        }
        coef[i] = wv;
        if (wr0 < sw) {
            row[wr0] |= u << sh;
            if (sh && wr0 + 1 < sw) row[wr0 + 1] |= u >> (64 - sh);
        }
        row[sw] = place_bits(u, sw, wr0, sh);
    }
}

// ---------------------------------------------------------------------------
// k_m4rm: C[rows, words] ^= sum_b T_b[byte b of coef[row]] over one column
// tile of TILE_W words per block.  T_b (b < 8) holds all 256 sums of B rows
// 8b .. 8b+7 restricted to the tile (MakeTable); each row adds one entry per
// non-zero byte (AddRowsFromTable).  With `rec` the rows are rec->r .. m-1
// and B has rec->rbar rows; without it, rows 0 .. m-1 and `nbits` rows.
// Block -> (tile, chunk) with tiles fastest; consecutive logical blocks are
// placed on the same XCD so neighbouring tiles share L2 lines.
// ---------------------------------------------------------------------------
constexpr int M4_UNROLL = 4;

__global__ __launch_bounds__(WIDE_THREADS) void k_m4rm(uint64_t *__restrict__ C, int64_t ldc, int64_t m,
                                                       const uint64_t *__restrict__ coef, int64_t coef_ld,
                                                       const uint64_t *__restrict__ B, int64_t ldb, int nbits,
                                                       int64_t w_begin, int64_t w_end, int ntiles, int nchunks,
                                                       const PassRec *__restrict__ rec) {
    __shared__ uint64_t T[8][256][TILE_W];
    __shared__ uint64_t Bt[KW][TILE_W];

    int64_t row0 = 0;
    if (rec) {
        if (!rec->active) return;
        row0 = rec->r;
        nbits = rec->rbar;
    }
    const int G = gridDim.x;
    const int bid = blockIdx.x;
    const int xcd = bid & 7, jx = bid >> 3;
    const int g8 = G >> 3, rem = G & 7;
    const int logical = xcd * g8 + (xcd < rem ? xcd : rem) + jx;
    const int tile = logical % ntiles;
    const int chunk = logical / ntiles;
    if (chunk >= nchunks) return;
    const int64_t rows = m - row0;
    const int64_t per = (rows + nchunks - 1) / nchunks;
    const int64_t rb = row0 + (int64_t)chunk * per;
    const int64_t re = rb + per < m ? rb + per : m;
    if (rb >= re) return;
    const int64_t wt0 = w_begin + (int64_t)tile * TILE_W;
    const int tid = threadIdx.x;

    for (int e = tid; e < KW * TILE_W; e += WIDE_THREADS) {
        const int k = e / TILE_W, wl = e % TILE_W;
        const int64_t w = wt0 + wl;
        Bt[k][wl] = (k < nbits && w < w_end) ? B[(int64_t)k * ldb + w] : 0ull;
    }
    __syncthreads();
    const int nbytes = (nbits + 7) >> 3;
    for (int e = tid; e < 8 * 256 * TILE_W; e += WIDE_THREADS) {
        const int wl = e % TILE_W;
        const int x = (e / TILE_W) & 255;
        const int b = e / (TILE_W * 256);
        uint64_t acc = 0;
        if (b < nbytes) {
#pragma unroll
            for (int t = 0; t < 8; t++)
                if ((x >> t) & 1) acc ^= Bt[8 * b + t][wl];
        }
        T[b][x][wl] = acc;
    }
    __syncthreads();

    const int wl = tid % TILE_W;
    const int rs = tid / TILE_W;
    constexpr int RS = WIDE_THREADS / TILE_W;
    const int64_t w = wt0 + wl;
    const bool wok = w < w_end;
    for (int64_t i0 = rb + rs; i0 < re; i0 += (int64_t)RS * M4_UNROLL) {
        uint64_t cw[M4_UNROLL], x[M4_UNROLL];
#pragma unroll
        for (int u = 0; u < M4_UNROLL; u++) {
            const int64_t i = i0 + (int64_t)u * RS;
            cw[u] = i < re ? coef[i * coef_ld] : 0ull;
            x[u] = (i < re && wok) ? C[i * ldc + w] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < M4_UNROLL; u++) {
            uint64_t acc = 0;
#pragma unroll
            for (int b = 0; b < 8; b++)
                if (b < nbytes) acc ^= T[b][(cw[u] >> (8 * b)) & 255][wl];
            x[u] ^= acc;
        }
#pragma unroll
        for (int u = 0; u < M4_UNROLL; u++) {
            const int64_t i = i0 + (int64_t)u * RS;
            if (i < re && wok && cw[u]) C[i * ldc + w] = x[u];
        }
    }
}

// ---------------------------------------------------------------------------
// Echelon from L\E: clear the L part, zero the rows at or past the rank.
// ---------------------------------------------------------------------------
__global__ void k_echelon(uint64_t *A, int64_t m, int64_t ldw, const int64_t *rank) {
    const int64_t r = *rank;
    const int64_t total = m * ldw;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ldw, w = e - i * ldw;
        if (i >= r) {
            A[e] = 0;
        } else {
            const int64_t lw = i >> 6;
            if (w < lw) A[e] = 0;
            else if (w == lw) A[e] &= ~((1ull << (i & 63)) - 1ull);
        }
    }
}

// Padding check: any bit at a column >= n sets *flag.
__global__ void k_padding(const uint64_t *A, int64_t m, int64_t n, int64_t ldw, int *flag) {
    const int64_t nw = words_for(n);
    const uint64_t tailmask = (n & 63) ? ~((1ull << (n & 63)) - 1ull) : 0ull;
    const int64_t total = m * ldw;
    int hit = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ldw, w = e - i * ldw;
        const uint64_t v = A[e];
        if (w >= nw) hit |= v != 0;
        else if (w == nw - 1) hit |= (v & tailmask) != 0;
    }
    if (hit) atomicOr(flag, 1);
}

// MakeTable by Gray code: one thread per word column walks i = 1 .. 2^k - 1;
// g(i) = i ^ (i >> 1) differs from g(i-1) in bit ctz(i), i.e. row k-1-ctz(i)
// of the most-significant-first ordering.
__global__ void k_make_table(const uint64_t *rows, int64_t ldr, int k, int64_t nw, uint64_t *T, int64_t ldt) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= ldt) return;
    uint64_t cur = 0;
    T[w] = 0;
    const int size = 1 << k;
    for (int i = 1; i < size; i++) {
        const int bit = __builtin_ctz(i);
        if (w < nw) cur ^= rows[(int64_t)(k - 1 - bit) * ldr + w];
        const int g = i ^ (i >> 1);
        T[(int64_t)g * ldt + w] = w < nw ? cur : 0ull;
    }
}

// ---------------------------------------------------------------------------
// launch wrappers (host side)
// ---------------------------------------------------------------------------
hipError_t launch_init(int64_t *P, int64_t m, int64_t *Q, int64_t mn, int64_t *rank, PassRec *rec, hipStream_t s) {
    int64_t work = m > mn ? m : mn;
    int blocks = (int)((work + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(256), 0, s, P, m, Q, mn, rank, rec);
    return hipGetLastError();
}

hipError_t launch_pass(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t c, PassRec *rec, int64_t *P,
                       int64_t *Q, int64_t *rank, uint64_t *coef, uint64_t *PB, uint64_t *gsv, int32_t *gsid,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_panel, dim3(1), dim3(64), 0, s, (const uint64_t *)A, m, n, ldw, c, rec, P, Q, rank, gsv, gsid);
    const int nA = (int)((ldw + 63) / 64);
    int64_t rows_est = m - (c < m ? c : m);
    if (rows_est < 1) rows_est = 1;
    int nB = (int)((rows_est + WIDE_THREADS - 1) / WIDE_THREADS);
    if (nB > 256) nB = 256;
    if (nB < 1) nB = 1;
    hipLaunchKernelGGL(k_permute, dim3(nA + nB), dim3(WIDE_THREADS), 0, s, A, m, ldw, c, (const PassRec *)rec, coef, PB,
                       nA);
    const int64_t nw = words_for(n);
    const int64_t tw0 = (c >> 6) + 1;
    if (tw0 < nw) {
        const int ntiles = (int)((nw - tw0 + TILE_W - 1) / TILE_W);
        int nchunks = (int)((rows_est + 127) / 128);
        const int want = (512 + ntiles - 1) / ntiles;
        if (nchunks > want) nchunks = want;
        if (nchunks < 1) nchunks = 1;
        hipLaunchKernelGGL(k_m4rm, dim3(ntiles * nchunks), dim3(WIDE_THREADS), 0, s, A, ldw, m, (const uint64_t *)coef,
                           (int64_t)1, (const uint64_t *)PB, ldw, KW, tw0, nw, ntiles, nchunks, (const PassRec *)rec);
    }
    return hipGetLastError();
}

hipError_t launch_m4rm(uint64_t *C, int64_t ldc, int64_t m, const uint64_t *coef, int64_t coef_ld, const uint64_t *B,
                       int64_t ldb, int nbits, int64_t w_begin, int64_t w_end, hipStream_t s) {
    if (w_begin >= w_end || m <= 0) return hipSuccess;
    const int ntiles = (int)((w_end - w_begin + TILE_W - 1) / TILE_W);
    int nchunks = (int)((m + 127) / 128);
    const int want = (512 + ntiles - 1) / ntiles;
    if (nchunks > want) nchunks = want;
    if (nchunks < 1) nchunks = 1;
    hipLaunchKernelGGL(k_m4rm, dim3(ntiles * nchunks), dim3(WIDE_THREADS), 0, s, C, ldc, m, coef, coef_ld, B, ldb, nbits,
                       w_begin, w_end, ntiles, nchunks, (const PassRec *)nullptr);
    return hipGetLastError();
}

hipError_t launch_echelon(uint64_t *A, int64_t m, int64_t ldw, const int64_t *rank, hipStream_t s) {
    int64_t total = m * ldw;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_echelon, dim3(blocks), dim3(256), 0, s, A, m, ldw, rank);
    return hipGetLastError();
}

hipError_t launch_padding(const uint64_t *A, int64_t m, int64_t n, int64_t ldw, int *flag, hipStream_t s) {
    int64_t total = m * ldw;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_padding, dim3(blocks), dim3(256), 0, s, A, m, n, ldw, flag);
    return hipGetLastError();
}

hipError_t launch_make_table(const uint64_t *rows, int64_t ldr, int k, int64_t nw, uint64_t *T, int64_t ldt,
                             hipStream_t s) {
    int blocks = (int)((ldt + 255) / 256);
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_make_table, dim3(blocks), dim3(256), 0, s, rows, ldr, k, nw, T, ldt);
    return hipGetLastError();
}

}  // namespace gf2
