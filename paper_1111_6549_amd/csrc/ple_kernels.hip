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
#include <hip/hip_ext.h>

#include "m4rm.h"
#include "panel.h"

namespace gf2 {

// ---------------------------------------------------------------------------
// k_init: P = identity, Q = -1, rank = 0, empty pass record.
// ---------------------------------------------------------------------------
__global__ void k_init(int64_t *P, int64_t m, int64_t *Q, int64_t mn, int64_t *rank, PassRec *recs) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = i; t < m; t += stride) P[t] = t;
    for (int64_t t = i; t < mn; t += stride) Q[t] = -1;
    if (i < NREC && recs) {
        if (i == 0) *rank = 0;
        recs[i].r = 0;
        recs[i].rbar = 0;
        recs[i].nspec = 0;
        recs[i].active = 0;
        recs[i].slow = 0;
    }
}

// ---------------------------------------------------------------------------
// k_panel: one wave runs the panel of the stripe at column c.
// ---------------------------------------------------------------------------
// waves of a standalone panel's block (wave 0 runs the panel, all of them its
// slow search).  Eight, two per SIMD, with 16 registers of kept rows per lane,
// repeat less per-wave work per column than sixteen; four lengthen the scan
// and the register loops more than they save.
constexpr int PANEL_WAVES = 8;

// SR: rows of the all-rows search kept in LDS.  The look-ahead panel runs
// beside the update kernels on their CUs, so it uses SR = 0 (workspace) and
// a raised wave priority.  NW > 1: a block of NW waves, all of which run the
// slow search (staged in the LDS rows).
template <int WQ, int SR, int NW = 1>
__global__ __launch_bounds__(64 * NW) void k_panel(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t c,
                                                   const PassRec *prev, PassRec *rec, int64_t *P, int64_t *Q,
                                                   int64_t *rank_out, uint64_t *gsv, int32_t *gsid, PanelFix fix) {
    __shared__ PanelLdsT<SR> L;
    if (SR == 0) __builtin_amdgcn_s_setprio(3);
    if constexpr (NW > 1) {
        static_assert(SR >= MW_SLOTS, "the staging holds every slot");
        __shared__ MwX<NW> X;
        MwCtx mc;
        mc.x = &X;
        mc.stv = L.sv;
        mc.stp = L.spos;
        mc.cap = SR;
        mc.hv = L.sv;
        mc.hp = L.spos;
        mc.hi = L.sid;
        panel_body<WQ, SR, true, NW>(A, m, n, ldw, c, prev, rec, P, Q, rank_out, gsv, gsid, L, threadIdx.x & 63, fix,
                                     uni(threadIdx.x >> 6), mc);
    } else {
        panel_body<WQ, SR>(A, m, n, ldw, c, prev, rec, P, Q, rank_out, gsv, gsid, L, threadIdx.x, fix);
    }
}

// ---------------------------------------------------------------------------
// k_permute: swaps, pivot staging, coefficients, L bits.
//   blocks [0, nA): PERM_A_COLS word columns each, every special row (read all, then
//                   write all, so the permutation is applied in place);
//   blocks [nA, ..): grid-stride over the other rows.
// MODE 0: serial pass loop.
// MODE 1: look-ahead.  The special rows' next stripe word (sw + 1) stays in
//         place: its new value goes to the record (spec_next, from the first
//         row block) for the next panel, which reads that column meanwhile;
//         the other rows' next stripe word gets the pass's update here
//         (tables of the pivots' old words at sw + 1).
// MODE 2: second pass u of a fused pair (t, u = t + 1): as MODE 1, and pass
//         t's update is still pending on every word right of sw for the rows
//         from r_t on: its coefficient words (coefT, by position before this
//         pass's swaps) are carried to the rows' new positions (coefP), and
//         the next stripe word gets both passes' updates (pass u's pivots'
//         words there first get pass t's).
// ---------------------------------------------------------------------------
// Word columns per special-row block: 16 (128-byte row pieces) spreads the
// special rows over four times as many blocks as 64 would, with two rows per
// thread instead of eight, which shortens the chain of dependent loads.
constexpr int PERM_A_COLS = 16;

template <int MODE>
__global__ __launch_bounds__(WIDE_THREADS) void k_permute(uint64_t *__restrict__ A, int64_t m, int64_t ldw, int64_t c,
                                                          PassRec *__restrict__ rec, uint64_t *__restrict__ coef,
                                                          uint64_t *__restrict__ PB, int nA, int64_t nw,
                                                          const PassRec *__restrict__ rect,
                                                          const uint64_t *__restrict__ coefT,
                                                          uint64_t *__restrict__ coefP,
                                                          const uint64_t *__restrict__ PBt, int64_t wlo) {
    __shared__ uint64_t tw[16][16], tu[16][16], tn[16][16], tt[MODE == 2 ? 16 : 1][16];
    __shared__ uint64_t simg_w[KW], simg_u[KW], simg_n[KW], spbt[KW];
    __shared__ int64_t sp_dst[MAX_SPEC], sp_src[MAX_SPEC], smaxdisp;
    __shared__ uint64_t sp_coef[MAX_SPEC];
    constexpr bool LA = MODE >= 1;

    const int tid = threadIdx.x;
    const int64_t sw = c >> 6;
    const bool nxt = LA && sw + 1 < nw;
    // A row block's first rows are read before the record's header is in,
    // at the rows they take when every pass so far had full rank (the first
    // row is then the stripe's column); they are read again if not.
    const int64_t gfirst = (MODE == 2 ? c - KW : c) + ((int64_t)blockIdx.x - nA) * WIDE_THREADS + tid;
    uint64_t g_sw = 0, g_nx = 0, g_ct = 0;
    if ((int)blockIdx.x >= nA && gfirst < m) {
        const uint64_t *row = A + gfirst * ldw;
        g_sw = row[sw];
        if (nxt) g_nx = row[sw + 1];
        if (MODE == 2) g_ct = coefT[gfirst];
    }
    // the row blocks read the record's special-row entries beside its header
    // (every entry exists), so the loads that take a special row's position
    // wait for one round trip, not two
    int64_t s_src = 0, s_dst = 0;
    uint64_t s_coef = 0;
    if ((int)blockIdx.x >= nA && tid < MAX_SPEC) {
        s_src = rec->spec_src[tid];
        s_dst = rec->spec_dst[tid];
        s_coef = rec->spec_coef[tid];
    }
    // the record's header (r < 0 never holds: the test keeps the load of r
    // ahead of the branch, beside the others)
    const int64_t r = rec->r;
    const int rbar_rec = rec->rbar, nspec_rec = rec->nspec;
    const int active = rec->active;
    if (MODE != 2 && (!active || r < 0)) return;
    const int rbar = active ? rbar_rec : 0;
    const int nspec = active ? nspec_rec : 0;
    const int64_t wr0 = r >> 6;
    const int sh = (int)(r & 63);

    if ((int)blockIdx.x < nA) {
        constexpr int SLOTS = WIDE_THREADS / PERM_A_COLS;  // 64
        constexpr int PER = MAX_SPEC / SLOTS;              // 2
        // the whole row moves: words [wlo, wlo + ldw) relative to A (wlo < 0
        // when A points into a row, at a right-hand block of the matrix)
        const int64_t w = wlo + (int64_t)blockIdx.x * PERM_A_COLS + (tid % PERM_A_COLS);
        const int64_t wend = wlo + ldw;
        const int slot = tid / PERM_A_COLS;
        uint64_t nv[PER];
        int64_t srcs[PER];
#pragma unroll
        for (int t = 0; t < PER; t++) srcs[t] = rec->spec_src[slot + SLOTS * t];  // (every entry exists)
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int k = slot + SLOTS * t;
            nv[t] = 0;
            if (k < nspec && w < wend && !(LA && w == sw + 1)) {
                const uint64_t old = A[srcs[t] * ldw + w];
                if (k < rbar && w > sw) PB[(int64_t)k * ldw + w] = old;
                nv[t] = special_word(old, w, sw, wr0, sh, rec->spec_lbits[k], rec->spec_stripe[k]);
            }
        }
        __syncthreads();  // every read of these columns precedes every write
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int k = slot + SLOTS * t;
            if (k < nspec && w < wend && !(LA && w == sw + 1)) {
                const int64_t src = rec->spec_src[k], dst = rec->spec_dst[k];
                if (dst != src || (w >= wr0 && w <= sw)) A[dst * ldw + w] = nv[t];
            }
        }
        return;
    }

    // ---- other rows ----
    // Every global read that does not depend on another is issued first (this
    // thread's first row, the pass maps, the pivots' next-stripe words), so
    // the launch costs about one memory round trip before the table builds.
    const int ndisp = nspec - rbar;
    const int rt = (MODE == 2 && rect->active) ? rect->rbar : 0;
    const int64_t nB = (int64_t)gridDim.x - nA;
    const int64_t row0 = MODE == 2 ? rect->r : r;
    const int64_t istep = nB * WIDE_THREADS;
    const int64_t ifirst = row0 + ((int64_t)blockIdx.x - nA) * WIDE_THREADS + tid;
    // first row: special rows read here are rewritten by group A meanwhile,
    // but their values are not used (the loop skips them)
    uint64_t f_sw = g_sw, f_nx = g_nx, f_ct = g_ct;
    if (ifirst != gfirst && ifirst < m) {
        const uint64_t *row = A + ifirst * ldw;
        f_sw = row[sw];
        if (nxt) f_nx = row[sw + 1];
        if (MODE == 2) f_ct = coefT[ifirst];
    }
    uint64_t pn = 0, pct = 0;  // pivot tid's next-stripe word and (MODE 2) pass t coefficient
    // the first row block also finishes the special rows' next-stripe words
    const bool spec_blk = nxt && (int)blockIdx.x == nA;
    uint64_t so = 0, sct = 0, scf = 0;  // special row tid: old next-stripe word, pass t and own coefficients
    if (spec_blk && tid < nspec) {
        so = A[s_src * ldw + sw + 1];
        if (MODE == 2) sct = coefT[s_src];
        scf = s_coef;
    }
    if (tid < MAX_SPEC) {
        sp_dst[tid] = s_dst;
        sp_src[tid] = s_src;
        sp_coef[tid] = s_coef;
    }
    if (tid < KW) {
        simg_w[tid] = active ? rec->img_w[tid] : 0ull;
        simg_u[tid] = active ? rec->img_u[tid] : 0ull;
        if (MODE == 2) spbt[tid] = (nxt && tid < rt) ? PBt[(int64_t)tid * ldw + sw + 1] : 0ull;
        // group A leaves the next stripe word of the special rows alone, so
        // these are the pivots' words there as they stand at the pass start
        if (nxt && tid < rbar) {
            pn = A[s_src * ldw + sw + 1];
            if (MODE == 2) pct = coefT[s_src];
        }
    }
    // the pivots' next-stripe words as they stand (MODE 2 adds pass t's update
    // below, once its pivots' words are in LDS)
    if (MODE != 2 && nxt && tid < KW) simg_n[tid] = pn;
    __syncthreads();
    // the displaced rows are entries rbar .. nspec - 1: the largest position
    // they take (read after the tables' barrier)
    if (tid < 64) {
        int64_t dv = tid < ndisp ? sp_dst[rbar + tid] : -1;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int64_t ov = __shfl_xor(dv, o);
            dv = ov > dv ? ov : dv;
        }
        if (tid == 0) smaxdisp = dv;
    }
    if (MODE == 2 && nxt && tid < KW) {
        uint64_t v = pn;
        if (tid < rbar) {
            for (int b = 0; b < KW; b++)
                if ((pct >> b) & 1ull) v ^= spbt[b];
        }
        simg_n[tid] = v;
    }
    // nibble tables, 256 threads each: the maps w and u, and pass t's update
    // of the next stripe word (MODE 2) or this pass's (the others)
    static_assert(WIDE_THREADS == 4 * 256, "four groups of 256 threads build the tables");
    const int tb = (tid & 255) >> 4, tx = tid & 15;
    auto build = [&](const uint64_t *img) {
        uint64_t a = 0;
#pragma unroll
        for (int t = 0; t < 4; t++)
            if ((tx >> t) & 1) a ^= img[4 * tb + t];
        return a;
    };
    if (tid < 256) tw[tb][tx] = build(simg_w);
    else if (tid < 512) tu[tb][tx] = build(simg_u);
    else if (tid < 768) {
        if (MODE == 2) tt[tb][tx] = build(spbt);
    } else if (MODE != 2 && nxt) {
        tn[tb][tx] = build(simg_n);
    }
    __syncthreads();
    const int64_t maxdisp = smaxdisp;
    if (MODE == 2) {
        if (nxt && tid < 256) tn[tb][tx] = build(simg_n);
        __syncthreads();
    }
    if (spec_blk && tid < nspec) {
        // old word, then (MODE 2) pass t's update, then this pass's: the
        // pivots' words in tn already carry pass t's update
        uint64_t v = so;
        if (MODE == 2) {
#pragma unroll
            for (int b = 0; b < 16; b++) v ^= tt[b][(sct >> (4 * b)) & 15];
        }
#pragma unroll
        for (int b = 0; b < 16; b++) v ^= tn[b][(scf >> (4 * b)) & 15];
        rec->spec_next[tid] = v;
    }
    for (int64_t i = ifirst; i < m; i += istep) {
        uint64_t *row = A + i * ldw;
        const bool first = i == ifirst;
        uint64_t ct = 0;
        if (MODE == 2) {
            ct = first ? f_ct : coefT[i];
            if (i < r) {  // pass t's pivot rows: only its update (the TRSM) is pending
                coefP[i] = ct;
                coef[i] = 0;
                if (nxt && ct) {
                    uint64_t acc = 0;
#pragma unroll
                    for (int b = 0; b < 16; b++) acc ^= tt[b][(ct >> (4 * b)) & 15];
                    row[sw + 1] = (first ? f_nx : row[sw + 1]) ^ acc;
                }
                continue;
            }
        }
        if (i < r + rbar) {
            coef[i] = sp_coef[i - r];
            if (MODE == 2) coefP[i] = coefT[sp_src[i - r]];
            continue;
        }
        if (i <= maxdisp) {
            // no early exit, so the compares' LDS reads can all be in flight
            int hit = -1;
            for (int d = 0; d < ndisp; d++) hit = sp_dst[rbar + d] == i ? rbar + d : hit;
            if (hit >= 0) {
                coef[i] = sp_coef[hit];
                if (MODE == 2) coefP[i] = coefT[sp_src[hit]];
                continue;
            }
        }
        if (MODE == 2) coefP[i] = ct;
        const uint64_t v = first ? f_sw : row[sw];
        uint64_t wv = 0;
        if (v) {
            uint64_t u = 0;
#pragma unroll
            for (int b = 0; b < 16; b++) {
                const int x = (int)((v >> (4 * b)) & 15);
                wv ^= tw[b][x];
                u ^= tu[b][x];
            }
            if (wr0 < sw) {
                row[wr0] |= u << sh;
                if (sh && wr0 + 1 < sw) row[wr0 + 1] |= u >> (64 - sh);
            }
            row[sw] = place_bits(u, sw, wr0, sh);
        }
        coef[i] = wv;
        if (nxt && (wv || ct)) {
            uint64_t acc = 0;
#pragma unroll
            for (int b = 0; b < 16; b++) acc ^= tn[b][(wv >> (4 * b)) & 15];
            if (MODE == 2) {
#pragma unroll
                for (int b = 0; b < 16; b++) acc ^= tt[b][(ct >> (4 * b)) & 15];
            }
            row[sw + 1] = (first ? f_nx : row[sw + 1]) ^ acc;
        }
    }
}

// ---------------------------------------------------------------------------
// k_m4rm / k_m4rm_w: the trailing update (m4rm.h).  With `rec` the rows are
// rec->r .. m-1 and B has rec->rbar rows; without it, rows 0 .. m-1 and
// `nbits` rows.  Column tiles are aligned to absolute multiples of the tile
// width (the first may be partial).  Block -> (tile, row chunk) with tiles
// fastest, so the blocks running at one time sweep whole rows together.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool m4_block_rows(int64_t m, int64_t row0, int ntiles, int nchunks, int *tile,
                                              int64_t *rb, int64_t *re) {
    const int logical = xcd_logical(blockIdx.x, gridDim.x);
    *tile = logical % ntiles;
    const int chunk = logical / ntiles;
    if (chunk >= nchunks) return false;
    const int64_t rows = m - row0;
    const int64_t per = (rows + nchunks - 1) / nchunks;
    *rb = row0 + (int64_t)chunk * per;
    *re = *rb + per < m ? *rb + per : m;
    return *rb < *re;
}

template <int TW, int NT, int U>
__global__ __launch_bounds__(NT) void k_m4rm(uint64_t *__restrict__ C, int64_t ldc, int64_t m,
                                             const uint64_t *__restrict__ coef, int64_t coef_ld,
                                             const uint64_t *__restrict__ B, int64_t ldb, int nbits, int64_t w_begin,
                                             int64_t w_end, int ntiles, int nchunks, const PassRec *__restrict__ rec) {
    __shared__ M4Lds<TW> L;
    int64_t row0 = 0;
    if (rec) {
        if (!rec->active) return;
        row0 = rec->r;
        nbits = rec->rbar;
    }
    int tile;
    int64_t rb, re;
    if (!m4_block_rows(m, row0, ntiles, nchunks, &tile, &rb, &re)) return;
    const int64_t wt0 = (w_begin & ~(int64_t)(TW - 1)) + (int64_t)tile * TW;
    m4_build_tables<TW, NT>(L, B, ldb, nbits, wt0, w_begin, w_end, threadIdx.x);
    m4_rows<TW, NT, U>(L, C, ldc, coef, coef_ld, nbits, rb, re, wt0, w_begin, w_end, threadIdx.x);
}

template <int NT, int U>
__global__ __launch_bounds__(NT) void k_m4rm_w(uint64_t *__restrict__ C, int64_t ldc, int64_t m,
                                               const uint64_t *__restrict__ coef, int64_t coef_ld,
                                               const uint64_t *__restrict__ B, int64_t ldb, int nbits, int64_t w_begin,
                                               int64_t w_end, int ntiles, int nchunks, const PassRec *__restrict__ rec) {
    __shared__ uint64_t T[16 * 16 * WR_TW];
    int64_t row0 = 0;
    if (rec) {
        if (!rec->active) return;
        row0 = rec->r;
        nbits = rec->rbar;
    }
    int tile;
    int64_t rb, re;
    if (!m4_block_rows(m, row0, ntiles, nchunks, &tile, &rb, &re)) return;
    const int64_t wt0 = (w_begin & ~(int64_t)(WR_TW - 1)) + (int64_t)tile * WR_TW;
    m4w_build_tables<NT>(T, B, ldb, nbits, wt0, w_begin, w_end, threadIdx.x);
    m4w_rows<NT, U>(T, C, ldc, coef, coef_ld, nbits, rb, re, wt0, w_begin, w_end, threadIdx.x);
}

// ---------------------------------------------------------------------------
// k_m4rm_pair: the updates of a fused pair of passes (t, u = t + 1) in one
// sweep over rows r_t .. m-1 and words [w_begin, w_end):
//   C[i][w] ^= T_t[coefP[i]][w] ^ T_u[coefU[i]][w],
// T_t the sixteen 4-bit tables of pass t's staged pivot rows (PBt), T_u
// those of pass u's (PBu, staged before pass t's update reached them, so
// they first get it: coefficient coefT[src] of their position then).
// Tiles of 32 words; 16 lanes per row, two words per lane, 128-bit table
// reads; 128 KB of tables per block.
//
// The panel of pass t + 2 runs inside the same launch: its stripe word lies
// left of the words this sweep writes, so the two are independent, and no
// event between two streams is needed to order them.  It runs either on the
// last wave of block 0 (raised priority), once the block's tables are built,
// that block's row chunk shortened to the share its other waves can do in
// the time the other blocks take, or (pp.share < 0) in a block of its own.
// ---------------------------------------------------------------------------
constexpr int PR_TW = 32;
// kept rows of the slow search of the panel inside the pair update that fit
// in the LDS beside the 128 KB of tables
constexpr int PAIR_PANEL_ROWS = 1536;
// sweeps estimated shorter than this (us) give the panel a block of its own
constexpr double PAIR_OWN_PANEL_US = 30.0;

template <int BASE, int NT>
__device__ __forceinline__ void pair_combos(uint64_t (*T)[16][PR_TW], int tid) {
    for (int e = tid; e < 16 * 16 * PR_TW; e += NT) {
        const int wl = e % PR_TW;
        const int x = (e / PR_TW) & 15;
        const int q = e / (PR_TW * 16);
        if (__popc(x) < 2) continue;
        uint64_t acc = 0;
#pragma unroll
        for (int b = 0; b < 4; b++)
            if ((x >> b) & 1) acc ^= T[BASE + q][1 << b][wl];
        T[BASE + q][x][wl] = acc;
    }
}

// Rows of block `logical`: tile = logical % ntiles, chunk = logical / ntiles.
// With `short0`, chunk 0 of tile 0 (the block that also runs the panel) gets
// share / 65536 of an even chunk and the tile's other chunks split the rest.
__device__ __forceinline__ bool pair_block_rows(int64_t m, int64_t row0, int ntiles, int nchunks, int logical,
                                                bool short0, int share, int *tile, int64_t *rb, int64_t *re) {
    *tile = logical % ntiles;
    const int chunk = logical / ntiles;
    if (chunk >= nchunks) return false;
    const int64_t rows = m - row0;
    if (short0 && *tile == 0 && nchunks > 1) {
        const int64_t a = rows * share / (65536 * (int64_t)nchunks);
        if (chunk == 0) {
            *rb = row0;
            *re = row0 + a;
        } else {
            const int64_t per = (rows - a + nchunks - 2) / (nchunks - 1);
            *rb = row0 + a + (int64_t)(chunk - 1) * per;
            *re = *rb + per < m ? *rb + per : m;
        }
    } else {
        const int64_t per = (rows + nchunks - 1) / nchunks;
        *rb = row0 + (int64_t)chunk * per;
        *re = *rb + per < m ? *rb + per : m;
    }
    return *rb < *re;
}

template <int NT, int U, int G, bool PF, bool RP = false>
__global__ __launch_bounds__(NT) void k_m4rm_pair(uint64_t *__restrict__ C, int64_t ldc, int64_t m,
                                                  const uint64_t *__restrict__ coefP,
                                                  const uint64_t *__restrict__ coefU,
                                                  const uint64_t *__restrict__ coefT,
                                                  const uint64_t *__restrict__ PBt, const uint64_t *__restrict__ PBu,
                                                  int64_t ldb, int64_t w_begin, int64_t w_end, int ntiles, int nchunks,
                                                  const PassRec *__restrict__ rect, const PassRec *__restrict__ recu,
                                                  PairPanel pp) {
    __shared__ __align__(16) uint64_t T[32][16][PR_TW];
    __shared__ PanelLdsT<PAIR_PANEL_ROWS> PL;
    const int tid = threadIdx.x;
    // share < 0: the panel has a block of its own (logical block 0, one
    // extra block in the grid), and the sweep's blocks are the rest
    const bool own = pp.on && pp.share < 0;
    const int logical = xcd_logical(blockIdx.x, gridDim.x) - (own ? 1 : 0);
    const bool panel_here = pp.on && logical == (own ? -1 : 0);
    // pass t + 2's panel: the pair's special rows' words in its stripe come
    // from the second pass's record
    auto run_panel = [&]() {
        __builtin_amdgcn_s_setprio(3);
        PanelFix f;
        f.mode = 1;
        panel_body<2, PAIR_PANEL_ROWS>(C, m, pp.n, ldc, pp.c, recu, pp.rec, pp.P, pp.Q, pp.rank, pp.gsv, pp.gsid, PL, tid & 63, f);
    };
    if (own && panel_here) {
        // a block of its own: every wave joins the slow search, which stages
        // its kept rows where the tables would be
        static_assert(MW_SLOTS * 12 + sizeof(MwX<NT / 64>) <= sizeof(T), "staging in the tables' LDS");
        __builtin_amdgcn_s_setprio(3);
        PanelFix f;
        f.mode = 1;
        MwCtx mc;
        uint64_t *tb = &T[0][0][0];
        mc.stv = tb;
        mc.stp = (int32_t *)(tb + MW_SLOTS);
        mc.x = (void *)(tb + MW_SLOTS + MW_SLOTS / 2);
        mc.cap = MW_SLOTS;
        mc.hv = PL.sv;
        mc.hp = PL.spos;
        mc.hi = PL.sid;
        panel_body<2, PAIR_PANEL_ROWS, true, NT / 64, true>(C, m, pp.n, ldc, pp.c, recu, pp.rec, pp.P, pp.Q, pp.rank,
                                                     pp.gsv, pp.gsid, PL, tid & 63, f, uni(tid >> 6), mc);
        return;
    }
    const int at = rect->active, au = recu->active;
    const int nbt = at ? rect->rbar : 0, nbu = au ? recu->rbar : 0;
    int tile = 0;
    int64_t rb = 0, re = 0;
    const bool rows_here =
        (at || au) && pair_block_rows(m, rect->r, ntiles, nchunks, logical, pp.on && !own, pp.share, &tile, &rb, &re);
    if (!rows_here) {
        if (panel_here && tid < 64) run_panel();
        return;
    }
    const int64_t wt0 = (w_begin & ~(int64_t)(PR_TW - 1)) + (int64_t)tile * PR_TW;
    // every global read of the table build first: pass u's staged pivot
    // words and their pass-t coefficients (two dependent loads) then travel
    // beside pass t's words and the first table build
    constexpr int IT = (KW * PR_TW + NT - 1) / NT;
    uint64_t pbu[IT], ctu[IT];
#pragma unroll
    for (int it = 0; it < IT; it++) {
        const int e = tid + it * NT;
        const int k = e / PR_TW;
        const int64_t w = wt0 + e % PR_TW;
        const bool on = e < KW * PR_TW && k < nbu && w >= w_begin && w < w_end;
        pbu[it] = on ? PBu[(int64_t)k * ldb + w] : 0ull;
        ctu[it] = on && nbt ? coefT[recu->spec_src[k]] : 0ull;
    }
    for (int e = tid; e < KW * PR_TW; e += NT) {
        const int k = e / PR_TW, wl = e % PR_TW;
        const int64_t w = wt0 + wl;
        const int q = k >> 2, b = k & 3;
        T[q][1 << b][wl] = (k < nbt && w >= w_begin && w < w_end) ? PBt[(int64_t)k * ldb + w] : 0ull;
        if (b == 0) T[q][0][wl] = 0ull;
    }
    __syncthreads();
    pair_combos<0, NT>(T, tid);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; it++) {
        const int e = tid + it * NT;
        if (e >= KW * PR_TW) break;
        const int k = e / PR_TW, wl = e % PR_TW;
        const int q = k >> 2, b = k & 3;
        uint64_t v = pbu[it];
        const uint64_t ct = ctu[it];
#pragma unroll
        for (int qq = 0; qq < 16; qq++) v ^= T[qq][(ct >> (4 * qq)) & 15][wl];
        T[16 + q][1 << b][wl] = v;
        if (b == 0) T[16 + q][0][wl] = 0ull;
    }
    __syncthreads();
    pair_combos<16, NT>(T, tid);
    __syncthreads();
    if (panel_here && tid >= NT - 64) {
        run_panel();
        return;
    }

    // rows: every table is read (those past a pass's pivots are zero), so the
    // 32 reads of a row carry no branch and can all be in flight at once
    constexpr int LPR = PR_TW / 2;                       // lanes per row
    const int RS = (panel_here ? NT - 64 : NT) / LPR;  // rows per step
    const int wp = tid % LPR, rs = tid / LPR;
    const int64_t w2 = wt0 + 2 * wp;
    const bool ok0 = w2 >= w_begin && w2 < w_end, ok1 = w2 + 1 >= w_begin && w2 + 1 < w_end;
    const uint32_t tbase = (uint32_t)(2 * wp) * 8u;  // byte offset of this lane's pair of words
    // a lane's two words are 16-byte aligned when the row stride is even
    // (tiles start at even words): then they move as one 16-byte access
    const bool wide = (ldc & 1) == 0 && ((uintptr_t)C & 15) == 0;
    // a row's words: one 16-byte access when aligned, else two
    auto load_row = [&](const int64_t i, const bool on, uint64_t &v0, uint64_t &v1) {
        if (wide && on && ok0 && ok1) {
            const ulonglong2 v = *(const ulonglong2 *)(C + i * ldc + w2);
            v0 = v.x;
            v1 = v.y;
        } else {
            v0 = (on && ok0) ? C[i * ldc + w2] : 0ull;
            v1 = (on && ok1) ? C[i * ldc + w2 + 1] : 0ull;
        }
    };
    if constexpr (RP) {
        // two steps in flight: the next step's coefficient words and row
        // words load while this step's tables are read
        static_assert(U == 1, "row prefetch keeps one row per step");
        int64_t i = rb + rs;
        uint64_t ncp1 = i < re ? coefP[i] : 0ull, ncu1 = i < re ? coefU[i] : 0ull, nx0 = 0, nx1 = 0;
        load_row(i, i < re, nx0, nx1);
        for (; i < re; i += RS) {
            const uint64_t cp = ncp1, cu = ncu1, x0 = nx0, x1 = nx1;
            const int64_t in = i + RS;
            ncp1 = in < re ? coefP[in] : 0ull;
            ncu1 = in < re ? coefU[in] : 0ull;
            load_row(in, in < re, nx0, nx1);
            const uint32_t h[4] = {(uint32_t)cp, (uint32_t)(cp >> 32), (uint32_t)cu, (uint32_t)(cu >> 32)};
            uint64_t a0 = 0, a1 = 0;
#pragma unroll
            for (int g = 0; g < 32; g += G) {
                ulonglong2 t[G];
#pragma unroll
                for (int j = 0; j < G; j++) {
                    const int q = g + j;
                    const uint32_t nib = (h[q >> 3] >> (4 * (q & 7))) & 15u;
                    t[j] = *(const ulonglong2 *)((const char *)&T[0][0][0] + tbase +
                                                 ((uint32_t)q * 16u + nib) * (uint32_t)(PR_TW * 8));
                }
                if constexpr (G % 2 == 0) {
#pragma unroll
                    for (int j = 0; j < G; j += 2) {
                        a0 = xor3_64(a0, t[j].x, t[j + 1].x);
                        a1 = xor3_64(a1, t[j].y, t[j + 1].y);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < G; j++) {
                        a0 ^= t[j].x;
                        a1 ^= t[j].y;
                    }
                }
                // materialise the partial sums here: otherwise the xor chain is
                // reassociated into one tree that keeps all 32 reads live
                __asm__ volatile("" : "+v"(a0), "+v"(a1));
            }
            if (cp | cu) {
                if (wide && ok0 && ok1) {
                    ulonglong2 v;
                    v.x = x0 ^ a0;
                    v.y = x1 ^ a1;
                    *(ulonglong2 *)(C + i * ldc + w2) = v;
                } else {
                    if (ok0) C[i * ldc + w2] = x0 ^ a0;
                    if (ok1) C[i * ldc + w2 + 1] = x1 ^ a1;
                }
            }
        }
        return;
    }
    // PF: the next step's coefficient words are loaded during this step's
    // lookups, so a step starts with its row loads and lookups at once
    uint64_t ncp[U], ncu[U];
    if constexpr (PF) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = rb + rs + (int64_t)u * RS;
            ncp[u] = i < re ? coefP[i] : 0ull;
            ncu[u] = i < re ? coefU[i] : 0ull;
        }
    }
    for (int64_t i0 = rb + rs; i0 < re; i0 += (int64_t)RS * U) {
        uint64_t cp[U], cu[U], x0[U], x1[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = i0 + (int64_t)u * RS;
            if constexpr (PF) {
                cp[u] = ncp[u];
                cu[u] = ncu[u];
            } else {
                cp[u] = i < re ? coefP[i] : 0ull;
                cu[u] = i < re ? coefU[i] : 0ull;
            }
            const bool any = i < re && (cp[u] | cu[u]);
            if (wide && any && ok0 && ok1) {
                // one 16-byte load: the row's 16 lanes read 256 contiguous bytes
                const ulonglong2 v = *(const ulonglong2 *)(C + i * ldc + w2);
                x0[u] = v.x;
                x1[u] = v.y;
            } else {
                x0[u] = (any && ok0) ? C[i * ldc + w2] : 0ull;
                x1[u] = (any && ok1) ? C[i * ldc + w2 + 1] : 0ull;
            }
        }
        if constexpr (PF) {
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int64_t i = i0 + (int64_t)(U + u) * RS;
                ncp[u] = i < re ? coefP[i] : 0ull;
                ncu[u] = i < re ? coefU[i] : 0ull;
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = i0 + (int64_t)u * RS;
            // coefficient halves: tables 0-7, 8-15 (pass t), 16-23, 24-31 (pass u)
            const uint32_t h[4] = {(uint32_t)cp[u], (uint32_t)(cp[u] >> 32), (uint32_t)cu[u],
                                   (uint32_t)(cu[u] >> 32)};
            uint64_t a0 = 0, a1 = 0;
#pragma unroll
            for (int g = 0; g < 32; g += G) {
                ulonglong2 t[G];
#pragma unroll
                for (int j = 0; j < G; j++) {
                    const int q = g + j;
                    const uint32_t nib = (h[q >> 3] >> (4 * (q & 7))) & 15u;
                    t[j] = *(const ulonglong2 *)((const char *)&T[0][0][0] + tbase +
                                                 ((uint32_t)q * 16u + nib) * (uint32_t)(PR_TW * 8));
                }
                if constexpr (G % 2 == 0) {
#pragma unroll
                    for (int j = 0; j < G; j += 2) {
                        a0 = xor3_64(a0, t[j].x, t[j + 1].x);
                        a1 = xor3_64(a1, t[j].y, t[j + 1].y);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < G; j++) {
                        a0 ^= t[j].x;
                        a1 ^= t[j].y;
                    }
                }
                // materialise the partial sums here: otherwise the xor chain is
                // reassociated into one tree that keeps all 32 reads live
                __asm__ volatile("" : "+v"(a0), "+v"(a1));
            }
            if (i < re && (cp[u] | cu[u])) {
                if (wide && ok0 && ok1) {
                    ulonglong2 v;
                    v.x = x0[u] ^ a0;
                    v.y = x1[u] ^ a1;
                    *(ulonglong2 *)(C + i * ldc + w2) = v;
                } else {
                    if (ok0) C[i * ldc + w2] = x0[u] ^ a0;
                    if (ok1) C[i * ldc + w2 + 1] = x1[u] ^ a1;
                }
            }
        }
    }
}

// Schedules of the update kernel (index = M4Variant id).
struct M4Variant {
    int tw, nt, u;
    const char *name;
};
constexpr int M4_NVARIANTS = 12;
static const M4Variant kM4Variants[M4_NVARIANTS] = {
    {8, 1024, 4, "tw8_nt1024_u4"},   {8, 1024, 2, "tw8_nt1024_u2"},   {8, 512, 8, "tw8_nt512_u8"},
    {8, 512, 4, "tw8_nt512_u4"},     {4, 512, 8, "tw4_nt512_u8"},     {4, 256, 16, "tw4_nt256_u16"},
    {4, 1024, 4, "tw4_nt1024_u4"},   {8, 256, 16, "tw8_nt256_u16"},   {64, 1024, 4, "row_nt1024_u4"},
    {64, 1024, 8, "row_nt1024_u8"},  {64, 512, 8, "row_nt512_u8"},    {64, 512, 16, "row_nt512_u16"},
};

// Default schedule of one update launch, from sweeps on MI355X: the
// wave-per-row kernel (512-byte row segments) when the trailing block does
// not fit the 256 MB Infinity Cache, the 8-word tiles otherwise.
static int m4_auto(int64_t rows, int64_t words) {
    const double bytes = (double)rows * (double)words * 8.0;
    if (words >= 48 && bytes > 192.0 * 1024 * 1024) return 9;
    return 0;
}

static void m4_launch_variant(int v, dim3 grid, hipStream_t s, uint64_t *C, int64_t ldc, int64_t m, const uint64_t *coef,
                              int64_t coef_ld, const uint64_t *B, int64_t ldb, int nbits, int64_t w_begin,
                              int64_t w_end, int ntiles, int nchunks, const PassRec *rec) {
#define M4_CASE(ID, TW, NT, U)                                                                                       \
    case ID:                                                                                                          \
        hipLaunchKernelGGL((k_m4rm<TW, NT, U>), grid, dim3(NT), 0, s, C, ldc, m, coef, coef_ld, B, ldb, nbits,      \
                           w_begin, w_end, ntiles, nchunks, rec);                                                     \
        break;
    switch (v) {
        M4_CASE(0, 8, 1024, 4)
        M4_CASE(1, 8, 1024, 2)
        M4_CASE(2, 8, 512, 8)
        M4_CASE(3, 8, 512, 4)
        M4_CASE(4, 4, 512, 8)
        M4_CASE(5, 4, 256, 16)
        M4_CASE(6, 4, 1024, 4)
        M4_CASE(7, 8, 256, 16)
#define M4W_CASE(ID, NT, U)                                                                                         \
    case ID:                                                                                                          \
        hipLaunchKernelGGL((k_m4rm_w<NT, U>), grid, dim3(NT), 0, s, C, ldc, m, coef, coef_ld, B, ldb, nbits, w_begin,  \
                           w_end, ntiles, nchunks, rec);                                                              \
        break;
        M4W_CASE(8, 1024, 4)
        M4W_CASE(9, 1024, 8)
        M4W_CASE(10, 512, 8)
        M4W_CASE(11, 512, 16)
#undef M4W_CASE
        default:
            break;
    }
#undef M4_CASE
}

// Grid of one update launch over words [w_begin, w_end): ntiles aligned
// column tiles x nchunks row chunks.  The chunk count is chosen so that the
// blocks fill whole rounds of the device's block slots (one block with
// 128 KB of tables per CU, two with 64 KB): e.g. 15 tiles x 17 chunks = 255
// blocks on 256 CUs rather than 270 blocks that need a second round.
// `target` > 0 asks for about that many blocks instead.
static int g_cus = 0;
static int device_cus() {
    if (g_cus <= 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            g_cus = cus;
        else
            g_cus = 256;
    }
    return g_cus;
}

int device_cu_count() { return device_cus(); }

static void m4_grid(int v, int64_t rows_est, int64_t w_begin, int64_t w_end, int target, int *ntiles, int *nchunks) {
    const int tw = kM4Variants[v].tw;
    const int64_t base = w_begin & ~(int64_t)(tw - 1);
    const int nt = (int)((w_end - base + tw - 1) / tw);
    *ntiles = nt;
    int64_t maxc = rows_est / 128;  // at least 128 rows per chunk
    if (maxc < 1) maxc = 1;
    if (target > 0) {
        int64_t nc = (target + nt - 1) / nt;
        *nchunks = (int)(nc < 1 ? 1 : (nc > maxc ? maxc : nc));
        return;
    }
    const int64_t slots = (int64_t)device_cus() * (tw == 4 ? 2 : 1);
    if (maxc > 4 * slots) maxc = 4 * slots;
    int best = 1;
    double best_eff = -1.0;
    for (int64_t nc = 1; nc <= maxc; nc++) {
        const int64_t g = nt * nc;
        const int64_t rounds = (g + slots - 1) / slots;
        // filled share of the rounds, discounted slightly per extra round
        const double eff = (double)g / (double)(rounds * slots) - 0.02 * (double)(rounds - 1);
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best = (int)nc;
        }
    }
    *nchunks = best;
}

static int m4_pick(int variant, int64_t rows, int64_t words) {
    return (variant > 0 && variant <= M4_NVARIANTS) ? variant - 1 : m4_auto(rows, words);
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
    ProfScope ps(KID_INIT, s);
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(256), 0, s, P, m, Q, mn, rank, rec);
    return hipGetLastError();
}

// fix: what the previous pass(es) left in this stripe word; beside: the
// panel runs on a second stream beside an update kernel (no LDS window,
// raised wave priority).
// done: if given, recorded when the kernel completes (carried by the
// kernel's own completion signal rather than a separate marker)
hipError_t launch_panel(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t c, const PassRec *prev, PassRec *rec,
                        int64_t *P, int64_t *Q, int64_t *rank, uint64_t *gsv, int32_t *gsid, int panel_regs,
                        const PanelFix &fix, bool beside, hipStream_t s, hipEvent_t done) {
    ProfScope ps(KID_PANEL, s);
#define PANEL_LAUNCH(WQ, SR)                                                                                      \
    hipExtLaunchKernelGGL((k_panel<WQ, SR>), dim3(1), dim3(64), 0, s, nullptr, done, 0, A, m, n, ldw, c, prev, rec, P, \
                          Q, rank, gsv, gsid, fix)
    if (panel_regs == 0 || panel_regs == 2) {
        // the default panel: a block of PANEL_WAVES waves for the slow search
        if (beside) PANEL_LAUNCH(2, 0);
        else
            hipExtLaunchKernelGGL((k_panel<2, SLOW_LDS_ROWS, PANEL_WAVES>), dim3(1), dim3(64 * PANEL_WAVES), 0, s,
                                  nullptr, done, 0, A, m, n, ldw, c, prev, rec, P, Q, rank, gsv, gsid, fix);
    } else if (panel_regs == 4) {
        if (beside) PANEL_LAUNCH(4, 0);
        else PANEL_LAUNCH(4, SLOW_LDS_ROWS);
    } else {
        if (beside) PANEL_LAUNCH(8, 0);
        else PANEL_LAUNCH(8, SLOW_LDS_ROWS);
    }
#undef PANEL_LAUNCH
    return hipGetLastError();
}

hipError_t launch_permute(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t c, PassRec *rec,
                          uint64_t *coef, uint64_t *PB, int mode, const PassRec *rect, const uint64_t *coefT,
                          uint64_t *coefP, const uint64_t *PBt, hipStream_t s, hipEvent_t done, int64_t wlo) {
    const int nA = (int)((ldw + PERM_A_COLS - 1) / PERM_A_COLS);
    int64_t rows_est = m - (c < m ? c : m);
    if (mode == 2) rows_est += KW;  // also the first pass's pivot rows
    if (rows_est < 1) rows_est = 1;
    int nB = (int)((rows_est + WIDE_THREADS - 1) / WIDE_THREADS);
    if (nB > 256) nB = 256;
    if (nB < 1) nB = 1;
    const int64_t nw = words_for(n);
    ProfScope ps(KID_PERMUTE, s);
#define PERMUTE_LAUNCH(MODE)                                                                                    \
    hipExtLaunchKernelGGL(k_permute<MODE>, dim3(nA + nB), dim3(WIDE_THREADS), 0, s, nullptr, done, 0, A, m, ldw, c, \
                          rec, coef, PB, nA, nw, rect, coefT, coefP, PBt, wlo)
    if (mode == 0) PERMUTE_LAUNCH(0);
    else if (mode == 1) PERMUTE_LAUNCH(1);
    else PERMUTE_LAUNCH(2);
#undef PERMUTE_LAUNCH
    return hipGetLastError();
}

// Trailing update of one pass over words [sw + first, nw): first = 1 for the
// whole trailing block, 2 when the next stripe was updated on its own.
hipError_t launch_update(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t c, const PassRec *rec,
                         const uint64_t *coef, const uint64_t *PB, int first, int m4_variant, int m4_target,
                         hipStream_t s) {
    const int64_t nw = words_for(n);
    const int64_t tw0 = (c >> 6) + first;
    if (tw0 >= nw) return hipSuccess;
    int64_t rows_est = m - (c < m ? c : m);
    if (rows_est < 1) rows_est = 1;
    const int v = m4_pick(m4_variant, rows_est, nw - tw0);
    int ntiles, nchunks;
    m4_grid(v, rows_est, tw0, nw, m4_target, &ntiles, &nchunks);
    ProfScope ps(KID_M4RM, s);
    m4_launch_variant(v, dim3(ntiles * nchunks), s, A, ldw, m, coef, (int64_t)1, PB, ldw, KW, tw0, nw, ntiles, nchunks,
                      rec);
    return hipGetLastError();
}

// Fused update of a pair (t, u): words [sw_t + 3, nw) of rows r_t .. m-1,
// and with pp.on the panel of pass t + 2 (inside the same launch, or alone
// when no word is left to update).
// The fused two-block sweep of the back-substitution: rows [0, m) and words
// [w_begin, w_end) get two blocks' updates at once (the second block's rows
// first take the first's), on the pair kernel's default schedule.
hipError_t launch_rref_pair(uint64_t *A, int64_t ldw, int64_t m, const uint64_t *coefT, const uint64_t *coefU,
                            const uint64_t *PBt, const uint64_t *PBu, int64_t w_begin, int64_t w_end,
                            const PassRec *rect, const PassRec *recu, hipStream_t s) {
    if (w_begin >= w_end || m <= 0) return hipSuccess;
    const int64_t base = w_begin & ~(int64_t)(PR_TW - 1);
    const int nt = (int)((w_end - base + PR_TW - 1) / PR_TW);
    const int64_t slots = device_cus();
    int64_t maxc = m / 256;
    if (maxc < 1) maxc = 1;
    if (maxc > 4 * slots) maxc = 4 * slots;
    int nchunks = 1;
    double best_eff = -1.0;
    for (int64_t nc = 1; nc <= maxc; nc++) {
        const int64_t g = nt * nc;
        const int64_t rounds = (g + slots - 1) / slots;
        const double eff = (double)g / (double)(rounds * slots) - 0.02 * (double)(rounds - 1);
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            nchunks = (int)nc;
        }
    }
    const PairPanel none;
    ProfScope ps(KID_M4RM, s);
    hipLaunchKernelGGL((k_m4rm_pair<1024, 1, 2, true, true>), dim3(nt * nchunks), dim3(1024), 0, s, A, ldw, m, coefT,
                       coefU, coefT, PBt, PBu, ldw, w_begin, w_end, nt, nchunks, rect, recu, none);
    return hipGetLastError();
}

hipError_t launch_update_pair(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t ct, const PassRec *rect,
                              const PassRec *recu, const uint64_t *coefP, const uint64_t *coefU,
                              const uint64_t *coefT, const uint64_t *PBt, const uint64_t *PBu, int m4_target,
                              int pair_variant, const PairPanel &pp, hipStream_t s) {
    const int64_t nw = words_for(n);
    const int64_t tw0 = (ct >> 6) + 3;
    if (tw0 >= nw) {
        if (!pp.on) return hipSuccess;
        PanelFix f;
        f.mode = 1;
        return launch_panel(A, m, n, ldw, pp.c, recu, pp.rec, pp.P, pp.Q, pp.rank, pp.gsv, pp.gsid, 2, f, false, s,
                            nullptr);
    }
    int64_t rows_est = m - (ct < m ? ct : m);
    if (rows_est < 1) rows_est = 1;
    const int64_t base = tw0 & ~(int64_t)(PR_TW - 1);
    const int nt = (int)((nw - base + PR_TW - 1) / PR_TW);
    // The next panel gets a block (a CU) of its own when the sweep is short:
    // the panel then starts at once, alone on its CU, instead of after block
    // 0's tables and beside its sweep (about 25 us there), which is most of
    // such a launch.  Variants 13 and 14 force the two forms.
    const double upd_us = (double)rows_est * (double)(nw - tw0) * 16.0 / 3.3e6;
    const bool own = pp.on && (pair_variant == 13 || (pair_variant != 14 && upd_us < PAIR_OWN_PANEL_US));
    int nchunks = 1;
    if (m4_target > 0) {
        nchunks = (m4_target + nt - 1) / nt;
    } else {
        // whole rounds of one block per CU (less the panel's)
        const int64_t slots = device_cus() - (own ? 1 : 0);
        int64_t maxc = rows_est / 256;
        if (maxc < 1) maxc = 1;
        if (maxc > 4 * slots) maxc = 4 * slots;
        double best_eff = -1.0;
        for (int64_t nc = 1; nc <= maxc; nc++) {
            const int64_t g = nt * nc;
            const int64_t rounds = (g + slots - 1) / slots;
            const double eff = (double)g / (double)(rounds * slots) - 0.02 * (double)(rounds - 1);
            if (eff > best_eff + 1e-9) {
                best_eff = eff;
                nchunks = (int)nc;
            }
        }
    }
    if (nchunks < 1) nchunks = 1;
    // block 0 (16 waves) loses its panel wave for about the panel's time: its share of a
    // chunk is the rest (about 25 us of panel against an update streaming
    // its bytes at about 3.3 TB/s)
    PairPanel ppl = pp;
    if (own) {
        ppl.share = -1;
    } else if (pp.on) {
        const double busy = upd_us > 0.0 ? (25.0 / upd_us < 1.0 ? 25.0 / upd_us : 1.0) : 1.0;
        ppl.share = (int)(65536.0 * (16.0 - busy) / 16.0);
    }
    const unsigned grid = (unsigned)(nt * nchunks + (own ? 1 : 0));
    ProfScope ps(KID_M4RM, s);
#define PAIR_LAUNCH(NT, U, G, PF)                                                                                 \
    hipLaunchKernelGGL((k_m4rm_pair<NT, U, G, PF>), dim3(grid), dim3(NT), 0, s, A, ldw, m, coefP, coefU, coefT,     \
                       PBt, PBu, ldw, tw0, nw, nt, nchunks, rect, recu, ppl)
#define PAIR_LAUNCH_RP(NT, G)                                                                                     \
    hipLaunchKernelGGL((k_m4rm_pair<NT, 1, G, true, true>), dim3(grid), dim3(NT), 0, s, A, ldw, m, coefP, coefU,    \
                       coefT, PBt, PBu, ldw, tw0, nw, nt, nchunks, rect, recu, ppl)
    // (threads, rows in flight per thread, table reads per group, coefficient
    // prefetch[, row prefetch]); the default was the fastest on MI355X for the
    // 65536^2 PLE
    switch (pair_variant) {
        case 1: PAIR_LAUNCH(1024, 2, 2, false); break;
        case 3: PAIR_LAUNCH(1024, 4, 1, false); break;
        case 4: PAIR_LAUNCH(1024, 4, 2, false); break;
        case 5: PAIR_LAUNCH(1024, 1, 4, false); break;
        case 2: PAIR_LAUNCH(1024, 2, 4, false); break;
        case 6: PAIR_LAUNCH(1024, 2, 4, true); break;
        case 8: PAIR_LAUNCH(1024, 1, 8, true); break;
        case 9: PAIR_LAUNCH(1024, 1, 2, true); break;
        case 10: PAIR_LAUNCH_RP(1024, 4); break;
        case 11: PAIR_LAUNCH(1024, 1, 4, true); break;
        case 12: PAIR_LAUNCH_RP(1024, 8); break;
        default: PAIR_LAUNCH_RP(1024, 2); break;
    }
#undef PAIR_LAUNCH
#undef PAIR_LAUNCH_RP
    return hipGetLastError();
}

hipError_t launch_pass(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t c, const PassRec *prev, PassRec *rec,
                       int64_t *P, int64_t *Q, int64_t *rank, uint64_t *coef, uint64_t *PB, uint64_t *gsv,
                       int32_t *gsid, int m4_variant, int m4_target, int panel_regs, hipStream_t s) {
    hipError_t e =
        launch_panel(A, m, n, ldw, c, prev, rec, P, Q, rank, gsv, gsid, panel_regs, PanelFix(), false, s, nullptr);
    if (e != hipSuccess) return e;
    if ((e = launch_permute(A, m, n, ldw, c, rec, coef, PB, 0, nullptr, nullptr, nullptr, nullptr, s, nullptr, 0)) !=
        hipSuccess)
        return e;
    return launch_update(A, m, n, ldw, c, rec, coef, PB, 1, m4_variant, m4_target, s);
}

hipError_t launch_m4rm(uint64_t *C, int64_t ldc, int64_t m, const uint64_t *coef, int64_t coef_ld, const uint64_t *B,
                       int64_t ldb, int nbits, int64_t w_begin, int64_t w_end, int m4_variant, int m4_target,
                       hipStream_t s) {
    if (w_begin >= w_end || m <= 0) return hipSuccess;
    const int v = m4_pick(m4_variant, m, w_end - w_begin);
    int ntiles, nchunks;
    m4_grid(v, m, w_begin, w_end, m4_target, &ntiles, &nchunks);
    ProfScope ps(KID_M4RM, s);
    m4_launch_variant(v, dim3(ntiles * nchunks), s, C, ldc, m, coef, coef_ld, B, ldb, nbits, w_begin, w_end, ntiles,
                      nchunks, (const PassRec *)nullptr);
    return hipGetLastError();
}

hipError_t launch_echelon(uint64_t *A, int64_t m, int64_t ldw, const int64_t *rank, hipStream_t s) {
    int64_t total = m * ldw;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    ProfScope ps(KID_ECHELON, s);
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
