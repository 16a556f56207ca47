// The panel of one pass: Algorithm 1 (PartialPle) on a 64-column stripe,
// run by one wavefront.  Included by the kernels that launch it.
//
// Search.  For each stripe column j in turn, the pivot is the first row at or
// below the current rank position, in the current row order, whose entry is
// 1 after reduction by the pivots already found (Algorithm 1's search loop);
// it is swapped in whole.  Laziness (Algorithm 1): rows are fetched and
// reduced only when the search reaches them, 64 at a time into the wave's
// registers (lane = row, ballot = "which rows have a 1 in column j").  If the
// register window (WQ x 64 rows) runs out, the search restarts over every
// remaining row in LDS or workspace ("slow" path).
//
// Replay.  The pass's maps (Section 3.2's T and T') come out of one more run
// of the same eliminations that carries, next to each stripe word, the sum h
// of the pivot "histories" it was reduced by and the set u of pivots used.
// A pivot row's history starts as its own unit vector, so it ends as its row
// of L11^-1 (the TRSM of Algorithm 2); a non-pivot row ends with h = its
// coefficients on the pivot rows as they were (Orig) and u = its L bits.
// Replaying the 64 unit stripe vectors gives both maps for every other row
// by linearity: a row with stripe word v becomes row + w*Orig with
// w = xor of h(e_j) over the set bits j of v, and gets the L bits
// u = xor of u(e_j).
#pragma once
#include "dev.h"

namespace gf2 {

// LDS of the panel: the special-row lists and up to SR rows of the slow
// search (beyond that it uses the workspace arrays).
template <int SR>
struct PanelLdsT {
    int64_t dst[MAX_SPEC], src[MAX_SPEC];
    uint64_t sv[SR > 0 ? SR : 1];
    int32_t sid[SR > 0 ? SR : 1];
    int32_t spos[SR > 0 ? SR : 1];
    int32_t sgrp[SR > 0 ? SR / 64 + 1 : 1];
};
using PanelLds = PanelLdsT<SLOW_LDS_ROWS>;

// Stripe words are read past the L1 cache (the panel itself may just have
// rewritten some of them): a relaxed load at device scope, which, unlike a
// volatile one, lets several loads be in flight at once.
__device__ __forceinline__ uint64_t ld_stripe(const uint64_t *p) { return ld_dev(p); }

// The rows a fix wrote: lane l's entries l and 64 + l (position d, -1 if
// none, and the new stripe word n).
struct FixOut {
    uint64_t n0 = 0, n1 = 0;
    int64_t d0 = -1, d1 = -1;
};

// Order this wave's LDS accesses before and after the call: a compiler
// barrier and a wave barrier (the LDS executes one wave's accesses in order).
__device__ __forceinline__ void lds_order() {
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
}

__device__ __forceinline__ void fix_wait() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// With the look-ahead, the previous pass's permute leaves the special rows'
// (its pivots' and the rows they displaced) word of this stripe in place and
// puts their new values in its record: the panel writes them to their
// positions.  One wave, entries lane and 64 + lane.  With `wait` the writes
// are complete on return.
__device__ __forceinline__ FixOut fix_from_record(uint64_t *A, int64_t ldw, int64_t sw, const PassRec *pr,
                                                  const int lane, const bool wait) {
    FixOut o;
    const int fn = pr->active ? pr->nspec : 0;
    if (fn <= 0) return o;
    const bool h0 = lane < fn, h1 = 64 + lane < fn;
    o.d0 = h0 ? pr->spec_dst[lane] : -1;
    o.d1 = h1 ? pr->spec_dst[64 + lane] : -1;
    o.n0 = h0 ? pr->spec_next[lane] : 0ull;
    o.n1 = h1 ? pr->spec_next[64 + lane] : 0ull;
    if (h0) A[o.d0 * ldw + sw] = o.n0;
    if (h1) A[o.d1 * ldw + sw] = o.n1;
    if (wait) fix_wait();
    return o;
}

// What the previous pass left for the panel to finish in its stripe word:
// mode 1 after a look-ahead permute (the special rows' words are in the
// previous record).
struct PanelFix {
    int mode = 0;
};

// A panel launched inside a fused pair's update kernel: pass t + 2 on the
// stripe at c, writing record `rec` (the pair's second record is its
// previous one).
struct PairPanel {
    int on = 0;
    int share = 65536;  // block 0's row share relative to the others, in 1/65536

    int64_t n = 0, c = 0;
    PassRec *rec = nullptr;
    int64_t *P = nullptr, *Q = nullptr, *rank = nullptr;
    uint64_t *gsv = nullptr;
    int32_t *gsid = nullptr;
};

// Slow search bookkeeping: a row with a zero stripe word sits at position
// npiv and goes to position `found` (the pivot's).  Lane d of dzp/dzi holds
// the d-th such row: where it is now and where it started (-1: none).  A row
// moved before moves on; at most one new row per pivot.
__device__ __forceinline__ void move_zero_row(int &dzp, int &dzi, const int npiv, const int found, const int lane) {
    if (__ballot(dzp == npiv)) {
        dzp = dzp == npiv ? found : dzp;
    } else {
        const int nd = __popcll(__ballot(dzp >= 0));
        if (lane == nd) {
            dzp = found;
            dzi = npiv;
        }
    }
}

// The special-row list of a slow search, finished by one wave: entries
// [npiv, nsp) already hold the kept rows that moved, in any order.  Adds the
// pivots in order at [0, npiv) and the zero-word rows that moved, then ranks
// the displaced rows (at most npiv) by position.  Returns the list's length.
template <int SR>
__device__ __forceinline__ int finish_special(PanelLdsT<SR> &L, const int64_t r, const int npiv, int nsp,
                                              const int my_id, const int dzp, const int dzi, const int lane) {
    const uint64_t lt = (1ull << lane) - 1ull;
    if (lane < npiv) {
        L.dst[lane] = r + lane;
        L.src[lane] = r + my_id;
    }
    {
        const uint64_t msk = __ballot(dzp >= 0);
        if (dzp >= 0) {
            const int idx = nsp + __popcll(msk & lt);
            L.dst[idx] = r + dzp;
            L.src[idx] = r + dzi;
        }
        nsp += __popcll(msk);
    }
    const int nspec = uni(nsp);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int nd = nspec - npiv;  // <= npiv <= 64
    int64_t dd = 0, ds = 0;
    if (lane < nd) {
        dd = L.dst[npiv + lane];
        ds = L.src[npiv + lane];
    }
    const int dpos = (int)(dd - r);
    int rank = 0;
    for (int k = 0; k < nd; k++) rank += readlane32(dpos, k) < dpos ? 1 : 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (lane < nd) {
        L.dst[npiv + rank] = dd;
        L.src[npiv + rank] = ds;
    }
    return nspec;
}

// ---- the slow search on every wave of the block ----------------------------
// When the panel has a block of NW waves, its slow search runs on all of
// them.  The scan over the remaining rows is split into rounds of NW * 64 * 4
// rows, one part per wave, and the kept rows (non-zero stripe word, in row
// order) are staged in LDS, then taken into registers: slot k lives in
// register k / (64 NW) of wave (k / 64) % NW, lane k % 64, so each wave's
// slots ascend with its register and lane.  A column then costs one barrier:
// every wave posts its first active slot and its first active slot with the
// column's bit, every wave reads the NW posts and takes the smallest, and
// all apply the same move and the same elimination to the slots they hold.
// A slot keeps its position and a swap exchanges word and first position,
// as in the one-wave search below; but where a pivot takes a zero row's
// place, that row moves into the pivot's slot (as a word of 0) instead of
// the slot retiring, so the active slots stay a range.  The elimination is
// eager: each pivot leaves every active slot that has its bit at once.
constexpr int MW_SLOTS = 8192;  // kept rows held in registers, over all waves

// Minimum and sum over lanes 0..15 (one DPP row), in each of those lanes:
// exchanges within pairs, within quads, across the two quads of each half
// and across the two halves.
__device__ __forceinline__ int row16_min(int v) {
    int o = __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    v = o < v ? o : v;
    o = __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    v = o < v ? o : v;
    o = __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v = o < v ? o : v;
    o = __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false);  // row_mirror
    return o < v ? o : v;
}
__device__ __forceinline__ int row16_sum(int v) {
    v += __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false);
    return v + __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false);
}

// LDS exchange of the multi-wave search.
template <int NW>
struct MwX {
    struct Post {
        uint64_t word;
        int32_t slot, pos, id, pad;
    };
    Post fm[2][NW], fa[2][NW];  // per column, alternating: first slot with the bit, first active slot
    int32_t cnt[2][NW];         // per scan round, alternating: kept rows of each wave
    uint64_t orv[NW];
    int32_t lcount, flag;
#ifdef GF2_PANEL_TIMING
    uint64_t tph[4];  // wave 0's clock: start, scan done, columns done, end
#endif
};

// Where the multi-wave search stages the kept rows (LDS, cap entries) and
// keeps its exchange (an MwX<NW>), and the one-wave search's LDS arrays
// (word, position, first position), to which it may hand few kept rows.
struct MwCtx {
    void *x = nullptr;
    uint64_t *stv = nullptr;
    int32_t *stp = nullptr;
    int cap = 0;
    uint64_t *hv = nullptr;
    int32_t *hp = nullptr, *hi = nullptr;
};

// Up to this many kept rows wave 0 alone (no barrier per column) takes over
// from the multi-wave search after the shared scan.
constexpr int MW_ALONE = 512;
enum MwResult { MW_FALLBACK = 0, MW_HANDED = 1, MW_DONE = 2 };

// The column search of the multi-wave slow search over the first RR of the
// R registers of slots (the others are empty).  No slot retires: when a row
// with a zero stripe word sits at the rank position, it moves into the
// pivot's slot as a word of 0.  Slot positions ascend with the slot and never
// change, so the active slots are the range [kthr, nc) and the first active
// slot is kthr.  One barrier per column with a possible pivot: every wave
// posts its first active slot with the column's bit, and the owner of slot
// kthr posts that slot's word, position and first position; then every wave
// reads the posts (lane w takes wave w's) and picks the smallest slot.
template <int NW, int RR, int R>
__device__ __forceinline__ void mw_columns(MwX<NW> &X, uint64_t (&wd)[R], int (&cpos)[R], int (&cid)[R],
                                           const int lane, const int wave, const uint64_t orv, const int kp,
                                           const int nc, const int64_t rows, int &npiv, int &kthr, int &my_q,
                                           uint64_t &my_fin, int &my_p, int &my_id) {
    using Post = typename MwX<NW>::Post;
    uint64_t or_pe = 0;
    int par = 0;
    // one column; HI: j >= 32, whose bit and part above it lie in the high
    // half of each word (one 32-bit test, one half to update)
    auto column = [&](const int j, auto hi_c) {
        constexpr bool HI = decltype(hi_c)::value;
        const uint32_t bj = 1u << (j & 31);
        auto half = [&](const uint64_t w) { return HI ? (uint32_t)(w >> 32) : (uint32_t)w; };
        if (!(((orv | or_pe) >> j) & 1ull)) return;  // no row can have a 1 here
        // this wave's first active slot with bit j (register qm, lane lm);
        // each lane keeps its own entry of that register
        int qm = RR, lm = 0;
        uint64_t wm = 0;
        int pm = 0, im = 0;
#pragma unroll
        for (int q = 0; q < RR; q++) {
            if (qm == RR) {
                const uint64_t cm = __ballot(cpos[q] >= npiv && (half(wd[q]) & bj) != 0);
                if (cm) {
                    qm = q;
                    lm = (int)__builtin_ctzll(cm);
                    wm = wd[q];
                    pm = cpos[q];
                    im = cid[q];
                }
            }
        }
        // slot h = kthr's owner: this wave or not, its register and lane
        const int h = kthr;
        const bool oh = h < nc && (h >> 6) % NW == wave;
        const int rh = (h >> 6) / NW, lh = h & 63;
        if (lane == lm) X.fm[par][wave] = Post{wm, qm == RR ? INT32_MAX : (qm * NW + wave) * 64 + lm, pm, im, 0};
        if (oh) {
            uint64_t w_h = 0;
            int p_h = 0, i_h = 0;
#pragma unroll
            for (int q = 0; q < RR; q++) {
                if (q == rh) {
                    w_h = wd[q];
                    p_h = cpos[q];
                    i_h = cid[q];
                }
            }
            if (lane == lh) X.fa[par][0] = Post{w_h, h, p_h, i_h, 0};
        }
        if constexpr (NW > 1) {
            __syncthreads();
        } else {
            lds_order();  // one wave: its own posts, in program order
        }
        Post em;
        em.slot = INT32_MAX;
        if (lane < NW) em = X.fm[par][lane];
        const Post eh = X.fa[par][0];
        par ^= 1;  // the next column posts to the other half: no second barrier
        const int kf = uni(row16_min(em.slot));
        if (kf == INT32_MAX) return;  // column j has no pivot
        const int wf = (int)__builtin_ctzll(__ballot(em.slot == kf));
        const uint64_t pv = readlane64(em.word, wf);
        const int found = readlane32(em.pos, wf), pid = readlane32(em.id, wf);
        const uint64_t vh = readlane64(eh.word, 0);  // kf exists, so slot h does
        const int ph = uni(eh.pos), idh = uni(eh.id);
        const bool of = (kf >> 6) % NW == wave;
        const int rf = (kf >> 6) / NW, lf = kf & 63;
        if (ph == npiv) {
            // the row at npiv is slot h: h now holds the pivot (and leaves the
            // range) and kf that row (kf == h: the pivot is in place)
            if (kf != h) {
#pragma unroll
                for (int q = 0; q < RR; q++) {
                    if (oh && q == rh) {
                        wd[q] = lane == lh ? pv : wd[q];
                        cid[q] = lane == lh ? pid : cid[q];
                    }
                    if (of && q == rf) {
                        wd[q] = lane == lf ? vh : wd[q];
                        cid[q] = lane == lf ? idh : cid[q];
                    }
                }
            }
            kthr = h + 1;
        } else {
            // a row with a zero stripe word is at npiv, where it has always
            // been: it moves into the pivot's slot
#pragma unroll
            for (int q = 0; q < RR; q++) {
                if (of && q == rf) {
                    wd[q] = lane == lf ? 0ull : wd[q];
                    cid[q] = lane == lf ? npiv : cid[q];
                }
            }
        }
        // every later active slot with bit j leaves it
        const uint64_t pe = pv & above(j);
        const uint32_t pel = (uint32_t)pe, peh = (uint32_t)(pe >> 32);
#pragma unroll
        for (int q = 0; q < RR; q++) {
            uint32_t lo = (uint32_t)wd[q], hi = (uint32_t)(wd[q] >> 32);
            const bool e = cpos[q] > npiv && ((HI ? hi : lo) & bj) != 0;
            if (!HI) lo = e ? lo ^ pel : lo;  // a high column's part above it has no low bits
            hi = e ? hi ^ peh : hi;
            wd[q] = ((uint64_t)hi << 32) | lo;
        }
        my_q = writelane32(my_q, j, npiv);
        my_fin = writelane64(my_fin, pv, npiv);
        my_p = writelane32(my_p, found, npiv);
        my_id = writelane32(my_id, pid, npiv);
        or_pe |= pe;
        npiv++;
    };
    const int k32 = kp < 32 ? kp : 32;
    for (int j = 0; j < k32 && npiv < rows; j++) column(j, std::false_type());
    for (int j = 32; j < kp && npiv < rows; j++) column(j, std::true_type());
}

// Wave 0 alone, after the scan, on at most MW_ALONE kept rows: slot k in
// register k / 64, lane k mod 64; the column loop of the multi-wave search
// with one wave (its posts need no barrier), then the list.  Uses the LDS of
// the exchange as an MwX<1> (the other waves read none of it any more).
template <int NW, int SR>
__device__ __forceinline__ void mw_alone(const MwCtx &mc, PanelLdsT<SR> &L, const int nc, const uint64_t orv,
                                         const int64_t r, const int64_t rows, const int kp, const int lane,
                                         int &npiv_out, int &my_q, uint64_t &my_fin, int &my_p, int &nspec_out) {
    static_assert(sizeof(MwX<1>) <= sizeof(MwX<NW>) && offsetof(MwX<NW>, orv) >= sizeof(MwX<1>),
                  "the one-wave exchange stays clear of what the others still read");
    MwX<1> &X = *(MwX<1> *)mc.x;
    constexpr int R = MW_ALONE / 64;
    uint64_t wd[R];
    int cpos[R], cid[R];  // position now (-1: retired or empty), first position
#pragma unroll
    for (int q = 0; q < R; q++) {
        const int k = q * 64 + lane;
        const bool in = k < nc;
        wd[q] = in ? mc.stv[k] : 0ull;
        cpos[q] = in ? mc.stp[k] : -1;
        cid[q] = cpos[q];
    }
    my_q = 0;
    my_fin = 0;
    my_p = 0;
    int npiv = 0, kthr = 0, my_id = 0;
    const int rr = (nc + 63) / 64;
    static_assert(R == 8, "register counts 1, 2, 4, 8");
    if (rr <= 1)
        mw_columns<1, 1, R>(X, wd, cpos, cid, lane, 0, orv, kp, nc, rows, npiv, kthr, my_q, my_fin, my_p, my_id);
    else if (rr <= 2)
        mw_columns<1, 2, R>(X, wd, cpos, cid, lane, 0, orv, kp, nc, rows, npiv, kthr, my_q, my_fin, my_p, my_id);
    else if (rr <= 4)
        mw_columns<1, 4, R>(X, wd, cpos, cid, lane, 0, orv, kp, nc, rows, npiv, kthr, my_q, my_fin, my_p, my_id);
    else
        mw_columns<1, 8, R>(X, wd, cpos, cid, lane, 0, orv, kp, nc, rows, npiv, kthr, my_q, my_fin, my_p, my_id);
    // kept rows that moved: listed after the pivots, in any order
    const uint64_t lt = (1ull << lane) - 1ull;
    int nsp = npiv;
#pragma unroll
    for (int q = 0; q < R; q++) {
        const bool f = cpos[q] >= npiv && cpos[q] != cid[q];
        const uint64_t msk = __ballot(f);
        if (f) {
            const int idx = nsp + __popcll(msk & lt);
            L.dst[idx] = r + cpos[q];
            L.src[idx] = r + cid[q];
        }
        nsp += __popcll(msk);
    }
    npiv_out = npiv;
    nspec_out = finish_special(L, r, npiv, nsp, my_id, -1, 0, lane);
}

// Run by every wave of the block (wave = its index, uniform); the result is
// the same on every wave.  At most MW_ALONE kept rows: with ALONE, wave 0
// searches them in its registers; otherwise they go to the one-wave search.  MW_FALLBACK: the kept rows exceed what the
// registers or the staging hold (nothing was written but the exchange and
// the staging).  MW_HANDED: at most MW_ALONE kept rows, now in the one-wave
// search's arrays (nc_out, orv_out: their count and union).  MW_DONE: wave 0
// holds the pivots (lane l: column, reduced stripe word, position found) and
// L the special rows.
template <int NW, bool ALONE, int SR>
__device__ __forceinline__ MwResult slow_search_mw(const uint64_t *A, const int64_t ldw, const int64_t sw,
                                                   const int64_t r, const int64_t rows, const uint64_t kmask,
                                                   const int kp, const int lane, const int wave, const MwCtx &mc,
                                                   PanelLdsT<SR> &L, int &npiv_out, int &my_q, uint64_t &my_fin,
                                                   int &my_p, int &nspec_out, int &nc_out, uint64_t &orv_out) {
    constexpr int R = MW_SLOTS / (NW * 64);  // slots per lane
    constexpr int SB = 4;                    // row loads in flight per lane
    static_assert(R * NW * 64 == MW_SLOTS, "slots per lane");
    static_assert(NW <= 16, "the waves' posts fit one DPP row");
    MwX<NW> &X = *(MwX<NW> *)mc.x;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int cap = mc.cap < MW_SLOTS ? mc.cap : MW_SLOTS;
    if (wave == 0 && lane == 0) X.lcount = 0;
#ifdef GF2_PANEL_TIMING
    if (wave == 0 && lane == 0) X.tph[0] = wall_clock64();
#define MW_STAMP(k) \
    if (wave == 0 && lane == 0) X.tph[k] = wall_clock64();
#else
#define MW_STAMP(k)
#endif

    // ---- scan: every wave takes 64 * SB rows of each round ----
    int nc = 0, par = 0;
    uint64_t orv = 0;
    for (int64_t b0 = 0; b0 < rows; b0 += (int64_t)NW * 64 * SB) {
        const int64_t wb = b0 + (int64_t)wave * 64 * SB;
        uint64_t v[SB];
#pragma unroll
        for (int u = 0; u < SB; u++) {
            const int64_t pos = wb + 64 * u + lane;
            v[u] = ld_stripe(A + (r + (pos < rows ? pos : rows - 1)) * ldw + sw);
        }
        int cw = 0;
#pragma unroll
        for (int u = 0; u < SB; u++) {
            v[u] = wb + 64 * u + lane < rows ? v[u] & kmask : 0ull;
            cw += __popcll(__ballot(v[u] != 0));
            orv |= v[u];
        }
        if (lane == 0) X.cnt[par][wave] = cw;
        __syncthreads();
        // this wave's first slot: the rows the waves before it keep
        const int cl = lane < NW ? X.cnt[par][lane] : 0;
        const int total = uni(row16_sum(cl));
        int k0 = nc + uni(row16_sum(lane < wave ? cl : 0));
#pragma unroll
        for (int u = 0; u < SB; u++) {
            const uint64_t msk = __ballot(v[u] != 0);
            const int k = k0 + __popcll(msk & lt);
            if (v[u] && k < cap) {
                mc.stv[k] = v[u];
                mc.stp[k] = (int32_t)(wb + 64 * u + lane);
            }
            k0 += __popcll(msk);
        }
        nc += total;
        par ^= 1;
    }
    orv = wave_or64(orv);
    if (lane == 0) X.orv[wave] = orv;
    __syncthreads();  // also completes the staging
    orv = wave_or64(lane < NW ? X.orv[lane] : 0ull);
    MW_STAMP(1)
    if (nc > cap) return MW_FALLBACK;
    if (nc <= MW_ALONE) {
        // few kept rows: wave 0 alone holds them, and its columns take no
        // barrier (the others leave; nothing they read is written below)
        if constexpr (ALONE) {
            if (wave == 0) mw_alone<NW>(mc, L, nc, orv, r, rows, kp, lane, npiv_out, my_q, my_fin, my_p, nspec_out);
            return MW_DONE;
        }
        for (int k = wave * 64 + lane; k < nc; k += NW * 64) {
            if (mc.hv != mc.stv) mc.hv[k] = mc.stv[k];
            const int32_t p = mc.stp[k];
            mc.hp[k] = p;
            mc.hi[k] = p;
        }
        __syncthreads();
        nc_out = nc;
        orv_out = orv;
        return MW_HANDED;
    }

    // ---- the kept rows into registers ----
    uint64_t wd[R];
    int cpos[R], cid[R];  // position now (-1: retired or empty), first position
#pragma unroll
    for (int q = 0; q < R; q++) {
        const int k = (q * NW + wave) * 64 + lane;
        const bool in = k < nc;
        wd[q] = in ? mc.stv[k] : 0ull;
        cpos[q] = in ? mc.stp[k] : -1;
        cid[q] = cpos[q];
    }

    // ---- column search, on the registers in use ----
    my_q = 0;
    my_fin = 0;
    my_p = 0;
    int npiv = 0, kthr = 0, my_id = 0;
    static_assert(R == 8 || R == 16, "register counts 1, 2, 4, 8 (, 16)");
    const int rr = (nc + NW * 64 - 1) / (NW * 64);
    if (rr <= 1)
        mw_columns<NW, 1, R>(X, wd, cpos, cid, lane, wave, orv, kp, nc, rows, npiv, kthr, my_q, my_fin, my_p,
                              my_id);
    else if (rr <= 2)
        mw_columns<NW, 2, R>(X, wd, cpos, cid, lane, wave, orv, kp, nc, rows, npiv, kthr, my_q, my_fin, my_p,
                              my_id);
    else if (rr <= 4)
        mw_columns<NW, 4, R>(X, wd, cpos, cid, lane, wave, orv, kp, nc, rows, npiv, kthr, my_q, my_fin, my_p,
                              my_id);
    else if (R == 8 || rr <= 8)
        mw_columns<NW, 8, R>(X, wd, cpos, cid, lane, wave, orv, kp, nc, rows, npiv, kthr, my_q, my_fin, my_p,
                              my_id);
    else
        mw_columns<NW, (R > 8 ? 16 : 8), R>(X, wd, cpos, cid, lane, wave, orv, kp, nc, rows, npiv, kthr, my_q, my_fin,
                                             my_p, my_id);
    MW_STAMP(2)

    // ---- kept rows that moved: listed after the pivots, in any order ----
#pragma unroll
    for (int q = 0; q < R; q++) {
        const bool f = cpos[q] >= npiv && cpos[q] != cid[q];
        const uint64_t msk = __ballot(f);
        if (msk) {
            int base = 0;
            if (lane == 0) base = atomicAdd(&X.lcount, (int)__popcll(msk));
            base = uni(base);
            if (f) {
                const int idx = npiv + base + __popcll(msk & lt);
                L.dst[idx] = r + cpos[q];
                L.src[idx] = r + cid[q];
            }
        }
    }
    __syncthreads();
    npiv_out = npiv;
    if (wave != 0) return MW_DONE;
    nspec_out = finish_special(L, r, npiv, npiv + uni(X.lcount), my_id, -1, 0, lane);
    MW_STAMP(3)
#undef MW_STAMP
    return MW_DONE;
}

// One wave (lane = threadIdx.x & 63) computes the panel of the stripe at
// column c.  `prev` is the previous pass's record (its r + rbar is this
// pass's r; it is read before `rec` is written, so the two may be the same
// record), `rec` receives this pass.  Writes P[r..r+rbar), Q[r..r+rbar)
// and *rank_out = r + rbar.  With NW > 1 every wave of the block calls it
// (`wave` = its index): wave 0 runs the panel, and the others join it for
// the slow search (mc: its LDS; ALONE: few kept rows in wave 0's registers
// rather than the one-wave search's LDS arrays: faster on sparse stripes, but
// in the standalone panel the larger kernel cost its dense launches time).
template <int WQ, int SR, bool KEPT = true, int NW = 1, bool ALONE = false>
__device__ __forceinline__ void panel_body(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t c,
                                           const PassRec *prev, PassRec *rec, int64_t *P, int64_t *Q,
                                           int64_t *rank_out, uint64_t *gsv, int32_t *gsid, PanelLdsT<SR> &L,
                                           const int lane, PanelFix fix = PanelFix(), const int wave = 0,
                                           const MwCtx &mc = MwCtx()) {
    static_assert(NW == 1 || (WQ == 2 && KEPT), "the multi-wave slow search follows the "
                                                                     "two-register window");
#ifdef GF2_PANEL_TIMING
    uint64_t *dbg = gsv + (c >> 6) * 8;
    uint64_t *dbg2 = gsv + 2048 + (c >> 6) * 8;  // phase sums of the kept-row search
#define PANEL_STAMP(k) \
    if (lane == 0 && wave == 0) dbg[k] = wall_clock64();
#define PANEL_T0(t) const uint64_t t = wall_clock64();
#define PANEL_ACC(k, t) \
    if (lane == 0 && wave == 0) dbg2[k] += wall_clock64() - t;
#else
#define PANEL_STAMP(k)
#define PANEL_T0(t)
#define PANEL_ACC(k, t)
#endif
    PANEL_STAMP(0)
    const int64_t r = prev->r + prev->rbar;
    // the two-register window takes the fixed rows into its registers
    // directly (their stores need not land before the window is read); the
    // other paths read rows back from A, so the fix completes first
    const bool patch = WQ == 2 && fix.mode != 0 && r < m && c < n;
    auto run_fix = [&](const bool wait) -> FixOut { return fix_from_record(A, ldw, c >> 6, prev, lane, wait); };
    if (fix.mode != 0 && c < n && !patch && wave == 0) run_fix(true);
    if (r >= m || c >= n) {
        if (lane == 0 && wave == 0) {
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
    // The other waves stay for the slow search only when the previous pass
    // needed one (sparse stripes come in runs); otherwise wave 0 goes on alone
    // and no barrier is taken.  (With prev == rec, wave 0 may rewrite the
    // flag before another wave reads it: then always alone.)
    bool mw = false;
    if constexpr (NW > 1) {
        mw = prev != rec && prev->slow != 0;
        if (!mw && wave != 0) return;
    }

    // lane l keeps pivot l: stripe column, reduced stripe word, window position
    int my_q = 0;
    uint64_t my_fin = 0;
    int my_p = 0;
    int npiv = 0;
    int nspec = 0;
    bool slow = false;

    // ---- search over a register window ---------------------------------------
    // (wave 0 alone when the block has several)
    if (NW == 1 || wave == 0) {
        if constexpr (WQ == 2) {
            // Two registers (128 rows), loaded at once, kept as 32-bit halves:
            // lane l holds positions l (x0) and 64 + l (x1).  Per column the
            // candidate masks are ballots of one half, the pivot is their first
            // set bit, and every move is a select on a scalar lane mask: the
            // rows with the bit (but the pivot) get the pivot's part above the
            // column, the row at npiv moves to the pivot's place and the pivot
            // row to npiv.  Positions below npiv are never written again, so at
            // the end they hold the pivot rows as found.  No branch but the exit.
            const int nmax = (int)(rows < 128 ? rows : 128);
            uint32_t x0l, x0h, x1l, x1h;
            {
                const int64_t row0 = r + (lane < rows ? lane : rows - 1);
                const int64_t row1 = r + (64 + lane < rows ? 64 + lane : rows - 1);
                // the fix's record entries load first (every entry, masked once
                // the header is in), so waiting for them never waits for the
                // stripe words behind them
                FixOut fo;
                int fa = 0, fnr = 0;
                if (patch) {
                    fa = prev->active;
                    fnr = prev->nspec;
                    fo.d0 = prev->spec_dst[lane];
                    fo.d1 = prev->spec_dst[64 + lane];
                    fo.n0 = prev->spec_next[lane];
                    fo.n1 = prev->spec_next[64 + lane];
                }
                __builtin_amdgcn_sched_barrier(0);
                uint64_t t0 = ld_stripe(A + row0 * ldw + sw);
                uint64_t t1 = ld_stripe(A + row1 * ldw + sw);
                __builtin_amdgcn_sched_barrier(0);
                if (patch) {
                    // the previous pass(es)' special rows in the window: their
                    // loaded words are stale, the fix's new words replace them
                    // (LDS scratch of this wave: its LDS accesses execute in
                    // program order, and the compiler barriers keep that order)
                    const int fn = fa ? fnr : 0;
                    if (lane >= fn) fo.d0 = -1;
                    if (64 + lane >= fn) fo.d1 = -1;
                    if (fo.d0 >= 0) A[fo.d0 * ldw + sw] = fo.n0;
                    if (fo.d1 >= 0) A[fo.d1 * ldw + sw] = fo.n1;
                    int64_t *pf = L.src;
                    uint64_t *pw = (uint64_t *)L.dst;
                    pf[lane] = -1;
                    pf[64 + lane] = -1;
                    lds_order();
                    if (fo.d0 >= r && fo.d0 < r + 128) {
                        pw[fo.d0 - r] = fo.n0;
                        pf[fo.d0 - r] = 1;
                    }
                    if (fo.d1 >= r && fo.d1 < r + 128) {
                        pw[fo.d1 - r] = fo.n1;
                        pf[fo.d1 - r] = 1;
                    }
                    lds_order();
                    if (pf[lane] >= 0) t0 = pw[lane];
                    if (pf[64 + lane] >= 0) t1 = pw[64 + lane];
                    lds_order();
                }
                const uint64_t v0 = lane < nmax ? (t0 & kmask) : 0ull;
                const uint64_t v1 = 64 + lane < nmax ? (t1 & kmask) : 0ull;
                x0l = (uint32_t)v0;
                x0h = (uint32_t)(v0 >> 32);
                x1l = (uint32_t)v1;
                x1h = (uint32_t)(v1 >> 32);
            }
            PANEL_STAMP(1)
            int id0 = lane, id1 = 64 + lane;  // original position of the row each lane holds
            uint64_t act0 = nmax >= 64 ? ~0ull : ((1ull << nmax) - 1ull);
            uint64_t act1 = nmax >= 128 ? ~0ull : (nmax <= 64 ? 0ull : ((1ull << (nmax - 64)) - 1ull));
            int my_qp = 0;  // pivot column | (window position where it was found) << 8
            // Columns [jb, je) of one half (HI: the high half holds their bits).
            // The inner loop takes the usual column, whose pivot is in register
            // 0, without a branch; a column with no candidate in register 0
            // leaves it for the general step (pivot in register 1, no pivot, or
            // rows past the window).  Once every row is a pivot, the candidate
            // masks are empty and the remaining columns cost a ballot each.
            bool go = true;
            auto run = [&](const int jb, const int je, const bool HI) {
                int j = jb;
                while (j < je && go) {
                    // one exit: m0 is empty when column j has no candidate in
                    // register 0 or j reaches je
                    uint64_t m0 = __ballot(((HI ? x0h : x0l) & (1u << (j & 31))) != 0) & act0;
                    while (m0) {
                        const uint32_t bj = 1u << (j & 31);
                        const uint64_t m1 = __ballot(((HI ? x1h : x1l) & bj) != 0) & act1;
                        const int lf = (int)__builtin_ctzll(m0);
                        const uint32_t pvl = (uint32_t)readlane32((int)x0l, lf);
                        const uint32_t pvh = (uint32_t)readlane32((int)x0h, lf);
                        const int idp = readlane32(id0, lf);
                        const uint32_t vrl = (uint32_t)readlane32((int)x0l, npiv);
                        const uint32_t vrh = (uint32_t)readlane32((int)x0h, npiv);
                        const int idr = readlane32(id0, npiv);
                        // the pivot's part strictly above column j leaves the other
                        // rows that have the bit
                        const uint32_t pel = HI ? 0u : (j == 31 ? 0u : pvl & (~0u << (j + 1)));
                        const uint32_t peh = HI ? (j == 63 ? 0u : pvh & (~0u << ((j & 31) + 1))) : pvh;
                        const uint64_t lbit = 1ull << lf, nbit = 1ull << npiv;
                        // lane masks as all-ones/zero words, opaque to the compiler,
                        // so that each update below is one three-input logic
                        // instruction with the scalar operand (a select on a scalar
                        // mask would first copy the scalar into a vector register)
                        uint32_t e0 = __builtin_amdgcn_inverse_ballot_w64(m0 & ~lbit) ? ~0u : 0u;
                        uint32_t e1 = __builtin_amdgcn_inverse_ballot_w64(m1) ? ~0u : 0u;
                        uint32_t s0 = __builtin_amdgcn_inverse_ballot_w64(lbit) ? ~0u : 0u;
                        uint32_t sn = __builtin_amdgcn_inverse_ballot_w64(nbit) ? ~0u : 0u;
                        __asm__ volatile("" : "+v"(e0), "+v"(e1), "+v"(s0), "+v"(sn));
                        if (!HI) {
                            x0l ^= pel & e0;
                            x1l ^= pel & e1;
                        }
                        x0h ^= peh & e0;
                        x1h ^= peh & e1;
                        // the row at npiv to the pivot's place, the pivot to npiv
                        x0l = (x0l & ~s0) | (vrl & s0);
                        x0h = (x0h & ~s0) | (vrh & s0);
                        id0 = (int)(((uint32_t)id0 & ~s0) | ((uint32_t)idr & s0));
                        x0l = (x0l & ~sn) | (pvl & sn);
                        x0h = (x0h & ~sn) | (pvh & sn);
                        id0 = (int)(((uint32_t)id0 & ~sn) | ((uint32_t)idp & sn));
                        my_qp = (int)(((uint32_t)my_qp & ~sn) | ((uint32_t)(j | (lf << 8)) & sn));
                        act0 &= ~nbit;
                        npiv++;
                        j++;
                        const uint64_t nx = __ballot(((HI ? x0h : x0l) & (1u << (j & 31))) != 0) & act0;
                        m0 = j < je ? nx : 0ull;
                    }
                    if (j >= je) return;
                    // general step for column j: no candidate in register 0
                    const uint32_t bj = 1u << (j & 31);
                    const uint64_t m1 = __ballot(((HI ? x1h : x1l) & bj) != 0) & act1;
                    if (!m1) {
                        if (nmax < rows) {  // a row outside the window may hold the pivot
                            slow = true;
                            go = false;
                            return;
                        }
                        j++;  // column j has no pivot
                        continue;
                    }
                    const int lf = (int)__builtin_ctzll(m1);
                    const uint32_t pvl = (uint32_t)readlane32((int)x1l, lf), pvh = (uint32_t)readlane32((int)x1h, lf);
                    const int idp = readlane32(id1, lf);
                    const uint32_t vrl = (uint32_t)readlane32((int)x0l, npiv);
                    const uint32_t vrh = (uint32_t)readlane32((int)x0h, npiv);
                    const int idr = readlane32(id0, npiv);
                    const uint32_t pel = HI ? 0u : (j == 31 ? 0u : pvl & (~0u << (j + 1)));
                    const uint32_t peh = HI ? (j == 63 ? 0u : pvh & (~0u << ((j & 31) + 1))) : pvh;
                    const uint64_t lbit = 1ull << lf, nbit = 1ull << npiv;
                    const bool e1 = __builtin_amdgcn_inverse_ballot_w64(m1 & ~lbit);
                    if (!HI) x1l = e1 ? x1l ^ pel : x1l;
                    x1h = e1 ? x1h ^ peh : x1h;
                    const bool s1 = __builtin_amdgcn_inverse_ballot_w64(lbit);
                    x1l = s1 ? vrl : x1l;
                    x1h = s1 ? vrh : x1h;
                    id1 = s1 ? idr : id1;
                    const bool sn = __builtin_amdgcn_inverse_ballot_w64(nbit);
                    x0l = sn ? pvl : x0l;
                    x0h = sn ? pvh : x0h;
                    id0 = sn ? idp : id0;
                    my_qp = sn ? (j | ((64 + lf) << 8)) : my_qp;
                    act0 &= ~nbit;
                    npiv++;
                    j++;
                }
            };
            run(0, kp < 32 ? kp : 32, false);
            if (go && kp > 32) run(32, kp, true);
            my_fin = lane < npiv ? (((uint64_t)x0h << 32) | x0l) : 0ull;
            my_q = my_qp & 255;
            my_p = my_qp >> 8;
            npiv = uni(npiv);
            PANEL_STAMP(2)
            if (!slow) {
                int base = 0;
#pragma unroll
                for (int q = 0; q < 2; q++) {
                    const int pos = 64 * q + lane;
                    const int idq = q ? id1 : id0;
                    const bool f = pos < nmax && (pos < npiv || idq != pos);
                    const uint64_t msk = __ballot(f);
                    const int idx = base + __popcll(msk & ((1ull << lane) - 1ull));
                    if (f) {
                        L.dst[idx] = r + pos;
                        L.src[idx] = r + idq;
                    }
                    base += __popcll(msk);
                }
                nspec = uni(base);
            }
        } else {

            uint64_t val[WQ];
            int id[WQ];
#pragma unroll
            for (int q = 0; q < WQ; q++) {
                val[q] = 0;
                id[q] = 64 * q + lane;
            }
            const int nmax = (int)(rows < 64 * WQ ? rows : 64 * WQ);
            const int nregmax = (nmax + 63) >> 6;
            int nreg = 0;
            // fetch registers [nreg, want) and reduce them by the pivots so far
            auto extend = [&](int want) {
                uint64_t tmp[WQ];
#pragma unroll
                for (int q = 0; q < WQ; q++) {
                    if (q >= nreg && q < want) {
                        const int pos = 64 * q + lane;
                        const int64_t row = r + (pos < rows ? pos : rows - 1);
                        tmp[q] = ld_stripe(A + row * ldw + sw);
                    }
                }
#pragma unroll
                for (int q = 0; q < WQ; q++) {
                    if (q >= nreg && q < want) val[q] = (64 * q + lane) < nmax ? (tmp[q] & kmask) : 0ull;
                }
                for (int l = 0; l < npiv; l++) {
                    const int ql = uni(readlane32(my_q, l));
                    const uint64_t fl = readlane64(my_fin, l) & above(ql);
#pragma unroll
                    for (int q = 0; q < WQ; q++) {
                        if (q >= nreg && q < want && ((val[q] >> ql) & 1ull)) val[q] ^= fl;
                    }
                }
                nreg = want;
            };
            extend(nregmax < 2 ? nregmax : 2);
            PANEL_STAMP(1)

            // act[q]: lanes of register q that are candidates (loaded, position
            // >= npiv, row < m); kept as scalar masks and updated as npiv grows
            uint64_t act[WQ];
#pragma unroll
            for (int q = 0; q < WQ; q++) act[q] = __ballot(q < nreg && 64 * q + lane < nmax);
            for (int j = 0; j < kp; j++) {
                uint64_t msk[WQ];
                int found = -1;
                for (;;) {
#pragma unroll
                    for (int q = 0; q < WQ; q++) msk[q] = __ballot(((val[q] >> j) & 1ull) != 0) & act[q];
                    found = -1;
#pragma unroll
                    for (int q = WQ - 1; q >= 0; q--)
                        if (msk[q]) found = 64 * q + (int)__builtin_ctzll(msk[q]);
                    found = uni(found);
                    if (found >= 0 || nreg >= nregmax) break;
                    extend(uni(nreg + 1));
#pragma unroll
                    for (int q = 0; q < WQ; q++)
                        act[q] = __ballot(q < nreg && 64 * q + lane < nmax && 64 * q + lane >= npiv);
                }
                if (found < 0) {
                    if (nmax < rows) {  // a row outside the window may hold the pivot
                        slow = true;
                        break;
                    }
                    continue;  // column j has no pivot
                }
                const int qf = found >> 6, lf = found & 63;
                // the pivot row (at `found`) and the row at npiv (register 0, npiv < 64)
                uint64_t pv = 0;
                int idp = 0;
#pragma unroll
                for (int q = 0; q < WQ; q++) {
                    const uint64_t t = readlane64(val[q], lf);
                    const int ti = readlane32(id[q], lf);
                    pv = q == qf ? t : pv;
                    idp = q == qf ? ti : idp;
                }
                const uint64_t vr = readlane64(val[0], npiv);
                const int idr = readlane32(id[0], npiv);
                // swap the two rows, then eliminate column j from the later rows
                // that have it (the row now at `found` never has it)
                const uint64_t pe = pv & above(j);
#pragma unroll
                for (int q = 0; q < WQ; q++) {
                    uint64_t e = msk[q];
                    if (q == 0) e &= ~(1ull << npiv);
                    if (q == qf) e &= ~(1ull << lf);
                    const bool at_found = (q == qf) && lane == lf;
                    const bool at_npiv = (q == 0) && lane == npiv;
                    uint64_t v = at_found ? vr : val[q];
                    v = at_npiv ? pv : v;
                    id[q] = at_npiv ? idp : (at_found ? idr : id[q]);
                    val[q] = v ^ (pe & (0ull - ((e >> lane) & 1ull)));
                }
                act[0] &= ~(1ull << npiv);
                const bool me = lane == npiv;
                my_q = me ? j : my_q;
                my_fin = me ? pv : my_fin;
                my_p = me ? found : my_p;
                npiv = uni(npiv + 1);
                if (npiv == rows) break;
            }
            PANEL_STAMP(2)
            if (!slow) {
                int base = 0;
#pragma unroll
                for (int q = 0; q < WQ; q++) {
                    if (q < nreg) {
                        const int pos = 64 * q + lane;
                        const bool f = pos < nmax && (pos < npiv || id[q] != pos);
                        const uint64_t msk = __ballot(f);
                        const int idx = base + __popcll(msk & ((1ull << lane) - 1ull));
                        if (f) {
                            L.dst[idx] = r + pos;
                            L.src[idx] = r + id[q];
                        }
                        base += __popcll(msk);
                    }
                }
                nspec = uni(base);
            }
        }
    }

    // ---- slow path: every remaining row -------------------------------------
    // The one-wave panels first make one pass over the remaining rows and keep
    // those whose stripe word is not zero (word, position, first position, in
    // row order): a row with a zero stripe word is never a pivot and no
    // elimination changes it; only its position can change, when a pivot is
    // swapped into its place.  The search then runs on the kept rows alone,
    // in LDS or workspace.  The batched kernels' panels (KEPT = false) search
    // every row in place.  A block of several waves first tries the
    // multi-wave search above, with the one-wave search as its fallback.
    bool slow_done = false, handed = false;
    int h_nc = 0;
    uint64_t h_orv = 0;
    if constexpr (NW > 1) {
        if (mw) {
            MwX<NW> &X = *(MwX<NW> *)mc.x;
            if (wave == 0) {
                if (slow && patch) fix_wait();  // the fix's stores, before the other waves read rows back
                if (lane == 0) X.flag = slow ? 1 : 0;
            }
            __syncthreads();
            slow = X.flag != 0;
            if (slow) {
                const MwResult res = slow_search_mw<NW, ALONE>(A, ldw, sw, r, rows, kmask, kp, lane, wave, mc, L, npiv,
                                                        my_q, my_fin, my_p, nspec, h_nc, h_orv);
                slow_done = res == MW_DONE;
                handed = res == MW_HANDED;
#ifdef GF2_PANEL_TIMING
                if (wave == 0 && lane == 0) {
                    dbg2[3] += X.tph[1] - X.tph[0];
                    if (slow_done) {
                        dbg2[4] += X.tph[2] - X.tph[1];
                        dbg2[5] += X.tph[3] - X.tph[2];
                    }
                    dbg2[6] += (uint64_t)res;
                }
#endif
            }
            if (wave != 0) return;
        }
    }
    if (slow && !slow_done) {
        if (patch) fix_wait();  // the fix's stores, before every row is read back
        npiv = 0;
        my_q = 0;
        my_fin = 0;
        my_p = 0;
        if constexpr (!KEPT) {
            uint64_t *sv = rows <= SR ? L.sv : gsv;
            int32_t *sid = rows <= SR ? L.sid : gsid;
            uint64_t orv = 0;
            for (int64_t pos = lane; pos < rows; pos += 64) {
                const uint64_t v = ld_stripe(A + (r + pos) * ldw + sw) & kmask;
                sv[pos] = v;
                sid[pos] = (int32_t)pos;
                orv |= v;
            }
            orv = wave_or64(orv);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            for (int j = 0; j < kp && npiv < rows; j++) {
                if (!((orv >> j) & 1ull)) continue;  // no remaining row has a 1 here
                int64_t found = -1;
                for (int64_t base = npiv & ~(int64_t)63; base < rows; base += 64) {
                    const int64_t pos = base + lane;
                    const bool b = pos >= npiv && pos < rows && ((sv[pos] >> j) & 1ull);
                    const uint64_t msk = __ballot(b);
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
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                if (lane == 0) {
                    sv[found] = vr;
                    sid[found] = idr;
                    sv[npiv] = pv;
                    sid[npiv] = idp;
                }
                my_q = writelane32(my_q, j, npiv);
                my_fin = writelane64(my_fin, pv, npiv);
                my_p = writelane32(my_p, (int)found, npiv);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
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
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                npiv = uni(npiv + 1);
            }
            int base = 0;
            for (int64_t pb = 0; pb < rows; pb += 64) {
                const int64_t pos = pb + lane;
                const bool f = pos < rows && (pos < npiv || sid[pos] != (int32_t)pos);
                const uint64_t msk = __ballot(f);
                const int idx = base + __popcll(msk & ((1ull << lane) - 1ull));
                if (f) {
                    L.dst[idx] = r + pos;
                    L.src[idx] = r + sid[pos];
                }
                base += __popcll(msk);
            }
            nspec = uni(base);
        } else {
            const uint64_t lt = (1ull << lane) - 1ull;
            constexpr int SB = 8;  // row loads in flight per lane
            // kept rows: word, position now, first position (written and read
            // by this wave only, ordered by the fences between the steps)
            uint64_t *cv = gsv;
            int32_t *ci = gsid;
            int32_t *cp = gsid + m;
            int32_t *rg = gsid + 2 * m;  // per 64-slot group: pivots applied
            if constexpr (SR > 0) {
                cv = L.sv;
                ci = L.sid;
                cp = L.spos;
                rg = L.sgrp;
            }
            int nc = 0;
            uint64_t orv = 0;
            auto keep = [&](const int cap) {
                nc = 0;
                orv = 0;
                for (int64_t b0 = 0; b0 < rows; b0 += 64 * SB) {
                    uint64_t v[SB];
                    // every lane loads (past the end: the last row, unused), so
                    // no load sits under a branch and all SB are in flight
#pragma unroll
                    for (int u = 0; u < SB; u++) {
                        const int64_t pos = b0 + 64 * u + lane;
                        v[u] = ld_stripe(A + (r + (pos < rows ? pos : rows - 1)) * ldw + sw);
                    }
#pragma unroll
                    for (int u = 0; u < SB; u++) v[u] = b0 + 64 * u + lane < rows ? v[u] & kmask : 0ull;
#pragma unroll
                    for (int u = 0; u < SB; u++) {
                        const uint64_t msk = __ballot(v[u] != 0);
                        const int k = nc + __popcll(msk & lt);
                        if (v[u] && k < cap) {
                            const int32_t pos = (int32_t)(b0 + 64 * u + lane);
                            cv[k] = v[u];
                            ci[k] = pos;
                            cp[k] = pos;
                        }
                        nc += __popcll(msk);
                        orv |= v[u];
                    }
                }
                orv = wave_or64(orv);
                nc = uni(nc);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            };
            if (handed) {  // the multi-wave scan's rows, already in LDS
                nc = h_nc;
                orv = h_orv;
            } else {
                keep(SR > 0 ? SR : INT32_MAX);
                if (SR > 0 && nc > SR) {  // more kept rows than the LDS holds
                    cv = gsv;
                    ci = gsid;
                    cp = gsid + m;
                    rg = gsid + 2 * m;
                    keep(INT32_MAX);
                }
            }
            // lane d: a row with a zero stripe word moved to position dzp (it
            // started at dzi); -1 = none.  At most one per pivot.
            int dzp = -1, dzi = 0;
            int my_id = 0;
            int nsp = 0;  // special rows listed
            // The kept rows are searched in row order and reduced lazily.
            // A slot's position never changes, and the active slots (position
            // at or below npiv) are in position order: a swap exchanges the
            // pivot's and the npiv row's word and first position between their
            // two slots, and a pivot that takes a zero row's place is retired
            // (position -1).  A column's pivot is then the first active slot
            // with its bit.  Each 64-slot group records how many pivots have
            // been applied to it (in order); a group is brought up to date
            // when the search reaches it, so no elimination pass is needed.
            // Whether a column can have a pivot at all is bounded by the union
            // of the rows as read and the pivots' parts above their columns.
            int head = 0;  // slots before head are not active
            uint64_t or_pe = 0;
            for (int g = lane; g < (nc + 63) / 64; g += 64) rg[g] = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            for (int j = 0; j < kp && npiv < rows; j++) {
                if (!(((orv | or_pe) >> j) & 1ull)) continue;  // no row can have a 1 here
                PANEL_T0(ts0)
                // from head: the first active slot (h) and the first with bit j
                int h = -1, kf = -1;
                for (int s0 = head & ~63; s0 < nc; s0 += 64) {
                    const int g = s0 >> 6;
                    const int k = s0 + lane;
                    const bool in = k < nc;
                    uint64_t v = in ? cv[k] : 0ull;
                    const int p = in ? cp[k] : -1;
                    const int done = uni(rg[g]);
                    if (done < npiv) {
                        for (int l = done; l < npiv; l++) {
                            const int ql = readlane32(my_q, l);
                            const uint64_t pel = readlane64(my_fin, l) & above(ql);
                            v = ((v >> ql) & 1ull) ? v ^ pel : v;
                        }
                        if (in) cv[k] = v;
                        if (lane == 0) rg[g] = npiv;
                    }
                    const bool act = p >= npiv;
                    const uint64_t am = __ballot(act);
                    if (h < 0 && am) h = s0 + (int)__builtin_ctzll(am);
                    const uint64_t cm = __ballot(act && ((v >> j) & 1ull));
                    if (cm) {
                        kf = s0 + (int)__builtin_ctzll(cm);
                        break;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                PANEL_ACC(1, ts0)
                if (kf < 0) continue;  // column j has no pivot
                PANEL_T0(tx0)
                h = uni(h);
                kf = uni(kf);
                const int found = cp[kf];
                const int ph = cp[h];
                const uint64_t pv = cv[kf];
                const int pid = ci[kf];
                const uint64_t vh = cv[h];
                const int idh = ci[h];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                if (ph == npiv) {
                    // the row at npiv is slot h: h now holds the pivot and kf
                    // that row (kf == h: the pivot is in place)
                    if (kf != h && lane == 0) {
                        cv[h] = pv;
                        ci[h] = pid;
                        cv[kf] = vh;
                        ci[kf] = idh;
                    }
                    head = h + 1;
                } else {
                    // a row with a zero stripe word is at npiv: it takes the
                    // pivot's place, and the pivot's slot retires
                    move_zero_row(dzp, dzi, npiv, found, lane);
                    if (lane == 0) cp[kf] = -1;
                    if (kf == h) head = h + 1;
                }
                my_q = writelane32(my_q, j, npiv);
                my_fin = writelane64(my_fin, pv, npiv);
                my_p = writelane32(my_p, found, npiv);
                my_id = writelane32(my_id, pid, npiv);
                or_pe |= pv & above(j);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                PANEL_ACC(2, tx0)
                npiv = uni(npiv + 1);
            }
            // slots that never moved have their first position
            nsp = npiv;
            for (int b0 = 0; b0 < nc; b0 += 64) {
                const int k = b0 + lane;
                const int p = k < nc ? cp[k] : -1;
                const int i0 = k < nc ? ci[k] : -1;
                const bool f = p >= npiv && p != i0;
                const uint64_t msk = __ballot(f);
                if (f) {
                    const int idx = nsp + __popcll(msk & lt);
                    L.dst[idx] = r + p;
                    L.src[idx] = r + i0;
                }
                nsp += __popcll(msk);
            }
            // special rows: the pivots in order, then the displaced rows by
            // position (listed above in any order, ranked there)
            nspec = finish_special(L, r, npiv, nsp, my_id, dzp, dzi, lane);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    PANEL_STAMP(3)

    // ---- replay with histories ---------------------------------------------
    const int rbar = uni(npiv);
    const int ndisp = nspec - rbar;  // <= rbar <= 64
    // displaced rows (lane d <-> special entry rbar + d): their stripe words as
    // they were when the pass began
    uint64_t vD = 0;
    if (patch) fix_wait();  // long since complete: the fix's stores precede these reads
    if (lane < ndisp) vD = ld_stripe(A + L.src[rbar + lane] * ldw + sw) & kmask;
    // 32-bit halves throughout: every update below is one three-input logic
    // instruction per half
    uint32_t vVl = 0, vVh = 0;  // unit stripe vectors
    if (lane < kp) {
        vVl = lane < 32 ? 1u << lane : 0u;
        vVh = lane >= 32 ? 1u << (lane - 32) : 0u;
    }
    uint32_t vDl = (uint32_t)vD, vDh = (uint32_t)(vD >> 32);
    uint32_t hPl = 0, hPh = 0, uPl = 0, uPh = 0;
    if (lane < rbar) {
        hPl = lane < 32 ? 1u << lane : 0u;
        hPh = lane >= 32 ? 1u << (lane - 32) : 0u;
    }
    uint32_t hVl = 0, hVh = 0, uVl = 0, uVh = 0, hDl = 0, hDh = 0, uDl = 0, uDh = 0;
    // a pivot row's bits below its own pivot column are its L bits: bit q_l
    // of them is set only on later pivots reduced by pivot l
    const uint64_t finL = lane < rbar ? my_fin & ((1ull << my_q) - 1ull) : 0ull;
    const uint32_t fLl = (uint32_t)finL, fLh = (uint32_t)(finL >> 32);
    // pivot columns increase with l: those in the low half come first
    const int nlo = __popcll(__ballot(lane < rbar && my_q < 32));
    // HIQ: pivot column ql >= 32; HIL: pivot index l >= 32 (its L bit in the
    // high half).  Both are fixed per loop, so each update touches only the
    // halves that can change.
    // per pivot (lane): its part above its column and its bit offset in its half
    const uint64_t pe_lane = lane < rbar ? my_fin & above(my_q) : 0ull;
    const uint32_t pe_lo = (uint32_t)pe_lane, pe_hi = (uint32_t)(pe_lane >> 32);
    const int qs_lane = my_q & 31;
    auto step = [&](const int l, const bool HIQ, const bool HIL) {
        const uint32_t pel = HIQ ? 0u : (uint32_t)readlane32((int)pe_lo, l);
        const uint32_t peh = (uint32_t)readlane32((int)pe_hi, l);
        // final: pivot l is reduced by pivots < l only
        const uint32_t hll = (uint32_t)readlane32((int)hPl, l), hlh = (uint32_t)readlane32((int)hPh, l);
        const uint32_t bl = 1u << (l & 31);
        const int sh = readlane32(qs_lane, l);
        const uint32_t mp = (uint32_t)__builtin_amdgcn_sbfe((int)(HIQ ? fLh : fLl), sh, 1);
        const uint32_t mv = (uint32_t)__builtin_amdgcn_sbfe((int)(HIQ ? vVh : vVl), sh, 1);
        const uint32_t md = (uint32_t)__builtin_amdgcn_sbfe((int)(HIQ ? vDh : vDl), sh, 1);
        hPl ^= hll & mp;
        hPh ^= hlh & mp;
        if (!HIQ) vVl ^= pel & mv;
        vVh ^= peh & mv;
        hVl ^= hll & mv;
        hVh ^= hlh & mv;
        if (!HIQ) vDl ^= pel & md;
        vDh ^= peh & md;
        hDl ^= hll & md;
        hDh ^= hlh & md;
        if (HIL) {
            uPh |= bl & mp;
            uVh |= bl & mv;
            uDh |= bl & md;
        } else {
            uPl |= bl & mp;
            uVl |= bl & mv;
            uDl |= bl & md;
        }
    };
    const int l32 = rbar < 32 ? rbar : 32;
    const int e1 = nlo < l32 ? nlo : l32;
    for (int l = 0; l < e1; l++) step(l, false, false);       // column < 32 implies l < 32
    for (int l = e1; l < l32; l++) step(l, true, false);
    for (int l = l32 > nlo ? l32 : nlo; l < rbar; l++) step(l, true, true);
    const uint64_t hP = ((uint64_t)hPh << 32) | hPl, uP = ((uint64_t)uPh << 32) | uPl;
    const uint64_t hV = ((uint64_t)hVh << 32) | hVl, uV = ((uint64_t)uVh << 32) | uVl;
    const uint64_t hD = ((uint64_t)hDh << 32) | hDl, uD = ((uint64_t)uDh << 32) | uDl;
    PANEL_STAMP(4)
    rec->img_w[lane] = hV;
    rec->img_u[lane] = uV;
    for (int kb = 0; kb < nspec; kb += 64) {
        const int k = kb + lane;
        if (k < nspec) {
            rec->spec_dst[k] = L.dst[k];
            rec->spec_src[k] = L.src[k];
        }
    }
    if (lane < ndisp) {
        rec->spec_coef[rbar + lane] = hD;
        rec->spec_lbits[rbar + lane] = uD;
        rec->spec_stripe[rbar + lane] = 0;
    }
    if (lane < rbar) {
        rec->spec_coef[lane] = hP ^ (1ull << lane);  // row of L11^-1 without its diagonal
        rec->spec_lbits[lane] = uP;                   // row of L11
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
    PANEL_STAMP(5)
#undef PANEL_STAMP
#undef PANEL_T0
#undef PANEL_ACC
}

}  // namespace gf2
