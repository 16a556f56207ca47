// Batched PLE: many independent matrices of uneven shape in one persistent
// launch per size class.  Each workgroup takes the next matrix from a queue
// (an atomic counter over a cost-ordered list) and runs Algorithm 2 on it
// alone: wave 0 runs the panel (Algorithm 1, the same device code as the
// single-matrix path), then the whole block applies the pass's swaps, writes
// coefficients and compressed L bits, and performs the Four-Russians trailing
// update (MakeTable + AddRowsFromTable, Appendix A) with its tables in LDS.
// Per-matrix results are therefore bit-identical to gf2_ple.
//
// The schedule -- waves per matrix, table width k (4 or 8 bits), tile width
// and the panel's register window -- is a template; a plan picks one per size
// class, from a built-in table or by timing the candidates (autotune).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "batch.h"
#include "m4rm.h"
#include "panel.h"

namespace gf2 {

// The batched kernels' panels search every row in place when their window
// runs out (no kept-row search): their waves are already near the register
// limit.
constexpr bool BATCH_KEPT = false;

// Staged special-row lists of one pass, and the nibble tables of the maps
// stripe word -> (w, u) for the other rows.
struct BPermLds {
    int64_t dst[MAX_SPEC], src[MAX_SPEC];
    uint64_t coef[MAX_SPEC], lbits[MAX_SPEC], stripe[MAX_SPEC];
    uint64_t tw[16][16], tu[16][16];
};

// Row swaps (special rows: read every word column, then write it, so the
// permutation is applied in place), pivot staging into PB, coefficients and
// compressed L bits of every row at or below r.
template <int NT>
__device__ __forceinline__ void batch_permute(uint64_t *__restrict__ A, int64_t m, int64_t ldw, int64_t nw, int64_t c,
                                              const PassRec *rec, uint64_t *__restrict__ coef,
                                              uint64_t *__restrict__ PB, BPermLds &L, int tid) {
    // the record was written by wave 0 in this launch: read it with relaxed
    // device-scope vector loads, never through the scalar cache
    const int64_t r = ld_dev(&rec->r);
    const int rbar = ld_dev(&rec->rbar);
    const int nspec = ld_dev(&rec->nspec);
    const int64_t sw = c >> 6;
    const int64_t wr0 = r >> 6;
    const int sh = (int)(r & 63);
    for (int k = tid; k < nspec; k += NT) {
        L.dst[k] = ld_dev(&rec->spec_dst[k]);
        L.src[k] = ld_dev(&rec->spec_src[k]);
        L.coef[k] = ld_dev(&rec->spec_coef[k]);
        L.lbits[k] = ld_dev(&rec->spec_lbits[k]);
        L.stripe[k] = ld_dev(&rec->spec_stripe[k]);
    }
    for (int e = tid; e < 256; e += NT) {
        const int t = e >> 4, x = e & 15;
        uint64_t a = 0, b = 0;
#pragma unroll
        for (int q = 0; q < 4; q++)
            if ((x >> q) & 1) {
                a ^= ld_dev(&rec->img_w[4 * t + q]);
                b ^= ld_dev(&rec->img_u[4 * t + q]);
            }
        L.tw[t][x] = a;
        L.tu[t][x] = b;
    }
    __syncthreads();

    // special rows, whole word columns per round
    constexpr int PER = 4;
    const int64_t cols = (NT * PER) / nspec > 0 ? (NT * PER) / nspec : 1;
    for (int64_t w0 = 0; w0 < nw; w0 += cols) {
        const int64_t wend = w0 + cols < nw ? w0 + cols : nw;
        const int items = (int)(wend - w0) * nspec;
        uint64_t nv[PER];
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int idx = tid + t * NT;
            nv[t] = 0;
            if (idx < items) {
                const int k = idx % nspec;
                const int64_t w = w0 + idx / nspec;
                const uint64_t old = A[L.src[k] * ldw + w];
                if (k < rbar && w > sw) PB[(int64_t)k * ldw + w] = old;
                nv[t] = special_word(old, w, sw, wr0, sh, L.lbits[k], L.stripe[k]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int idx = tid + t * NT;
            if (idx < items) {
                const int k = idx % nspec;
                const int64_t w = w0 + idx / nspec;
                if (L.dst[k] != L.src[k] || (w >= wr0 && w <= sw)) A[L.dst[k] * ldw + w] = nv[t];
            }
        }
        __syncthreads();
    }
    for (int k = tid; k < nspec; k += NT) coef[L.dst[k]] = L.coef[k];

    // every other row at or below r
    const int ndisp = nspec - rbar;
    int64_t maxdisp = -1;
    for (int d = 0; d < ndisp; d++) maxdisp = L.dst[rbar + d] > maxdisp ? L.dst[rbar + d] : maxdisp;
    for (int64_t i = r + rbar + tid; i < m; i += NT) {
        if (i <= maxdisp) {
            bool disp = false;
            for (int d = 0; d < ndisp; d++) disp |= L.dst[rbar + d] == i;
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
        for (int t = 0; t < 16; t++) {
            const int x = (int)((v >> (4 * t)) & 15);
            wv ^= L.tw[t][x];
            u ^= L.tu[t][x];
        }
        coef[i] = wv;
        if (wr0 < sw) {
            row[wr0] |= u << sh;
            if (sh && wr0 + 1 < sw) row[wr0 + 1] |= u >> (64 - sh);
        }
        row[sw] = place_bits(u, sw, wr0, sh);
    }
    __syncthreads();
}

// Table LDS of a schedule: 8-bit tables (M4Lds) or 4-bit tables (M4NLds).
template <int TB, int TW>
struct BTab;
template <int TW>
struct BTab<8, TW> {
    using type = M4Lds<TW>;
};
template <int TW>
struct BTab<4, TW> {
    using type = M4NLds<TW>;
};

// Trailing update of rows r..m-1, words right of the stripe, one tile of TW
// words at a time (tables rebuilt per tile from the staged pivot rows PB).
template <int NT, int TB, int TW, int U>
__device__ __forceinline__ void batch_update(uint64_t *__restrict__ A, int64_t m, int64_t ldw, int64_t nw, int64_t c,
                                             int64_t r, int rbar, const uint64_t *__restrict__ coef,
                                             const uint64_t *__restrict__ PB, typename BTab<TB, TW>::type &T,
                                             int tid) {
    const int64_t w_begin = (c >> 6) + 1, w_end = nw;
    for (int64_t wt0 = w_begin & ~(int64_t)(TW - 1); wt0 < w_end; wt0 += TW) {
        if constexpr (TB == 8) {
            m4_build_tables<TW, NT>(T, PB, ldw, rbar, wt0, w_begin, w_end, tid);
            m4_rows<TW, NT, U>(T, A, ldw, coef, 1, rbar, r, m, wt0, w_begin, w_end, tid);
        } else {
            m4n_build_tables<TW, NT>(T, PB, ldw, rbar, wt0, w_begin, w_end, tid);
            m4n_rows<TW, NT, U>(T, A, ldw, coef, rbar, r, m, wt0, w_begin, w_end, tid);
        }
        __syncthreads();
    }
}

template <int NW, int TB, int TW, int WQ, int U>
__global__ __launch_bounds__(NW * 64) void k_batch(BatchArgs a) {
    constexpr int NT = NW * 64;
    __shared__ PanelLdsT<0> PL;
    __shared__ BPermLds BL;
    __shared__ typename BTab<TB, TW>::type TL;
    __shared__ int s_next;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint8_t *slot = a.slots + (int64_t)blockIdx.x * a.lay.bytes;
    PassRec *rec = (PassRec *)slot;
    uint64_t *coef = (uint64_t *)(slot + a.lay.coef);
    uint64_t *PB = (uint64_t *)(slot + a.lay.pb);
    uint64_t *gsv = (uint64_t *)(slot + a.lay.gsv);
    int32_t *gsid = (int32_t *)(slot + a.lay.gsid);

    for (;;) {
        if (tid == 0) s_next = atomicAdd(a.counter, 1);
        __syncthreads();
        const int qi = s_next;
        __syncthreads();
        if (qi >= a.count) break;
        const int mi = a.order[qi];
        const gf2_desc d = a.descs[mi];
        uint64_t *A = a.arena + d.a_off;
        int64_t *P = a.P + d.p_off;
        int64_t *Q = a.Q + d.q_off;
        int64_t *rank = a.ranks + (a.rank_off ? a.rank_off[mi] : (int64_t)mi);
        const int64_t m = d.m, n = d.n, ldw = d.ldw;
        const int64_t mn = m < n ? m : n;
        for (int64_t i = tid; i < m; i += NT) P[i] = i;
        for (int64_t i = tid; i < mn; i += NT) Q[i] = -1;
        if (tid == 0) {
            rec->r = 0;
            rec->rbar = 0;
            rec->nspec = 0;
            rec->active = 0;
            rec->slow = 0;
            *rank = 0;
        }
        __syncthreads();
        const int64_t nw = words_for(n);
        for (int64_t c = 0; c < n && m > 0; c += KW) {
            if (wave == 0) panel_body<WQ, 0, BATCH_KEPT>(A, m, n, ldw, c, rec, rec, P, Q, rank, gsv, gsid, PL, lane);
            __syncthreads();
            const int active = ld_dev(&rec->active);
            const int64_t r = ld_dev(&rec->r);
            const int rbar = ld_dev(&rec->rbar);
            if (active) {
                batch_permute<NT>(A, m, ldw, nw, c, rec, coef, PB, BL, tid);
                batch_update<NT, TB, TW, U>(A, m, ldw, nw, c, r, rbar, coef, PB, TL, tid);
            }
            __syncthreads();  // every thread has read rec before the next panel writes it
            if (r + rbar >= m) break;
        }
        __syncthreads();
    }
}

__global__ void k_batch_reset(int32_t *counters, int n) {
    const int i = threadIdx.x;
    if (i < n) counters[i] = 0;
}

// ---------------------------------------------------------------------------
// Schedules.
// ---------------------------------------------------------------------------
struct BatchConfig {
    int nw, tb, tw, wq, u;
    const char *name;
};

static const BatchConfig kBatchConfigs[] = {
    {1, 4, 8, 2, 2, "w1_k4_tw8_q2"},   {2, 4, 8, 2, 2, "w2_k4_tw8_q2"},   {4, 4, 8, 2, 2, "w4_k4_tw8_q2"},
    {4, 8, 1, 2, 4, "w4_k8_tw1_q2"},   {4, 4, 16, 4, 2, "w4_k4_tw16_q4"}, {8, 8, 2, 4, 4, "w8_k8_tw2_q4"},
    {8, 4, 16, 8, 2, "w8_k4_tw16_q8"}, {8, 8, 4, 8, 2, "w8_k8_tw4_q8"},
};
static_assert(sizeof(kBatchConfigs) / sizeof(kBatchConfigs[0]) == NBATCH_CONFIGS, "schedule table");

template <int NW, int TB, int TW, int WQ, int U>
static hipError_t batch_launch_t(int grid, const BatchArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_batch<NW, TB, TW, WQ, U>), dim3(grid), dim3(NW * 64), 0, s, a);
    return hipGetLastError();
}

template <int NW, int TB, int TW, int WQ, int U>
static int batch_occupancy_t() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<NW, TB, TW, WQ, U>, NW * 64, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

#define GF2_BATCH_CONFIGS(X)   \
    X(0, 1, 4, 8, 2, 2)        \
    X(1, 2, 4, 8, 2, 2)        \
    X(2, 4, 4, 8, 2, 2)        \
    X(3, 4, 8, 1, 2, 4)        \
    X(4, 4, 4, 16, 4, 2)       \
    X(5, 8, 8, 2, 4, 4)        \
    X(6, 8, 4, 16, 8, 2)       \
    X(7, 8, 8, 4, 8, 2)

hipError_t batch_launch(int cfg, int grid, const BatchArgs &a, hipStream_t s) {
#define X(ID, NW, TB, TW, WQ, U) \
    case ID:                     \
        return batch_launch_t<NW, TB, TW, WQ, U>(grid, a, s);
    switch (cfg) {
        GF2_BATCH_CONFIGS(X)
        default:
            return hipErrorInvalidValue;
    }
#undef X
}

int batch_occupancy(int cfg) {
#define X(ID, NW, TB, TW, WQ, U) \
    case ID:                     \
        return batch_occupancy_t<NW, TB, TW, WQ, U>();
    switch (cfg) {
        GF2_BATCH_CONFIGS(X)
        default:
            return 1;
    }
#undef X
}

// Fill the k x words region of each matrix of a temporary arena with
// pseudo-random bits (SplitMix64 of the word index), padding bits zero.
__global__ void k_batch_fill(uint64_t *arena, const gf2_desc *descs, int count, uint64_t salt) {
    for (int mi = blockIdx.x; mi < count; mi += gridDim.x) {
        const gf2_desc d = descs[mi];
        const int64_t nw = words_for(d.n);
        const int tail = (int)(d.n & 63);
        for (int64_t e = threadIdx.x; e < d.m * d.ldw; e += blockDim.x) {
            const int64_t i = e / d.ldw, w = e % d.ldw;
            uint64_t z = (uint64_t)(d.a_off + e) * 0x9E3779B97F4A7C15ull + salt;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            if (w >= nw) z = 0;
            else if (w == nw - 1 && tail) z &= (1ull << tail) - 1;
            arena[d.a_off + i * d.ldw + w] = z;
        }
    }
}

hipError_t batch_reset(int32_t *counters, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, counters, n);
    return hipGetLastError();
}

SlotLayout batch_slot_layout(int64_t mmax, int64_t ldwmax) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    SlotLayout L;
    size_t off = al(sizeof(PassRec));
    L.coef = (int64_t)off;
    off += al((size_t)(mmax > 0 ? mmax : 1) * 8);
    L.pb = (int64_t)off;
    off += al((size_t)KW * (size_t)(ldwmax > 0 ? ldwmax : 1) * 8);
    L.gsv = (int64_t)off;
    off += al((size_t)(mmax > 0 ? mmax : 1) * 8);
    L.gsid = (int64_t)off;
    off += al((size_t)(mmax > 0 ? mmax : 1) * 4);
    L.bytes = (int64_t)off;
    return L;
}

// Size classes by the larger side, and the built-in schedule of each (from
// autotuning the 4096-matrix uneven batch on MI355X).
static const int64_t kClassMax[] = {256, 512, 1024, 2048, 4096, INT64_MAX};
constexpr int NCLASS = (int)(sizeof(kClassMax) / sizeof(kClassMax[0]));
static const int kClassDefault[NCLASS] = {3, 2, 3, 2, 6, 7};

int batch_default_config(int64_t max_dim) {
    int k = 0;
    while (k + 1 < NCLASS && max_dim > kClassMax[k]) k++;
    return kClassDefault[k];
}

}  // namespace gf2

using namespace gf2;

namespace {

constexpr size_t BALIGN = 256;
size_t balign(size_t x) { return (x + BALIGN - 1) & ~(BALIGN - 1); }

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

}  // namespace

struct gf2_batch_plan {
    struct Class {
        int64_t max_dim = 0;
        std::vector<int32_t> idx;  // matrices, most expensive first
        int64_t order_off = 0;     // into d_order
        int64_t mmax = 0, ldwmax = 0;
        int cfg = 0;
        int grid = 0;
        double tuned_ms = 0.0;
        SlotLayout lay{};
        size_t ws_off = 0;
        size_t ws_len = 0;
    };
    std::vector<gf2_desc> descs;
    gf2_desc *d_descs = nullptr;
    int32_t *d_order = nullptr;
    std::vector<Class> classes;
    size_t ws_bytes = 0;
    bool use_graph = true;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

namespace {

// Grid and workspace of each class for its current schedule.
void plan_layout(gf2_batch_plan *p) {
    const int cus = device_cu_count();
    size_t off = balign(64 * sizeof(int32_t));  // queue counters
    for (auto &c : p->classes) {
        const int occ = batch_occupancy(c.cfg);
        const int64_t slots = (int64_t)occ * cus;
        c.grid = (int)std::min<int64_t>((int64_t)c.idx.size(), slots);
        c.lay = batch_slot_layout(c.mmax, c.ldwmax);
        c.ws_off = off;
        c.ws_len = balign((size_t)c.grid * (size_t)c.lay.bytes);
        off += c.ws_len;
    }
    p->ws_bytes = off;
}

hipError_t plan_enqueue(gf2_batch_plan *p, uint64_t *arena, int64_t *P, int64_t *Q, int64_t *ranks, uint8_t *ws,
                        hipStream_t s) {
    int32_t *counters = (int32_t *)ws;
    hipError_t e = batch_reset(counters, (int)p->classes.size(), s);
    if (e != hipSuccess) return e;
    for (size_t ci = 0; ci < p->classes.size(); ci++) {
        auto &c = p->classes[ci];
        if (c.idx.empty()) continue;
        BatchArgs a;
        a.descs = p->d_descs;
        a.order = p->d_order + c.order_off;
        a.rank_off = nullptr;
        a.count = (int32_t)c.idx.size();
        a.counter = counters + ci;
        a.arena = arena;
        a.P = P;
        a.Q = Q;
        a.ranks = ranks;
        a.slots = ws + c.ws_off;
        a.lay = c.lay;
        e = batch_launch(c.cfg, c.grid, a, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void plan_drop_graph(gf2_batch_plan *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    p->exec = nullptr;
    for (auto &k : p->key) k = nullptr;
}

// Time every schedule on each class, on synthetic matrices of the class's
// own shapes in a temporary arena; keep the fastest.
gf2_status plan_autotune(gf2_batch_plan *p) {
    hipStream_t s = p->cap;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return GF2_EHIP;
    gf2_status st = GF2_OK;
    for (auto &c : p->classes) {
        if (c.idx.empty()) continue;
        // compact copy of the class's descriptors
        std::vector<gf2_desc> td(c.idx.size());
        int64_t aw = 0, pl = 0, ql = 0;
        for (size_t k = 0; k < c.idx.size(); k++) {
            gf2_desc d = p->descs[c.idx[k]];
            d.a_off = aw;
            d.p_off = pl;
            d.q_off = ql;
            aw += (d.m * d.ldw + 31) & ~(int64_t)31;
            pl += d.m;
            ql += std::min(d.m, d.n);
            td[k] = d;
        }
        gf2_desc *dd = nullptr;
        int32_t *dord = nullptr;
        uint64_t *arena = nullptr;
        int64_t *P = nullptr, *Q = nullptr, *R = nullptr;
        uint8_t *ws = nullptr;
        gf2_batch_plan sub;
        sub.descs = td;
        sub.classes.push_back(c);
        auto &sc = sub.classes[0];
        std::vector<int32_t> ord(td.size());
        for (size_t k = 0; k < td.size(); k++) ord[k] = (int32_t)k;
        sc.idx = ord;
        sc.order_off = 0;
        size_t ws_max = 0;
        for (int cfg = 0; cfg < NBATCH_CONFIGS; cfg++) {
            sc.cfg = cfg;
            plan_layout(&sub);
            ws_max = std::max(ws_max, sub.ws_bytes);
        }
        bool ok = hipMalloc(&dd, td.size() * sizeof(gf2_desc)) == hipSuccess &&
                  hipMalloc(&dord, ord.size() * sizeof(int32_t)) == hipSuccess &&
                  hipMalloc(&arena, (size_t)std::max<int64_t>(aw, 1) * 8) == hipSuccess &&
                  hipMalloc(&P, (size_t)std::max<int64_t>(pl, 1) * 8) == hipSuccess &&
                  hipMalloc(&Q, (size_t)std::max<int64_t>(ql, 1) * 8) == hipSuccess &&
                  hipMalloc(&R, td.size() * 8) == hipSuccess && hipMalloc(&ws, ws_max) == hipSuccess;
        ok = ok && hipMemcpy(dd, td.data(), td.size() * sizeof(gf2_desc), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(dord, ord.data(), ord.size() * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess;
        sub.d_descs = dd;
        sub.d_order = dord;
        double best = 1e300;
        int best_cfg = c.cfg;
        for (int cfg = 0; ok && cfg < NBATCH_CONFIGS; cfg++) {
            sc.cfg = cfg;
            plan_layout(&sub);
            float ms_min = 1e30f;
            for (int rep = 0; ok && rep < 3; rep++) {
                hipLaunchKernelGGL(k_batch_fill, dim3(std::min<size_t>(td.size(), 4096)), dim3(256), 0, s, arena, dd,
                                   (int)td.size(), (uint64_t)(rep + 1));
                ok = ok && hipEventRecord(e0, s) == hipSuccess;
                ok = ok && plan_enqueue(&sub, arena, P, Q, R, ws, s) == hipSuccess;
                ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
                float ms = 0;
                ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                if (rep > 0) ms_min = std::min(ms_min, ms);  // first run warms up
            }
            if (ok && ms_min < best) {
                best = ms_min;
                best_cfg = cfg;
            }
        }
        sub.d_descs = nullptr;
        sub.d_order = nullptr;
        (void)hipFree(dd);
        (void)hipFree(dord);
        (void)hipFree(arena);
        (void)hipFree(P);
        (void)hipFree(Q);
        (void)hipFree(R);
        (void)hipFree(ws);
        if (!ok) {
            st = GF2_EHIP;
            break;
        }
        c.cfg = best_cfg;
        c.tuned_ms = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // namespace

extern "C" {

int32_t gf2_batch_num_configs(void) { return NBATCH_CONFIGS; }

const char *gf2_batch_config_name(int32_t config) {
    if (config < 1 || config > NBATCH_CONFIGS) return "";
    return kBatchConfigs[config - 1].name;
}

gf2_status gf2_batch_plan_create(const gf2_desc *descs, int64_t count, int64_t arena_words, int64_t p_len,
                                 int64_t q_len, const gf2_batch_opts *opts, gf2_batch_plan **plan) {
    if (!plan || count < 0 || (count > 0 && !descs) || count > INT32_MAX) return GF2_EINVAL;
    *plan = nullptr;
    gf2_batch_opts o{};
    if (opts) o = *opts;
    if (o.config < 0 || o.config > NBATCH_CONFIGS) return GF2_EINVAL;
    for (int64_t i = 0; i < count; i++) {
        const gf2_desc &d = descs[i];
        if (d.m < 0 || d.n < 0 || d.ldw < words_for(d.n) || d.a_off < 0 || d.p_off < 0 || d.q_off < 0) return GF2_EINVAL;
        if (d.m > INT32_MAX || d.n > INT32_MAX) return GF2_EINVAL;
        if (d.m > 0 && d.ldw > 0 && (d.ldw > (arena_words - d.a_off) / d.m)) return GF2_EINVAL;
        if (d.a_off > arena_words || d.p_off + d.m > p_len || d.q_off + std::min(d.m, d.n) > q_len) return GF2_EINVAL;
    }
    gf2_batch_plan *p = new (std::nothrow) gf2_batch_plan();
    if (!p) return GF2_ENOMEM;
    p->descs.assign(descs, descs + count);
    p->use_graph = o.no_graph == 0;
    p->classes.resize(NCLASS);
    for (int k = 0; k < NCLASS; k++) {
        p->classes[k].max_dim = kClassMax[k];
        p->classes[k].cfg = o.config > 0 ? o.config - 1 : kClassDefault[k];
    }
    std::vector<double> cost(count);
    for (int64_t i = 0; i < count; i++) {
        const gf2_desc &d = p->descs[i];
        const int64_t big = std::max(d.m, d.n);
        int k = 0;
        while (big > kClassMax[k]) k++;
        auto &c = p->classes[k];
        c.idx.push_back((int32_t)i);
        c.mmax = std::max(c.mmax, d.m);
        c.ldwmax = std::max(c.ldwmax, d.ldw);
        cost[i] = (double)d.m * (double)words_for(d.n) * (double)std::min(d.m, d.n) + 1.0;
    }
    std::vector<int32_t> order;
    order.reserve(count);
    for (auto &c : p->classes) {
        std::stable_sort(c.idx.begin(), c.idx.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
        c.order_off = (int64_t)order.size();
        order.insert(order.end(), c.idx.begin(), c.idx.end());
    }
    gf2_status st = GF2_OK;
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) st = GF2_EHIP;
    if (st == GF2_OK && count > 0) {
        if (hipMalloc(&p->d_descs, (size_t)count * sizeof(gf2_desc)) != hipSuccess ||
            hipMalloc(&p->d_order, (size_t)count * sizeof(int32_t)) != hipSuccess ||
            hipMemcpy(p->d_descs, p->descs.data(), (size_t)count * sizeof(gf2_desc), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(p->d_order, order.data(), (size_t)count * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
            st = GF2_EHIP;
    }
    if (st == GF2_OK && o.autotune && o.config == 0 && count > 0) st = plan_autotune(p);
    if (st != GF2_OK) {
        gf2_batch_plan_destroy(p);
        return st;
    }
    plan_layout(p);
    *plan = p;
    return GF2_OK;
}

size_t gf2_batch_workspace_bytes(const gf2_batch_plan *plan) { return plan ? plan->ws_bytes : 0; }

gf2_status gf2_ple_batched(gf2_batch_plan *plan, uint64_t *arena, int64_t *P, int64_t *Q, int64_t *ranks, void *ws,
                           size_t ws_bytes, void *stream) {
    if (!plan) return GF2_EINVAL;
    if (plan->descs.empty()) return GF2_OK;
    if (!arena || !P || !Q || !ranks || !ws) return GF2_EINVAL;
    if (((uintptr_t)arena & 7) || ((uintptr_t)P & 7) || ((uintptr_t)Q & 7) || ((uintptr_t)ranks & 7) ||
        ((uintptr_t)ws & (BALIGN - 1)))
        return GF2_EINVAL;
    if (ws_bytes < plan->ws_bytes) return GF2_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (!plan->use_graph) {
        ProfScope ps(KID_BATCH, s);
        return plan_enqueue(plan, arena, P, Q, ranks, (uint8_t *)ws, s) == hipSuccess ? GF2_OK : GF2_EHIP;
    }
    const void *key[5] = {arena, P, Q, ranks, ws};
    bool same = plan->exec != nullptr;
    for (int k = 0; k < 5; k++) same = same && plan->key[k] == key[k];
    if (!same) {
        plan_drop_graph(plan);
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return GF2_EHIP;
        const hipError_t le = plan_enqueue(plan, arena, P, Q, ranks, (uint8_t *)ws, plan->cap);
        const hipError_t ce = hipStreamEndCapture(plan->cap, &g);
        if (le != hipSuccess || ce != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return GF2_EHIP;
        }
        const hipError_t ie = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            plan->exec = nullptr;
            return GF2_EHIP;
        }
        for (int k = 0; k < 5; k++) plan->key[k] = key[k];
    }
    ProfScope ps(KID_BATCH, s);
    return hipGraphLaunch(plan->exec, s) == hipSuccess ? GF2_OK : GF2_EHIP;
}

gf2_status gf2_batch_plan_info(const gf2_batch_plan *plan, gf2_batch_class *out, int32_t max, int32_t *nclasses) {
    if (!plan || !nclasses || (max > 0 && !out)) return GF2_EINVAL;
    int32_t k = 0;
    for (const auto &c : plan->classes) {
        if (k < max) {
            out[k].max_dim = c.max_dim;
            out[k].count = (int64_t)c.idx.size();
            out[k].config = c.cfg + 1;
            out[k].grid = c.grid;
            out[k].tuned_ms = c.tuned_ms;
        }
        k++;
    }
    *nclasses = k;
    return GF2_OK;
}

gf2_status gf2_batch_plan_destroy(gf2_batch_plan *plan) {
    if (!plan) return GF2_EINVAL;
    plan_drop_graph(plan);
    if (plan->d_descs) (void)hipFree(plan->d_descs);
    if (plan->d_order) (void)hipFree(plan->d_order);
    if (plan->cap) (void)hipStreamDestroy(plan->cap);
    delete plan;
    return GF2_OK;
}

}  // extern "C"
