// C-ABI entry points of libgf2ple (declared in include/gf2ple.h): argument
// checks, workspace layout and the pass loop of Algorithm 2.  All arithmetic
// runs in the HIP kernels of ple_kernels.hip / rref_kernels.hip.
#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/gf2ple.h"
#include "alg3.h"
#include "batch.h"
#include "common.h"
#include "m4ri_jobs.h"
#include "panel.h"

namespace gf2 {
hipError_t launch_init(int64_t *P, int64_t m, int64_t *Q, int64_t mn, int64_t *rank, PassRec *rec, hipStream_t s);
hipError_t launch_panel(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t c, const PassRec *prev, PassRec *rec,
                        int64_t *P, int64_t *Q, int64_t *rank, uint64_t *gsv, int32_t *gsid, int panel_regs,
                        const PanelFix &fix, bool beside, hipStream_t s, hipEvent_t done);
hipError_t launch_permute(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t c, PassRec *rec,
                          uint64_t *coef, uint64_t *PB, int mode, const PassRec *rect, const uint64_t *coefT,
                          uint64_t *coefP, const uint64_t *PBt, hipStream_t s, hipEvent_t done, int64_t wlo);
hipError_t launch_update_pair(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t ct, const PassRec *rect,
                              const PassRec *recu, const uint64_t *coefP, const uint64_t *coefU,
                              const uint64_t *coefT, const uint64_t *PBt, const uint64_t *PBu, int m4_target,
                              int pair_variant, const PairPanel &pp, hipStream_t s);
hipError_t launch_update(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t c, const PassRec *rec,
                         const uint64_t *coef, const uint64_t *PB, int first, int m4_variant, int m4_target,
                         hipStream_t s);
hipError_t launch_transpose_bits(const uint64_t *B, int64_t ldb, int64_t k, int64_t n, uint64_t *Bt, int64_t ldbt,
                                 hipStream_t s);
hipError_t launch_mfma_gf2(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda, const uint64_t *Bt, int64_t ldbt,
                           int64_t m, int64_t k, int64_t n, hipStream_t s, int fmt);
hipError_t launch_m4rm(uint64_t *C, int64_t ldc, int64_t m, const uint64_t *coef, int64_t coef_ld, const uint64_t *B,
                       int64_t ldb, int nbits, int64_t w_begin, int64_t w_end, int m4_variant, int m4_target,
                       hipStream_t s);
hipError_t launch_echelon(uint64_t *A, int64_t m, int64_t ldw, const int64_t *rank, hipStream_t s);
hipError_t launch_padding(const uint64_t *A, int64_t m, int64_t n, int64_t ldw, int *flag, hipStream_t s);
hipError_t launch_make_table(const uint64_t *rows, int64_t ldr, int k, int64_t nw, uint64_t *T, int64_t ldt,
                             hipStream_t s);
hipError_t launch_rref_block(uint64_t *A, int64_t ldw, int64_t nw, const int64_t *Q, int64_t j0, int64_t j1,
                             int64_t ws0, int64_t q0, int64_t jz, uint64_t *coef, uint64_t *PB, PassRec *rec,
                             hipStream_t s, const PassRec *drec = nullptr);
hipError_t launch_rref_block2(uint64_t *A, int64_t ldw, int64_t nw, const int64_t *Q, int64_t ws0, int64_t jz,
                              int64_t j0a, int64_t j1a, int64_t q0a, uint64_t *coefa, uint64_t *PBa, PassRec *reca,
                              int64_t j0b, int64_t j1b, int64_t q0b, uint64_t *coefb, uint64_t *PBb, PassRec *recb,
                              hipStream_t s, const PassRec *dreca = nullptr, const PassRec *drecb = nullptr);
hipError_t launch_rref_pair(uint64_t *A, int64_t ldw, int64_t m, const uint64_t *coefT, const uint64_t *coefU,
                            const uint64_t *PBt, const uint64_t *PBu, int64_t w_begin, int64_t w_end,
                            const PassRec *rect, const PassRec *recu, hipStream_t s);
}  // namespace gf2

using namespace gf2;

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

struct PleLayout {
    size_t rec, coef, coefp, coef2, pb, pb2, gsv, gsid, total;
};

// workspace of gf2_ple: pass records (a ring of NREC) | coef[m] | coefP[m] |
// coef2[m] | pivot block 64 x ldw | second pivot block | slow-search
// values[m] | slow-search ids[m], positions[m] and per-64-row group counts.
// coefP, coef2 and the second pivot block serve the fused update of a pair
// of passes.
PleLayout ple_layout(int64_t m, int64_t ldw) {
    PleLayout L;
    size_t off = 0;
    L.rec = off;
    off += align_up(NREC * sizeof(PassRec));
    L.coef = off;
    off += align_up((size_t)m * 8);
    L.coefp = off;
    off += align_up((size_t)m * 8);
    L.coef2 = off;
    off += align_up((size_t)m * 8);
    L.pb = off;
    off += align_up((size_t)KW * (size_t)ldw * 8);
    L.pb2 = off;
    off += align_up((size_t)KW * (size_t)ldw * 8);
    L.gsv = off;
    off += align_up((size_t)m * 8);
    L.gsid = off;
    off += align_up((size_t)m * 8 + ((size_t)m / 64 + 2) * 4);
    L.total = off;
    return L;
}

// workspace of gf2_rref_from_ple: coef[m] | second block's coef[m] | pivot
// block 64 x ldw | second pivot block | two block records (a fused pair of
// blocks per sweep)
struct RrefLayout {
    size_t coef, coef2, pb, pb2, rec, total;
};
RrefLayout rref_layout(int64_t m, int64_t ldw) {
    RrefLayout L;
    L.coef = 0;
    L.coef2 = align_up((size_t)m * 8);
    L.pb = L.coef2 + align_up((size_t)m * 8);
    L.pb2 = L.pb + align_up((size_t)KW * (size_t)ldw * 8);
    L.rec = L.pb2 + align_up((size_t)KW * (size_t)ldw * 8);
    L.total = L.rec + align_up(2 * sizeof(PassRec));
    return L;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// sizes: m, n >= 0, ldw >= ceil(n/64), m * ldw * 8 representable
bool sizes_ok(int64_t m, int64_t n, int64_t ldw) {
    if (m < 0 || n < 0 || ldw < 0) return false;
    if (ldw < words_for(n)) return false;
    if (ldw > 0 && m > (int64_t)(INT64_MAX / 8) / ldw) return false;
    if (m > (int64_t)INT32_MAX) return false;  // positions are kept as int32 in the slow search
    return true;
}

gf2_status hip_status(hipError_t e) { return e == hipSuccess ? GF2_OK : GF2_EHIP; }

// Per device: one int for the padding scan.  g_flag_mu is held for the whole
// scan (clear, launch, read back), so concurrent scans on one device take
// turns instead of sharing the flag.
std::mutex g_flag_mu;
std::vector<int *> g_flag;

int *device_flag_locked() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    if ((int)g_flag.size() <= dev) g_flag.resize(dev + 1, nullptr);
    if (!g_flag[dev]) {
        int *p = nullptr;
        if (hipMalloc(&p, sizeof(int)) != hipSuccess) return nullptr;
        g_flag[dev] = p;
    }
    return g_flag[dev];
}

}  // namespace

namespace gf2 {

// The second stream of the look-ahead and of the M4RI form's eliminations,
// and the events that order it against the caller's stream: made by the
// call that needs them and released when it returns (a stream or event
// still in use then is released once its work completes).  No stream of
// the library outlives a call, so a process's later streams (a serving
// session's, say) get the hardware queues as if the call had not run, and
// calls from different host threads share nothing.
struct LookCtx {
    hipStream_t s2 = nullptr;
    hipEvent_t evA = nullptr, evN = nullptr;
    hipEvent_t evJ[NREC] = {};  // M4RI: one per elimination job in flight
    LookCtx() = default;
    LookCtx(const LookCtx &) = delete;
    LookCtx &operator=(const LookCtx &) = delete;
    ~LookCtx() {
        if (evA) (void)hipEventDestroy(evA);
        if (evN) (void)hipEventDestroy(evN);
        for (int j = 0; j < NREC; j++)
            if (evJ[j]) (void)hipEventDestroy(evJ[j]);
        if (s2) (void)hipStreamDestroy(s2);
    }
    bool init() {
        if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess) {
            s2 = nullptr;
            return false;
        }
        // the events only order the two streams on this device: a
        // device-scope release and no timestamps (a default event also
        // writes back the caches for the host, which delays the next kernel
        // by microseconds)
        constexpr unsigned EV_FLAGS = hipEventDisableTiming | hipEventReleaseToDevice;
        bool ok = hipEventCreateWithFlags(&evA, EV_FLAGS) == hipSuccess &&
                  hipEventCreateWithFlags(&evN, EV_FLAGS) == hipSuccess;
        for (int j = 0; ok && j < NREC; j++) ok = hipEventCreateWithFlags(&evJ[j], EV_FLAGS) == hipSuccess;
        return ok;
    }
};

// Trailing blocks above this many bytes take the look-ahead in the default
// mode when a pass is not paired: their update outlasts the next panel.
constexpr double LOOKAHEAD_BYTES = 64.0 * 1024 * 1024;

size_t ple_workspace_total(int64_t m, int64_t ldw) { return ple_layout(m, ldw).total; }

// How each 64-column pass is run (host decision, made before any launch):
// serial; look-ahead (its update starts at the stripe + 2, the next panel
// runs beside it); or a fused pair (the first pass has no update, the second
// pass's update covers both from the first stripe + 3).  mode = the
// lookahead option (1: serial only).
enum PassKind { PK_SERIAL = 0, PK_LOOK = 1, PK_PAIR1 = 2, PK_PAIR2 = 3 };

static void pass_kinds(int64_t m, int64_t n, int mode, std::vector<int8_t> &kind) {
    const int64_t npasses = words_for(n);
    kind.assign((size_t)npasses, (int8_t)PK_SERIAL);
    auto rows = [&](int64_t t) {
        const int64_t c = t * KW;
        return m - (c < m ? c : m);
    };
    auto big = [&](int64_t t) { return (double)rows(t) * (double)(npasses - t - 2) * 8.0 > LOOKAHEAD_BYTES; };
    for (int64_t t = 0; t < npasses;) {
        // pairs while rows remain below the stripe (past that, the serial
        // loop stops as soon as the rank reaches m)
        if ((mode == 0 || mode == 3) && t + 3 < npasses && (mode == 3 || rows(t + 1) > 0)) {
            kind[t] = PK_PAIR1;
            kind[t + 1] = PK_PAIR2;
            t += 2;
            continue;
        }
        if (mode != 1 && t + 1 < npasses && (mode >= 2 || big(t))) kind[t] = PK_LOOK;
        t += 1;
    }
}

// The pass loop of Algorithm 2.  Pass t: panel(t) (Algorithm 1 on the stripe
// at c = 64 t), permute(t) (swaps, coefficients, compressed L bits), then the
// trailing update.  With look-ahead the next stripe word is brought up to
// date by permute(t) (ordinary rows) and panel(t + 1) (the pass's special
// rows), so panel(t + 1) -- which reads only that word -- runs on a second
// stream beside the update of the words beyond; the next permute waits for
// both.
// The M4RI form (Algorithms 5-8: every column block eliminated from all
// rows): after each pass (or fused pair of passes, a 128-column block), the
// block's pivot rows are brought to reduced form and removed from the rows
// above, with the back-substitution's kernels (coefficients, staged pivot
// rows and two records of its own).
struct M4riStep {
    uint64_t *coef = nullptr, *coef2 = nullptr;
    uint64_t *PB = nullptr, *PB2 = nullptr;
    PassRec *rec = nullptr;  // two
};

// wlo: first word of A's rows relative to A (0, or < 0 when A points at a
// right-hand block of a matrix): the swaps move the whole rows, words
// [wlo, wlo + ldw), while the passes eliminate only A's n columns.
static hipError_t pass_loop(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank,
                            void *ws, const gf2_ple_opts *opts, hipStream_t s, bool allow_sync, bool allow_s2,
                            const M4riStep *m4ri, int64_t wlo = 0) {
    const PleLayout L = ple_layout(m, ldw);
    const int64_t mn = m < n ? m : n;
    char *base = (char *)ws;
    PassRec *recs = (PassRec *)(base + L.rec);
    uint64_t *coef = (uint64_t *)(base + L.coef);
    uint64_t *coefP = (uint64_t *)(base + L.coefp);
    uint64_t *coef2 = (uint64_t *)(base + L.coef2);
    uint64_t *PB = (uint64_t *)(base + L.pb);
    uint64_t *PB2 = (uint64_t *)(base + L.pb2);
    uint64_t *gsv = (uint64_t *)(base + L.gsv);
    int32_t *gsid = (int32_t *)(base + L.gsid);
    const int m4v = opts ? opts->m4_variant : 0;
    const int m4t = opts ? opts->m4_blocks : 0;
    const int pr = opts ? opts->panel_regs : 0;
    const int mode = opts ? opts->lookahead : 0;
    const int pv = opts ? opts->pair_variant : 0;

    hipError_t e = launch_init(P, m, Q, mn, rank, recs, s);
    if (e != hipSuccess) return e;
    if (m == 0 || n == 0) return hipSuccess;

    const int64_t npasses = words_for(n);
    std::vector<int8_t> kind;
    pass_kinds(m, n, mode, kind);
    // the M4RI form keeps the second stream for its eliminations
    if (m4ri)
        for (auto &k : kind)
            if (k == PK_LOOK) k = PK_SERIAL;
    // the second stream serves look-ahead passes and the M4RI form's
    // eliminations; without it look-ahead passes run serially and the
    // eliminations on the caller's stream
    LookCtx ctx;
    const bool want_s2 = m4ri || std::find(kind.begin(), kind.end(), (int8_t)PK_LOOK) != kind.end();
    const bool have_s2 = allow_s2 && want_s2 && ctx.init();
    LookCtx *lc = have_s2 && !m4ri ? &ctx : nullptr;
    if (!lc)
        for (auto &k : kind)
            if (k == PK_LOOK) k = PK_SERIAL;
    auto want_pair = [&](int64_t t) { return kind[t] == PK_PAIR1; };
    auto want_la = [&](int64_t t) { return kind[t] == PK_LOOK; };
    auto rec_of = [&](int64_t t) { return &recs[t % NREC]; };
    if ((e = launch_panel(A, m, n, ldw, 0, rec_of(NREC - 1), rec_of(0), P, Q, rank, gsv, gsid, pr, PanelFix(), false,
                          s, nullptr)) != hipSuccess)
        return e;
    bool pending = false;  // this pass's panel ran on the second stream
    int64_t since_check = 0;
    // M4RI: a block's elimination from the rows above (a job) runs on the
    // second stream, behind the passes that follow it.  It writes only rows
    // above the next pass's first row (rows whose coefficients are zero are
    // not written), which no later pass touches.  It reads its passes'
    // records, so before a kernel writes the record of pass x, every job
    // that read the slot x shares in the ring (passes <= x - NREC) is done.
    LookCtx *mc = have_s2 && m4ri ? &ctx : nullptr;
    M4JobRing<NREC> jobs;
    auto m4_guard = [&](int64_t x) -> hipError_t {
        const int ev = jobs.guard(x);
        return ev >= 0 ? hipStreamWaitEvent(s, mc->evJ[ev], 0) : hipSuccess;
    };
    // a job over passes [t, t + np): both blocks' reduction and removal from
    // rows 0 .. min(c + 64 np, m) - 1 (rows r .. r + rbar - 1 of the passes
    // lie below c + 64 np, since r <= c)
    auto m4_job = [&](int64_t t, int np) -> hipError_t {
        const int64_t c = t * KW;
        const int64_t jz = c + np * KW < m ? c + np * KW : m;
        hipStream_t ms = mc ? mc->s2 : s;
        hipError_t err;
        if (mc) {
            if ((err = hipEventRecord(mc->evA, s)) != hipSuccess) return err;
            if ((err = hipStreamWaitEvent(ms, mc->evA, 0)) != hipSuccess) return err;
        }
        if (np == 2) {
            // the later block first (its update leaves the earlier block's
            // pivot columns as they are), the earlier block's rows taking it
            // in the sweep's table build, as in the back-substitution
            if ((err = launch_rref_block2(A, ldw, npasses, Q, c >> 6, jz, 0, 0, -2, m4ri->coef, m4ri->PB, m4ri->rec, 0,
                                          0, -2, m4ri->coef2, m4ri->PB2, m4ri->rec + 1, ms, rec_of(t + 1),
                                          rec_of(t))) != hipSuccess)
                return err;
            if ((err = launch_rref_pair(A, ldw, jz, m4ri->coef, m4ri->coef2, m4ri->PB, m4ri->PB2, c >> 6, npasses,
                                        m4ri->rec, m4ri->rec + 1, ms)) != hipSuccess)
                return err;
        } else {
            if ((err = launch_rref_block(A, ldw, npasses, Q, 0, 0, c >> 6, -2, jz, m4ri->coef, m4ri->PB, nullptr, ms,
                                         rec_of(t))) != hipSuccess)
                return err;
            if ((err = launch_m4rm(A, ldw, jz, m4ri->coef, 1, m4ri->PB, ldw, KW, c >> 6, npasses, 0, 0, ms)) !=
                hipSuccess)
                return err;
        }
        if (mc) {
            const int ev = jobs.push(t);
            if (ev < 0) return hipErrorUnknown;  // an unguarded record write
            if ((err = hipEventRecord(mc->evJ[ev], ms)) != hipSuccess) return err;
        }
        return hipSuccess;
    };
    for (int64_t t = 0; t < npasses;) {
        const int64_t c = t * KW;
        PassRec *rec = rec_of(t), *nxt = rec_of(t + 1);
        if (pending) {
            if ((e = hipStreamWaitEvent(s, lc->evN, 0)) != hipSuccess) return e;
            pending = false;
        }
        if (want_pair(t)) {
            // pass t: permute with the next stripe word updated; its bulk
            // update waits for pass t + 1
            if ((e = launch_permute(A, m, n, ldw, c, rec, coef, PB, 1, nullptr, nullptr, nullptr, nullptr, s,
                                    nullptr, wlo)) != hipSuccess)
                return e;
            PanelFix f1;
            f1.mode = 1;
            if (mc && (e = m4_guard(t + 1)) != hipSuccess) return e;
            if ((e = launch_panel(A, m, n, ldw, c + KW, rec, nxt, P, Q, rank, gsv, gsid, pr, f1, false, s,
                                  nullptr)) != hipSuccess)
                return e;
            // pass u = t + 1 carries pass t's coefficients along; the pair's
            // update also runs the panel of pass t + 2 (no second stream)
            if ((e = launch_permute(A, m, n, ldw, c + KW, nxt, coef2, PB2, 2, rec, coef, coefP, PB, s, nullptr, wlo)) !=
                hipSuccess)
                return e;
            PairPanel pp;
            pp.on = 1;
            pp.n = n;
            pp.c = c + 2 * KW;
            pp.rec = rec_of(t + 2);
            pp.P = P;
            pp.Q = Q;
            pp.rank = rank;
            pp.gsv = gsv;
            pp.gsid = gsid;
            if (mc && (e = m4_guard(t + 2)) != hipSuccess) return e;
            if ((e = launch_update_pair(A, m, n, ldw, c, rec, nxt, coefP, coef2, coef, PB, PB2, m4t, pv, pp, s)) !=
                hipSuccess)
                return e;
            if (m4ri && (e = m4_job(t, 2)) != hipSuccess) return e;
            t += 2;
            continue;
        }
        if (want_la(t)) {
            // permute also updates the next stripe word of the ordinary rows;
            // the next panel finishes the special rows' one, then searches,
            // while the update of the words beyond runs
            if ((e = launch_permute(A, m, n, ldw, c, rec, coef, PB, 1, nullptr, nullptr, nullptr, nullptr, s,
                                    lc->evA, wlo)) != hipSuccess)
                return e;
            if ((e = launch_update(A, m, n, ldw, c, rec, coef, PB, 2, m4v, m4t, s)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(lc->s2, lc->evA, 0)) != hipSuccess) return e;
            PanelFix f1;
            f1.mode = 1;
            if ((e = launch_panel(A, m, n, ldw, c + KW, rec, nxt, P, Q, rank, gsv, gsid, pr, f1, true, lc->s2,
                                  lc->evN)) != hipSuccess)
                return e;
            pending = true;
            t += 1;
            continue;
        }
        if ((e = launch_permute(A, m, n, ldw, c, rec, coef, PB, 0, nullptr, nullptr, nullptr, nullptr, s,
                                nullptr, wlo)) != hipSuccess)
            return e;
        if ((e = launch_update(A, m, n, ldw, c, rec, coef, PB, 1, m4v, m4t, s)) != hipSuccess) return e;
        if (m4ri && (e = m4_job(t, 1)) != hipSuccess) return e;
        if (t + 1 >= npasses) break;
        if (c + KW >= m && allow_sync) {
            // rank <= m: once it reaches m the remaining passes are empty
            if (since_check == 0) {
                int64_t host_rank = 0;
                if ((e = hipMemcpyAsync(&host_rank, rank, 8, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
                if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
                if (host_rank >= m) break;
            }
            since_check = (since_check + 1) % 8;
        }
        if (mc && (e = m4_guard(t + 1)) != hipSuccess) return e;
        if ((e = launch_panel(A, m, n, ldw, c + KW, rec, nxt, P, Q, rank, gsv, gsid, pr, PanelFix(), false, s,
                              nullptr)) != hipSuccess)
            return e;
        t += 1;
    }
    if (mc && jobs.last() >= 0 && (e = hipStreamWaitEvent(s, mc->evJ[jobs.last()], 0)) != hipSuccess) return e;
    return hipGetLastError();
}

gf2_status ple_check_args(const uint64_t *A, int64_t m, int64_t n, int64_t ldw, const int64_t *P, const int64_t *Q,
                          const int64_t *rank, const gf2_ple_opts *opts) {
    if (!sizes_ok(m, n, ldw)) return GF2_EINVAL;
    const int64_t mn = m < n ? m : n;
    if (!rank || !aligned(rank, 8)) return GF2_EINVAL;
    if (m > 0 && (!P || !aligned(P, 8))) return GF2_EINVAL;
    if (mn > 0 && (!Q || !aligned(Q, 8))) return GF2_EINVAL;
    if (m > 0 && ldw > 0 && (!A || !aligned(A, 8))) return GF2_EINVAL;
    if (opts && (opts->update < 0 || opts->update > 4 || opts->m4_variant < 0 || opts->m4_blocks < 0)) return GF2_EINVAL;
    if (opts && (opts->rec_levels < 0 || opts->rec_levels > 16)) return GF2_EINVAL;
    if (opts && (opts->rec_split < 0 || opts->rec_split % 64 != 0)) return GF2_EINVAL;
    if (opts && opts->panel_regs != 0 && opts->panel_regs != 2 && opts->panel_regs != 4 && opts->panel_regs != 8)
        return GF2_EINVAL;
    if (opts && (opts->lookahead < 0 || opts->lookahead > 3)) return GF2_EINVAL;
    if (opts && (opts->pair_variant < 0 || opts->pair_variant > 14)) return GF2_EINVAL;
    if (opts && (opts->product_split < -1 || opts->product_split > 1)) return GF2_EINVAL;
    return GF2_OK;
}

hipError_t ple_block(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank, void *ws,
                     const gf2_ple_opts *opts, hipStream_t s, int64_t wlo) {
    return pass_loop(A, m, n, ldw, P, Q, rank, ws, opts, s, true, true, nullptr, wlo);
}

// update = 2 / 3 / 4: Algorithm 3 levels (fp4 matrix-core / table / int8
// matrix-core products)
static bool recursive(const gf2_ple_opts *opts) { return opts && opts->update >= 2; }
static int rec_levels(const gf2_ple_opts *opts) { return opts && opts->rec_levels > 0 ? opts->rec_levels : 1; }
static int rec_products(const gf2_ple_opts *opts) { return opts->update == 2 ? 1 : (opts->update == 4 ? 2 : 0); }
static int64_t rec_split(const gf2_ple_opts *opts) { return opts ? opts->rec_split : 0; }
// Strassen's split applies to the fp4 products only
static int prod_split(const gf2_ple_opts *opts) { return rec_products(opts) == 1 ? opts->product_split : -1; }

hipError_t ple_enqueue(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank,
                       void *ws, const gf2_ple_opts *opts, hipStream_t s, bool allow_sync, bool allow_s2) {
    return pass_loop(A, m, n, ldw, P, Q, rank, ws, opts, s, allow_sync, allow_s2, nullptr);
}

}  // namespace gf2

extern "C" {

const char *gf2_version(void) { return "gf2ple 0.1.0 gfx950"; }

const char *gf2_status_str(gf2_status s) {
    switch (s) {
        case GF2_OK: return "ok";
        case GF2_EINVAL: return "invalid argument";
        case GF2_EWORKSPACE: return "workspace too small";
        case GF2_ENOMEM: return "out of memory";
        case GF2_EBUDGET: return "request exceeds the device budget";
        case GF2_EHIP: return "HIP runtime error";
        case GF2_EPADDING: return "non-zero bit at a column >= n";
        case GF2_EBUSY: return "no such pending request";
    }
    return "unknown status";
}

size_t gf2_ple_workspace_bytes(int64_t m, int64_t n, int64_t ldw, const gf2_ple_opts *opts) {
    if (!sizes_ok(m, n, ldw)) return 0;
    if (recursive(opts))
        return align_up(ple_layout(m, ldw).total) +
               alg3_extra_bytes(m, n, ldw, rec_levels(opts), rec_products(opts) != 0, rec_split(opts),
                                prod_split(opts));
    return ple_layout(m, ldw).total;
}

gf2_status gf2_check_padding(const uint64_t *A, int64_t m, int64_t n, int64_t ldw, void *stream) {
    if (!sizes_ok(m, n, ldw)) return GF2_EINVAL;
    if (m == 0 || ldw == 0) return GF2_OK;
    if (!A || !aligned(A, 8)) return GF2_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_flag_mu);
    int *flag = device_flag_locked();
    if (!flag) return GF2_EHIP;
    if (hipMemsetAsync(flag, 0, sizeof(int), s) != hipSuccess) return GF2_EHIP;
    if (launch_padding(A, m, n, ldw, flag, s) != hipSuccess) return GF2_EHIP;
    int host = 0;
    if (hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return GF2_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return GF2_EHIP;
    return host ? GF2_EPADDING : GF2_OK;
}

gf2_status gf2_ple(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank, void *ws,
                   size_t ws_bytes, const gf2_ple_opts *opts, void *stream) {
    const gf2_status chk = ple_check_args(A, m, n, ldw, P, Q, rank, opts);
    if (chk != GF2_OK) return chk;
    if (!ws || !aligned(ws, ALIGN)) return GF2_EINVAL;
    if (ws_bytes < gf2_ple_workspace_bytes(m, n, ldw, opts)) return GF2_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (opts && opts->check_padding) {
        gf2_status st = gf2_check_padding(A, m, n, ldw, stream);
        if (st != GF2_OK) return st;
    }
    if (recursive(opts))
        return hip_status(
            ple_alg3(A, m, n, ldw, P, Q, rank, ws, opts, s, rec_levels(opts), rec_products(opts), rec_split(opts),
                     prod_split(opts)));
    return hip_status(ple_enqueue(A, m, n, ldw, P, Q, rank, ws, opts, s, true, true));
}

int64_t gf2_product_plan(int64_t m, int64_t k, int64_t n, int32_t split, int64_t lda, int64_t ldbt, int64_t ldc,
                         gf2_plan_step *steps, int64_t max, int64_t *ws_words) {
    return product_plan(m, k, n, split, lda, ldbt, ldc, steps, max, ws_words);
}

int64_t gf2_ple_schedule(int64_t m, int64_t n, const gf2_ple_opts *opts, int32_t *kinds, int64_t max) {
    if (m < 0 || n < 0) return -1;
    const int mode = opts ? opts->lookahead : 0;
    if (mode < 0 || mode > 3) return -1;
    std::vector<int8_t> kind;
    pass_kinds(m, n, mode, kind);
    const int64_t np = (int64_t)kind.size();
    for (int64_t t = 0; t < np && t < max && kinds; t++) kinds[t] = kind[t];
    return np;
}

gf2_status gf2_echelon_from_ple(uint64_t *A, int64_t m, int64_t n, int64_t ldw, const int64_t *rank, void *stream) {
    if (!sizes_ok(m, n, ldw)) return GF2_EINVAL;
    if (!rank || !aligned(rank, 8)) return GF2_EINVAL;
    if (m == 0 || ldw == 0) return GF2_OK;
    if (!A || !aligned(A, 8)) return GF2_EINVAL;
    return hip_status(launch_echelon(A, m, ldw, rank, (hipStream_t)stream));
}

size_t gf2_rref_workspace_bytes(int64_t m, int64_t n, int64_t ldw) {
    if (!sizes_ok(m, n, ldw)) return 0;
    return rref_layout(m, ldw).total;
}

gf2_status gf2_rref_from_ple(uint64_t *A, int64_t m, int64_t n, int64_t ldw, const int64_t *Q, const int64_t *rank,
                             void *ws, size_t ws_bytes, void *stream) {
    if (!sizes_ok(m, n, ldw)) return GF2_EINVAL;
    if (!rank || !aligned(rank, 8)) return GF2_EINVAL;
    const int64_t mn = m < n ? m : n;
    if (mn > 0 && (!Q || !aligned(Q, 8))) return GF2_EINVAL;
    if (m == 0 || ldw == 0) return GF2_OK;
    if (!A || !aligned(A, 8)) return GF2_EINVAL;
    const RrefLayout L = rref_layout(m, ldw);
    if (!ws || !aligned(ws, ALIGN)) return GF2_EINVAL;
    if (ws_bytes < L.total) return GF2_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (launch_echelon(A, m, ldw, rank, s) != hipSuccess) return GF2_EHIP;
    // the number of pivot blocks and their first columns size the launches
    int64_t r = 0;
    if (hipMemcpyAsync(&r, rank, 8, hipMemcpyDeviceToHost, s) != hipSuccess) return GF2_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return GF2_EHIP;
    if (r <= 0) return GF2_OK;
    std::vector<int64_t> hq((size_t)r);
    if (hipMemcpy(hq.data(), Q, (size_t)r * 8, hipMemcpyDeviceToHost) != hipSuccess) return GF2_EHIP;
    char *base = (char *)ws;
    uint64_t *coef = (uint64_t *)(base + L.coef);
    uint64_t *coef2 = (uint64_t *)(base + L.coef2);
    uint64_t *PB = (uint64_t *)(base + L.pb);
    uint64_t *PB2 = (uint64_t *)(base + L.pb2);
    PassRec *rect = (PassRec *)(base + L.rec), *recu = rect + 1;
    const int64_t nw = words_for(n);
    const int64_t nblk = (r + KW - 1) / KW;
    // contiguous pivot columns (the full-rank case): their bits are one
    // funnel shift of a row's words; -1 otherwise
    auto first_col = [&](int64_t j0, int64_t j1) {
        int64_t q0 = hq[(size_t)j0];
        for (int64_t t = j0 + 1; t < j1; t++)
            if (hq[(size_t)t] != hq[(size_t)j0] + (t - j0)) q0 = -1;
        return q0;
    };
    for (int64_t b = nblk - 1; b >= 0;) {
        const int64_t j0 = b * KW;
        const int64_t j1 = j0 + KW < r ? j0 + KW : r;
        const int64_t wq0 = hq[(size_t)j0] >> 6;
        if (b >= 1) {
            // blocks b and b - 1 in one sweep.  Block b's update leaves the
            // bits at block b - 1's pivot columns (left of its own) as they
            // are, so both blocks' coefficients come from the rows as they
            // stand; block b - 1's rows first take block b's update in the
            // sweep's table build.
            const int64_t j0u = j0 - KW;
            const int64_t wq0u = hq[(size_t)j0u] >> 6;
            if (launch_rref_block2(A, ldw, nw, Q, wq0u, j1, j0, j1, first_col(j0, j1), coef, PB, rect, j0u, j0,
                                   first_col(j0u, j0), coef2, PB2, recu, s) != hipSuccess)
                return GF2_EHIP;
            if (launch_rref_pair(A, ldw, j1, coef, coef2, PB, PB2, wq0u, nw, rect, recu, s) != hipSuccess)
                return GF2_EHIP;
            b -= 2;
        } else {
            if (launch_rref_block(A, ldw, nw, Q, j0, j1, wq0, first_col(j0, j1), j1, coef, PB, nullptr, s) !=
                hipSuccess)
                return GF2_EHIP;
            if (launch_m4rm(A, ldw, j1, coef, 1, PB, ldw, (int)(j1 - j0), wq0, nw, 0, 0, s) != hipSuccess)
                return GF2_EHIP;
            b -= 1;
        }
    }
    return hip_status(hipGetLastError());
}

// workspace of gf2_m4ri_rref: that of gf2_ple | coef[m] | coef2[m] |
// PB[64 x ldw] | PB2[64 x ldw] | two records | P[m]
struct M4riLayout {
    size_t coef, coef2, pb, pb2, rec, p, total;
};
static M4riLayout m4ri_layout(int64_t m, int64_t ldw) {
    M4riLayout L;
    size_t off = ple_layout(m, ldw).total;
    L.coef = off;
    off += align_up((size_t)m * 8);
    L.coef2 = off;
    off += align_up((size_t)m * 8);
    L.pb = off;
    off += align_up((size_t)KW * (size_t)ldw * 8);
    L.pb2 = off;
    off += align_up((size_t)KW * (size_t)ldw * 8);
    L.rec = off;
    off += align_up(2 * sizeof(PassRec));
    L.p = off;
    off += align_up((size_t)m * 8);
    L.total = off;
    return L;
}

size_t gf2_m4ri_rref_workspace_bytes(int64_t m, int64_t n, int64_t ldw) {
    if (!sizes_ok(m, n, ldw)) return 0;
    return m4ri_layout(m, ldw).total;
}

gf2_status gf2_m4ri_rref(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *Q, int64_t *rank, void *ws,
                         size_t ws_bytes, void *stream) {
    if (!sizes_ok(m, n, ldw)) return GF2_EINVAL;
    const int64_t mn = m < n ? m : n;
    if (!rank || !aligned(rank, 8)) return GF2_EINVAL;
    if (mn > 0 && (!Q || !aligned(Q, 8))) return GF2_EINVAL;
    if (m > 0 && ldw > 0 && (!A || !aligned(A, 8))) return GF2_EINVAL;
    if (!ws || !aligned(ws, ALIGN)) return GF2_EINVAL;
    if (ws_bytes < gf2_m4ri_rref_workspace_bytes(m, n, ldw)) return GF2_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const M4riLayout L = m4ri_layout(m, ldw);
    char *base = (char *)ws;
    M4riStep st;
    st.coef = (uint64_t *)(base + L.coef);
    st.coef2 = (uint64_t *)(base + L.coef2);
    st.PB = (uint64_t *)(base + L.pb);
    st.PB2 = (uint64_t *)(base + L.pb2);
    st.rec = (PassRec *)(base + L.rec);
    int64_t *P = (int64_t *)(base + L.p);
    // the default schedule: fused pairs of passes, each pair's 128-column
    // block then eliminated from the rows above in one sweep
    gf2_ple_opts o{};
    hipError_t e = pass_loop(A, m, n, ldw, P, Q, rank, ws, &o, s, true, true, &st);
    if (e != hipSuccess) return hip_status(e);
    if (m == 0 || ldw == 0) return GF2_OK;
    return hip_status(launch_echelon(A, m, ldw, rank, s));
}

size_t gf2_rref_full_workspace_bytes(int64_t m, int64_t n, int64_t ldw, const gf2_ple_opts *opts) {
    size_t a = gf2_ple_workspace_bytes(m, n, ldw, opts);
    size_t b = gf2_rref_workspace_bytes(m, n, ldw);
    if (!a || !b) return 0;
    return a > b ? a : b;
}

gf2_status gf2_rref(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank, void *ws,
                    size_t ws_bytes, const gf2_ple_opts *opts, void *stream) {
    gf2_status st = gf2_ple(A, m, n, ldw, P, Q, rank, ws, ws_bytes, opts, stream);
    if (st != GF2_OK) return st;
    return gf2_rref_from_ple(A, m, n, ldw, Q, rank, ws, ws_bytes, stream);
}

// update 2: fp4 matrix cores; 4: int8 matrix cores; 0, 1, 3: tables
static bool addmul_mfma(const gf2_ple_opts *opts) { return opts && (opts->update == 2 || opts->update == 4); }

size_t gf2_addmul_workspace_bytes(int64_t m, int64_t k, int64_t n, const gf2_ple_opts *opts) {
    if (m < 0 || k < 0 || n < 0) return 0;
    if (!addmul_mfma(opts)) return 0;
    return (size_t)words_for(n) * 64 * (size_t)words_for(k) * 8;
}

gf2_status gf2_addmul(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda, const uint64_t *B, int64_t ldb,
                      int64_t m, int64_t k, int64_t n, void *ws, size_t ws_bytes, const gf2_ple_opts *opts,
                      void *stream) {
    if (m < 0 || k < 0 || n < 0) return GF2_EINVAL;
    if (ldc < words_for(n) || lda < words_for(k) || ldb < words_for(n)) return GF2_EINVAL;
    if (opts && (opts->update < 0 || opts->update > 4 || opts->m4_variant < 0 || opts->m4_blocks < 0)) return GF2_EINVAL;
    if (m == 0 || n == 0 || k == 0) return GF2_OK;
    if (!C || !A || !B || !aligned(C, 8) || !aligned(A, 8) || !aligned(B, 8)) return GF2_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nw = words_for(n);
    if (addmul_mfma(opts)) {
        // matrix cores: B bit-transposed into the caller's workspace first
        const int64_t kw = words_for(k);
        if (!ws || !aligned(ws, 8)) return GF2_EINVAL;
        if (ws_bytes < gf2_addmul_workspace_bytes(m, k, n, opts)) return GF2_EWORKSPACE;
        hipError_t e = launch_transpose_bits(B, ldb, k, n, (uint64_t *)ws, kw, s);
        if (e == hipSuccess)
            e = launch_mfma_gf2(C, ldc, A, lda, (const uint64_t *)ws, kw, m, k, n, s, opts->update == 4 ? 1 : 0);
        return hip_status(e);
    }
    for (int64_t kb = 0; kb * KW < k; kb++) {
        const int nb = (int)(k - kb * KW < KW ? k - kb * KW : KW);
        if (launch_m4rm(C, ldc, m, A + kb, lda, B + kb * KW * ldb, ldb, nb, 0, nw, opts ? opts->m4_variant : 0,
                        opts ? opts->m4_blocks : 0, s) != hipSuccess)
            return GF2_EHIP;
    }
    return hip_status(hipGetLastError());
}

gf2_status gf2_make_table(const uint64_t *rows, int64_t ldr, int32_t k, int64_t n, uint64_t *T, int64_t ldt,
                          void *stream) {
    if (k < 1 || k > 8 || n < 0) return GF2_EINVAL;
    const int64_t nw = words_for(n);
    if (ldr < nw || ldt < nw) return GF2_EINVAL;
    if (ldt == 0) return GF2_OK;
    if (!rows || !T || !aligned(rows, 8) || !aligned(T, 8)) return GF2_EINVAL;
    return hip_status(launch_make_table(rows, ldr, k, nw, T, ldt, (hipStream_t)stream));
}

}  // extern "C"
