// Kernel timing with HIP events (gf2_profile_start / gf2_profile_stop).
// While enabled, each launch site records one event before and one after its
// kernel on the launch stream; stop() waits for the events and sums the
// elapsed times per kernel.  Events are pooled and reused.
#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/gf2ple.h"
#include "common.h"

namespace gf2 {
namespace {

struct Mark {
    int kid;
    hipEvent_t b, e;
};

std::mutex g_mu;
std::atomic<bool> g_on{false};
std::vector<Mark> g_marks;
std::vector<hipEvent_t> g_pool;

const char *kNames[KID_COUNT] = {"panel", "permute", "m4rm",  "init",     "rref_block",
                                 "echelon", "mfma",  "batch", "trsm", "transpose", "sums"};

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void recycle_marks() {
    for (auto &m : g_marks) {
        if (m.b) g_pool.push_back(m.b);
        if (m.e) g_pool.push_back(m.e);
    }
    g_marks.clear();
}

}  // namespace

bool prof_enabled() { return g_on.load(std::memory_order_relaxed); }

void prof_mark(int kid, hipStream_t s, bool begin) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (begin) {
        hipEvent_t ev = take_event();
        if (!ev) return;
        (void)hipEventRecord(ev, s);
        g_marks.push_back(Mark{kid, ev, nullptr});
        return;
    }
    for (auto it = g_marks.rbegin(); it != g_marks.rend(); ++it) {
        if (it->kid == kid && it->e == nullptr) {
            hipEvent_t ev = take_event();
            if (!ev) return;
            (void)hipEventRecord(ev, s);
            it->e = ev;
            return;
        }
    }
}

}  // namespace gf2

using namespace gf2;

extern "C" {

gf2_status gf2_profile_start(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    recycle_marks();
    g_on.store(true);
    return GF2_OK;
}

gf2_status gf2_profile_stop(gf2_kernel_time *out, int32_t max_entries, int32_t *count) {
    g_on.store(false);
    std::lock_guard<std::mutex> lk(g_mu);
    gf2_kernel_time acc[KID_COUNT];
    std::memset(acc, 0, sizeof(acc));
    gf2_status st = GF2_OK;
    for (auto &m : g_marks) {
        if (!m.e) continue;
        float ms = 0.f;
        if (hipEventSynchronize(m.e) != hipSuccess || hipEventElapsedTime(&ms, m.b, m.e) != hipSuccess) {
            st = GF2_EHIP;
            continue;
        }
        gf2_kernel_time &a = acc[m.kid];
        if (a.launches == 0 || ms < a.min_ms) a.min_ms = ms;
        if (ms > a.max_ms) a.max_ms = ms;
        a.total_ms += ms;
        a.launches++;
    }
    recycle_marks();
    int32_t n = 0;
    for (int k = 0; k < KID_COUNT; k++) {
        if (acc[k].launches == 0) continue;
        if (out && n < max_entries) {
            out[n] = acc[k];
            std::strncpy(out[n].name, kNames[k], sizeof(out[n].name) - 1);
            out[n].name[sizeof(out[n].name) - 1] = 0;
        }
        n++;
    }
    if (count) *count = n;
    return st;
}

}  // extern "C"
