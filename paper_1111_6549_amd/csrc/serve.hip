// Serving session (gf2_serve_*): a host thread that admits requests in
// arrival order into a device-memory pool of fixed budget and launches them
// as they arrive -- all admitted small requests together in one batched
// launch (the persistent kernel of the batched path), every large request in
// its own pass loop of gf2_ple -- on several streams, so that new requests
// join the next launch while earlier launches still run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.h"

using namespace gf2;

namespace {

constexpr size_t SALIGN = 256;
size_t sal(size_t x) { return (x + SALIGN - 1) & ~(SALIGN - 1); }

// First-fit allocator over the session's one device allocation (byte
// offsets, 256-byte granules, neighbours merged on release).
class Pool {
   public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
        used_ = peak_ = 0;
    }
    int64_t alloc(size_t bytes) {
        bytes = sal(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return (int64_t)off;
        }
        return -1;
    }
    void release(size_t off, size_t bytes) {
        bytes = sal(bytes ? bytes : 1);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const {
        size_t b = 0;
        for (auto &f : free_) b = std::max(b, f.second);
        return b;
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

   private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0, peak_ = 0;
};

struct Req {
    int64_t id = 0, m = 0, n = 0, ldw = 0;
    std::vector<uint64_t> host;      // host copy of the input (host submissions)
    const uint64_t *dsrc = nullptr;  // device input (device submissions)
    int state = GF2_REQ_QUEUED;
    int status = GF2_OK;
    bool small = true;
    bool fetching = false;
    size_t bytes = 0;
    int64_t off = -1;                          // region in the pool
    size_t a_rel = 0, p_rel = 0, q_rel = 0, r_rel = 0, ws_rel = 0;  // parts of the region
    double t_submit = 0, t_admit = 0, t_done = 0;
};

struct Launch {
    int stream = 0;
    std::vector<int64_t> ids;
    std::vector<gf2_desc> descs;  // host sources of the descriptor uploads, kept until done
    std::vector<int64_t> roff;
    std::vector<int32_t> order;
};

// Per-stream reserved area of batched launches.
struct Aux {
    size_t descs = 0, roff = 0, order = 0, counter = 0, slots = 0;
};

}  // namespace

struct gf2_serve {
    gf2_serve_opts o{};
    int dev = 0;
    uint8_t *base = nullptr;
    size_t budget = 0;
    Pool pool;
    size_t reserved = 0;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<char> busy;
    std::vector<Aux> aux;
    SlotLayout lay{};
    int64_t slot_cap = 0;  // workgroup slots reserved per stream
    int64_t small_ldw = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::unordered_map<int64_t, std::unique_ptr<Req>> reqs;
    std::deque<int64_t> queue;  // waiting for admission
    std::deque<int64_t> ready;  // admitted, not launched
    std::vector<std::unique_ptr<Launch>> inflight;
    int64_t next_id = 1;
    int64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_batched = 0, n_single = 0;
    bool stop = false;
    std::thread th;
    std::chrono::steady_clock::time_point t0;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
    void run();
    // Enqueue a launch without holding mu: rs are its requests (admitted and
    // running, so no other thread changes or frees them meanwhile).
    hipError_t enqueue(Launch &L, const std::vector<Req *> &rs, bool *single);
};

namespace {

void region_layout(Req &r, bool small) {
    const int64_t mn = std::min(r.m, r.n);
    size_t off = 0;
    r.a_rel = off;
    off += sal((size_t)r.m * (size_t)r.ldw * 8);
    r.p_rel = off;
    off += sal((size_t)r.m * 8);
    r.q_rel = off;
    off += sal((size_t)mn * 8);
    r.r_rel = off;
    off += SALIGN;
    r.ws_rel = off;
    if (!small) off += sal(ple_workspace_total(r.m, r.ldw));
    r.bytes = off;
}

double cost_of(const Req &r) { return (double)r.m * (double)words_for(r.n) * (double)std::min(r.m, r.n) + 1.0; }

}  // namespace

hipError_t gf2_serve::enqueue(Launch &L, const std::vector<Req *> &rs, bool *single) {
    hipStream_t st = streams[L.stream];
    hipError_t e = hipSuccess;
    int64_t maxdim = 0;
    for (Req *rp : rs) {
        Req &r = *rp;
        const size_t nb = (size_t)r.m * (size_t)r.ldw * 8;
        uint8_t *dst = base + r.off + r.a_rel;
        if (nb) {
            if (!r.host.empty())
                e = hipMemcpyAsync(dst, r.host.data(), nb, hipMemcpyHostToDevice, st);
            else
                e = hipMemcpyAsync(dst, r.dsrc, nb, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return e;
        }
        maxdim = std::max(maxdim, std::max(r.m, r.n));
    }
    *single = rs.size() == 1 && !rs[0]->small;
    if (*single) {
        Req &r = *rs[0];
        uint8_t *p = base + r.off;
        // the default pass schedule (fused pairs), every kernel on this
        // stream (no look-ahead on the library's second stream)
        gf2_ple_opts o{};
        e = ple_enqueue((uint64_t *)(p + r.a_rel), r.m, r.n, r.ldw, (int64_t *)(p + r.p_rel), (int64_t *)(p + r.q_rel),
                        (int64_t *)(p + r.r_rel), p + r.ws_rel, &o, st, false, false);
        if (e != hipSuccess) return e;
    } else {
        const Aux &x = aux[L.stream];
        const size_t cnt = L.ids.size();
        L.descs.resize(cnt);
        L.roff.resize(cnt);
        L.order.resize(cnt);
        for (size_t k = 0; k < cnt; k++) {
            const Req &r = *rs[k];
            gf2_desc d;
            d.a_off = (int64_t)((r.off + r.a_rel) / 8);
            d.m = r.m;
            d.n = r.n;
            d.ldw = r.ldw;
            d.p_off = (int64_t)((r.off + r.p_rel) / 8);
            d.q_off = (int64_t)((r.off + r.q_rel) / 8);
            L.descs[k] = d;
            L.roff[k] = (int64_t)((r.off + r.r_rel) / 8);
        }
        std::iota(L.order.begin(), L.order.end(), 0);
        std::stable_sort(L.order.begin(), L.order.end(),
                         [&](int32_t a, int32_t b) { return cost_of(*rs[a]) > cost_of(*rs[b]); });
        if ((e = hipMemcpyAsync(base + x.descs, L.descs.data(), cnt * sizeof(gf2_desc), hipMemcpyHostToDevice, st)) !=
                hipSuccess ||
            (e = hipMemcpyAsync(base + x.roff, L.roff.data(), cnt * 8, hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(base + x.order, L.order.data(), cnt * 4, hipMemcpyHostToDevice, st)) != hipSuccess)
            return e;
        if ((e = batch_reset((int32_t *)(base + x.counter), 1, st)) != hipSuccess) return e;
        const int cfg = batch_default_config(maxdim);
        // at most the reserved slots; beyond the resident capacity the extra
        // workgroups start as others finish
        const int64_t grid = std::min<int64_t>((int64_t)cnt, slot_cap);
        BatchArgs a;
        a.descs = (const gf2_desc *)(base + x.descs);
        a.order = (const int32_t *)(base + x.order);
        a.rank_off = (const int64_t *)(base + x.roff);
        a.count = (int32_t)cnt;
        a.counter = (int32_t *)(base + x.counter);
        a.arena = (uint64_t *)base;
        a.P = (int64_t *)base;
        a.Q = (int64_t *)base;
        a.ranks = (int64_t *)base;
        a.slots = base + x.slots;
        a.lay = lay;
        if ((e = batch_launch(cfg, (int)grid, a, st)) != hipSuccess) return e;
    }
    return hipEventRecord(events[L.stream], st);
}

void gf2_serve::run() {
    (void)hipSetDevice(dev);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progress = false;
        // completions
        for (size_t k = 0; k < inflight.size();) {
            Launch &L = *inflight[k];
            const hipError_t q = hipEventQuery(events[L.stream]);
            if (q == hipErrorNotReady) {
                k++;
                continue;
            }
            const double t = now();
            for (int64_t id : L.ids) {
                Req &r = *reqs[id];
                r.state = q == hipSuccess ? GF2_REQ_DONE : GF2_REQ_FAILED;
                r.status = q == hipSuccess ? GF2_OK : GF2_EHIP;
                r.t_done = t;
                std::vector<uint64_t>().swap(r.host);
                if (q == hipSuccess)
                    n_completed++;
                else
                    n_failed++;
            }
            busy[L.stream] = 0;
            inflight.erase(inflight.begin() + k);
            progress = true;
        }
        if (progress) cv_done.notify_all();
        // admission, in arrival order
        while (!stop && !queue.empty()) {
            Req &r = *reqs[queue.front()];
            const int64_t off = pool.alloc(r.bytes);
            if (off < 0) break;
            r.off = off;
            r.state = GF2_REQ_RUNNING;
            r.t_admit = now();
            ready.push_back(r.id);
            queue.pop_front();
            progress = true;
        }
        // launches
        while (!ready.empty()) {
            int s = -1;
            for (int k = 0; k < (int)streams.size(); k++)
                if (!busy[k]) {
                    s = k;
                    break;
                }
            if (s < 0) break;
            auto L = std::unique_ptr<Launch>(new Launch());
            L->stream = s;
            if (!reqs[ready.front()]->small) {
                L->ids.push_back(ready.front());
                ready.pop_front();
            } else {
                std::deque<int64_t> rest;
                while (!ready.empty()) {
                    const int64_t id = ready.front();
                    ready.pop_front();
                    if (reqs[id]->small && (int)L->ids.size() < o.max_batch)
                        L->ids.push_back(id);
                    else
                        rest.push_back(id);
                }
                ready.swap(rest);
            }
            std::vector<Req *> rs;
            rs.reserve(L->ids.size());
            for (int64_t id : L->ids) rs.push_back(reqs[id].get());
            // host inputs are copied (pageable, so the copy may wait) and the
            // launches enqueued without the lock: submit, poll and wait go on
            busy[s] = 1;
            bool single = false;
            lk.unlock();
            const hipError_t e = enqueue(*L, rs, &single);
            lk.lock();
            if (e != hipSuccess) {
                // the launch could not be enqueued: fail its requests
                (void)hipStreamSynchronize(streams[s]);
                const double t = now();
                for (Req *r : rs) {
                    r->state = GF2_REQ_FAILED;
                    r->status = GF2_EHIP;
                    r->t_done = t;
                    n_failed++;
                }
                busy[s] = 0;
                cv_done.notify_all();
            } else {
                (single ? n_single : n_batched)++;
                inflight.push_back(std::move(L));
            }
            progress = true;
        }
        if (stop && inflight.empty()) break;
        if (!progress) {
            if (inflight.empty())
                cv_work.wait_for(lk, std::chrono::milliseconds(50));
            else
                cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

extern "C" {

gf2_status gf2_serve_create(const gf2_serve_opts *opts, gf2_serve **session) {
    if (!session) return GF2_EINVAL;
    *session = nullptr;
    gf2_serve_opts o{};
    if (opts) o = *opts;
    if (o.budget_bytes < 0 || o.streams < 0 || o.streams > 16 || o.max_batch < 0 || o.small_max_dim < 0 ||
        o.small_max_dim > 4096)
        return GF2_EINVAL;
    if (o.budget_bytes == 0) o.budget_bytes = (int64_t)64 << 30;
    // three launch streams: with the process's default stream they fit the
    // four hardware queues a process gets by default (GPU_MAX_HW_QUEUES)
    if (o.streams == 0) o.streams = 3;
    if (o.max_batch == 0) o.max_batch = 4096;
    if (o.small_max_dim == 0) o.small_max_dim = 2048;

    gf2_serve *S = new (std::nothrow) gf2_serve();
    if (!S) return GF2_ENOMEM;
    S->o = o;
    S->t0 = std::chrono::steady_clock::now();
    S->budget = (size_t)o.budget_bytes & ~(SALIGN - 1);
    S->small_ldw = words_for(o.small_max_dim);
    S->lay = batch_slot_layout(o.small_max_dim, S->small_ldw);
    int cus = 256;
    gf2_status st = GF2_OK;
    if (hipGetDevice(&S->dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->dev) != hipSuccess)
        st = GF2_EHIP;
    // workgroup slots a batched launch may use: the largest persistent grid of
    // the schedules small requests can get
    int64_t cap = 1;
    for (int64_t d : {(int64_t)256, (int64_t)512, (int64_t)1024, (int64_t)2048, (int64_t)4096}) {
        if (d > 2 * (int64_t)o.small_max_dim) break;
        cap = std::max<int64_t>(cap, (int64_t)batch_occupancy(batch_default_config(d)) * cus);
    }
    S->slot_cap = cap;
    // reserved per stream: descriptors, rank offsets, order, counter, slots
    std::vector<Aux> aux(o.streams);
    size_t off = 0;
    for (auto &x : aux) {
        x.descs = off;
        off += sal((size_t)o.max_batch * sizeof(gf2_desc));
        x.roff = off;
        off += sal((size_t)o.max_batch * 8);
        x.order = off;
        off += sal((size_t)o.max_batch * 4);
        x.counter = off;
        off += SALIGN;
        x.slots = off;
        off += sal((size_t)cap * (size_t)S->lay.bytes);
    }
    S->reserved = off;
    if (st == GF2_OK && S->reserved + ((size_t)1 << 20) > S->budget) st = GF2_EINVAL;
    if (st == GF2_OK && hipMalloc(&S->base, S->budget) != hipSuccess) {
        S->base = nullptr;
        st = GF2_ENOMEM;
    }
    if (st == GF2_OK) {
        S->pool.init(S->budget);
        const int64_t r0 = S->pool.alloc(S->reserved);  // first-fit on an empty pool: offset 0
        if (r0 != 0) st = GF2_EHIP;
        S->aux = aux;
        S->streams.resize(o.streams, nullptr);
        S->events.resize(o.streams, nullptr);
        S->busy.assign(o.streams, 0);
        for (int k = 0; st == GF2_OK && k < o.streams; k++) {
            if (hipStreamCreateWithFlags(&S->streams[k], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&S->events[k], hipEventDisableTiming) != hipSuccess)
                st = GF2_EHIP;
        }
    }
    if (st == GF2_OK) {
        try {
            S->th = std::thread([S] { S->run(); });
        } catch (...) {
            st = GF2_ENOMEM;
        }
    }
    if (st != GF2_OK) {
        for (auto s : S->streams)
            if (s) (void)hipStreamDestroy(s);
        for (auto e : S->events)
            if (e) (void)hipEventDestroy(e);
        if (S->base) (void)hipFree(S->base);
        delete S;
        return st;
    }
    *session = S;
    return GF2_OK;
}

gf2_status gf2_serve_submit(gf2_serve *S, const uint64_t *A, int32_t a_on_device, int64_t m, int64_t n, int64_t ldw,
                            int64_t *ticket) {
    if (!S || !ticket) return GF2_EINVAL;
    const double t_arrive = S->now();
    if (m < 0 || n < 0 || ldw < words_for(n) || m > INT32_MAX || n > INT32_MAX) return GF2_EINVAL;
    if (ldw > 0 && m > (int64_t)(INT64_MAX / 16) / ldw) return GF2_EINVAL;
    if (m > 0 && ldw > 0 && (!A || ((uintptr_t)A & 7))) return GF2_EINVAL;
    std::unique_ptr<Req> r(new (std::nothrow) Req());
    if (!r) return GF2_ENOMEM;
    r->m = m;
    r->n = n;
    r->ldw = ldw;
    r->small = std::max(m, n) <= S->o.small_max_dim && ldw <= S->small_ldw;
    region_layout(*r, r->small);
    if (r->bytes > S->budget - S->reserved) return GF2_EBUDGET;
    const size_t nb = (size_t)m * (size_t)ldw;
    if (nb) {
        if (a_on_device) {
            r->dsrc = A;
        } else {
            try {
                r->host.assign(A, A + nb);
            } catch (...) {
                return GF2_ENOMEM;
            }
        }
    }
    r->t_submit = t_arrive;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r->id = S->next_id++;
        *ticket = r->id;
        S->queue.push_back(r->id);
        S->reqs.emplace(r->id, std::move(r));
        S->n_submitted++;
    }
    S->cv_work.notify_one();
    return GF2_OK;
}

static void fill_info(const Req &r, gf2_serve_info *info) {
    info->state = r.state;
    info->status = r.status;
    info->m = r.m;
    info->n = r.n;
    info->ldw = r.ldw;
    info->t_submit = r.t_submit;
    info->t_admit = r.t_admit;
    info->t_done = r.t_done;
}

gf2_status gf2_serve_poll(gf2_serve *S, int64_t ticket, gf2_serve_info *info) {
    if (!S || !info) return GF2_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return GF2_EBUSY;
    fill_info(*it->second, info);
    return GF2_OK;
}

gf2_status gf2_serve_wait(gf2_serve *S, int64_t ticket, gf2_serve_info *info) {
    if (!S) return GF2_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return GF2_EBUSY;
    Req *r = it->second.get();
    S->cv_done.wait(lk, [&] { return r->state == GF2_REQ_DONE || r->state == GF2_REQ_FAILED; });
    if (info) fill_info(*r, info);
    return GF2_OK;
}

static void release_locked(gf2_serve *S, std::unordered_map<int64_t, std::unique_ptr<Req>>::iterator it) {
    Req &r = *it->second;
    if (r.off >= 0) S->pool.release((size_t)r.off, r.bytes);
    S->reqs.erase(it);
}

gf2_status gf2_serve_fetch(gf2_serve *S, int64_t ticket, uint64_t *LE, int64_t ldw_out, int64_t *P, int64_t *Q,
                           int64_t *rank, int32_t to_device) {
    if (!S) return GF2_EINVAL;
    Req *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end() || it->second->fetching) return GF2_EBUSY;
        r = it->second.get();
        if (r->state == GF2_REQ_FAILED) {
            const gf2_status st = (gf2_status)r->status;
            release_locked(S, it);
            S->cv_work.notify_one();
            return st;
        }
        if (r->state != GF2_REQ_DONE) return GF2_EBUSY;
        if (LE && ldw_out < words_for(r->n)) return GF2_EINVAL;
        r->fetching = true;
    }
    // the region is not reused before the release below; the copies run on
    // the default stream (no stream of the session's own, so the session's
    // launch streams keep the hardware queues to themselves)
    const hipMemcpyKind kind = to_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const uint8_t *p = S->base + r->off;
    hipStream_t fs = nullptr;
    hipError_t e = hipSuccess;
    const int64_t mn = std::min(r->m, r->n);
    const int64_t wcopy = LE ? std::min(ldw_out, r->ldw) : 0;
    if (LE && r->m > 0 && wcopy > 0)
        e = hipMemcpy2DAsync(LE, (size_t)ldw_out * 8, p + r->a_rel, (size_t)r->ldw * 8, (size_t)wcopy * 8, (size_t)r->m,
                             kind, fs);
    if (e == hipSuccess && LE && r->m > 0 && ldw_out > wcopy && to_device)
        e = hipMemset2DAsync(LE + wcopy, (size_t)ldw_out * 8, 0, (size_t)(ldw_out - wcopy) * 8, (size_t)r->m, fs);
    if (e == hipSuccess && P && r->m > 0) e = hipMemcpyAsync(P, p + r->p_rel, (size_t)r->m * 8, kind, fs);
    if (e == hipSuccess && Q && mn > 0) e = hipMemcpyAsync(Q, p + r->q_rel, (size_t)mn * 8, kind, fs);
    if (e == hipSuccess && rank) e = hipMemcpyAsync(rank, p + r->r_rel, 8, kind, fs);
    if (e == hipSuccess) e = hipStreamSynchronize(fs);
    if (e == hipSuccess && LE && r->m > 0 && ldw_out > wcopy && !to_device)
        for (int64_t i = 0; i < r->m; i++) memset(LE + i * ldw_out + wcopy, 0, (size_t)(ldw_out - wcopy) * 8);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        release_locked(S, S->reqs.find(ticket));
    }
    S->cv_work.notify_one();
    return e == hipSuccess ? GF2_OK : GF2_EHIP;
}

gf2_status gf2_serve_release(gf2_serve *S, int64_t ticket) {
    if (!S) return GF2_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end() || it->second->fetching) return GF2_EBUSY;
        const int st = it->second->state;
        if (st != GF2_REQ_DONE && st != GF2_REQ_FAILED) return GF2_EBUSY;
        release_locked(S, it);
    }
    S->cv_work.notify_one();
    return GF2_OK;
}

gf2_status gf2_serve_stats_get(gf2_serve *S, gf2_serve_stats *st) {
    if (!S || !st) return GF2_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    st->submitted = S->n_submitted;
    st->completed = S->n_completed;
    st->failed = S->n_failed;
    st->queued = (int64_t)S->queue.size();
    int64_t running = 0;
    for (auto &kv : S->reqs) running += kv.second->state == GF2_REQ_RUNNING;
    st->running = running;
    st->launches_batched = S->n_batched;
    st->launches_single = S->n_single;
    st->bytes_in_use = (int64_t)S->pool.used();
    st->bytes_peak = (int64_t)S->pool.peak();
    st->budget_bytes = (int64_t)S->budget;
    st->now = S->now();
    return GF2_OK;
}

gf2_status gf2_serve_destroy(gf2_serve *S) {
    if (!S) return GF2_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->th.joinable()) S->th.join();
    for (auto s : S->streams) (void)hipStreamSynchronize(s);
    for (auto s : S->streams) (void)hipStreamDestroy(s);
    for (auto e : S->events) (void)hipEventDestroy(e);
    if (S->base) (void)hipFree(S->base);
    delete S;
    return GF2_OK;
}

}  // extern "C"
