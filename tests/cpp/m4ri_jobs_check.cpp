// Model check of M4JobRing (the M4RI form's job bookkeeping) on random pass
// schedules: the guard calls and pushes follow the pass loop (a fused pair
// writes the records of passes t + 1 and t + 2, then pushes its job; a
// serial pass pushes its job, then its successor's panel writes record
// t + 1).  After every guard no outstanding job may read the slot about to
// be written, event indices of outstanding jobs stay distinct, and last()
// names the newest job.  Prints "ok" and returns 0, else names the failure.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "m4ri_jobs.h"

struct Job {
    long long first;
    int np, ev;
};

template <int R>
static bool run(std::mt19937_64 &rng, int npasses) {
    gf2::M4JobRing<R> ring;
    std::vector<Job> out;  // the model's outstanding jobs, oldest first
    auto guard = [&](long long x) {
        const int e = ring.guard(x);
        if (e >= 0) {  // jobs finish in order: the waited job and all before it are done
            int k = -1;
            for (int i = 0; i < (int)out.size(); i++)
                if (out[i].ev == e && out[i].first <= x - R) k = i;
            if (k < 0) {
                std::printf("R=%d guard(%lld) returned event %d of no eligible job\n", R, x, e);
                return false;
            }
            out.erase(out.begin(), out.begin() + k + 1);
        }
        for (const Job &j : out)
            for (int p = 0; p < j.np; p++)
                if ((j.first + p) % R == x % R && j.first + p < x) {
                    std::printf("R=%d: record %lld written while the job at pass %lld reads it\n", R, x, j.first);
                    return false;
                }
        return true;
    };
    auto push = [&](long long t, int np) {
        const int e = ring.push(t);
        if (e < 0) {
            std::printf("R=%d push(%lld) refused: %d jobs outstanding\n", R, t, (int)out.size());
            return false;
        }
        for (const Job &j : out)
            if (j.ev == e) {
                std::printf("R=%d: event %d reused while the job at pass %lld is outstanding\n", R, e, j.first);
                return false;
            }
        out.push_back({t, np, e});
        if (ring.last() != e) {
            std::printf("R=%d: last() %d, newest job's event %d\n", R, ring.last(), e);
            return false;
        }
        return true;
    };
    std::uniform_int_distribution<int> coin(0, 3);
    for (long long t = 0; t < npasses;) {
        if (t + 3 < npasses && coin(rng) != 0) {  // a fused pair
            if (!guard(t + 1) || !guard(t + 2) || !push(t, 2)) return false;
            t += 2;
            continue;
        }
        if (!push(t, 1)) return false;
        if (t + 1 >= npasses) break;
        if (!guard(t + 1)) return false;
        t += 1;
    }
    return true;
}

int main() {
    std::mt19937_64 rng(12345);
    for (int it = 0; it < 2000; it++) {
        const int np = 1 + (int)(rng() % 300);
        if (!run<8>(rng, np) || !run<4>(rng, np) || !run<3>(rng, np) || !run<2>(rng, np)) return 1;
    }
    std::printf("ok\n");
    return 0;
}
