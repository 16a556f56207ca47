// Bookkeeping of the M4RI form's eliminations (Appendix, Algorithms 5-8: each
// column block removed from the rows above its pivots), which run as jobs on
// a second stream behind the PLE passes that follow them.
//
// A job over passes first .. first + np - 1 reads those passes' records from
// the ring of R records (pass t's record is slot t mod R).  Before a kernel
// writes the record of pass x, every job that read the slot x shares must be
// done: the jobs over passes <= x - R.  Jobs finish in order (one stream), so
// waiting for the last such job covers the earlier ones.  Each job records
// one of R events; at most R jobs are outstanding once every record write is
// guarded, so an event is not recorded again while its job is waited on.
//
// Host code only, no allocation.
#pragma once
#include <cstdint>

namespace gf2 {

template <int R>
struct M4JobRing {
    int64_t first[R] = {};
    int ev[R] = {};
    int head = 0, count = 0;
    int64_t njobs = 0;

    // A new job whose first pass is `first_pass`: the event index it records.
    // Returns -1 when R jobs are already outstanding (a missing guard).
    int push(int64_t first_pass) {
        if (count == R) return -1;
        const int e = (int)(njobs++ % R);
        const int slot = (head + count) % R;
        first[slot] = first_pass;
        ev[slot] = e;
        count++;
        return e;
    }

    // Before a kernel writes the record of pass x: the event to wait for, or
    // -1 when no outstanding job read that record's slot.
    int guard(int64_t x) {
        int e = -1;
        while (count > 0 && first[head] <= x - R) {
            e = ev[head];
            head = (head + 1) % R;
            count--;
        }
        return e;
    }

    // The event of the last job pushed, or -1 (to join the streams at the end).
    int last() const { return count > 0 ? ev[(head + count - 1) % R] : -1; }
};

}  // namespace gf2
