// Internal interface of the batched kernel, shared by the batched-plan
// entry points (batch.hip) and the serving session (serve.hip).
#pragma once
#include "../../include/gf2ple.h"
#include "common.h"

namespace gf2 {

// Where one workgroup's scratch lives inside its slot of the workspace.
struct SlotLayout {
    int64_t coef, pb, gsv, gsid, bytes;  // offsets from the slot start; PassRec at 0
};

struct BatchArgs {
    const gf2_desc *descs;
    const int32_t *order;     // matrix indices, most expensive first
    const int64_t *rank_off;  // NULL: rank of matrix i at ranks[i]; else at ranks[rank_off[i]]
    int32_t count;
    int32_t *counter;  // next position in `order` (zeroed before the launch)
    uint64_t *arena;
    int64_t *P;
    int64_t *Q;
    int64_t *ranks;
    uint8_t *slots;
    SlotLayout lay;
};

constexpr int NBATCH_CONFIGS = 8;

SlotLayout batch_slot_layout(int64_t mmax, int64_t ldwmax);
hipError_t batch_launch(int cfg, int grid, const BatchArgs &a, hipStream_t s);
hipError_t batch_reset(int32_t *counters, int n, hipStream_t s);
int batch_occupancy(int cfg);
// built-in schedule (0-based) for matrices whose larger side is at most max_dim
int batch_default_config(int64_t max_dim);

// gf2_ple after its argument checks.  allow_sync = false never waits on the
// stream (all passes are enqueued; those past full rank exit at once);
// allow_s2 = false keeps every kernel on `s` (look-ahead passes run
// serially instead of using the library's second stream).
hipError_t ple_enqueue(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank,
                       void *ws, const gf2_ple_opts *opts, hipStream_t s, bool allow_sync, bool allow_s2);
size_t ple_workspace_total(int64_t m, int64_t ldw);
// gf2_ple's argument checks (sizes, pointers, options), made before any
// device call.
gf2_status ple_check_args(const uint64_t *A, int64_t m, int64_t n, int64_t ldw, const int64_t *P, const int64_t *Q,
                          const int64_t *rank, const gf2_ple_opts *opts);

}  // namespace gf2
