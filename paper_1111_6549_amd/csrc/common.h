// Internal declarations shared by the HIP kernels and the host driver of
// libgf2ple.  Not part of the public ABI (that is include/gf2ple.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gf2 {

// One pass of Algorithm 2 eliminates a stripe of KW columns.  KW = 64 keeps
// the stripe one aligned 64-bit word per row, since c advances by the full
// stripe width every pass whatever the stripe's rank.
constexpr int KW = 64;
// Largest pivot-search window held in registers by the panel wave: WIN_Q x 64 rows.
constexpr int WIN_Q = 8;
// Pivot rows plus rows displaced by the pass's swaps (each swap moves <= 2).
constexpr int MAX_SPEC = 2 * KW;
// Rows the slow pivot search keeps in LDS; beyond this it uses workspace.
constexpr int SLOW_LDS_ROWS = 9216;
// Pass records kept in the workspace ring: a pass's record is still read by
// the fused update of its pair while the panel two passes later writes its own,
// and by the M4RI form's elimination from the rows above, which runs behind
// the passes on a second stream (at most NREC passes behind).
constexpr int NREC = 8;
// Columns per trailing-update tile (words): 8 words = 64 B of each row.
constexpr int TILE_W = 8;
// Threads per block of the wide kernels.
constexpr int WIDE_THREADS = 1024;

// Everything a pass's later kernels need from its panel (Algorithm 1 on the
// stripe).  Notation: Orig_l = pivot row l as it stood when the pass began
// (after the swaps), w = coefficients of a row's update with respect to the
// Orig rows, u = the row's L bits (multipliers of the reduced pivot rows).
struct PassRec {
    int64_t r;       // rank before the pass (first row of the stripe's block)
    int32_t rbar;    // pivots found in the stripe
    int32_t nspec;   // special rows: rbar pivot positions, then displaced rows
    int32_t active;  // rbar > 0
    int32_t slow;    // 1 if the search needed more rows than the register window
    int64_t spec_dst[MAX_SPEC];      // position after the pass's swaps
    int64_t spec_src[MAX_SPEC];      // position of that row before the swaps
    uint64_t spec_coef[MAX_SPEC];    // w of the row
    uint64_t spec_lbits[MAX_SPEC];   // u of the row (rbar bits, placed at column r)
    uint64_t spec_stripe[MAX_SPEC];  // E part of the stripe word (pivot rows), else 0
    // look-ahead permutes only: the row's word of the next stripe with the
    // pass's update (after a pair, both passes'), for the next panel to take
    uint64_t spec_next[MAX_SPEC];
    uint64_t img_w[KW];  // stripe bit j -> w of a row whose stripe is e_j (linear map)
    uint64_t img_u[KW];  // stripe bit j -> u
};

__host__ __device__ inline int64_t words_for(int64_t n) { return (n + 63) >> 6; }

// Kernel timing: when enabled (gf2_profile_start), every launch site brackets
// its kernel with HIP events on the launch stream.
enum KernelId {
    KID_PANEL = 0,
    KID_PERMUTE,
    KID_M4RM,
    KID_INIT,
    KID_RREF,
    KID_ECHELON,
    KID_MFMA,
    KID_BATCH,
    KID_TRSM,
    KID_TRANSPOSE,
    KID_SUMS,
    KID_COUNT
};
bool prof_enabled();
void prof_mark(int kid, hipStream_t s, bool begin);

struct ProfScope {
    int kid;
    hipStream_t s;
    bool on;
    ProfScope(int k, hipStream_t st) : kid(k), s(st), on(prof_enabled()) {
        if (on) prof_mark(kid, s, true);
    }
    ~ProfScope() {
        if (on) prof_mark(kid, s, false);
    }
};

}  // namespace gf2
