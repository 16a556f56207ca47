// gf2_ple_noalloc: gf2_ple with its workspace in a static device array of
// the library instead of caller memory, for callers that cannot allocate.
//
// The array `scratch` is file-scope device memory: every GPU the library
// runs on holds its own copy (NOALLOC_SCRATCH_BYTES) until the process ends.
// Host code never passes `scratch` itself to a kernel (in host code that
// name is a host-side stand-in, not a device address); it passes the device
// address hipGetSymbolAddress returns, looked up once per device with that
// device current and kept in g_scratch_ptr.
#include <mutex>
#include <vector>

#include "../../include/gf2ple.h"
#include "batch.h"
#include "common.h"

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // per device: device address of `scratch`

// Device address of this device's copy of `scratch` (looked up on the first
// call on each device), or nullptr on a runtime error.
void *scratch_ptr() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_ptr[(size_t)dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[(size_t)dev] = p;
    }
    return g_scratch_ptr[(size_t)dev];
}

}  // namespace

extern "C" {

size_t gf2_ple_noalloc_max_workspace(void) { return NOALLOC_SCRATCH_BYTES; }

gf2_status gf2_ple_noalloc(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank,
                           const gf2_ple_opts *opts, void *stream) {
    const gf2_status chk = gf2::ple_check_args(A, m, n, ldw, P, Q, rank, opts);
    if (chk != GF2_OK) return chk;
    // the padding scan keeps a device flag of its own, and the recursive
    // schedules wait on the stream: neither is available here
    if (opts && (opts->check_padding || opts->update >= 2)) return GF2_EINVAL;
    if (gf2::ple_workspace_total(m, ldw) > NOALLOC_SCRATCH_BYTES) return GF2_EWORKSPACE;
    void *ws = scratch_ptr();
    if (!ws) return GF2_EHIP;
    // gf2_ple's workspace needs no initial contents, so nothing is cleared;
    // no host wait (passes past full rank exit at once) and no second stream
    const hipError_t e = gf2::ple_enqueue(A, m, n, ldw, P, Q, rank, ws, opts, (hipStream_t)stream, false, false);
    return e == hipSuccess ? GF2_OK : GF2_EHIP;
}

}  // extern "C"
