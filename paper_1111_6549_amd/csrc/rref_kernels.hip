// RREF from a PLE result (Section 2: the reduced row echelon form is unique;
// Section 5 computes it from the PLE output).  Back-substitution by blocks
// of 64 pivots, last block first, each block being one Four-Russians
// product:
//   U     = block rows at the block's pivot columns (unit upper triangular),
//   Y     = U^-1,
//   new block rows   = Y * block            (rows become reduced on the block)
//   rows above (i<j0): row_i ^= (c_i Y) * block, c_i = row_i at the pivot columns.
// k_rref_block computes Y (per workgroup), stages the block rows and writes
// every row's coefficient word; the update itself is k_m4rm.
#include "common.h"

namespace gf2 {

__device__ __forceinline__ uint64_t rl64(uint64_t v, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

constexpr int RREF_THREADS = 256;

// Bits q0 .. q0 + nb - 1 of a row, from its words holding column q0 (w0)
// and the next one (w1, zero when q0 is word-aligned or the row ends).
__device__ __forceinline__ uint64_t funnel_bits(uint64_t w0, uint64_t w1, int64_t q0, int nb) {
    const int sh = (int)(q0 & 63);
    uint64_t c = w0 >> sh;
    if (sh) c |= w1 << (64 - sh);
    return nb == 64 ? c : (c & ((1ull << nb) - 1ull));
}

// A row's bits at the block's pivot columns, bit t = column Q[j0 + t].  With
// contiguous pivot columns (q0 = the first, q0 >= 0) that is one funnel
// shift of the two words holding them; otherwise one bit at a time.
__device__ __forceinline__ uint64_t pivot_bits(const uint64_t *row, const int64_t *sq, int nb, int64_t q0,
                                               int64_t nw) {
    if (q0 >= 0) {
        const int64_t w = q0 >> 6;
        const int sh = (int)(q0 & 63);
        uint64_t c = row[w] >> sh;
        if (sh && w + 1 < nw) c |= row[w + 1] << (64 - sh);
        return nb == 64 ? c : (c & ((1ull << nb) - 1ull));
    }
    int64_t cw = -1;
    uint64_t cur = 0, c = 0;
    for (int t = 0; t < nb; t++) {
        const int64_t q = sq[t];
        if ((q >> 6) != cw) {
            cw = q >> 6;
            cur = row[cw];
        }
        c |= ((cur >> (q & 63)) & 1ull) << t;
    }
    return c;
}

// Rows [j1, jz) get a zero coefficient (rows below the block that a fused
// pair's sweep also covers).  With rec, the block is described there as a
// pass of pivots j0 .. j1 - 1 (their rows' positions in spec_src) for the
// fused pair update.
//
// With drec (the forward elimination of the M4RI form), the block is that
// pass's pivot rows, r .. r + rbar - 1, just left by a PLE pass: a pivot
// row's columns left of its pivot column hold L bits, which are masked
// (only its E part enters U and the staged rows), and q0 = -2 asks the
// kernel to find out itself whether the pivot columns are contiguous.
struct RrefBlockArgs {
    int64_t j0, j1, ws0, q0, jz;
    uint64_t *coef, *PB;
    PassRec *rec;
    const PassRec *drec;
    int nA;  // staging workgroups; the rest of the set's nwg write coefficients
    int nwg;
};

// One workgroup (bid of the set's nwg) of a block's job.
__device__ __forceinline__ void rref_block_body(const uint64_t *__restrict__ A, int64_t ldw, int64_t nw,
                                                const int64_t *__restrict__ Q, const RrefBlockArgs &a, int bid,
                                                int64_t *sq, uint64_t *sY, uint64_t (*tab)[256], int64_t *sq0) {
    const bool mask_l = a.drec != nullptr;
    int64_t j0 = a.j0, j1 = a.j1, q0 = a.q0;
    if (a.drec) {
        j0 = a.drec->r;
        j1 = j0 + (a.drec->active ? a.drec->rbar : 0);
    }
    const int tid = threadIdx.x;
    const int nb = (int)(j1 - j0);

    if (bid < a.nA) {  // stage the block rows' words >= ws0
        const int64_t w = a.ws0 + (int64_t)bid * 64 + (tid & 63);
        if (w >= nw) return;
        // every load before the first store (the stores could alias the
        // rows for all the compiler knows, which would serialise the copy)
        constexpr int RG = RREF_THREADS / 64;  // row groups
        constexpr int PER = KW / RG;            // rows per thread
        uint64_t v[PER];
        int64_t q[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int k = (tid >> 6) + RG * u;
            v[u] = k < nb ? A[(j0 + k) * ldw + w] : 0ull;
            q[u] = (mask_l && k < nb) ? Q[j0 + k] : 0;
        }
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int k = (tid >> 6) + RG * u;
            if (k >= nb) break;
            uint64_t x = v[u];
            if (mask_l) {  // the row's E part: columns from its pivot column on
                const int64_t b = w * 64;
                x = q[u] >= b + 64 ? 0ull : (q[u] > b ? x & ~((1ull << (q[u] - b)) - 1ull) : x);
            }
            a.PB[(int64_t)k * ldw + w] = x;
        }
        return;
    }

    // The words this thread will need are loaded first, on the guess that
    // the pivot columns are contiguous from qs = Q[j0] (always so at full
    // rank): the row it finishes (at most one per thread when the grid
    // covers jz) and, in wave 0, its pivot row's.  They arrive while U, Y
    // and the tables are worked out; a wrong guess falls back to pivot_bits.
    const int64_t i0 = (int64_t)(bid - a.nA) * RREF_THREADS + tid;
    const int64_t qs = q0 >= 0 ? q0 : (q0 == -2 && nb > 0 ? Q[j0] : -1);
    uint64_t rw0 = 0, rw1 = 0, uw0 = 0, uw1 = 0;
    if (qs >= 0) {
        const int64_t w = qs >> 6;
        const bool two = (qs & 63) && w + 1 < nw;
        if (i0 < j0) {
            rw0 = A[i0 * ldw + w];
            if (two) rw1 = A[i0 * ldw + w + 1];
        }
        if (tid < nb) {
            uw0 = A[(j0 + tid) * ldw + w];
            if (two) uw1 = A[(j0 + tid) * ldw + w + 1];
        }
    }
    if (tid < KW) sq[tid] = tid < nb ? Q[j0 + tid] : 0;
    if (a.rec && bid == a.nA) {
        if (tid < nb) a.rec->spec_src[tid] = j0 + tid;
        if (tid == 0) {
            a.rec->r = 0;
            a.rec->rbar = nb;
            a.rec->nspec = nb;
            a.rec->active = nb > 0;
            a.rec->slow = 0;
        }
    }
    __syncthreads();
    if (q0 == -2) {  // contiguous pivot columns?
        if (tid == 0) {
            int64_t f = nb > 0 ? sq[0] : -1;
            for (int t = 1; t < nb; t++)
                if (sq[t] != sq[0] + t) f = -1;
            *sq0 = f;
        }
        __syncthreads();
        q0 = *sq0;
    }
    if (tid < 64) {  // wave 0: Y = U^-1
        const int lane = tid;
        uint64_t U = 0;
        if (lane < nb) U = (q0 >= 0 && q0 == qs) ? funnel_bits(uw0, uw1, q0, nb) : pivot_bits(A + (j0 + lane) * ldw, sq, nb, q0, nw);
        if (mask_l) U &= ~((1ull << lane) - 1ull);  // L bits (pivot columns left of its own)
        uint64_t Y = 1ull << lane;
        for (int t = nb - 1; t >= 0; t--) {
            const uint64_t yt = rl64(Y, t);
            if (lane < t && ((U >> t) & 1ull)) Y ^= yt;
        }
        sY[lane] = Y;
    }
    __syncthreads();
    for (int e = tid; e < 8 * 256; e += RREF_THREADS) {
        const int b = e >> 8, x = e & 255;
        uint64_t y = 0;
        for (int t = 0; t < 8; t++)
            if (((x >> t) & 1) && 8 * b + t < nb) y ^= sY[8 * b + t];
        tab[b][x] = y;
    }
    __syncthreads();
    const int64_t nG = (int64_t)a.nwg - a.nA;
    for (int64_t i = (int64_t)(bid - a.nA) * RREF_THREADS + tid; i < a.jz; i += nG * RREF_THREADS) {
        if (i >= j1) {
            a.coef[i] = 0;
            continue;
        }
        if (i >= j0) {
            a.coef[i] = sY[i - j0] ^ (1ull << (i - j0));
            continue;
        }
        const uint64_t c = (i == i0 && q0 >= 0 && q0 == qs) ? funnel_bits(rw0, rw1, q0, nb)
                                                             : pivot_bits(A + i * ldw, sq, nb, q0, nw);
        uint64_t w = 0;
        if (c) {
#pragma unroll
            for (int b = 0; b < 8; b++) w ^= tab[b][(c >> (8 * b)) & 255];
        }
        a.coef[i] = w;
    }
}

__global__ __launch_bounds__(RREF_THREADS) void k_rref_block(const uint64_t *__restrict__ A, int64_t ldw, int64_t nw,
                                                             const int64_t *__restrict__ Q, RrefBlockArgs a) {
    __shared__ int64_t sq[KW];
    __shared__ uint64_t sY[KW];
    __shared__ uint64_t tab[8][256];
    __shared__ int64_t sq0;
    rref_block_body(A, ldw, nw, Q, a, (int)blockIdx.x, sq, sY, tab, &sq0);
}

// Two blocks' jobs in one launch (the two blocks of a fused back-substitution
// sweep read the rows as they stand and write separate outputs): workgroups
// below a.nwg take the first, the rest the second.
__global__ __launch_bounds__(RREF_THREADS) void k_rref_block2(const uint64_t *__restrict__ A, int64_t ldw,
                                                              int64_t nw, const int64_t *__restrict__ Q,
                                                              RrefBlockArgs a, RrefBlockArgs b) {
    __shared__ int64_t sq[KW];
    __shared__ uint64_t sY[KW];
    __shared__ uint64_t tab[8][256];
    __shared__ int64_t sq0;
    const int bid = (int)blockIdx.x;
    if (bid < a.nwg)
        rref_block_body(A, ldw, nw, Q, a, bid, sq, sY, tab, &sq0);
    else
        rref_block_body(A, ldw, nw, Q, b, bid - a.nwg, sq, sY, tab, &sq0);
}

static RrefBlockArgs rref_args(int64_t nw, int64_t j0, int64_t j1, int64_t ws0, int64_t q0, int64_t jz,
                               uint64_t *coef, uint64_t *PB, PassRec *rec, const PassRec *drec) {
    RrefBlockArgs a;
    a.j0 = j0;
    a.j1 = j1;
    a.ws0 = ws0;
    a.q0 = q0;
    a.jz = jz;
    a.coef = coef;
    a.PB = PB;
    a.rec = rec;
    a.drec = drec;
    a.nA = (int)((nw - ws0 + 63) / 64);
    int nG = (int)((jz + RREF_THREADS - 1) / RREF_THREADS);
    if (nG > 512) nG = 512;
    if (nG < 1) nG = 1;
    a.nwg = a.nA + nG;
    return a;
}

hipError_t launch_rref_block(uint64_t *A, int64_t ldw, int64_t nw, const int64_t *Q, int64_t j0, int64_t j1,
                             int64_t ws0, int64_t q0, int64_t jz, uint64_t *coef, uint64_t *PB, PassRec *rec,
                             hipStream_t s, const PassRec *drec) {
    const RrefBlockArgs a = rref_args(nw, j0, j1, ws0, q0, jz, coef, PB, rec, drec);
    ProfScope ps(KID_RREF, s);
    hipLaunchKernelGGL(k_rref_block, dim3(a.nwg), dim3(RREF_THREADS), 0, s, (const uint64_t *)A, ldw, nw, Q, a);
    return hipGetLastError();
}

hipError_t launch_rref_block2(uint64_t *A, int64_t ldw, int64_t nw, const int64_t *Q, int64_t ws0, int64_t jz,
                              int64_t j0a, int64_t j1a, int64_t q0a, uint64_t *coefa, uint64_t *PBa, PassRec *reca,
                              int64_t j0b, int64_t j1b, int64_t q0b, uint64_t *coefb, uint64_t *PBb, PassRec *recb,
                              hipStream_t s, const PassRec *dreca, const PassRec *drecb) {
    const RrefBlockArgs a = rref_args(nw, j0a, j1a, ws0, q0a, jz, coefa, PBa, reca, dreca);
    const RrefBlockArgs b = rref_args(nw, j0b, j1b, ws0, q0b, jz, coefb, PBb, recb, drecb);
    ProfScope ps(KID_RREF, s);
    hipLaunchKernelGGL(k_rref_block2, dim3(a.nwg + b.nwg), dim3(RREF_THREADS), 0, s, (const uint64_t *)A, ldw, nw, Q,
                       a, b);
    return hipGetLastError();
}

}  // namespace gf2
