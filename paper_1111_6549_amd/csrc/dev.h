// Small device helpers shared by the kernels (wave64 cross-lane moves).
#pragma once
#include "common.h"

namespace gf2 {

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int readlane32(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// lane l takes the (uniform) value v, the other lanes keep theirs
__device__ __forceinline__ uint64_t writelane64(uint64_t old, uint64_t v, int l) {
    return (int)__lane_id() == l ? v : old;
}

__device__ __forceinline__ int writelane32(int old, int v, int l) { return (int)__lane_id() == l ? v : old; }

// a value the whole wave agrees on, kept in a scalar register
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        lo |= (uint32_t)__shfl_xor((int)lo, off, 64);
        hi |= (uint32_t)__shfl_xor((int)hi, off, 64);
    }
    return ((uint64_t)hi << 32) | lo;
}

// A relaxed device-scope load: a vector load past the L1 cache (never the
// scalar cache), with no wait of its own, for data another wave of the
// launch may have written.
template <typename T>
__device__ __forceinline__ T ld_dev(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, off, 64);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), off, 64);
        const uint64_t o = ((uint64_t)hi << 32) | lo;
        v = o < v ? o : v;
    }
    return v;
}

// bits strictly above column j of a word
__device__ __forceinline__ uint64_t above(int j) { return j >= 63 ? 0ull : (~0ull << (j + 1)); }

// The part of the rbar-bit vector u (bit l = column r + l) that falls into word w.
__device__ __forceinline__ uint64_t place_bits(uint64_t u, int64_t w, int64_t wr0, int sh) {
    if (w == wr0) return u << sh;
    if (sh && w == wr0 + 1) return u >> (64 - sh);
    return 0;
}

// a ^ b ^ c in one instruction per 32-bit half (v_bitop3_b32 with the
// three-input XOR truth table 0x96).
__device__ __forceinline__ uint64_t xor3_64(uint64_t a, uint64_t b, uint64_t c) {
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, 0x96);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), 0x96);
    return ((uint64_t)hi << 32) | lo;
}

// New value of word w of a special row (a pivot or a row displaced by the
// pass's swaps): the stripe word becomes its L bits and, for a pivot, its E
// part; the words holding columns [r, c) get the L bits or-ed in; the rest
// move unchanged.
__device__ __forceinline__ uint64_t special_word(uint64_t old, int64_t w, int64_t sw, int64_t wr0, int sh,
                                                 uint64_t lbits, uint64_t stripe) {
    if (w == sw) return place_bits(lbits, w, wr0, sh) | stripe;
    if (w >= wr0 && w < sw) return old | place_bits(lbits, w, wr0, sh);
    return old;
}

}  // namespace gf2
