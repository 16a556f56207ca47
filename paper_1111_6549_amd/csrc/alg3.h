// Internal interface of the block-recursive PLE (Algorithm 3, Section 3.3):
// the recursion in alg3.hip drives the block-iterative pass loop of api.hip
// on column blocks of the matrix.
#pragma once
#include "../../include/gf2ple.h"
#include "common.h"

namespace gf2 {

// The pass loop of Algorithm 2 on the m x n block at A (row stride ldw),
// whose swaps move whole rows: words [wlo, wlo + ldw) relative to A (wlo <= 0).
// May synchronise the stream (the early stop at full rank).
hipError_t ple_block(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank, void *ws,
                     const gf2_ple_opts *opts, hipStream_t s, int64_t wlo);
size_t ple_workspace_total(int64_t m, int64_t ldw);

// Extra workspace of the recursion beyond the pass loop's, for an m x n
// matrix: the sub-ranks and, with matrix-core products, the bit transpose of
// the largest product's right operand.
size_t alg3_extra_bytes(int64_t m, int64_t n, int64_t ldw, int levels, bool mfma, int64_t split, int psplit);

// Algorithm 3 with `levels` levels of column splits (then Algorithm 2):
// products on the Four-Russians tables (products = 0), the fp4 matrix cores
// (1) or the int8 matrix cores (2).  split = 0: halves, both recursing;
// split > 0: a left strip of `split` columns (a leaf) and the recursion in
// the right block.  Synchronises the stream once per split (to size the
// products by the left block's rank).
// psplit: Strassen's split of the fp4 products (gf2_ple_opts.product_split).
hipError_t ple_alg3(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank, void *ws,
                    const gf2_ple_opts *opts, hipStream_t s, int levels, int products, int64_t split, int psplit);

// The steps of an m x k x n product C ^= A B on the fp4 matrix cores: one
// product, or one level of Strassen's split (gf2_product_plan).
int64_t product_plan(int64_t m, int64_t k, int64_t n, int split, int64_t lda, int64_t ldbt, int64_t ldc,
                     gf2_plan_step *st, int64_t max, int64_t *ws_words);
int64_t product_plan_ws_bound(int64_t m, int64_t k, int64_t n);

}  // namespace gf2
