/*
 * gf2ple: PLE decomposition over GF(2) on MI355X (gfx950), C ABI.
 *
 * Method: Albrecht, Bard, Pernet, "Efficient Dense Gaussian Elimination over
 * the Finite Field with Two Elements" -- block-iterative PLE (Algorithm 2)
 * whose trailing update is the Method of Four Russians: all 2^k sums of k
 * pivot rows in a table (MakeTable, Appendix A) and one table row added per
 * matrix row (AddRowsFromTable, Appendix A).
 *
 * Packed format (Section 1.1, Section 2 "row major representation"):
 *   an m x n matrix over GF(2) is m rows of `ldw` 64-bit words, row-major;
 *   column j of row i is bit (j & 63) of word A[i*ldw + (j >> 6)].
 *   ldw >= ceil(n/64); every bit at a column >= n must be zero.
 *
 * Conventions shared by all calls:
 *   - Every matrix, permutation, rank and workspace pointer is a DEVICE
 *     pointer owned by the caller; the library never frees or keeps them.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     stream-ordered and return once the work is enqueued, except where a
 *     call says it synchronises.
 *   - Errors are return codes.  An error found before launch leaves every
 *     output untouched.  After GF2_EHIP the outputs are undefined
 *     (hipGetLastError() has the runtime's detail).
 *   - Calls on different streams with disjoint buffers are independent.
 */
#ifndef GF2PLE_H
#define GF2PLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gf2_status {
    GF2_OK = 0,
    GF2_EINVAL = 1,     /* negative size, ldw < ceil(n/64), NULL or misaligned pointer, bad option */
    GF2_EWORKSPACE = 2, /* workspace smaller than the matching *_workspace_bytes() */
    GF2_ENOMEM = 3,     /* a host-side allocation failed (serving sessions) */
    GF2_EBUDGET = 4,    /* serving: request larger than the whole device budget */
    GF2_EHIP = 5,       /* HIP runtime error */
    GF2_EPADDING = 6,   /* check_padding: a bit at a column >= n is set */
    GF2_EBUSY = 7       /* serving: no ticket of that number is pending */
} gf2_status;

/* Schedule options.  A NULL pointer or a zeroed struct selects the defaults. */
typedef struct gf2_ple_opts {
    int32_t check_padding; /* 1: scan for set bits at columns >= n first (synchronises) */
    int32_t update;        /* 0 = default = 1: Algorithm 2, every trailing update by the Four-Russians tables;
                              2 = Algorithm 3 (block-recursive PLE, Section 3.3): split the columns (in
                              halves, or a left strip of rec_split columns), PLE of the left block,
                              A01 <- L00^-1 A01, then A11 <- A11 + L10 A01 as a product on the fp4 matrix
                              cores, PLE of A11, and the two blocks' P, Q and L combined; rec_levels levels
                              of splits, Algorithm 2 below them.  Bit-identical to Algorithm 2.
                              Synchronises once per split.
                              3 = the same recursion with its products on the Four-Russians tables;
                              4 = the same recursion with its products on the int8 matrix cores.
                              gf2_addmul: 2 = fp4 matrix cores, 4 = int8 matrix cores, else tables */
    int32_t rec_levels;    /* update = 2 or 3: levels of Algorithm 3 splits (0 = 1, at most 16) */
    int32_t m4_variant;    /* Four-Russians update schedule: 0 = default, 1..8 = a fixed (tile, threads, unroll) */
    int32_t m4_blocks;     /* target blocks per update launch (0 = default 512) */
    int32_t panel_regs;    /* pivot-search register window of the panel: 0 = default, 2, 4 or 8 x 64 rows */
    int32_t lookahead;     /* 0 = pairs of passes share one trailing update (the later pass's next panel runs
                              inside that update) while rows remain below the stripe, then serial passes;
                              1 = serial passes only; 2 = look-ahead on every pass (next panel on a second
                              stream beside the update), no pairs; 3 = pairs on every pass */
    int32_t pair_variant;  /* schedule of the fused pair update: 0 = default; 1..12 = a fixed (threads, rows in
                              flight, table reads per group, coefficient prefetch); 13 / 14 = the default
                              schedule with the next panel always / never in a block of its own (the
                              default gives it one when the sweep is short) */
    int32_t rec_split;     /* update = 2, 3 or 4: 0 = split each block's columns in halves (both halves
                              recurse); > 0 (a multiple of 64) = the left block of every split is a strip of
                              rec_split columns done by Algorithm 2, and the splits go on in the right block
                              while levels remain and it is wider than rec_split */
    int32_t product_split; /* update = 2: Strassen's split of the fp4 products (see gf2_product_plan):
                              0 = default (one level on products whose three sizes are all at least
                              GF2_PLAN_MIN_BITS), 1 = one level on every product the split allows, -1 = none */
} gf2_ple_opts;

/* Library version string, e.g. "gf2ple 0.1.0 gfx950". */
const char *gf2_version(void);

/* Text for a status code (static storage). */
const char *gf2_status_str(gf2_status s);

/* Bytes of device workspace gf2_ple needs for an m x n matrix with row
 * stride ldw (tables, per-row coefficients, pivot block, pass record and
 * the pivot-search scratch).  Returns 0 for invalid sizes. */
size_t gf2_ple_workspace_bytes(int64_t m, int64_t n, int64_t ldw, const gf2_ple_opts *opts);

/*
 * PLE decomposition A = P L E (Section 2, definition of the PLE
 * decomposition; computed by Algorithm 2 with Algorithm 1's pivot rule).
 *
 *   A    [in/out] m x n packed, row stride ldw words.  Overwritten by L\E in
 *        the space-sharing form of Section 1.2, "clean" variant:
 *          row i <  r: columns < i hold L[i][0..i-1]; columns >= i hold row i
 *                      of E (zero before its pivot Q[i], 1 at Q[i]);
 *          row i >= r: columns < r hold L[i][0..r-1]; columns >= r are zero.
 *   P    [out] m entries, LAPACK-style swap vector (Section 1.2): P^T A is A
 *        with rows i and P[i] swapped for i = 0, 1, ... in order; P[i] = i
 *        for i >= r.
 *   Q    [out] min(m, n) entries: Q[i] = column of the i-th pivot (the column
 *        rank profile, Section 2), -1 for i >= r.
 *   rank [out] one int64: r.
 *   ws   device workspace of at least gf2_ple_workspace_bytes(m, n, ldw)
 *        bytes, 256-byte aligned; its contents need not be initialised.
 *
 * The pivot of each column is the first row at or below the current rank in
 * the current row order (Algorithm 1), swapped in whole; so P, L, E are
 * unique and bit-identical to plain Gaussian elimination with that rule.
 * When n > m the call may synchronise the stream once the rank can have
 * reached m, to skip passes that have nothing left to do.
 */
gf2_status gf2_ple(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank,
                   void *ws, size_t ws_bytes, const gf2_ple_opts *opts, void *stream);

/*
 * gf2_ple without caller workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as gf2_ple, except:
 *   - the workspace is a static device array of the library, one per GPU,
 *     gf2_ple_noalloc_max_workspace() bytes (16 MiB), held from the first
 *     call on that GPU until the process ends; GF2_EWORKSPACE when
 *     gf2_ple_workspace_bytes(m, n, ldw) exceeds it (e.g. m = 65536 with
 *     ldw = 1024 needs about 4 MiB);
 *   - every call on one GPU shares that array, so calls that overlap on one
 *     GPU (on different streams, or from different host threads without
 *     ordering) race and give undefined results: order them on one stream;
 *   - it never waits on the stream and never uses a second stream (the
 *     passes past full rank are enqueued and exit at once);
 *   - opts->check_padding and opts->update >= 2 are rejected (GF2_EINVAL).
 * It calls no hipMalloc / hipFree.
 */
size_t gf2_ple_noalloc_max_workspace(void);
gf2_status gf2_ple_noalloc(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank,
                           const gf2_ple_opts *opts, void *stream);

/*
 * The pass schedule gf2_ple follows for an m x n matrix with these options
 * (host only, no device call): kinds[t] for each 64-column pass t of
 * Algorithm 2, for up to max passes:
 *   0 serial: panel, permute, update of every word right of the stripe;
 *   1 look-ahead: the update covers the words from the stripe + 2 (permute
 *     and the next panel take the next stripe word) and the next panel runs
 *     on a second stream beside it;
 *   2, 3 a fused pair: pass 2 has no update of its own, pass 3's update
 *     covers both passes on the words from the pair's first stripe + 3.
 * Returns the number of passes, ceil(n/64), or -1 for invalid arguments.
 * (Where the look-ahead's second stream cannot be made, the passes run
 * serially instead.)
 */
int64_t gf2_ple_schedule(int64_t m, int64_t n, const gf2_ple_opts *opts, int32_t *kinds, int64_t max);

/* A block of a product plan step: rows [row0, row0 + rows) and bits [0, bits) starting at word word0 of
 * a buffer whose rows are ld words apart.  buf: 0 = the left operand A, 1 = the bit transpose of the
 * right operand B (one row per column of B, zero past the inner size), 2 = the result C, 3 = the
 * plan's workspace (row0 = 0, word0 = the block's offset in words).  rows = 0: no block. */
typedef struct {
    int64_t buf, row0, word0, ld, rows, bits;
} gf2_plan_block;

/* A step.  kind 0, a sum: b[0] = b[1] ^ b[2] over b[0]'s rows and bits, b[1] and b[2] read as zero
 * outside their own rows and bits.  kind 1, a product: the product of b[0] (rows x inner size
 * b[0].bits) and the matrix whose bit transpose is b[1] (b[1].rows columns) is added to b[2] and,
 * if b[3].rows > 0, to b[3], each over its own rows and bits (at most the product's). */
typedef struct {
    int64_t kind;
    gf2_plan_block b[4];
} gf2_plan_step;

#define GF2_PLAN_MIN_BITS 8192
#define GF2_PLAN_MAX_STEPS 17

/*
 * The plan by which gf2_ple (update = 2, Algorithm 3 of Section 3.3) adds a product C (m x n) ^= A (m x k)
 * * B (k x n) on the fp4 matrix cores (host only, no device call).  Section 3.3 notes that the paper's
 * implementation multiplies by Strassen-Winograd; with split = 1 (or 0 and all three sizes at least
 * GF2_PLAN_MIN_BITS, and n a multiple of 64) the plan is one level of Strassen's split: C, A and B in
 * 2 x 2 blocks (the rows of A and C split at their middle rounded up to a multiple of 256, the inner
 * size at its middle rounded up to an even number of words, the columns at their middle rounded up to
 * a multiple of 256 bits; where that rounding leaves no second part, at the middle itself), ten block
 * sums in the workspace, then seven products of half size, each added to one or two blocks of C.  Over GF(2) every sign of
 * Strassen's formulas is a plus.  Otherwise (split = -1, or sizes too small to split) the plan is one
 * product.  lda, ldbt, ldc fill the ld of the blocks in buffers 0, 1, 2.  Writes up to max steps
 * (at most GF2_PLAN_MAX_STEPS) and *ws_words (the workspace in 8-byte words); returns the number of
 * steps, or -1 for invalid arguments.
 */
int64_t gf2_product_plan(int64_t m, int64_t k, int64_t n, int32_t split, int64_t lda, int64_t ldbt, int64_t ldc,
                         gf2_plan_step *steps, int64_t max, int64_t *ws_words);

/* Echelon form from a PLE result (Section 2, row echelon form): in place,
 * A <- E: rows i < r keep columns >= i (their L part is cleared), rows
 * i >= r become zero.  `rank` is the device int64 written by gf2_ple. */
gf2_status gf2_echelon_from_ple(uint64_t *A, int64_t m, int64_t n, int64_t ldw, const int64_t *rank, void *stream);

/* Bytes of workspace gf2_rref_from_ple needs. */
size_t gf2_rref_workspace_bytes(int64_t m, int64_t n, int64_t ldw);

/* Reduced row echelon form from a PLE result (Section 2: the RREF is unique;
 * Section 5 recovers it from the PLE output): in place, A <- RREF of the
 * original matrix in rows 0..r-1 and zero below.  Q and rank are the device
 * outputs of gf2_ple. */
gf2_status gf2_rref_from_ple(uint64_t *A, int64_t m, int64_t n, int64_t ldw, const int64_t *Q, const int64_t *rank,
                             void *ws, size_t ws_bytes, void *stream);

/* gf2_ple followed by gf2_rref_from_ple (the "PLE" timing of Section 5).
 * P and Q are still required (they are outputs of the decomposition). */
size_t gf2_rref_full_workspace_bytes(int64_t m, int64_t n, int64_t ldw, const gf2_ple_opts *opts);
gf2_status gf2_rref(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t *rank,
                    void *ws, size_t ws_bytes, const gf2_ple_opts *opts, void *stream);

/* Bytes of workspace gf2_m4ri_rref needs. */
size_t gf2_m4ri_rref_workspace_bytes(int64_t m, int64_t n, int64_t ldw);

/* Reduced row echelon form in the M4RI form (Appendix, Algorithms 5-8: each
 * block of columns is eliminated from every row, above and below its
 * pivots): in place, A <- RREF in rows 0..r-1 and zero below.  The blocks
 * are the passes of gf2_ple's default schedule (a fused pair of 64-column
 * passes is one 128-column block: pivot search, swaps, update of the rows
 * below); each block is then reduced and eliminated from the rows above, on
 * the same table kernels, on a second stream of the library's own behind the
 * passes that follow (joined into `stream` before the call's last kernel).
 * Q[0..r) receives the pivot columns, *rank the
 * rank (device pointers, caller-owned); ws is device workspace of at least
 * gf2_m4ri_rref_workspace_bytes, 256-byte aligned.  Stream-ordered; one
 * host synchronisation once the rank may have reached m.  Errors as
 * gf2_ple. */
gf2_status gf2_m4ri_rref(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *Q, int64_t *rank, void *ws,
                         size_t ws_bytes, void *stream);

/*
 * C ^= A * B over GF(2): the Four-Russians product that Algorithm 2 applies
 * to the trailing block (A22 <- L21 A12 + A22; M4RM, Section 3.2), as a
 * standalone call.  A is m x k (row stride lda words), B is k x n (ldb),
 * C is m x n (ldc).  For each 64-column slice of A the 64 matching rows of B
 * are tabulated 8 at a time (256-entry tables) and one table row per byte of
 * A's word is added to C.  opts->update = 2 selects the matrix-core product
 * instead (the product Algorithm 3 hands to matrix multiplication;
 * bit-identical): B is bit-transposed into the workspace, the bits become
 * fp4 (e2m1) operands 0.0 / 1.0 and the exact fp32 sums are taken mod 2;
 * opts->update = 4 does the same with int8 operands and int32 sums.
 *   ws  device workspace of at least gf2_addmul_workspace_bytes(m, k, n,
 *       opts) bytes (0 for the table product, where ws may be NULL).
 */
size_t gf2_addmul_workspace_bytes(int64_t m, int64_t k, int64_t n, const gf2_ple_opts *opts);
gf2_status gf2_addmul(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda, const uint64_t *B, int64_t ldb,
                      int64_t m, int64_t k, int64_t n, void *ws, size_t ws_bytes, const gf2_ple_opts *opts,
                      void *stream);

/*
 * MakeTable (Appendix A): T[x] = sum of the rows t of `rows` whose bit
 * (k-1-t) is set in x, i.e. the first row is the most significant index bit
 * (the order of Appendix A's figure).  rows: k x n packed (stride ldr),
 * 1 <= k <= 8; T: 2^k rows of ldt words (ldt >= ceil(n/64)).  Built by the
 * Gray-code enumeration, 2^k - 1 row additions.
 */
gf2_status gf2_make_table(const uint64_t *rows, int64_t ldr, int32_t k, int64_t n, uint64_t *T, int64_t ldt,
                          void *stream);

/* Scan for set bits at columns >= n (padding); synchronises the stream.
 * Returns GF2_OK or GF2_EPADDING. */
gf2_status gf2_check_padding(const uint64_t *A, int64_t m, int64_t n, int64_t ldw, void *stream);

/*
 * Batched PLE: many independent matrices of uneven shape, each decomposed
 * exactly as gf2_ple would (same P, Q, rank and L\E, bit for bit), by one
 * persistent kernel per size class whose workgroups take matrices from a
 * device-side queue.  The method per matrix is Algorithm 2 with Algorithm 1
 * panels and a Four-Russians update (Section 3.2, Appendix A); batching is an
 * extension for throughput, not part of the paper.
 *
 * A plan is made once per set of shapes (host descriptors), then executed any
 * number of times on arenas holding those shapes.  The first execution with a
 * given (arena, P, Q, ranks, ws) records the plan's launches into a HIP graph
 * that later executions with the same pointers replay.
 */
typedef struct gf2_desc {
    int64_t a_off; /* first word of the matrix in the uint64 arena: m rows of ldw words */
    int64_t m, n, ldw;
    int64_t p_off; /* first of its m entries in the P arena */
    int64_t q_off; /* first of its min(m, n) entries in the Q arena */
} gf2_desc;

typedef struct gf2_batch_opts {
    int32_t autotune;  /* 1: time every candidate schedule per size class on synthetic matrices of the
                          plan's shapes when the plan is made, keep the fastest (allocates and
                          synchronises during gf2_batch_plan_create); 0: built-in choice */
    int32_t config;    /* 1..gf2_batch_num_configs(): force that schedule for every class; 0: choose */
    int32_t no_graph;  /* 1: launch directly on each execution instead of replaying a HIP graph */
    int32_t reserved[5];
} gf2_batch_opts;

typedef struct gf2_batch_plan gf2_batch_plan;

/* Class of a batch plan as chosen: matrices whose larger side is at most
 * max_dim, the schedule used for them, and the persistent grid size. */
typedef struct gf2_batch_class {
    int64_t max_dim;
    int64_t count;
    int32_t config;   /* 1-based schedule index */
    int32_t grid;     /* workgroups of the persistent launch */
    double tuned_ms;  /* time of the chosen schedule when autotuned, else 0 */
} gf2_batch_class;

/* Make a plan.  descs: `count` HOST descriptors (copied).  arena_words,
 * p_len, q_len: element counts of the arenas the plan will be executed on;
 * every descriptor must lie inside them (GF2_EINVAL otherwise), as must
 * ldw >= ceil(n/64), m, n >= 0.  Descriptors must not overlap (not checked).
 * Allocates device memory for the descriptors; *plan receives the handle. */
gf2_status gf2_batch_plan_create(const gf2_desc *descs, int64_t count, int64_t arena_words, int64_t p_len,
                                 int64_t q_len, const gf2_batch_opts *opts, gf2_batch_plan **plan);

/* Device workspace gf2_ple_batched needs with this plan (256-byte aligned). */
size_t gf2_batch_workspace_bytes(const gf2_batch_plan *plan);

/* Execute: every matrix of the plan is decomposed in place in `arena`
 * (device), its P and Q written at p_off / q_off of the device arenas P and
 * Q, and its rank to ranks[i] (device, `count` int64).  Stream-ordered.
 * Executions of one plan must not overlap unless they use distinct
 * workspaces; each execution needs the full workspace. */
gf2_status gf2_ple_batched(gf2_batch_plan *plan, uint64_t *arena, int64_t *P, int64_t *Q, int64_t *ranks, void *ws,
                           size_t ws_bytes, void *stream);

/* The chosen classes (up to max entries; *nclasses = number of classes). */
gf2_status gf2_batch_plan_info(const gf2_batch_plan *plan, gf2_batch_class *out, int32_t max, int32_t *nclasses);

/* Release a plan (waits for nothing: the caller makes sure no execution is in flight). */
gf2_status gf2_batch_plan_destroy(gf2_batch_plan *plan);

/* Number of batched schedules and the name of schedule i (1-based). */
int32_t gf2_batch_num_configs(void);
const char *gf2_batch_config_name(int32_t config);

/*
 * Serving session: a request loop that keeps packed matrices resident on the
 * device and decomposes them as they arrive.  Requests are admitted in
 * arrival order while their device memory (matrix, P, Q, rank, and for large
 * ones the PLE workspace) fits the session's budget; admitted requests are
 * launched at once on one of several streams -- all admitted small requests
 * together as one batched launch (the persistent kernel of gf2_ple_batched),
 * each large request as its own gf2_ple pass loop -- so requests that arrive
 * while others run join the next launch and overlap with the running ones
 * (continuous batching).  Each result is bit-identical to gf2_ple on that
 * matrix alone.  The session runs its own host thread; all calls are safe
 * from any host thread.  Serving is an extension for throughput, not part of
 * the paper.
 */
typedef struct gf2_serve_opts {
    int64_t budget_bytes;  /* device memory of the session, allocated once at create (0 = 64 GiB) */
    int32_t streams;       /* launch streams (0 = 3, at most 16) */
    int32_t max_batch;     /* most requests in one batched launch (0 = 4096) */
    int32_t small_max_dim; /* max(m, n) up to which a request runs in batched launches (0 = 2048, at most 4096) */
    int32_t reserved[3];
} gf2_serve_opts;

typedef struct gf2_serve gf2_serve;

enum { GF2_REQ_QUEUED = 0, GF2_REQ_RUNNING = 1, GF2_REQ_DONE = 2, GF2_REQ_FAILED = 3 };

typedef struct gf2_serve_info {
    int32_t state;  /* GF2_REQ_*: queued for admission, resident and launched, result in device memory, failed */
    int32_t status; /* gf2_status of a failed request */
    int64_t m, n, ldw;
    double t_submit, t_admit, t_done; /* seconds on the session's steady clock (0 = not yet) */
} gf2_serve_info;

typedef struct gf2_serve_stats {
    int64_t submitted, completed, failed, queued, running;
    int64_t launches_batched, launches_single;
    int64_t bytes_in_use, bytes_peak, budget_bytes;
    double now; /* current time on the session clock */
} gf2_serve_stats;

/* Create a session (allocates the budget on the current device and starts the
 * session thread).  GF2_EINVAL for bad options, GF2_ENOMEM / GF2_EHIP if the
 * budget cannot be allocated. */
gf2_status gf2_serve_create(const gf2_serve_opts *opts, gf2_serve **session);

/* Submit an m x n packed matrix (row stride ldw words).  a_on_device = 0: A is
 * host memory, copied before the call returns.  a_on_device = 1: A is device
 * memory whose contents must be complete when the call is made (the stream
 * that wrote them synchronised: the session's copy is not ordered after the
 * caller's streams) and must stay allocated and unchanged until the request
 * is done or failed (the copy into the session's pool runs when the request
 * is launched, which can be after admission).
 * *ticket receives the request id.  GF2_EBUDGET if the request could never
 * fit the budget; GF2_EINVAL for bad sizes. */
gf2_status gf2_serve_submit(gf2_serve *session, const uint64_t *A, int32_t a_on_device, int64_t m, int64_t n,
                            int64_t ldw, int64_t *ticket);

/* State of a request without waiting; GF2_EBUSY for an unknown ticket. */
gf2_status gf2_serve_poll(gf2_serve *session, int64_t ticket, gf2_serve_info *info);

/* Wait until the request is done or failed. */
gf2_status gf2_serve_wait(gf2_serve *session, int64_t ticket, gf2_serve_info *info);

/* Copy a finished request's results out -- L\E (m rows of ldw_out words,
 * ldw_out >= ceil(n/64), extra words zero), P (m), Q (min(m, n)), rank (1);
 * any pointer may be NULL -- to host memory (to_device = 0) or device memory
 * (to_device = 1), synchronously (on the default stream), then release the
 * request.  GF2_EBUSY if the
 * ticket is unknown or not done; a failed request returns its status and is
 * released. */
gf2_status gf2_serve_fetch(gf2_serve *session, int64_t ticket, uint64_t *LE, int64_t ldw_out, int64_t *P, int64_t *Q,
                           int64_t *rank, int32_t to_device);

/* Release a finished request without copying it out. */
gf2_status gf2_serve_release(gf2_serve *session, int64_t ticket);

/* Counters of the session. */
gf2_status gf2_serve_stats_get(gf2_serve *session, gf2_serve_stats *stats);

/* Stop the session thread after the running launches finish, free the budget
 * and every request. */
gf2_status gf2_serve_destroy(gf2_serve *session);

/*
 * Kernel timing.  Between gf2_profile_start() and gf2_profile_stop() every
 * kernel the library launches is bracketed by two HIP events recorded on its
 * launch stream (a small overhead per launch).  gf2_profile_stop waits for
 * the recorded events and writes up to max_entries per-kernel totals
 * (launch count, summed/min/max elapsed milliseconds) to `out` (host memory),
 * and the number of kernels seen to *count.  Process-wide; not for
 * concurrent use from several host threads.  Names: "panel", "permute",
 * "m4rm" (the Four-Russians updates), "init", "rref_block", "echelon",
 * "mfma" (matrix-core products), "batch", "trsm" (Algorithm 3's triangular
 * solve), "transpose" (bit transpose of a product's right operand) and "sums" (the block sums of
 * Strassen's split of a product).
 */
typedef struct gf2_kernel_time {
    char name[32];
    int64_t launches;
    double total_ms;
    double min_ms;
    double max_ms;
} gf2_kernel_time;

gf2_status gf2_profile_start(void);
gf2_status gf2_profile_stop(gf2_kernel_time *out, int32_t max_entries, int32_t *count);

#ifdef __cplusplus
}
#endif
#endif /* GF2PLE_H */
