/*
 * CPU ORACLE for PLE decomposition over GF(2).  TEST INFRASTRUCTURE ONLY:
 * nothing in the product library calls, links or loads this file; only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark use it.
 * It shares no code, header or table with the HIP library.
 *
 * Reference: Albrecht, Bard, Pernet, "Efficient Dense Gaussian Elimination
 * over the Finite Field with Two Elements".
 *
 * What it computes (Section 2, definition of the PLE decomposition, with the
 * pivoting rule of Algorithm 1 and the output contract of Algorithm 2):
 * plain column-by-column Gaussian elimination.  For each column, left to
 * right, the pivot is the first row at or below the current rank position,
 * in the current row order, whose fully reduced entry is 1 (Algorithm 1's
 * search loop); the whole pivot row is swapped into place and recorded
 * LAPACK-style (Section 1.2: P_i = "swap row i with row P_i", applied in
 * order); every row below with a 1 in the pivot column gets the pivot row
 * added to the right of the pivot column, the 1 itself being kept as the
 * multiplier L[i][r].  Afterwards L is compressed (Algorithm 1's and
 * Algorithm 2's "compress L" column swaps): for each pivot j the multiplier
 * column Q_j is moved to column j in the rows below row j.
 *
 * Blocking, laziness, the table width k and the recursion of Algorithms 2-3
 * change only the order of the XORs, never a pivot decision, so this plain
 * definition is the exact result they must reproduce.
 *
 * Output convention ("clean" L\E, overwriting A):
 *   row i < r : columns < i hold L[i][0..i-1]; columns >= i hold row i of E
 *               (zero on [i, Q_i), 1 at Q_i);
 *   row i >= r: columns < r hold L[i][0..r-1]; columns >= r are zero.
 *   P[i] = i for i >= r;  Q[i] = -1 for r <= i < min(m, n).
 * Then P^T A = L E where P^T A applies the swaps i = 0, 1, ... to the rows
 * of A, L is m x r unit lower trapezoidal and E is r x n in echelon form.
 *
 * Readings of the paper this file takes (the paper is silent or garbled):
 *  - pivot = first row in current order, whole-row swap (not a rotation);
 *  - additions start right of the pivot column, so earlier multipliers of the
 *    pivot row are never added;
 *  - compression moves a multiplier only in rows strictly below row j, so
 *    E keeps its pivot 1 at (j, Q_j);
 *  - P has m entries (identity past the rank), Q has min(m, n) entries
 *    (-1 past the rank).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline int getbit(const uint64_t *row, int64_t j) { return (int)((row[j >> 6] >> (j & 63)) & 1ULL); }
static inline void setbit(uint64_t *row, int64_t j, int v) {
    uint64_t mask = 1ULL << (j & 63);
    if (v) row[j >> 6] |= mask; else row[j >> 6] &= ~mask;
}

/* The elimination of gf2o_ple over columns 0 .. c_end - 1 only (each of
 * those steps exactly as in the whole run, rows still updated up to column
 * n), then the compression of L for the pivots found.  With c_end = n it is
 * gf2o_ple; a smaller c_end times a bounded share of a large elimination. */
int64_t gf2o_ple_cols(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q, int64_t c_end) {
    int64_t mn = m < n ? m : n;
    for (int64_t i = 0; i < m; i++) P[i] = i;
    for (int64_t i = 0; i < mn; i++) Q[i] = -1;
    int64_t r = 0;
    if (c_end > n) c_end = n;
    for (int64_t c = 0; c < c_end && r < m; c++) {
        /* first non-zero in column c at or below row r, current order */
        int64_t p = -1;
        for (int64_t i = r; i < m; i++)
            if (getbit(A + i * ldw, c)) { p = i; break; }
        if (p < 0) continue;                       /* no pivot in column c */
        if (p != r) {                              /* swap whole rows */
            uint64_t *a = A + r * ldw, *b = A + p * ldw;
            for (int64_t w = 0; w < ldw; w++) { uint64_t t = a[w]; a[w] = b[w]; b[w] = t; }
        }
        P[r] = p;
        Q[r] = c;
        /* eliminate below: add the pivot row right of column c */
        const uint64_t *pr = A + r * ldw;
        int64_t w0 = c >> 6;
        uint64_t head = (c & 63) == 63 ? 0 : (~0ULL << ((c & 63) + 1));
        int64_t nw = (n + 63) >> 6;
#pragma omp parallel for schedule(static) if ((m - r) * (nw - w0) > (1 << 18))
        for (int64_t i = r + 1; i < m; i++) {
            uint64_t *row = A + i * ldw;
            if (!getbit(row, c)) continue;
            row[w0] ^= pr[w0] & head;
            for (int64_t w = w0 + 1; w < nw; w++) row[w] ^= pr[w];
        }
        r++;
    }
    /* compress L: move multiplier column Q_j to column j, rows below j */
    for (int64_t j = 0; j < r; j++) {
        int64_t q = Q[j];
        if (q == j) continue;
        for (int64_t i = j + 1; i < m; i++) {
            uint64_t *row = A + i * ldw;
            setbit(row, j, getbit(row, q));
            setbit(row, q, 0);
        }
    }
    return r;
}

/* PLE decomposition (Section 2 definition; pivot rule of Algorithm 1).
 * Returns the rank r.  A is m x n, ldw words per row, overwritten by L\E. */
int64_t gf2o_ple(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t *P, int64_t *Q) {
    return gf2o_ple_cols(A, m, n, ldw, P, Q, n);
}

/* E from clean L\E (Section 2 definitions): clear the L part, keep E rows. */
void gf2o_echelon_from_ple(uint64_t *A, int64_t m, int64_t n, int64_t ldw, int64_t r) {
    (void)n;
    for (int64_t i = 0; i < m; i++) {
        uint64_t *row = A + i * ldw;
        int64_t lim = i < r ? i : r;       /* L occupies columns < min(i, r) */
        if (i >= r) { memset(row, 0, (size_t)ldw * 8); continue; }
        for (int64_t j = 0; j < lim; j++) setbit(row, j, 0);
    }
}

/* RREF from clean L\E (Section 2: the reduced row echelon form is unique).
 * Back-substitution: for pivots j = r-1 .. 0, clear column Q_j in the rows
 * above using row j of E. */
void gf2o_rref_from_ple(uint64_t *A, int64_t m, int64_t n, int64_t ldw, const int64_t *Q, int64_t r) {
    gf2o_echelon_from_ple(A, m, n, ldw, r);
    int64_t nw = (n + 63) >> 6;
    for (int64_t j = r - 1; j >= 0; j--) {
        const uint64_t *pr = A + j * ldw;
        int64_t q = Q[j];
        for (int64_t i = 0; i < j; i++) {
            uint64_t *row = A + i * ldw;
            if (getbit(row, q))
                for (int64_t w = q >> 6; w < nw; w++) row[w] ^= pr[w];
        }
    }
}

/* C ^= A * B over GF(2), from the definition of the product: row i of A*B is
 * the sum of the rows k of B with A[i][k] = 1.  A is m x k, B is k x n. */
void gf2o_addmul(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda, const uint64_t *B, int64_t ldb,
                 int64_t m, int64_t k, int64_t n) {
    int64_t nw = (n + 63) >> 6;
#pragma omp parallel for schedule(static) if (m * k * nw > (1 << 20))
    for (int64_t i = 0; i < m; i++) {
        uint64_t *crow = C + i * ldc;
        const uint64_t *arow = A + i * lda;
        for (int64_t t = 0; t < k; t++)
            if (getbit(arow, t)) {
                const uint64_t *brow = B + t * ldb;
                for (int64_t w = 0; w < nw; w++) crow[w] ^= brow[w];
            }
    }
}

/* Table of all 2^k combinations of k rows (Appendix A, MakeTable and the
 * "M4RI idea" figure), from its definition rather than by Gray code: entry x
 * is the sum of the rows t whose bit is set in x, the first row being the
 * most significant of the k index bits (the figure indexes T by the leading
 * bits read left to right, e.g. 011 -> 3).  T has 2^k rows of nw words. */
void gf2o_make_table(const uint64_t *rows, int64_t ldr, int64_t k, int64_t nw, uint64_t *T) {
    int64_t size = (int64_t)1 << k;
    for (int64_t x = 0; x < size; x++) {
        uint64_t *trow = T + x * nw;
        memset(trow, 0, (size_t)nw * 8);
        for (int64_t t = 0; t < k; t++)
            if ((x >> (k - 1 - t)) & 1)
                for (int64_t w = 0; w < nw; w++) trow[w] ^= rows[t * ldr + w];
    }
}

#ifdef _OPENMP
#include <omp.h>
int gf2o_threads(void) { return omp_get_max_threads(); }
void gf2o_set_threads(int t) { omp_set_num_threads(t); }
#else
int gf2o_threads(void) { return 1; }
void gf2o_set_threads(int t) { (void)t; }
#endif
