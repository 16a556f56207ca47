"""CPU model of the block-recursive PLE (Algorithm 3, Section 3.3) as the
library schedules it (update = 2 / 3): the steps in the library's order with
its index arithmetic -- the column split at a multiple of 64, the left PLE
whose swaps move whole rows, the triangular solve and product on the right
block, the right PLE, the P / Q / rank combination and the word walk that
moves the right block's L bits left -- with the oracle's PLE at the leaves.
The result must equal the oracle's PLE of the whole matrix (its arithmetic
is checked, not the kernels': those are compared with the oracle on the GPU).
"""
import numpy as np
import pytest

import oracle
from paper_1111_6549_amd import inputs
from tests import helpers as H


def _leaf(M, r0, c0, m, n, P, Q):
    """The pass loop on the block M[r0:r0+m, c0:c0+n], swaps of whole rows."""
    blk = H.pack(M[r0:r0 + m, c0:c0 + n])
    r, Pb, Qb = oracle.ple(blk, n)
    out = H.unpack(blk, n)
    for t in range(r):  # the same swaps on the rest of each row
        p = int(Pb[t])
        if p != t:
            for cols in (slice(0, c0), slice(c0 + n, M.shape[1])):
                a = M[r0 + t, cols].copy()
                M[r0 + t, cols] = M[r0 + p, cols]
                M[r0 + p, cols] = a
    M[r0:r0 + m, c0:c0 + n] = out
    P[r0:r0 + m] = Pb
    Q[r0:r0 + min(m, n)] = Qb
    return r


def _shift_words(row_words, r1, n1, nL):
    """The library's word walk for one row (k_alg3_shift): columns
    [n1, n1 + nL) move to [r1, r1 + nL), the columns they leave become 0."""
    def rbits(a, b, w):
        lo = 64 * w
        x0, x1 = max(a, lo), min(b, lo + 64)
        if x0 >= x1:
            return 0
        ln = x1 - x0
        return (((1 << ln) - 1) << (x0 - lo)) & ((1 << 64) - 1)
    d = n1 - r1
    s1 = n1 + nL
    wlast = (s1 - 1) >> 6
    row = [int(x) for x in row_words]
    full = (1 << 64) - 1
    for w in range(r1 >> 6, wlast + 1):
        md, ms = rbits(r1, r1 + nL, w), rbits(n1, s1, w)
        v = row[w] & ~ms & ~md & full
        if md:
            sc = 64 * w + d
            sw, sh = sc >> 6, sc & 63
            assert 0 <= sw <= wlast
            a = row[sw]
            b = row[sw + 1] if (sh and sw + 1 <= wlast) else 0
            sv = ((a >> sh) | (b << (64 - sh))) & full if sh else a
            v |= sv & md
        row[w] = v
    return np.array(row, dtype=np.uint64)


def _rec(M, r0, c0, m, n, P, Q, levels, split=0):
    if levels <= 0 or n <= 64 or m == 0 or (split > 0 and n <= split):
        return _leaf(M, r0, c0, m, n, P, Q)
    # halves (both recursing) or a left strip of `split` columns (a leaf)
    n1 = min(split, n) if split > 0 else (n // 2 + 63) // 64 * 64
    r1 = _rec(M, r0, c0, m, n1, P, Q, 0 if split > 0 else levels - 1, split)
    N = n - n1
    if r1 > 0:
        # A01 <- L00^-1 A01 (forward substitution), then A11 += L10 A01
        X = M[r0:r0 + r1, c0 + n1:c0 + n].astype(np.int64)
        L = np.tril(M[r0:r0 + r1, c0:c0 + r1].astype(np.int64), -1)
        for i in range(r1):
            X[i] = (X[i] + L[i, :i] @ X[:i]) & 1
        M[r0:r0 + r1, c0 + n1:c0 + n] = X
        if m > r1:
            L10 = M[r0 + r1:r0 + m, c0:c0 + r1].astype(np.int64)
            M[r0 + r1:r0 + m, c0 + n1:c0 + n] ^= ((L10 @ X) & 1).astype(np.uint8)
    if m <= r1:
        return r1
    r2 = _rec(M, r0 + r1, c0 + n1, m - r1, N, P, Q, levels - 1, split)
    mn = min(m, n)
    q_right = min(m - r1, N)
    for i in range(r1, max(m, mn)):
        if i < m:
            P[r0 + i] += r1
        if i < mn:
            if i < r1 + q_right:
                if Q[r0 + i] >= 0:
                    Q[r0 + i] += n1
            else:
                Q[r0 + i] = -1
    if r1 < n1:
        for i in range(r1, m):
            nL = min(i - r1, r2)
            if nL <= 0:
                continue
            words = H.pack(M[r0 + i:r0 + i + 1, c0:c0 + n])[0]
            M[r0 + i, c0:c0 + n] = H.unpack(_shift_words(words, r1, n1, nL)[None, :], n)[0]
    return r1 + r2


def model_alg3(A, n, levels, split=0):
    m = A.shape[0]
    M = H.unpack(A, n).copy()
    P = np.zeros(m, np.int64)
    Q = np.full(min(m, n), -1, np.int64)
    r = _rec(M, 0, 0, m, n, P, Q, levels, split)
    return r, P, Q, H.pack(M, A.shape[1])


def _case(kind, m, n, seed):
    n1 = (n // 2 + 63) // 64 * 64
    if kind == "u":
        return inputs.bernoulli(m, n, seed)
    if kind == "s":
        return inputs.bernoulli(m, n, seed, p=3.0 / n)
    if kind == "r":
        return inputs.known_rank(m, n, max(1, min(m, n) // 3), seed, seed + 1)
    if kind == "deficient_left":
        left = H.unpack(inputs.known_rank(m, n1, n1 // 2, seed, seed + 1), n1)
        right = H.unpack(inputs.bernoulli(m, n - n1, seed + 2), n - n1)
        return H.pack(np.concatenate([left, right], axis=1))
    if kind == "zero_left":
        right = H.unpack(inputs.bernoulli(m, n - n1, seed), n - n1)
        return H.pack(np.concatenate([np.zeros((m, n1), np.uint8), right], axis=1))
    raise ValueError(kind)


@pytest.mark.parametrize("m,n,kind,levels", [(200, 200, "u", 1), (130, 300, "u", 1), (300, 130, "u", 1),
                                             (250, 260, "deficient_left", 1), (150, 400, "deficient_left", 2),
                                             (400, 150, "deficient_left", 1), (200, 260, "zero_left", 1),
                                             (300, 300, "s", 2), (280, 330, "r", 3), (65, 130, "u", 1),
                                             (64, 65, "u", 1), (500, 700, "deficient_left", 3)])
def test_alg3_model_equals_oracle(m, n, kind, levels):
    A = _case(kind, m, n, 70 + m + n)
    r, P, Q, LE = model_alg3(A, n, levels)
    B = A.copy()
    ro, Po, Qo = oracle.ple(B, n)
    assert r == ro
    assert np.array_equal(Q, Qo)
    assert np.array_equal(P, Po)
    assert np.array_equal(LE, B)


@pytest.mark.parametrize("m,n,kind,levels,split", [(300, 300, "u", 16, 64), (400, 260, "deficient_left", 16, 128),
                                                   (200, 500, "u", 3, 128), (260, 400, "zero_left", 16, 64),
                                                   (350, 330, "r", 2, 192), (200, 640, "deficient_left", 16, 64),
                                                   (500, 700, "s", 16, 256)])
def test_alg3_strips_model_equals_oracle(m, n, kind, levels, split):
    """Left strips of `split` columns, the recursion going on in the right
    block (update = 2 / 3 / 4 with rec_split > 0)."""
    A = _case(kind, m, n, 90 + m + n)
    r, P, Q, LE = model_alg3(A, n, levels, split)
    B = A.copy()
    ro, Po, Qo = oracle.ple(B, n)
    assert r == ro
    assert np.array_equal(Q, Qo)
    assert np.array_equal(P, Po)
    assert np.array_equal(LE, B)


def _trsm_blocked_words(W, r, xw0, xw1):
    """The triangular solve as the library runs it, on packed words W (rows
    x words, the L bits of row i in its words left of column i): 128-row
    blocks in order; in each, the two-rows-per-lane forward substitution
    (first half from word lw's bits below the lane, second half from all of
    word lw then word lw + 1's bits below the lane), then the rows below the
    block take the block's rows selected by their words lw, lw + 1."""
    W = W.copy()
    for b in range(0, r, 128):
        _trsm_step_words(W, b, r, xw0, xw1)
    return W


def _trsm_step_words(W, b, r, xw0, xw1):
    """One 128-row step of the blocked solve, in place: rows b .. b + 127
    (up to r) by forward substitution, then rows b + 128 .. r - 1 lose them,
    on words [xw0, xw1)."""
    one = np.uint64(1)
    nb = min(128, r - b)
    lw = b // 64
    for w in range(xw0, xw1):
        x0 = [W[b + l, w] if l < nb else np.uint64(0) for l in range(64)]
        x1 = [W[b + 64 + l, w] if 64 + l < nb else np.uint64(0) for l in range(64)]
        below = [np.uint64(0) if l == 0 else np.uint64((1 << l) - 1) for l in range(64)]
        l0 = [W[b + l, lw] & below[l] if l < nb else np.uint64(0) for l in range(64)]
        l1a = [W[b + 64 + l, lw] if 64 + l < nb else np.uint64(0) for l in range(64)]
        l1b = [W[b + 64 + l, lw + 1] & below[l] if 64 + l < nb else np.uint64(0) for l in range(64)]
        for j in range(min(nb, 64)):
            xj = x0[j]
            for l in range(64):
                if (l0[l] >> np.uint64(j)) & one:
                    x0[l] ^= xj
                if (l1a[l] >> np.uint64(j)) & one:
                    x1[l] ^= xj
        for j in range(max(0, nb - 64 - 1)):
            xj = x1[j]
            for l in range(64):
                if (l1b[l] >> np.uint64(j)) & one:
                    x1[l] ^= xj
        for l in range(64):
            if l < nb:
                W[b + l, w] = x0[l]
            if 64 + l < nb:
                W[b + 64 + l, w] = x1[l]
    for i in range(b + nb, r):
        c = [W[i, lw], W[i, lw + 1]]
        for j in range(nb):
            if (c[j >> 6] >> np.uint64(j & 63)) & one:
                W[i, xw0:xw1] ^= W[b + j, xw0:xw1]


@pytest.mark.parametrize("r,ncols,seed", [(300, 200, 1), (128, 70, 2), (129, 64, 3), (256, 130, 4), (64, 64, 5),
                                          (20, 100, 6)])
def test_blocked_trsm_words_equal_forward_substitution(r, ncols, seed):
    """The library's blocked solve (its word indices and masks) equals plain
    forward substitution X <- L^-1 X for a random unit lower triangular L.
    The bits on and right of the diagonal of the L block (the E part of those
    rows in L\\E) are random too: the solve must not read them."""
    rng = np.random.default_rng(seed)
    nl = (r + 63) // 64 * 64
    Lb = np.tril(rng.integers(0, 2, (r, r), dtype=np.uint8), -1)
    Eb = np.triu(rng.integers(0, 2, (r, nl), dtype=np.uint8))
    Xb = rng.integers(0, 2, (r, ncols), dtype=np.uint8)
    M = np.zeros((r, nl + ncols), np.uint8)
    M[:, :nl] = Eb
    M[:, :r] |= Lb
    M[:, nl:] = Xb
    W = H.pack(M)
    xw0 = nl // 64
    got = H.unpack(_trsm_blocked_words(W, r, xw0, W.shape[1]), nl + ncols)[:, nl:]
    X = Xb.astype(np.int64)
    for i in range(r):
        X[i] = (X[i] + Lb[i, :i].astype(np.int64) @ X[:i]) & 1
    assert np.array_equal(got, X.astype(np.uint8))


def _solve_by_inverses_words(W, r, xw0, blk):
    """The solve as the library runs it with fp4 products and a rank above
    one diagonal block: the inverses of the diagonal blocks L_dd (blk rows)
    by the blocked forward substitution (_trsm_blocked_words) of each block
    on its own identity, every 128-row step covering only the words up to
    its rows' columns (an inverse's row has no bit past its own column);
    then per block, left-looking, X_d += L[d][0, d0) X[0, d0) and
    X_d += (L_dd^-1 + I) X_d, both as plain products mod 2."""
    W = W.copy()
    bw = blk // 64
    nblk = (r + blk - 1) // blk
    # Y: row i = row i - d0 of L_dd^-1, bw words, columns relative to d0
    Y = np.zeros((r, bw), dtype=np.uint64)
    for i in range(r):
        rel = i % blk
        Y[i, rel // 64] = np.uint64(1) << np.uint64(rel % 64)
    for d in range(nblk):
        d0, d1 = d * blk, min(r, (d + 1) * blk)
        K = d1 - d0
        # the block's L bits in its own columns (words d0 / 64 ..) next to Y
        Lblk = H.unpack(W[d0:d1, :], W.shape[1] * 64)[:, d0:d1]
        M = np.zeros((K, (K + 63) // 64 * 64 + blk), dtype=np.uint8)
        M[:, :K] = Lblk
        M[:, (K + 63) // 64 * 64:] = H.unpack(Y[d0:d1], blk)
        Mw = H.pack(M)
        xo = (K + 63) // 64
        for b in range(0, K, 128):
            # one 128-row step on the words up to its rows' columns only
            _trsm_step_words(Mw, b, K, xo, xo + min(bw, (b + 128) // 64))
        Y[d0:d1] = Mw[:, xo:xo + bw]
    # N = Y + I
    for i in range(r):
        rel = i % blk
        Y[i, rel // 64] ^= np.uint64(1) << np.uint64(rel % 64)
    nx = W.shape[1] - xw0
    X = H.unpack(W[:, xw0:], nx * 64).astype(np.int64)
    Lbits = H.unpack(W, W.shape[1] * 64)[:, :r].astype(np.int64)
    for d in range(nblk):
        d0, d1 = d * blk, min(r, (d + 1) * blk)
        if d0 > 0:
            X[d0:d1] = (X[d0:d1] + Lbits[d0:d1, :d0] @ X[:d0]) & 1
        N = H.unpack(Y[d0:d1], blk).astype(np.int64)[:, :d1 - d0]
        X[d0:d1] = (X[d0:d1] + N @ X[d0:d1]) & 1
    W[:, xw0:] = H.pack(X.astype(np.uint8), nx)
    return W


@pytest.mark.parametrize("r,ncols,blk,seed", [(300, 200, 128, 1), (520, 70, 256, 2), (1000, 130, 256, 3),
                                              (384, 64, 128, 4), (257, 100, 128, 5)])
def test_solve_by_block_inverses_equals_forward_substitution(r, ncols, blk, seed):
    """The solve by the diagonal blocks' inverses, left-looking between the
    blocks (X_d loses the solved blocks above it, then X_d += (L_dd^-1 + I)
    X_d), equals plain forward substitution X <- L^-1 X for a random unit
    lower triangular L, with random bits on and right of the diagonal of the
    L part (the E part of those rows), which the solve must not read."""
    rng = np.random.default_rng(seed)
    nl = (r + 63) // 64 * 64
    Lb = np.tril(rng.integers(0, 2, (r, r), dtype=np.uint8), -1)
    Eb = np.triu(rng.integers(0, 2, (r, nl), dtype=np.uint8))
    Xb = rng.integers(0, 2, (r, ncols), dtype=np.uint8)
    M = np.zeros((r, nl + ncols), np.uint8)
    M[:, :nl] = Eb
    M[:, :r] |= Lb
    M[:, nl:] = Xb
    W = H.pack(M)
    xw0 = nl // 64
    got = H.unpack(_solve_by_inverses_words(W, r, xw0, blk), nl + ncols)[:, nl:]
    X = Xb.astype(np.int64)
    for i in range(r):
        X[i] = (X[i] + Lb[i, :i].astype(np.int64) @ X[:i]) & 1
    assert np.array_equal(got, X.astype(np.uint8))
