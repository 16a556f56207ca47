"""Test-side checkers, written independently of both the oracle and the HIP
library: brute-force row spaces, reconstruction P^T A = L E from a packed
clean L\\E, the first-non-zero certificate for P, and golden-file parsing."""
import os

import numpy as np

from paper_1111_6549_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    """Parse a golden file: '# ...' comments, 'key:' starts a block of 0/1 rows,
    'key: a b c' is an inline integer list.  Repeated keys give lists."""
    blocks = []
    cur = None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if ":" in line:
                key, rest = line.split(":", 1)
                rest = rest.strip()
                if rest:
                    blocks.append((key, [int(x) for x in rest.split()]))
                    cur = None
                else:
                    cur = (key, [])
                    blocks.append(cur)
            else:
                cur[1].append([int(x) for x in line.split()])
    return blocks


def row_ints(bits):
    """0/1 rows -> python ints with bit j = column j."""
    out = []
    for row in np.asarray(bits):
        v = 0
        for j, b in enumerate(row):
            if b:
                v |= 1 << j
        out.append(v)
    return out


def brute_rowspace(rows):
    """All vectors of the row space (rows given as ints)."""
    space = {0}
    for v in rows:
        space |= {x ^ v for x in space}
    return space


def brute_facts(bits):
    """(rank, pivot columns, RREF rows) of a tiny 0/1 matrix by enumeration of
    its row space: the column rank profile is the set of leading positions of
    the non-zero row-space vectors; the RREF row of pivot q is the unique
    row-space vector led by q and zero on the other pivots."""
    bits = np.asarray(bits)
    space = brute_rowspace(row_ints(bits))
    rank = len(space).bit_length() - 1
    assert 1 << rank == len(space)
    lead = sorted({(v & -v).bit_length() - 1 for v in space if v})
    pivmask = 0
    for q in lead:
        pivmask |= 1 << q
    rref = []
    for q in lead:
        cands = [v for v in space if v and (v & -v) == (1 << q) and (v & pivmask) == (1 << q)]
        assert len(cands) == 1
        rref.append(cands[0])
    return rank, lead, rref


def split_LE(out_bits, r):
    """Clean L\\E (m x n 0/1) -> L (m x r, unit lower trapezoidal) and E (r x n)."""
    out_bits = np.asarray(out_bits, dtype=np.uint8)
    m, n = out_bits.shape
    L = np.zeros((m, r), dtype=np.uint8)
    E = np.zeros((r, n), dtype=np.uint8)
    for i in range(m):
        lim = min(i, r)
        L[i, :lim] = out_bits[i, :lim]
        if i < r:
            L[i, i] = 1
            E[i, i:] = out_bits[i, i:]
    return L, E


def apply_swaps(bits, P, r):
    """P^T A: apply the LAPACK-style swaps i = 0 .. r-1 to the rows of A."""
    B = np.array(bits, copy=True)
    for i in range(r):
        p = int(P[i])
        if p != i:
            B[[i, p]] = B[[p, i]]
    return B


def check_ple(A_bits, out_bits, r, P, Q):
    """Invariants of a PLE result in the clean L\\E convention; raises on failure."""
    A_bits = np.asarray(A_bits, dtype=np.uint8)
    out_bits = np.asarray(out_bits, dtype=np.uint8)
    m, n = A_bits.shape
    assert 0 <= r <= min(m, n)
    P = np.asarray(P)
    Q = np.asarray(Q)
    assert P.shape == (m,) and Q.shape == (min(m, n),)
    assert all(P[i] == i for i in range(r, m)), "P must be the identity past the rank"
    assert all(i <= P[i] < m for i in range(r)), "swap partner must be at or below"
    assert all(Q[i] == -1 for i in range(r, min(m, n))), "Q must be -1 past the rank"
    q = Q[:r]
    assert all(q[i] < q[i + 1] for i in range(r - 1)), "pivot columns increase"
    L, E = split_LE(out_bits, r)
    # non-pivot rows: zero from column r on
    for i in range(r, m):
        assert not out_bits[i, r:].any(), "rows past the rank are zero right of L"
    # E echelon with pivots q: zero left of q_i, 1 at q_i
    for i in range(r):
        assert not E[i, : q[i]].any(), "E row must be zero left of its pivot"
        assert E[i, q[i]] == 1, "E pivot entry must be 1"
    prod = (L.astype(np.int64) @ E.astype(np.int64)) & 1
    lhs = apply_swaps(A_bits, P, r)
    assert np.array_equal(lhs, prod.astype(np.uint8)), "P^T A != L E"


def check_first_nonzero(out_bits, r, P):
    """Certificate of the pivot rule: at step t the rows that sat at positions
    t .. P_t - 1 had a zero in the pivot column, so their final multiplier in
    column t of L is 0."""
    out_bits = np.asarray(out_bits)
    m = out_bits.shape[0]
    perm = list(range(m))          # perm[pos] = row id at that position
    steps = []
    for t in range(r):
        p = int(P[t])
        steps.append((t, [perm[pos] for pos in range(t, p)]))
        perm[t], perm[p] = perm[p], perm[t]
    final = {rid: pos for pos, rid in enumerate(perm)}
    for t, ids in steps:
        for rid in ids:
            pos = final[rid]
            assert pos > t, "a row skipped by pivot t must end below it"
            assert out_bits[pos, t] == 0, "row skipped by the pivot search has multiplier 1"


def xor_basis_rank(bits):
    """Rank of a 0/1 matrix by inserting its rows into a basis keyed by the
    highest set bit (a test-side routine, independent of both implementations)."""
    basis = {}
    rank = 0
    for v in row_ints(bits):
        while v:
            h = v.bit_length() - 1
            if h in basis:
                v ^= basis[h]
            else:
                basis[h] = v
                rank += 1
                break
    return rank


def gf2_rank_np(bits):
    """Rank over GF(2) of a medium 0/1 matrix (numpy, vectorised row reduction
    over the uint8 entries; test-side, independent of both implementations)."""
    M = np.array(bits, dtype=np.uint8) & 1
    m, n = M.shape
    r = 0
    for c in range(n):
        if r == m:
            break
        nz = np.nonzero(M[r:, c])[0]
        if nz.size == 0:
            continue
        p = r + nz[0]
        if p != r:
            M[[r, p]] = M[[p, r]]
        rows = np.nonzero(M[:, c])[0]
        rows = rows[rows != r]
        M[rows] ^= M[r]
        r += 1
    return r


def pack(bits, ldw=None):
    return inputs.pack(bits, ldw)


def unpack(A, n):
    return inputs.unpack(A, n)
