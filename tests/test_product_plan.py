"""The plan by which Algorithm 3 (Section 3.3) adds its products on the fp4
matrix cores (gf2_product_plan, host only): one product, or one level of
Strassen's split (the paper's implementation multiplies by
Strassen-Winograd).  The plan is executed here with numpy, reading whole
words the way the kernels do (a product reads every word its inner size
touches, junk bits past it included; the right operand is a bit transpose
that is zero past the inner size), on operands whose bits past k are junk,
and must give the oracle's product.  Every block must lie inside its buffer
and the workspace inside the library's bound."""
import numpy as np
import pytest

import oracle
from paper_1111_6549_amd import gf2ple as G
from paper_1111_6549_amd import inputs
from tests import helpers as H


def words(bits):
    return (bits + 63) // 64


def to_bits(W):
    """(r, w) uint64 words -> (r, 64 w) 0/1 array, bit j of word w = column 64 w + j."""
    b = np.unpackbits(np.ascontiguousarray(W).view(np.uint8), bitorder="little")
    return b.reshape(W.shape[0], W.shape[1] * 64)


def to_words(B):
    r, c = B.shape
    assert c % 64 == 0
    return np.packbits(B.astype(np.uint8), axis=1, bitorder="little").view(np.uint64).reshape(r, c // 64)


def last_mask(bits):
    return np.uint64((1 << (bits % 64)) - 1) if bits % 64 else np.uint64(0xFFFFFFFFFFFFFFFF)


def run_plan(plan, ws_words, A, Bt, C):
    """Execute the plan on A (lda words), Bt (ldbt), C (ldc) and a workspace."""
    ws = np.full(max(ws_words, 1), 0x5A5A5A5A5A5A5A5A, dtype=np.uint64)  # stale contents
    bufs = {0: A.reshape(-1), 1: Bt.reshape(-1), 2: C.reshape(-1), 3: ws}

    def view(b, nrows, nwords):
        buf, row0, word0, ld = b[0], b[1], b[2], b[3]
        flat = bufs[buf]
        out = np.zeros((nrows, nwords), dtype=np.uint64)
        for i in range(nrows):
            s = (row0 + i) * ld + word0
            assert 0 <= s and s + nwords <= flat.size, (b, i)
            out[i] = flat[s:s + nwords]
        return out

    def store(b, M, xor):
        buf, row0, word0, ld = b[0], b[1], b[2], b[3]
        flat = bufs[buf]
        for i in range(M.shape[0]):
            s = (row0 + i) * ld + word0
            assert 0 <= s and s + M.shape[1] <= flat.size, (b, i)
            if xor:
                flat[s:s + M.shape[1]] ^= M[i]
            else:
                flat[s:s + M.shape[1]] = M[i]

    for kind, b in plan:
        if kind == 0:
            d, x, y = b[0], b[1], b[2]
            dw = words(d[5])
            acc = np.zeros((d[4], dw), dtype=np.uint64)
            for src in (x, y):
                r, w = min(src[4], d[4]), min(words(src[5]), dw)
                if r and w:
                    v = view(src, r, w)
                    if w == words(src[5]):
                        v[:, w - 1] &= last_mask(src[5])
                    acc[:r, :w] ^= v
            acc[:, dw - 1] &= last_mask(d[5])
            store(d, acc, False)
        else:
            a, bt, o0, o1 = b
            kw = words(a[5])
            nrow = 64 * words(bt[4])  # the kernel reads whole words of columns
            P = (to_bits(view(a, a[4], kw)).astype(np.int64) @ to_bits(view(bt, nrow, kw)).astype(np.int64).T) & 1
            Pw = to_words(P)
            for o in (o0, o1):
                if o[4] == 0:
                    continue
                assert o[4] <= a[4] and words(o[5]) <= Pw.shape[1]
                store(o, Pw[:o[4], :words(o[5])], True)


def bit_transpose(B, k, n):
    """B (k x n bits, packed) -> Bt (64 words(n) rows x words(k) words), zero past k and n."""
    bits = np.zeros((64 * words(n), 64 * words(k)), dtype=np.uint8)
    bits[:n, :k] = H.unpack(B, n).T
    return to_words(bits)


CASES = [(2, 256, 128), (3, 300, 192), (300, 700, 640), (513, 1000, 1280), (257, 4100, 704),
         (1000, 64 * 7 + 5, 64 * 9), (600, 512, 256 * 3), (1200, 2048, 1024), (40, 64 * 5, 64 * 3)]


@pytest.mark.parametrize("m,k,n", CASES)
@pytest.mark.parametrize("split", [-1, 0, 1])
def test_plan_gives_the_product(m, k, n, split):
    seed = m + 3 * k + 7 * n + split
    A = inputs.bernoulli(m, k, seed)
    B = inputs.bernoulli(k, n, seed + 1)
    C0 = inputs.bernoulli(m, n, seed + 2)
    want = C0.copy()
    oracle.addmul(want, A, B, k, n)
    lda, ldc = A.shape[1] + 1, C0.shape[1] + 3  # row strides past the used words
    Aj = np.random.default_rng(seed).integers(0, 2**63, size=(m, lda), dtype=np.int64).view(np.uint64)
    Aw = A.view(np.uint64)
    for w in range(Aw.shape[1]):  # A's words, then junk past k (the rest of a wider matrix)
        keep = last_mask(k) if w == Aw.shape[1] - 1 else np.uint64(0xFFFFFFFFFFFFFFFF)
        Aj[:, w] = (Aw[:, w] & keep) | (Aj[:, w] & ~keep)
    Bt = bit_transpose(B, k, n)
    Cw = np.zeros((m, ldc), dtype=np.uint64)
    Cw[:, :C0.shape[1]] = C0.view(np.uint64)
    plan, ws_words = G.product_plan(m, k, n, split, lda, Bt.shape[1], ldc)
    halved = split == 1 and n % 64 == 0 and m >= 2 and words(k) >= 4 and words(n) >= 2
    assert len(plan) == (17 if halved else 1)
    run_plan(plan, ws_words, Aj, Bt, Cw)
    assert np.array_equal(Cw[:, :C0.shape[1]], want.view(np.uint64))


def test_default_split_sizes_and_workspace_bound():
    """The default splits only products whose three sizes are all at least
    GF2_PLAN_MIN_BITS; blocks stay inside their buffers and the workspace
    inside the bound the library sizes Algorithm 3's workspace by."""
    assert len(G.product_plan(8191, 40960, 40960, 0)[0]) == 1
    assert len(G.product_plan(40960, 8000, 40960, 0)[0]) == 1
    for m, k, n in [(40960, 24576, 40960), (8192, 8192, 8192), (65535, 24570, 40960), (20000, 9001, 12288),
                    (9000, 30000, 8192 + 64)]:
        lda, ldbt, ldc = words(k) + 5, words(k), words(n) + 7
        plan, ws = G.product_plan(m, k, n, 0, lda, ldbt, ldc)
        assert len(plan) == 17
        kl = words(k) // 2 + 3
        assert ws <= 5 * ((m // 2 + 256) * kl + 32) + 5 * ((n // 2 + 256) * kl + 32)
        lim = {0: (m, words(k), lda), 1: (64 * words(n), words(k), ldbt), 2: (m, words(n), ldc)}
        for kind, blocks in plan:
            for (buf, row0, word0, ld, rows, bits) in blocks:
                if rows == 0:
                    continue
                if buf == 3:
                    assert word0 % 32 == 0 and ld % 2 == 0 and word0 + (rows - 1) * ld + words(bits) <= ws
                else:
                    R, W, L = lim[buf]
                    assert ld == L and row0 + rows <= R and word0 + words(bits) <= W
            if kind == 1:
                assert blocks[0][5] == blocks[1][5]  # one inner size
                assert blocks[1][4] % 64 == 0


def test_plan_rejects_bad_arguments():
    lib = G.load()
    import ctypes
    steps = (G.PlanStep * 17)()
    ws = ctypes.c_int64(0)
    for args in [(-1, 64, 64, 0), (64, -1, 64, 0), (64, 64, -1, 0), (64, 64, 64, 2), (64, 64, 64, -2)]:
        assert lib.gf2_product_plan(*args, 1, 1, 1, steps, 17, ctypes.byref(ws)) == -1
