"""GPU parity of the matrix-core GF(2) products (gf2_addmul with update = 2,
fp4 operands, and update = 4, int8 operands) against the oracle's product by
definition, on ragged shapes that span several block tiles (256 x 256 for
fp4, 128 x 128 wave tiles for int8), partial words in every dimension, and k
from 1 to a few thousand; and agreement with the XOR-table product."""
import numpy as np
import pytest

import oracle
from paper_1111_6549_amd import gf2ple as G
from paper_1111_6549_amd import inputs
from tests.gpu_util import say, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (1, 64, 1), (64, 1, 64), (33, 17, 65), (100, 64, 70), (128, 128, 128), (300, 150, 900),
          (700, 1000, 130), (129, 33, 4097), (2048, 512, 2048), (1000, 2049, 300), (4100, 96, 640),
          (257, 4096, 513), (3000, 1100, 2500), (1500, 640, 1200), (600, 1400, 520)]


@pytest.mark.parametrize("m,k,n", SHAPES)
def test_mfma_addmul_matches_oracle(m, k, n):
    say("mfma addmul", m, k, n)
    C = inputs.bernoulli(m, n, 11 + m)
    A = inputs.bernoulli(m, k, 12 + k)
    B = inputs.bernoulli(k, n, 13 + n)
    want = C.copy()
    oracle.addmul(want, A, B, k, n)
    for update in (2, 4, 1):
        tC = to_dev(C)
        G.addmul(tC, to_dev(A), to_dev(B), k, n, update=update)
        got = to_host(tC)
        assert np.array_equal(got, want), "update=%d differs in %d words" % (update, int((got != want).sum()))


def test_mfma_addmul_sparse_and_strided():
    """Sparse operands, and row strides wider than the data (padding words
    must stay zero)."""
    say("mfma addmul sparse/strided")
    m, k, n = 500, 300, 700
    C = inputs.bernoulli(m, n, 21, ldw=inputs.words(n) + 3)
    A = inputs.bernoulli(m, k, 22, p=0.02, ldw=inputs.words(k) + 1)
    B = inputs.bernoulli(k, n, 23, p=0.05, ldw=inputs.words(n) + 2)
    want = C.copy()
    oracle.addmul(want, A, B, k, n)
    for update in (2, 4):
        tC = to_dev(C)
        G.addmul(tC, to_dev(A), to_dev(B), k, n, update=update)
        assert np.array_equal(to_host(tC), want), "update=%d" % update


@pytest.mark.parametrize("off,ld_extra", [(3, 0), (4, 7), (4, 640)])
def test_addmul_on_column_block_views(off, ld_extra):
    """C, A and B as views of column blocks of wider matrices (row strides
    of the wider matrices, even and odd; the view 16-byte aligned or not):
    the product reads and writes only the views' words, for every product
    kind."""
    import torch
    say("mfma addmul views", off, ld_extra)
    m, k, n = 1500, 1100, 900
    kw, nw = inputs.words(k), inputs.words(n)
    C = inputs.bernoulli(m, n, 31)
    A = inputs.bernoulli(m, k, 32)
    B = inputs.bernoulli(k, n, 33)
    want = C.copy()
    oracle.addmul(want, A, B, k, n)
    for update in (2, 4, 1):
        # each operand sits at word offset `off` of a wider matrix filled with a marker
        def wide(X, words):
            W = np.full((X.shape[0], words + off + ld_extra), 0x5A5A5A5A5A5A5A5A, np.uint64)
            W[:, off:off + X.shape[1]] = X
            return to_dev(W)
        tC, tA, tB = wide(C, nw), wide(A, kw), wide(B, nw)
        G.addmul(tC[:, off:off + nw], tA[:, off:off + kw], tB[:, off:off + nw], k, n, update=update)
        got = to_host(tC)
        assert np.array_equal(got[:, off:off + nw], want), "update=%d" % update
        assert np.all(got[:, :off] == 0x5A5A5A5A5A5A5A5A) and np.all(got[:, off + nw:] == 0x5A5A5A5A5A5A5A5A)
        torch.cuda.synchronize()
    # the in-place PLE works on whole rows: a column-block view is refused
    with pytest.raises(ValueError):
        G.ple(tC[:, off:off + nw], n)
