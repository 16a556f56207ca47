"""gf2_ple_noalloc (static device workspace, no allocation) against gf2_ple
on the same inputs, bit for bit, on consecutive calls -- the second smaller
than the first, so it runs on what the first left in the shared array."""
import numpy as np
import pytest
import torch

from paper_1111_6549_amd import gf2ple as G
from paper_1111_6549_amd import inputs
from tests.gpu_util import oracle_ple, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _run(fn, A, n, **kw):
    t = to_dev(A)
    P, Q, rank = fn(t, n, **kw)
    torch.cuda.synchronize()
    return int(rank.item()), P.cpu().numpy(), Q.cpu().numpy(), to_host(t)


def _same(a, b, label):
    assert a[0] == b[0], "%s rank %d != %d" % (label, a[0], b[0])
    for x, y, what in ((a[1], b[1], "P"), (a[2], b[2], "Q"), (a[3], b[3], "L\\E")):
        assert np.array_equal(x, y), "%s %s differs" % (label, what)


@pytest.mark.parametrize("shapes", [((3000, 2500, "u"), (700, 900, "r")),
                                    ((16384, 16384, "u"), (1500, 1300, "u")),
                                    ((4000, 4000, "s"), (64, 64, "u"))])
def test_noalloc_matches_ple_twice(shapes):
    for i, (m, n, kind) in enumerate(shapes):
        say("noalloc call", i, m, n, kind)
        if kind == "u":
            A = inputs.bernoulli(m, n, 300 + m + i)
        elif kind == "r":
            A = inputs.known_rank(m, n, min(m, n) // 2, 17, 19)
        else:
            A = inputs.bernoulli(m, n, 301 + m, p=4.0 / n)
        got = _run(G.ple_noalloc, A, n)
        want = _run(G.ple, A, n)
        _same(got, want, "%dx%d noalloc vs gf2_ple" % (m, n))
        if m * n <= 4000 * 4000:
            _same(got, oracle_ple(A, n), "%dx%d noalloc vs oracle" % (m, n))


def test_noalloc_rejects_oversize():
    say("noalloc oversize")
    limit = int(G.load().gf2_ple_noalloc_max_workspace())
    m, n = 600000, 64
    assert G.workspace_bytes(m, n, 1) > limit
    t = torch.zeros((m, 1), dtype=torch.int64, device="cuda")
    with pytest.raises(G.GF2Error) as ei:
        G.ple_noalloc(t, n)
    assert ei.value.status == 2
