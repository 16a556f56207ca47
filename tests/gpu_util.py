"""Shared helpers of the GPU tests: host <-> device packing and the two
sides of a parity comparison (the HIP library through its C ABI, and the CPU
oracle)."""
import sys

import numpy as np
import torch

import oracle
from paper_1111_6549_amd import gf2ple as G


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(A):
    return torch.from_numpy(np.ascontiguousarray(A).view(np.int64).copy()).cuda()


def to_host(t):
    return t.cpu().numpy().view(np.uint64)


def gpu_ple(A, n, **kw):
    t = to_dev(A)
    P, Q, rank = G.ple(t, n, **kw)
    torch.cuda.synchronize()
    return int(rank.item()), P.cpu().numpy(), Q.cpu().numpy(), to_host(t)


def oracle_ple(A, n):
    B = np.array(A, copy=True)
    r, P, Q = oracle.ple(B, n)
    return r, P, Q, B


def assert_same_ple(g, o, label=""):
    rg, Pg, Qg, Ag = g
    ro, Po, Qo, Ao = o
    assert rg == ro, "%s rank %d != oracle %d" % (label, rg, ro)
    assert np.array_equal(Qg, Qo), "%s Q differs at %s" % (label, np.nonzero(Qg != Qo)[0][:8])
    assert np.array_equal(Pg, Po), "%s P differs at %s" % (label, np.nonzero(Pg != Po)[0][:8])
    if not np.array_equal(Ag, Ao):
        rows = np.nonzero((Ag != Ao).any(axis=1))[0]
        raise AssertionError("%s L\\E differs in %d rows, first %s" % (label, rows.size, rows[:8]))
