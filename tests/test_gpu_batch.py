"""GPU parity of the batched PLE (gf2_ple_batched, through the C ABI): every
matrix of a batch must equal the CPU oracle's PLE of that matrix alone, bit
for bit (rank, P, Q, L\\E), whatever the schedule, the size class, the order
in which workgroups pick matrices up, and across replays of the captured
graph."""
import numpy as np
import pytest
import torch

from paper_1111_6549_amd import gf2ple as G
from paper_1111_6549_amd import inputs
from tests.gpu_util import assert_same_ple, oracle_ple, say

pytestmark = pytest.mark.gpu


def _matrix(m, n, kind, seed):
    if m == 0 or n == 0:
        return np.zeros((m, inputs.words(n)), dtype=np.uint64)
    if kind == "rank":
        rho = max(1, min(m, n) // 2 + seed % 7)
        rho = min(rho, m, n)
        return inputs.known_rank(m, n, rho, 31 + seed, 37 + seed)
    p = {"dense": 0.5, "sparse": 0.05, "vsparse": 0.003}[kind]
    return inputs.bernoulli(m, n, 1000 + seed, p=p)


def mixed_batch(count, hi, seed, extra=()):
    """Seeded shapes in [0, hi] plus explicit edge cases, mixed densities and
    known-rank products."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = ["dense", "dense", "sparse", "rank", "vsparse"]
    shapes = list(extra)
    for i in range(count):
        m = int(rng.integers(1, hi + 1))
        n = int(rng.integers(1, hi + 1))
        shapes.append((m, n, kinds[i % len(kinds)]))
    mats = [_matrix(m, n, k, seed * 1000 + i) for i, (m, n, k) in enumerate(shapes)]
    return [(m, n) for m, n, _ in shapes], mats


EDGES = [(0, 0, "dense"), (0, 7, "dense"), (9, 0, "dense"), (1, 1, "dense"), (1, 200, "dense"), (200, 1, "dense"),
         (64, 64, "dense"), (65, 63, "sparse"), (63, 65, "rank"), (128, 128, "vsparse"), (300, 300, "rank")]


def pack_arena(shapes, mats):
    descs, aw, pl, ql = G.batch_layout(shapes)
    arena = np.zeros(max(aw, 1), dtype=np.uint64)
    for d, A in zip(descs, mats):
        k = d["m"] * d["ldw"]
        if k:
            arena[d["a_off"]:d["a_off"] + k] = A.reshape(-1)
    return descs, arena, aw, pl, ql


class Batch:
    def __init__(self, shapes, mats, **plan_kw):
        self.shapes, self.mats = shapes, mats
        self.descs, self.host, aw, pl, ql = pack_arena(shapes, mats)
        self.plan = G.BatchPlan(self.descs, aw, pl, ql, **plan_kw)
        self.arena = torch.from_numpy(self.host.view(np.int64).copy()).cuda()
        self.P = torch.full((max(pl, 1),), -7, dtype=torch.int64, device="cuda")
        self.Q = torch.full((max(ql, 1),), -7, dtype=torch.int64, device="cuda")
        self.R = torch.full((max(len(shapes), 1),), -7, dtype=torch.int64, device="cuda")
        self.ws = G.alloc_workspace(self.plan.workspace_bytes())

    def restore(self):
        self.arena.copy_(torch.from_numpy(self.host.view(np.int64)))
        self.P.fill_(-7)
        self.Q.fill_(-7)
        self.R.fill_(-7)

    def run(self):
        self.plan.run(self.arena, self.P, self.Q, self.R, self.ws)
        torch.cuda.synchronize()

    def result(self, i):
        d = self.descs[i]
        m, n, ldw = d["m"], d["n"], d["ldw"]
        out = self.arena[d["a_off"]:d["a_off"] + m * ldw].cpu().numpy().view(np.uint64).reshape(m, ldw)
        P = self.P[d["p_off"]:d["p_off"] + m].cpu().numpy()
        Q = self.Q[d["q_off"]:d["q_off"] + min(m, n)].cpu().numpy()
        return int(self.R[i].item()), P, Q, out


_ORACLE_CACHE = {}


def oracle_of(key, i, A, n):
    k = (key, i)
    if k not in _ORACLE_CACHE:
        _ORACLE_CACHE[k] = oracle_ple(A, n)
    return _ORACLE_CACHE[k]


def check_all(b, key, label, indices=None):
    for i in (range(len(b.shapes)) if indices is None else indices):
        m, n = b.shapes[i]
        assert_same_ple(b.result(i), oracle_of(key, i, b.mats[i], n), "%s #%d %dx%d" % (label, i, m, n))


def test_batch_mixed_default():
    say("batch mixed default plan")
    shapes, mats = mixed_batch(150, 400, 1, EDGES)
    b = Batch(shapes, mats)
    b.run()
    check_all(b, "mixed1", "default")
    b.plan.close()


@pytest.mark.parametrize("config", list(range(1, 9)))
def test_batch_each_config(config):
    say("batch config", config, G.batch_config_name(config))
    shapes, mats = mixed_batch(40, 700, 2, EDGES)
    b = Batch(shapes, mats, config=config)
    info = b.plan.info()
    assert all(c["config"] == config for c in info)
    b.run()
    check_all(b, "mixed2", "config %d" % config)
    b.plan.close()


def test_batch_graph_replays_and_recapture():
    """Each replay of the captured graph is checked on its own; a second
    arena at another address makes the plan capture again."""
    say("batch graph replays")
    shapes, mats = mixed_batch(60, 500, 3, EDGES)
    b = Batch(shapes, mats)
    for rep in range(3):
        b.restore()
        torch.cuda.synchronize()
        b.run()
        check_all(b, "mixed3", "replay %d" % rep)
    # eager work between replays, then a different arena buffer
    other = torch.from_numpy(b.host.view(np.int64).copy()).cuda()
    b.arena, old = other, b.arena
    b.run()
    check_all(b, "mixed3", "recaptured")
    del old
    b.plan.close()


def test_batch_no_graph_matches():
    say("batch without graph")
    shapes, mats = mixed_batch(60, 500, 4, EDGES)
    b = Batch(shapes, mats, graph=False)
    b.run()
    check_all(b, "mixed4", "no graph")
    b.plan.close()


def test_batch_autotune():
    say("batch autotune")
    shapes, mats = mixed_batch(120, 1500, 5, EDGES)
    b = Batch(shapes, mats, autotune=True)
    info = b.plan.info()
    say("tuned classes", [(c["max_dim"], c["count"], c["config_name"], round(c["tuned_ms"], 3)) for c in info])
    assert any(c["tuned_ms"] > 0 for c in info if c["count"])
    b.run()
    check_all(b, "mixed5", "autotuned")
    b.plan.close()


def test_batch_large_classes():
    """Matrices in the 2048, 4096 and unbounded classes, including the slow
    pivot search over more rows than the register window."""
    say("batch large classes")
    shapes = [(2048, 2048), (2048, 64), (64, 2048), (3000, 500), (500, 3000), (5000, 100), (4100, 300)]
    kinds = ["dense", "rank", "dense", "rank", "sparse", "rank", "vsparse"]
    mats = [_matrix(m, n, k, 77 + i) for i, ((m, n), k) in enumerate(zip(shapes, kinds))]
    b = Batch(shapes, mats)
    b.run()
    check_all(b, "large", "large")
    b.plan.close()


@pytest.mark.slow
def test_batch_full_4096_sampled():
    """The full uneven batch (4096 matrices, m, n uniform in [64, 2048], every
    fourth a known-rank product) in the launch configuration the benchmark
    times: all ranks of the known-rank matrices are exact, every rank is
    within bounds, and 48 sampled matrices equal the oracle bit for bit."""
    say("batch full 4096 sampled")
    shapes_d = inputs.batch_shapes(4096, 7)
    mats = [inputs.batch_matrix(s, 7, i, device="cuda") for i, s in enumerate(shapes_d)]
    shapes = [(s["m"], s["n"]) for s in shapes_d]
    b = Batch(shapes, mats, autotune=True)
    b.run()
    ranks = b.R.cpu().numpy()
    for i, s in enumerate(shapes_d):
        assert 0 <= ranks[i] <= min(s["m"], s["n"])
        if s["kind"] == "known_rank":
            assert ranks[i] == s["rank"], (i, s, ranks[i])
    rng = np.random.Generator(np.random.PCG64(99))
    sample = sorted(set(rng.integers(0, 4096, size=48).tolist()) | {0, 3, 4095})
    check_all(b, "full4096", "full", sample)
    b.plan.close()
