"""GPU tests of the serving session (gf2_serve_*, through the C ABI): each
request's result, served in a mix of other requests that arrive while it
runs, equals the PLE of that matrix alone (gf2_ple, itself bit-exact against
the oracle; small requests are also compared with the oracle directly), for
batched and single launches, host and device inputs, and under an HBM budget
that forces admission to wait."""
import time

import numpy as np
import pytest
import torch

from paper_1111_6549_amd import gf2ple as G
from paper_1111_6549_amd import inputs
from tests.gpu_util import assert_same_ple, gpu_ple, oracle_ple, say

pytestmark = pytest.mark.gpu


def _mat(m, n, p, seed, rank=None):
    if m == 0 or n == 0:
        return np.zeros((m, inputs.words(n)), dtype=np.uint64)
    if rank is not None:
        return inputs.known_rank(m, n, rank, 5 + seed, 9 + seed, device="cuda")
    return inputs.bernoulli(m, n, seed, p=p)


def _alone(A, n):
    return gpu_ple(A, n)


def test_serve_mix_equals_alone():
    say("serve mix")
    specs = [(0, 0, .5), (0, 9, .5), (7, 0, .5), (1, 1, .5), (64, 64, .5), (200, 100, .05), (100, 200, .5),
             (1000, 1000, .5), (1000, 500, .05), (2048, 2048, .5), (2048, 1024, .05), (2049, 2049, .5),
             (3000, 1500, .5), (4500, 4500, .05), (6000, 3000, .5)]
    rng = np.random.Generator(np.random.PCG64(3))
    for i in range(45):
        s = int(np.exp(rng.uniform(np.log(64), np.log(2600))))
        specs.append((s, s if i % 2 else -(-s // 2), 0.5 if i % 3 else 0.05))
    mats = []
    for i, (m, n, p) in enumerate(specs):
        rank = min(m, n) // 3 if (i % 7 == 6 and min(m, n) > 8) else None
        mats.append(_mat(m, n, p, 100 + i, rank))
    S = G.ServeSession(budget_bytes=4 << 30)
    tickets = []
    for i, ((m, n, p), A) in enumerate(zip(specs, mats)):
        if i % 2:
            tickets.append(S.submit(A, n))  # host input
        else:
            tickets.append(S.submit(torch.from_numpy(A.view(np.int64).copy()).cuda(), n))  # device input
        if i % 10 == 9:
            time.sleep(0.002)  # later requests arrive while earlier ones run
    results = []
    for t, (m, n, p) in zip(tickets, specs):
        info = S.wait(t)
        assert info["state"] == "done", info
        assert info["t_submit"] <= info["t_admit"] <= info["t_done"]
        results.append(S.fetch(t, m, n))
    st = S.stats()
    say("serve stats", st)
    assert st["completed"] == len(specs) and st["failed"] == 0
    assert st["launches_batched"] >= 1 and st["launches_single"] >= 4
    assert st["bytes_peak"] <= st["budget_bytes"]
    S.close()
    for i, ((m, n, p), A, g) in enumerate(zip(specs, mats, results)):
        assert_same_ple(g, _alone(A, n), "served #%d %dx%d vs alone" % (i, m, n))
        if max(m, n) <= 1200:
            assert_same_ple(g, oracle_ple(A, n), "served #%d %dx%d vs oracle" % (i, m, n))


def test_serve_budget_forces_waiting():
    """A budget that holds a few large requests at a time: the others wait for
    admission until earlier results are fetched; all results stay exact and
    the pool never exceeds the budget.  A request larger than the whole
    budget is refused."""
    say("serve budget")
    S = G.ServeSession(budget_bytes=160 << 20, streams=2, small_max_dim=1024)
    n = 12000  # 18 MB per request: 8 of them do not fit the ~124 MB left after the per-stream reserve
    A0 = inputs.bernoulli(n, n, 41)
    too_big = np.zeros((40000, inputs.words(40000)), dtype=np.uint64)  # 200 MB
    with pytest.raises(G.GF2Error) as e:
        S.submit(too_big, 40000)
    assert e.value.status == 4  # GF2_EBUDGET
    mats = [A0] + [inputs.bernoulli(n, n, 42 + k) for k in range(7)]
    tickets = [S.submit(A, n) for A in mats]
    time.sleep(0.05)
    st = S.stats()
    say("after submit", st)
    assert st["queued"] >= 1  # not everything fits at once
    out = []
    for t in tickets:
        S.wait(t)
        out.append(S.fetch(t, n, n))
    st = S.stats()
    say("after fetch", st)
    assert st["completed"] == len(mats) and st["bytes_peak"] <= st["budget_bytes"]
    assert st["bytes_in_use"] < st["budget_bytes"]
    S.close()
    for k in (0, 3, 7):
        assert_same_ple(out[k], _alone(mats[k], n), "budget #%d" % k)


def test_serve_fetch_to_device_and_release():
    say("serve fetch to device")
    S = G.ServeSession(budget_bytes=1 << 30)
    m, n = 700, 900
    A = inputs.bernoulli(m, n, 55)
    t1 = S.submit(A, n)
    t2 = S.submit(A, n)
    S.wait(t1)
    ldw_out = inputs.words(n) + 3
    LE = torch.full((m, ldw_out), -1, dtype=torch.int64, device="cuda")
    P = torch.empty(m, dtype=torch.int64, device="cuda")
    Q = torch.empty(min(m, n), dtype=torch.int64, device="cuda")
    r = torch.empty(1, dtype=torch.int64, device="cuda")
    S.fetch_device(t1, LE, P, Q, r)
    LEh = LE.cpu().numpy().view(np.uint64)
    assert (LEh[:, inputs.words(n):] == 0).all()
    g = (int(r.item()), P.cpu().numpy(), Q.cpu().numpy(), np.ascontiguousarray(LEh[:, :inputs.words(n)]))
    assert_same_ple(g, oracle_ple(A, n), "fetched to device")
    S.wait(t2)
    S.release(t2)
    with pytest.raises(G.GF2Error):
        S.poll(t2)  # released tickets are unknown
    S.close()


SERVE_BENCH_COUNT = 3000  # the request stream bench.py serves (seed 8)


def test_serve_bench_stream_vs_oracle():
    """Requests of the benchmark's serving stream (inputs.serving_requests
    with its count and seed 8, sides up to 16384, density 0.5 or 0.05): the
    first 30, and the first two of side >= 12000 at each density, served
    together in one session from device inputs, each equal to the oracle."""
    reqs = inputs.serving_requests(SERVE_BENCH_COUNT, seed=8)
    pick = list(range(30))
    for p in (0.05, 0.5):
        pick += [i for i, r in enumerate(reqs) if max(r["m"], r["n"]) >= 12000 and r["p"] == p and i >= 30][:2]
    say("serve bench stream", len(pick), "requests", [(reqs[i]["m"], reqs[i]["n"], reqs[i]["p"]) for i in pick[30:]])
    mats = [inputs.bernoulli(reqs[i]["m"], reqs[i]["n"], reqs[i]["seed"], p=reqs[i]["p"]) for i in pick]
    S = G.ServeSession(budget_bytes=64 << 30)
    tickets = [S.submit(torch.from_numpy(A.view(np.int64).copy()).cuda(), reqs[i]["n"]) for i, A in zip(pick, mats)]
    out = []
    for t, i in zip(tickets, pick):
        info = S.wait(t)
        assert info["state"] == "done", info
        out.append(S.fetch(t, reqs[i]["m"], reqs[i]["n"]))
    S.close()
    for i, A, g in zip(pick, mats, out):
        say("  oracle", i, reqs[i]["m"], reqs[i]["n"], reqs[i]["p"])
        assert_same_ple(g, oracle_ple(A, reqs[i]["n"]), "bench request #%d" % i)


def test_serve_device_input_kept_until_done():
    """A device input is copied when its request is launched, which can be
    after admission: with one launch stream, requests admitted behind a
    running one wait with their inputs uncopied.  The binding keeps each
    input tensor referenced until its request is done, so freeing the
    caller's tensors and filling fresh ones of the same size (which the
    caching allocator may place on the same memory) cannot change a result."""
    say("serve device input lifetime")
    n = 6000
    mats = [inputs.bernoulli(n, n, 70 + k) for k in range(5)]
    S = G.ServeSession(budget_bytes=8 << 30, streams=1, small_max_dim=1024)
    tickets = []
    for A in mats:
        t = torch.from_numpy(A.view(np.int64).copy()).cuda()
        tickets.append(S.submit(t, n))
        del t
    states = [S.poll(t)["state"] for t in tickets]
    say("  states after submit", states)
    junk = [torch.full((n, inputs.words(n)), -1, dtype=torch.int64, device="cuda") for _ in range(8)]
    torch.cuda.synchronize()
    out = []
    for t in tickets:
        assert S.wait(t)["state"] == "done"
        out.append(S.fetch(t, n, n))
    S.close()
    del junk
    for k, (A, g) in enumerate(zip(mats, out)):
        assert_same_ple(g, oracle_ple(A, n), "device input #%d" % k)
