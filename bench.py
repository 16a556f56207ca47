#!/usr/bin/env python
"""Benchmark: PLE decomposition of a dense 65536 x 65536 GF(2) matrix on one
MI355X through the C ABI (gf2_ple).

One step = one full PLE (every pass of Algorithm 2: panel, permute, trailing
update) of the resident matrix.  Before each step the input is restored from
a pristine device copy (a 512 MiB device-to-device copy, inside the timed
region, about 0.1 ms of a step).  Prints ONE JSON line on stdout; progress
goes to stderr.

  value      whole-job throughput in PLE decompositions per second
  roofline   the dominant kernel (the Four-Russians trailing update k_m4rm):
             algorithmic bytes per launch / average launch time, both from a
             second, event-timed repetition of the same steps (HIP events on
             the launch stream, recorded by the library itself)
  cpu_baseline  the CPU oracle (plain Gaussian elimination) timed on this
             host on a bounded sample, scaled by n^3 to the full matrix
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
KW = 64
# HBM bytes per trailing-update launch on the 65536^2 seed-5 workload:
# rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE, averaged over the update
# launches of one PLE and scaled by the same counters on the 512 MiB restore copy
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Reported only while the kernel
# sources hash to the value the counters were taken on.
TRAFFIC = {"source": "04ab9aea8fe485c0", "n": 65536, "seed": 5, "bytes_per_launch": 366610682}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes_m4rm(m, n, Q, r, kinds):
    """Algorithmic bytes of the trailing-update launches of one PLE, following
    the library's pass schedule (gf2_ple_schedule): one 8-byte read and one
    8-byte write per row word an update launch covers -- rows r_t .. m-1;
    words right of the stripe (serial pass), from the stripe + 2 (look-ahead
    pass) or, for a fused pair, from the pair's first stripe + 3, once for
    both passes.  Launches of passes without a pivot move nothing."""
    import numpy as np
    nw = (n + 63) // 64
    q = np.asarray(Q[:r], dtype=np.int64)
    counts = np.bincount(q // KW, minlength=nw) if r else np.zeros(nw, np.int64)
    r_at = np.concatenate([[0], np.cumsum(counts)])
    total = 0
    for t, k in enumerate(kinds):
        if k == 0 and counts[t] > 0 and t + 1 < nw:
            total += 16 * (m - r_at[t]) * (nw - t - 1)
        elif k == 1 and counts[t] > 0 and t + 2 < nw:
            total += 16 * (m - r_at[t]) * (nw - t - 2)
        elif k == 3 and (counts[t - 1] > 0 or counts[t] > 0) and t + 2 < nw:
            total += 16 * (m - r_at[t - 1]) * (nw - (t - 1) - 3)
    return int(total)


def alg_bytes_k64(m, n, Q, r):
    """The same count for a schedule of serial 64-column passes only (the
    byte count the paper's per-pass update implies): the reference figure
    for the whole-PLE rate."""
    return alg_bytes_m4rm(m, n, Q, r, [0] * ((n + 63) // 64))


def alg_bytes_rref_from_ple(n, Q, r):
    """Algorithmic bytes of the update launches of gf2_rref_from_ple: pivot
    blocks of 64 rows from the last to the first, two per sweep; a sweep
    covers rows 0 .. j1-1 (j1 = end of its later block) and the words from
    the first pivot column of its earlier block to the end, 16 B per row
    word (one read, one write)."""
    nw = (n + 63) // 64
    total = 0
    b = (r + KW - 1) // KW - 1
    while b >= 0:
        j0 = b * KW
        j1 = min(j0 + KW, r)
        if b >= 1:
            wq = int(Q[j0 - KW]) >> 6
            b -= 2
        else:
            wq = int(Q[j0]) >> 6
            b -= 1
        total += 16 * j1 * (nw - wq)
    return int(total)


def alg_bytes_m4ri_rref(m, n, Q, r, kinds):
    """Algorithmic bytes of the update launches of gf2_m4ri_rref on the pass
    schedule `kinds` (gf2_ple's, with look-ahead passes run serially): the
    passes' own updates (as alg_bytes_m4rm), and after each pass or fused
    pair with a pivot, the elimination of its block from the rows above the
    next pass's first row over the words from its first stripe to the end."""
    import numpy as np
    nw = (n + 63) // 64
    kinds = [0 if k == 1 else k for k in kinds]
    q = np.asarray(Q[:r], dtype=np.int64)
    counts = np.bincount(q // KW, minlength=nw) if r else np.zeros(nw, np.int64)
    r_at = np.concatenate([[0], np.cumsum(counts)])
    total = alg_bytes_m4rm(m, n, Q, r, kinds)
    t = 0
    while t < nw:
        np_ = 2 if kinds[t] == 2 else 1
        if counts[t:t + np_].sum() > 0:
            total += 16 * int(r_at[t + np_]) * (nw - t)
        t += np_
    return int(total)


def kernel_source_hash():
    """Hash of the sources the update kernels are compiled from (the fused
    pair update also runs the next panel)."""
    h = hashlib.sha256()
    for f in ("ple_kernels.hip", "m4rm.h", "dev.h", "common.h", "panel.h"):
        with open(os.path.join(ROOT, "paper_1111_6549_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


DENSITY_POINTS = (0.1, 0.2, 0.5, 1.0, 2.0, 3.0, 5.0, 8.0, 12.0, 20.0)


def cpu_baseline(n_full, sample):
    """The oracle, untouched, on a sample x sample Bernoulli(0.5) matrix."""
    import oracle
    from paper_1111_6549_amd import inputs
    A = inputs.bernoulli(sample, sample, 2)
    oracle.ple(A[:64, :1].copy(), 64)  # load/compile outside the timing
    t0 = time.perf_counter()
    r, _, _ = oracle.ple(A, sample)
    dt = time.perf_counter() - t0
    scale = (n_full / sample) ** 3
    return {
        "value": 1.0 / (dt * scale),
        "unit": "matrices/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": "%dx%d Bernoulli(0.5) seed 2, whole oracle PLE in %.2f s (rank %d), scaled by (%d/%d)^3; "
                  "the sample is small enough to stay in the host's caches, so the scaled rate overstates the "
                  "oracle on the full matrix" % (sample, sample, dt, r, n_full, sample),
    }


def run_density(args, log_fn):
    """The sparse sweep of Section 5's Figure 2 on this path: 10000 x 10000,
    Bernoulli(x / 10000) for x non-zero entries per row on average, seed 9 +
    the point's index.  Each point: the median of five gf2_ple calls, input
    restored from a device copy before each (outside the timing).  The oracle
    is timed beside three points."""
    import numpy as np
    import torch

    from paper_1111_6549_amd import gf2ple as G
    from paper_1111_6549_amd import inputs

    side = 10000
    ldw = inputs.words(side)
    ws = G.alloc_workspace(G.workspace_bytes(side, side, ldw))
    points = []
    oracle_pts = (1.0, 5.0, 20.0)
    for idx, x in enumerate(DENSITY_POINTS):
        A = inputs.bernoulli(side, side, 9 + idx, p=x / side)
        dev = torch.from_numpy(A.view(np.int64)).cuda()
        work = torch.empty_like(dev)
        times = []
        for rep in range(6):
            work.copy_(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P, Q, rank = G.ple(work, side, ws=ws, panel_regs=args.panel_regs, lookahead=args.lookahead)
            torch.cuda.synchronize()
            if rep:
                times.append((time.perf_counter() - t0) * 1000.0)
        times.sort()
        pt = {"nnz_per_row": x, "rank": int(rank.item()), "gpu_ms": round(times[len(times) // 2], 3)}
        if not args.no_cpu_baseline and x in oracle_pts:
            import oracle
            B = A.copy()
            t0 = time.perf_counter()
            oracle.ple(B, side)
            pt["oracle_ms"] = round((time.perf_counter() - t0) * 1000.0, 1)
            pt["oracle_cores"] = oracle.threads()
        points.append(pt)
        log_fn("density %.1f per row: %s" % (x, json.dumps(pt)))
        del dev, work
    return {"workload": "10000x10000, Bernoulli(x/10000), x non-zero entries per row, seed 9 + index; "
                        "median of 5 gf2_ple calls on resident input", "points": points}


def run_batched(args, log_fn):
    """The uneven batch: 4096 matrices, m and n uniform in [64, 2048], seed 7,
    every fourth a known-rank product.  Batched = one execution of an
    autotuned plan (graph replay); plain = gf2_ple called per matrix, one
    after another on the same stream, on the same matrices."""
    import numpy as np
    import torch

    from paper_1111_6549_amd import gf2ple as G
    from paper_1111_6549_amd import inputs

    count = args.batch_count
    shapes_d = inputs.batch_shapes(count, 7)
    mats = [inputs.batch_matrix(s, 7, i, device="cuda") for i, s in enumerate(shapes_d)]
    shapes = [(s["m"], s["n"]) for s in shapes_d]
    descs, aw, pl, ql = G.batch_layout(shapes)
    host = np.zeros(aw, np.uint64)
    for d, A in zip(descs, mats):
        host[d["a_off"]:d["a_off"] + d["m"] * d["ldw"]] = A.reshape(-1)
    pristine = torch.from_numpy(host.view(np.int64)).cuda()
    arena = pristine.clone()
    P = torch.empty(pl, dtype=torch.int64, device="cuda")
    Q = torch.empty(ql, dtype=torch.int64, device="cuda")
    R = torch.empty(count, dtype=torch.int64, device="cuda")
    t0 = time.perf_counter()
    plan = G.BatchPlan(descs, aw, pl, ql, autotune=True)
    tune_s = time.perf_counter() - t0
    ws = G.alloc_workspace(plan.workspace_bytes())
    for _ in range(args.warmup + 1):
        arena.copy_(pristine)
        plan.run(arena, P, Q, R, ws)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.batch_reps):
        arena.copy_(pristine)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.run(arena, P, Q, R, ws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    batched_s = sorted(times)[len(times) // 2]
    ranks = R.cpu().numpy()
    for i, s in enumerate(shapes_d):
        if s["kind"] == "known_rank" and ranks[i] != s["rank"]:
            raise RuntimeError("batched rank of matrix %d is %d, built with rank %d" % (i, ranks[i], s["rank"]))
    log_fn("batched: %d matrices, median %.3f ms (plan + autotune %.2f s)" % (count, batched_s * 1e3, tune_s))

    # plain path: the same matrices through gf2_ple one by one
    arena.copy_(pristine)
    wsz = max(G.workspace_bytes(m, n, (n + 63) // 64) for m, n in shapes)
    wsp = G.alloc_workspace(wsz)
    views = [arena[d["a_off"]:d["a_off"] + d["m"] * d["ldw"]].view(d["m"], d["ldw"]) for d in descs]
    for v, (m, n) in list(zip(views, shapes))[:16]:
        G.ple(v, n, ws=wsp)
    arena.copy_(pristine)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for v, (m, n) in zip(views, shapes):
        G.ple(v, n, ws=wsp)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    log_fn("plain: %d gf2_ple calls in %.3f s" % (count, plain_s))

    out = {
        "workload": "%d GF(2) matrices, m and n uniform in [64, 2048], Bernoulli(0.5), every 4th of exact rank "
                    "in [m/4, min(m, n)], seed 7, one 256-byte aligned arena" % count,
        "value": round(count / batched_s, 1),
        "unit": "matrices/s",
        "ms_per_batch": round(batched_s * 1e3, 3),
        "plain_value": round(count / plain_s, 1),
        "plain_ms": round(plain_s * 1e3, 1),
        "speedup_vs_plain": round(plain_s / batched_s, 1),
        "classes": [{"max_dim": c["max_dim"], "count": c["count"], "schedule": c["config_name"], "grid": c["grid"]}
                    for c in plan.info() if c["count"]],
    }
    if not args.no_cpu_baseline:
        import oracle
        sample = list(range(0, count, max(1, count // args.batch_cpu_sample)))[:args.batch_cpu_sample]
        t0 = time.perf_counter()
        for i in sample:
            B = np.array(mats[i], copy=True)
            oracle.ple(B, shapes[i][1])
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(len(sample) / dt, 2), "unit": "matrices/s", "cores": oracle.threads(),
                               "kind": "oracle", "sample": "%d of the %d matrices (every %d-th), %.2f s"
                                                            % (len(sample), count, count // len(sample), dt)}
    plan.close()
    return out


def run_serving(args, log_fn):
    """Serving: a request stream (sides log-uniform in [128, 16384], square or
    s x ceil(s/2), density 0.5 or 0.05; seed 8), inputs resident on the device.
    Plain = gf2_ple per request in arrival order on one stream.  Served = the
    serving session (64 GiB budget) fed Poisson arrivals at 0.9x the measured
    plain capacity (latency = arrival -> result in device memory), and the
    same requests all at once (saturated throughput).  The plain latency at
    the same arrivals is a FIFO replay of the measured plain service times."""
    import numpy as np
    import torch

    from paper_1111_6549_amd import gf2ple as G
    from paper_1111_6549_amd import inputs

    count = args.serve_count
    reqs = inputs.serving_requests(count, seed=8)
    dev = [torch.from_numpy(inputs.bernoulli(r["m"], r["n"], r["seed"], p=r["p"]).view(np.int64)).cuda() for r in reqs]
    torch.cuda.synchronize()
    log_fn("serving: %d requests resident (%.2f GB)" % (count, sum(t.numel() for t in dev) * 8 / 1e9))

    # plain: gf2_ple per request, each on a fresh copy, timed per request
    big = max(t.numel() for t in dev)
    scratch = torch.empty(big, dtype=torch.int64, device="cuda")
    wsz = max(G.workspace_bytes(r["m"], r["n"], (r["n"] + 63) // 64) for r in reqs)
    wsp = G.alloc_workspace(wsz)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in reqs]
    for r, t in list(zip(reqs, dev))[:8]:
        w = scratch[:t.numel()].view(t.shape)
        w.copy_(t)
        G.ple(w, r["n"], ws=wsp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (r, t), (a, b) in zip(zip(reqs, dev), ev):
        w = scratch[:t.numel()].view(t.shape)
        w.copy_(t)
        a.record()
        G.ple(w, r["n"], ws=wsp)
        b.record()
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    service = np.array([a.elapsed_time(b) * 1e-3 for a, b in ev])
    capacity = count / plain_s
    log_fn("serving: plain %.3f s (%.1f req/s)" % (plain_s, capacity))
    del scratch, wsp

    def serve(arrivals):
        S = G.ServeSession(budget_bytes=64 << 30, small_max_dim=args.serve_small_max)
        tickets = []
        start = time.perf_counter()
        for r, t, at in zip(reqs, dev, arrivals):
            while time.perf_counter() - start < at:
                pass
            tickets.append(S.submit(t, r["n"]))
        infos = [S.wait(tk) for tk in tickets]
        st = S.stats()
        for tk in tickets:
            S.release(tk)
        S.close()
        lat = np.array([i["t_done"] - i["t_submit"] for i in infos])
        span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
        return lat, span, st

    rate = 0.9 * capacity
    rng = np.random.Generator(np.random.PCG64(8))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    arrivals -= arrivals[0]
    lat, span, st = serve(arrivals)
    # FIFO replay of the plain service times at the same arrivals
    fin = 0.0
    plain_lat = np.empty(count)
    for i in range(count):
        fin = max(arrivals[i], fin) + service[i]
        plain_lat[i] = fin - arrivals[i]
    log_fn("serving: poisson %.1f req/s: p50 %.2f ms p99 %.2f ms" % (rate, np.median(lat) * 1e3,
                                                                     np.percentile(lat, 99) * 1e3))
    lat_sat, span_sat, st_sat = serve(np.zeros(count))
    log_fn("serving: saturated %.3f s for %d requests" % (span_sat, count))
    pct = lambda x, q: round(float(np.percentile(x, q)) * 1e3, 3)
    out = {
        "workload": "%d requests, sides log-uniform in [128, 16384], square or s x ceil(s/2), density 0.5 or 0.05, "
                    "seed 8, inputs resident on the device, 64 GiB budget" % count,
        "plain_capacity_per_s": round(capacity, 1),
        "poisson": {"rate_per_s": round(rate, 1), "served_p50_ms": pct(lat, 50), "served_p99_ms": pct(lat, 99),
                    "served_matrices_per_s": round(count / span, 1), "plain_fifo_p50_ms": pct(plain_lat, 50),
                    "plain_fifo_p99_ms": pct(plain_lat, 99),
                    "launches": {"batched": st["launches_batched"], "single": st["launches_single"]}},
        "saturated": {"served_matrices_per_s": round(count / span_sat, 1),
                      "plain_matrices_per_s": round(capacity, 1),
                      "speedup_vs_plain": round((count / span_sat) / capacity, 2),
                      "served_p50_ms": pct(lat_sat, 50), "served_p99_ms": pct(lat_sat, 99),
                      "launches": {"batched": st_sat["launches_batched"], "single": st_sat["launches_single"]}},
    }
    if not args.no_cpu_baseline:
        import oracle
        sample = [i for i in range(count) if max(reqs[i]["m"], reqs[i]["n"]) <= 8192][:args.serve_cpu_sample]
        t0 = time.perf_counter()
        for i in sample:
            B = dev[i].cpu().numpy().view(np.uint64).copy()
            oracle.ple(B, reqs[i]["n"])
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(len(sample) / dt, 2), "unit": "matrices/s", "cores": oracle.threads(),
                               "kind": "oracle", "sample": "the first %d requests with sides <= 8192, in order, "
                                                           "%.2f s" % (len(sample), dt)}
    return out


def run_helpers(m, n, A, Qh, r, log_fn):
    """The helpers of the paper's PLE-based reductions on the bench matrix (not
    in the timed step): echelon form and the reduced echelon form from L\\E
    (on the PLE result), and the reduced echelon form of the input in the
    M4RI form.  Runs after the serving leg: the M4RI form's second stream
    would otherwise change how the serving session's streams share the
    process's hardware queues."""
    import numpy as np
    import torch
    from paper_1111_6549_amd import gf2ple as G
    pristine = torch.from_numpy(A.view(np.int64)).cuda()
    work = pristine.clone()
    P, Q, rank = G.ple(work, n)
    torch.cuda.synchronize()
    res = work.clone()
    hk = {}
    for name in ("echelon", "rref_from_ple", "m4ri_rref"):
        times = []
        for rep in range(2):  # the first also sets up the workspace
            work.copy_(res)
            torch.cuda.synchronize()
            h0 = time.perf_counter()
            if name == "echelon":
                G.echelon_from_ple(work, n, rank)
            elif name == "rref_from_ple":
                G.rref_from_ple(work, n, Q, rank)
            else:  # the M4RI form on the original matrix (not on the PLE result)
                work.copy_(pristine)
                torch.cuda.synchronize()
                h0 = time.perf_counter()
                G.m4ri_rref(work, n)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - h0) * 1000.0)
        hk[name + "_ms"] = round(min(times), 3)
    # the update launches' algorithmic bytes over the whole call's time (a
    # lower bound on their own rate: the call also syncs once and reads Q back)
    for name, nb in (("rref_from_ple", alg_bytes_rref_from_ple(n, Qh, r)),
                     ("m4ri_rref", alg_bytes_m4ri_rref(m, n, Qh, r, G.ple_schedule(m, n, lookahead=0)))):
        gbps = nb / (hk[name + "_ms"] * 1e-3) / 1e9
        hk[name + "_update_bytes"] = nb
        hk[name + "_alg_GBps"] = round(gbps, 1)
        hk[name + "_frac_hbm"] = round(gbps / HBM_PEAK_GBPS, 4)
    del pristine, work, res
    torch.cuda.empty_cache()
    log_fn("helpers: %s" % json.dumps(hk))
    return hk


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=32768)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-helpers", action="store_true", help="skip timing the echelon / RREF helpers")
    ap.add_argument("--m4-variant", type=int, default=0, help="update schedule 1..8 (0 = library default)")
    ap.add_argument("--m4-blocks", type=int, default=0, help="target blocks per update launch (0 = default)")
    ap.add_argument("--panel-regs", type=int, default=0, help="panel register window 2/4/8 (0 = default)")
    ap.add_argument("--lookahead", type=int, default=0,
                    help="0 = library default, 1 = serial passes, 2 = look-ahead only, 3 = pairs everywhere")
    ap.add_argument("--pair-variant", type=int, default=0, help="fused pair update schedule 1..12 (0 = default)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain measurement")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--batch-cpu-sample", type=int, default=512)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-density", action="store_true", help="skip the 10000^2 density sweep")
    ap.add_argument("--serve-count", type=int, default=600)
    ap.add_argument("--serve-cpu-sample", type=int, default=60)
    ap.add_argument("--serve-small-max", type=int, default=0,
                    help="largest side served by batched launches (0 = library default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the PLE of one matrix is not split across GPUs here; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1111_6549_amd import gf2ple as G
    from paper_1111_6549_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    G.load()
    m = n = args.n
    ldw = inputs.words(n)
    log("generating %dx%d Bernoulli(0.5) seed %d" % (m, n, args.seed))
    A = inputs.bernoulli(m, n, args.seed)
    pristine = torch.from_numpy(A.view(np.int64)).cuda()
    if args.no_helpers:
        del A
    work = torch.empty_like(pristine)
    ws = G.alloc_workspace(G.workspace_bytes(m, n, ldw))
    torch.cuda.synchronize()

    sched = dict(m4_variant=args.m4_variant, m4_blocks=args.m4_blocks, panel_regs=args.panel_regs,
                 lookahead=args.lookahead, pair_variant=args.pair_variant)

    def step():
        work.copy_(pristine)
        return G.ple(work, n, ws=ws, **sched)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup %d done" % i)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        P, Q, rank = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    r = int(rank.item())
    log("timed %d steps: %.3f ms/step, rank %d" % (args.steps, ms_per_step, r))

    Qh = Q.cpu().numpy()
    kinds = G.ple_schedule(m, n, lookahead=args.lookahead)
    abytes = alg_bytes_m4rm(m, n, Qh, r, kinds)
    abytes64 = alg_bytes_k64(m, n, Qh, r)

    roofline = None
    kernels = None
    if not args.no_profile:
        G.profile_start()
        for i in range(args.steps):
            step()
        torch.cuda.synchronize()
        kernels = G.profile_stop()
        k = kernels.get("m4rm")
        if k and k["total_ms"] > 0:
            launches_per_step = k["launches"] / args.steps
            bytes_per_launch = abytes / launches_per_step
            avg_ms = k["total_ms"] / k["launches"]
            achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
            traffic = None
            if (TRAFFIC and TRAFFIC.get("source") == kernel_source_hash() and TRAFFIC.get("n") == args.n
                    and TRAFFIC.get("seed") == args.seed and not args.m4_variant and not args.m4_blocks
                    and not args.pair_variant and not args.lookahead):
                traffic = TRAFFIC["bytes_per_launch"]
            roofline = {
                "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "trailing update (k_m4rm_pair for fused pairs, with the next panel on one wave; "
                          "k_m4rm / k_m4rm_w otherwise)",
                "launches_per_step": launches_per_step,
                "alg_bytes_per_launch": round(bytes_per_launch), "avg_launch_ms": round(avg_ms, 5),
            }
        log("profiled: %s" % json.dumps(kernels))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on %d^2" % args.cpu_sample)
        cpu = cpu_baseline(n, args.cpu_sample)
        log("cpu baseline done: %s" % cpu["sample"])

    density = None
    if not args.no_density:
        density = run_density(args, log)

    batched = None
    if not args.no_batched:
        del work, pristine, ws
        torch.cuda.empty_cache()
        batched = run_batched(args, log)
    serving = None
    if not args.no_serving:
        if args.no_batched:
            del work, pristine, ws
            torch.cuda.empty_cache()
        serving = run_serving(args, log)
    helpers = None
    if not args.no_helpers:
        if args.no_batched and args.no_serving:
            del work, pristine, ws
            torch.cuda.empty_cache()
        helpers = run_helpers(m, n, A, Qh, r, log)
        del A

    out = {
        "metric": "PLE time & HBM GB/s (% roofline), 65536² GF(2); batched matrices/s vs plain",
        "value": round(1000.0 / ms_per_step, 4),
        "unit": "matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "PLE of a dense %dx%d GF(2) matrix, Bernoulli(0.5), seed %d, uint64 row words"
                               % (m, n, args.seed),
                   "m": m, "n": n, "pass_width_K": KW, "update": "xor-table",
                   "update_schedule": "pairs of passes: one sweep with 32 nibble tables x 32-word tiles, "
                                      "the next panel inside it; single passes past the last pair",
                   "schedule": sched},
        "rank": r,
        "schedule": {"passes": len(kinds), "serial": kinds.count(0), "lookahead": kinds.count(1),
                     "fused_pairs": kinds.count(3)},
        "update_alg_bytes_per_step": abytes,
        "k64_alg_bytes_per_step": abytes64,
        "k64_alg_GBps_whole_ple": round(abytes64 / (ms_per_step * 1e-3) / 1e9, 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "helpers": helpers,
        "density_sweep": density,
        "batched": batched,
        "serving": serving,
        "kernels_ms_per_step": {k: round(v["total_ms"] / args.steps, 3) for k, v in (kernels or {}).items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
