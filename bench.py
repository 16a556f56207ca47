#!/usr/bin/env python
"""Benchmark: PLE decomposition of a dense 65536 x 65536 GF(2) matrix on one
MI355X through the C ABI (gf2_ple).

One step = one full PLE of the resident matrix by Algorithm 3 with one
column split (Section 3.3; --alg 2 times Algorithm 2 alone): the left block
(3/8 of the columns) by the pass loop of Algorithm 2 (panel, permute,
trailing update), the triangular solve of the right block's top rows, the
Schur product on the fp4 matrix cores, and the lower-right block by the pass
loop again.  Before each step the input is restored from a pristine device
copy (a 512 MiB device-to-device copy, inside the timed region, about 0.1 ms
of a step).  Prints ONE JSON line on stdout; progress goes to stderr.

  value      whole-job throughput in PLE decompositions per second
  roofline   the dominant kernel (the Four-Russians trailing update k_m4rm
             of the two pass loops): algorithmic bytes per launch / average
             launch time, both from a second, event-timed repetition of the
             same steps (HIP events on the launch stream, recorded by the
             library itself); roofline_product and roofline_trsm give the
             same for the matrix-core product and the triangular solve
  cpu_baseline  the CPU oracle (plain Gaussian elimination) timed on this
             host on the benchmark matrix itself, over its first columns (a
             bounded share of the elimination), scaled to the whole by the
             expected row-word operations of the pivot sequence
Further legs (each can be skipped): Algorithm 3 and the product comparison,
the other configurations (1024^2, 16384^2 uniform and rank 12000,
32768 x 131072) with the oracle beside each, the 10000^2 density sweep, the
RREF helpers, the uneven batch and the serving stream.
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
FP4_PEAK_TFLOPS = 10100.0
TRSM_BLOCK = 2048  # Algorithm 3's diagonal blocks of the solve with fp4 products (csrc/alg3.hip)
KW = 64
# HBM bytes per trailing-update launch on the 65536^2 seed-5 workload (the
# default timed path: Algorithm 3 with one split at column 24576):
# rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE, averaged over the update
# launches of one PLE and scaled by the same counters on the 512 MiB restore
# copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Reported only for that
# configuration and while the kernel sources hash to the value the counters
# were taken on.
TRAFFIC = {"source": "54742199ad7df76a", "n": 65536, "seed": 5, "split": 24576, "bytes_per_launch": 158715144}


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_work(m, n, Q, r, c_end=None):
    """Expected row-word operations of the oracle's elimination up to column
    c_end (all columns if None): at the pivot of column c (rank t before it)
    every row below is tested (one word) and, for a uniformly random trailing
    block, half of them take the pivot row's words from c on (read and write)."""
    import numpy as np
    nw = (n + 63) // 64
    q = np.asarray(Q[:r], dtype=np.float64)
    t = np.arange(r, dtype=np.float64)
    keep = q < (n if c_end is None else c_end)
    cost = (m - t - 1) * (1.0 + (nw - np.floor(q / 64.0)) / 2.0)
    return float(cost[keep].sum())


def oracle_prefix(A, n, c_end, threads, Q_full, r_full):
    """The untouched oracle's elimination of the first c_end columns of A (a
    copy; the whole matrix, so nothing fits a cache that the full run would
    not), on `threads` threads; the time scaled to the whole elimination by
    the expected row-word operations (oracle_work) of the full pivot
    sequence.  Returns (scaled seconds, measured seconds, work fraction)."""
    import numpy as np
    import oracle
    m = A.shape[0]
    B = np.array(A, copy=True)
    oracle.set_threads(threads)
    try:
        t0 = time.perf_counter()
        oracle.ple_cols(B, n, c_end)
        dt = time.perf_counter() - t0
    finally:
        oracle.set_threads(os.cpu_count() or 1)
    frac = oracle_work(m, n, Q_full, r_full, c_end) / oracle_work(m, n, Q_full, r_full)
    return dt / frac, dt, frac


def cpu_baseline(A, n, Q, r, args, log_fn):
    """The oracle on the benchmark matrix itself (65536^2, seed 5): its first
    args.cpu_cols columns on every core, and its first args.cpu_cols_1core
    columns on one core, each scaled to the whole elimination by the expected
    row-word operations of the measured pivot sequence."""
    import oracle
    cores = oracle.threads()
    full, dt, frac = oracle_prefix(A, n, args.cpu_cols, cores, Q, r)
    log_fn("cpu baseline: first %d columns on %d threads in %.2f s (%.4f of the work)" % (args.cpu_cols, cores, dt,
                                                                                            frac))
    one, dt1, frac1 = oracle_prefix(A, n, args.cpu_cols_1core, 1, Q, r)
    log_fn("cpu baseline: first %d columns on 1 thread in %.2f s (%.4f of the work)" % (args.cpu_cols_1core, dt1,
                                                                                          frac1))
    return {
        "value": 1.0 / full,
        "unit": "matrices/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "the benchmark matrix itself (%dx%d, seed %d): the oracle's first %d column steps on %d threads "
                  "took %.2f s, %.4f of the whole elimination's expected row-word operations (from its pivot "
                  "sequence), so %.1f s for the whole PLE" % (A.shape[0], n, args.seed, args.cpu_cols, cores, dt,
                                                              frac, full),
        "cpu_model": cpu_model(),
        "one_core": {"value": 1.0 / one, "unit": "matrices/s", "cores": 1,
                     "sample": "first %d column steps in %.2f s, %.5f of the work, so %.0f s for the whole PLE"
                               % (args.cpu_cols_1core, dt1, frac1, one)},
    }


def run_configs(args, log_fn):
    """The other workloads of the method on one GPU, each next to the oracle:
    1024^2 (seed 1), 16384^2 uniform (seed 2), 16384^2 of rank 12000 (X seed
    3 times Y seed 4) and 32768 x 131072 (seed 6).  GPU: median of repeated
    gf2_ple calls on resident input (restored from a device copy outside the
    timing); the trailing-update launches' algorithmic bytes per launch over
    their mean event-timed duration (the HBM fraction of the dominant
    kernel; at these sizes the matrix fits the 256 MB Infinity Cache, so it is
    an upper bound of the HBM share).  Oracle: whole runs (median) where they
    take seconds, else the first columns scaled as for the headline."""
    import numpy as np
    import torch

    import oracle
    from paper_1111_6549_amd import gf2ple as G
    from paper_1111_6549_amd import inputs

    cores = oracle.threads()
    cases = [
        ("1024x1024 Bernoulli(0.5) seed 1", 1024, 1024, lambda: inputs.bernoulli(1024, 1024, 1), 20,
         {"all": ("whole", 20), "one": ("whole", 20)}),
        ("16384x16384 Bernoulli(0.5) seed 2", 16384, 16384, lambda: inputs.bernoulli(16384, 16384, 2), 10,
         {"all": ("whole", 3), "one": ("prefix", 2048)}),
        ("16384x16384 rank 12000: X (16384x12000, seed 3) Y (12000x16384, seed 4)", 16384, 16384,
         lambda: inputs.known_rank(16384, 16384, 12000, 3, 4, device="cuda"), 10,
         {"all": ("whole", 3), "one": ("prefix", 2048)}),
        ("32768x131072 Bernoulli(0.5) seed 6", 32768, 131072, lambda: inputs.bernoulli(32768, 131072, 6), 5,
         {"all": ("prefix", 2048)}),
    ]
    out = []
    for name, m, n, make, reps, cpu_plan in cases:
        A = make()
        ldw = inputs.words(n)
        dev = torch.from_numpy(A.view(np.int64)).cuda()
        work = torch.empty_like(dev)
        ws = G.alloc_workspace(G.workspace_bytes(m, n, ldw))
        times = []
        for rep in range(reps + 2):
            work.copy_(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P, Q, rank = G.ple(work, n, ws=ws)
            torch.cuda.synchronize()
            if rep >= 2:
                times.append((time.perf_counter() - t0) * 1000.0)
        times.sort()
        r = int(rank.item())
        Qh = Q.cpu().numpy()
        kinds = G.ple_schedule(m, n)
        abytes = alg_bytes_m4rm(m, n, Qh, r, kinds)
        G.profile_start()
        for rep in range(3):
            work.copy_(dev)
            G.ple(work, n, ws=ws)
        torch.cuda.synchronize()
        prof = G.profile_stop()
        pt = {"workload": name, "m": m, "n": n, "rank": r, "gpu_ms": round(times[len(times) // 2], 4),
              "reps": reps, "update_alg_bytes": abytes}
        k = prof.get("m4rm")
        if k and k["launches"] and abytes:
            per_launch = abytes / (k["launches"] / 3.0)
            avg_ms = k["total_ms"] / k["launches"]
            pt["update_avg_launch_ms"] = round(avg_ms, 5)
            pt["update_alg_GBps"] = round(per_launch / (avg_ms * 1e-3) / 1e9, 1)
            pt["update_frac_hbm"] = round(pt["update_alg_GBps"] / HBM_PEAK_GBPS, 4)
        pt["whole_ple_alg_GBps"] = round(abytes / (pt["gpu_ms"] * 1e-3) / 1e9, 1)
        if not args.no_cpu_baseline:
            for which, (how, count) in cpu_plan.items():
                th = cores if which == "all" else 1
                if how == "whole":
                    oracle.set_threads(th)
                    ts = []
                    for _ in range(count):
                        B = np.array(A, copy=True)
                        t0 = time.perf_counter()
                        oracle.ple(B, n)
                        ts.append(time.perf_counter() - t0)
                    oracle.set_threads(os.cpu_count() or 1)
                    ts.sort()
                    pt["oracle_%s" % which] = {"cores": th, "ms": round(ts[len(ts) // 2] * 1e3, 2),
                                               "sample": "whole PLE, median of %d" % count}
                else:
                    full, dt, frac = oracle_prefix(A, n, count, th, Qh, r)
                    pt["oracle_%s" % which] = {"cores": th, "ms": round(full * 1e3, 1),
                                               "sample": "first %d column steps in %.2f s, %.4f of the expected "
                                                         "row-word operations, scaled" % (count, dt, frac)}
        out.append(pt)
        log_fn("config: %s" % json.dumps(pt))
        del dev, work, ws, A
        torch.cuda.empty_cache()
    return {"cpu_model": cpu_model(), "points": out}


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
    # the batch's algorithmic bytes: per matrix, 16 B per trailing row word
    # per 64-column pass (the batched kernel runs single passes), from its
    # own pivot columns; a weak HBM bound, most of it served from the caches
    Qa, Ra = Q.cpu().numpy(), R.cpu().numpy()
    bbytes = 0
    for d, rk in zip(descs, Ra):
        qd = Qa[d["q_off"]:d["q_off"] + min(d["m"], d["n"])]
        bbytes += alg_bytes_m4rm(d["m"], d["n"], qd, int(rk), [0] * ((d["n"] + 63) // 64))
    out["alg_bytes"] = int(bbytes)
    out["alg_GBps"] = round(bbytes / batched_s / 1e9, 1)
    out["frac_hbm"] = round(bbytes / batched_s / 1e9 / HBM_PEAK_GBPS, 4)
    out["bound"] = "latency of the serial panels (about min(m, n)/64 per matrix) and LDS/VALU table work"
    if not args.no_cpu_baseline:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        cores = oracle.threads()
        host = [np.array(mt, copy=True) for mt in mats]

        def one(i):
            oracle.set_threads(1)  # this worker thread's elimination on one core
            oracle.ple(host[i], shapes[i][1])

        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=cores) as ex:
            list(ex.map(one, range(count)))
        dt = time.perf_counter() - t0
        sample = list(range(0, count, max(1, count // args.batch_cpu_sample)))[:args.batch_cpu_sample]
        host1 = [np.array(mats[i], copy=True) for i in sample]
        oracle.set_threads(1)
        t0 = time.perf_counter()
        for i, B in zip(sample, host1):
            oracle.ple(B, shapes[i][1])
        dt1 = time.perf_counter() - t0
        oracle.set_threads(os.cpu_count() or 1)
        out["cpu_baseline"] = {"value": round(count / dt, 2), "unit": "matrices/s", "cores": cores,
                               "kind": "oracle",
                               "sample": "all %d matrices, one matrix per thread on %d threads, %.2f s"
                                         % (count, cores, dt),
                               "one_core": {"value": round(len(sample) / dt1, 2), "unit": "matrices/s", "cores": 1,
                                            "sample": "%d of the %d matrices (every %d-th) in %.2f s"
                                                      % (len(sample), count, count // len(sample), dt1)}}
        log_fn("batched: oracle %.2f s on %d threads, %.2f s for %d on one" % (dt, cores, dt1, len(sample)))
    plan.close()
    return out


def run_serving(args, log_fn):
    """Serving: a request stream (sides log-uniform in [128, 16384], square or
    s x ceil(s/2), density 0.5 or 0.05; seed 8), inputs resident on the device.
    Plain = gf2_ple per request in arrival order on one stream.  Served = the
    serving session (64 GiB budget) fed Poisson arrivals at 0.5, 0.9 and 1.5x
    the measured plain capacity (latency = arrival -> result in device
    memory), and the same requests all at once (saturated throughput).  The
    plain latency at the same arrivals is a FIFO replay of the measured plain
    service times.  The oracle serves the first requests at the 0.9x arrivals,
    one request per core in arrival order."""
    import numpy as np
    import torch

    from paper_1111_6549_amd import gf2ple as G
    from paper_1111_6549_amd import inputs

    count = args.serve_count
    reqs = inputs.serving_requests(count, seed=8)
    dev = []
    host_first = []
    for k, r in enumerate(reqs):
        A = inputs.bernoulli(r["m"], r["n"], r["seed"], p=r["p"])
        dev.append(torch.from_numpy(A.view(np.int64)).cuda())
        if k < args.serve_cpu_sample:
            host_first.append(A)
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
    outs = []
    for (r, t), (a, b) in zip(zip(reqs, dev), ev):
        w = scratch[:t.numel()].view(t.shape)
        w.copy_(t)
        a.record()
        outs.append(G.ple(w, r["n"], ws=wsp))
        b.record()
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    service = np.array([a.elapsed_time(b) * 1e-3 for a, b in ev])
    capacity = count / plain_s
    log_fn("serving: plain %.3f s (%.1f req/s)" % (plain_s, capacity))
    # the stream's algorithmic bytes: per request, 16 B per trailing row word
    # per 64-column pass (a schedule-independent count), from its pivots
    sbytes = 0
    for r, (P, Q, rank) in zip(reqs, outs):
        rk = int(rank.item())
        sbytes += alg_bytes_k64(r["m"], r["n"], Q.cpu().numpy(), rk)
    del scratch, wsp, outs

    def serve(arrivals):
        S = G.ServeSession(budget_bytes=64 << 30, small_max_dim=args.serve_small_max, streams=args.serve_streams)
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

    def fifo(arrivals, service_s, servers=1):
        """Completion latencies of a FIFO queue with `servers` servers."""
        free = [0.0] * servers
        lat = np.empty(len(arrivals))
        for i, at in enumerate(arrivals):
            k = int(np.argmin(free))
            fin = max(at, free[k]) + service_s[i]
            free[k] = fin
            lat[i] = fin - at
        return lat

    pct = lambda x, q: round(float(np.percentile(x, q)) * 1e3, 3)
    rng = np.random.Generator(np.random.PCG64(8))
    unit_gaps = rng.exponential(1.0, size=count)  # one draw, scaled per rate
    poisson = []
    arrivals_09 = None
    for mult in (0.5, 0.9, 1.5):
        rate = mult * capacity
        arrivals = np.cumsum(unit_gaps / rate)
        arrivals -= arrivals[0]
        if mult == 0.9:
            arrivals_09 = arrivals
        lat, span, st = serve(arrivals)
        plain_lat = fifo(arrivals, service)
        pt = {"load": mult, "rate_per_s": round(rate, 1), "served_p50_ms": pct(lat, 50), "served_p99_ms": pct(lat, 99),
              "served_matrices_per_s": round(count / span, 1), "plain_fifo_p50_ms": pct(plain_lat, 50),
              "plain_fifo_p99_ms": pct(plain_lat, 99),
              "launches": {"batched": st["launches_batched"], "single": st["launches_single"]}}
        poisson.append(pt)
        log_fn("serving: poisson %s" % json.dumps(pt))
    lat_sat, span_sat, st_sat = serve(np.zeros(count))
    log_fn("serving: saturated %.3f s for %d requests" % (span_sat, count))
    frac_sat = round(sbytes / span_sat / 1e9 / HBM_PEAK_GBPS, 4)
    out = {
        "workload": "%d requests, sides log-uniform in [128, 16384], square or s x ceil(s/2), density 0.5 or 0.05, "
                    "seed 8, inputs resident on the device, 64 GiB budget" % count,
        "plain_capacity_per_s": round(capacity, 1),
        "k64_alg_bytes": int(sbytes),
        "plain_frac_hbm": round(sbytes / plain_s / 1e9 / HBM_PEAK_GBPS, 4),
        "saturated_frac_hbm": frac_sat,
        "bound": "latency of the requests' serial panels (small requests in batched launches, large ones in "
                 "their own pass loops, three at a time)",
        "poisson": poisson,
        "saturated": {"served_matrices_per_s": round(count / span_sat, 1),
                      "plain_matrices_per_s": round(capacity, 1),
                      "speedup_vs_plain": round((count / span_sat) / capacity, 2),
                      "served_p50_ms": pct(lat_sat, 50), "served_p99_ms": pct(lat_sat, 99),
                      "launches": {"batched": st_sat["launches_batched"], "single": st_sat["launches_single"]}},
    }
    if not args.no_cpu_baseline and host_first:
        import queue
        import threading

        import oracle
        cores = oracle.threads()
        K = len(host_first)
        arr = arrivals_09[:K]
        fin = np.zeros(K)
        q = queue.Queue()

        def worker():
            oracle.set_threads(1)
            while True:
                k = q.get()
                if k is None:
                    return
                B = np.array(host_first[k], copy=True)
                oracle.ple(B, reqs[k]["n"])
                fin[k] = time.perf_counter()

        ths = [threading.Thread(target=worker) for _ in range(cores)]
        for t in ths:
            t.start()
        start = time.perf_counter()
        for k in range(K):
            while time.perf_counter() - start < arr[k]:
                time.sleep(0.0002)
            q.put(k)
        for _ in ths:
            q.put(None)
        for t in ths:
            t.join()
        oracle.set_threads(os.cpu_count() or 1)
        lat = fin - start - arr
        span = fin.max() - start
        out["cpu_baseline"] = {"value": round(K / span, 2), "unit": "matrices/s", "cores": cores, "kind": "oracle",
                               "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                               "sample": "the first %d requests at the 0.9x Poisson arrivals, one request per "
                                         "thread on %d threads in arrival order, %.2f s" % (K, cores, span)}
        log_fn("serving: oracle %s" % json.dumps(out["cpu_baseline"]))
    return out


def run_products(log_fn, shapes=((65536, 256, 65536), (65536, 512, 65536), (65536, 1024, 65536))):
    """C ^= A B over GF(2) on the tables (update 1) and on the fp4 (2) and
    int8 (4) matrix cores, for m x k x n at each shape: the best of three
    calls after one untimed call; the tables' algorithmic HBM rate (16 bytes
    per row word of C per 64 inner bits) and the matrix cores' rate
    (2 m k n operations) against their dense peaks."""
    import torch
    from paper_1111_6549_amd import gf2ple as G
    from paper_1111_6549_amd import inputs
    prod = []
    for mm, k, nn in shapes:
        C = torch.zeros((mm, (nn + 63) // 64), dtype=torch.int64, device="cuda")
        Ak = torch.from_numpy(inputs.bernoulli(mm, k, 60 + k).view("int64")).cuda()
        Bk = torch.from_numpy(inputs.bernoulli(k, nn, 61 + k).view("int64")).cuda()
        row = {"m": mm, "k": k, "n": nn}
        for update in (1, 2, 4):
            times = []
            for rep in range(4):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                G.addmul(C, Ak, Bk, k, nn, update=update)
                torch.cuda.synchronize()
                if rep:
                    times.append((time.perf_counter() - t0) * 1000.0)
            t = min(times)
            if update == 1:
                row["tables_ms"] = round(t, 3)
                row["tables_alg_GBps"] = round(16.0 * mm * ((nn + 63) // 64) * (k / 64.0) / (t * 1e-3) / 1e9, 1)
            elif update == 2:
                pf = 2.0 * mm * k * nn / (t * 1e-3) / 1e15
                row["fp4_ms"] = round(t, 3)
                row["fp4_PFLOPs"] = round(pf, 3)
                row["fp4_frac_peak"] = round(pf / 10.1, 4)
            else:
                pops = 2.0 * mm * k * nn / (t * 1e-3) / 1e15
                row["int8_ms"] = round(t, 3)
                row["int8_POPS"] = round(pops, 3)
                row["int8_frac_peak"] = round(pops / 5.0, 4)
        prod.append(row)
        log_fn("product: %s" % json.dumps(row))
        del Ak, Bk, C
        torch.cuda.empty_cache()
    return prod


def run_alg3(args, m, n, pristine, work, log_fn):
    """Algorithm 3 (block-recursive PLE) against Algorithm 2 on the bench
    matrix: gf2_ple with update = 2 (products on the fp4 matrix cores), 3 (on
    the Four-Russians tables) and 4 (on the int8 matrix cores), one and two
    levels of column splits; each the best of two calls after one untimed
    call; one uneven split (a left block of 20480 to 28672 columns,
    rec_split with one level), and left strips of 16384 columns with the
    splits going on in the right block; Algorithm 2 beside them.  Then the
    product on its own, C ^= A B for 65536 x k x 65536 at
    k = 256, 512, 1024, on the tables and both matrix-core forms: time, the
    tables' HBM rate (16 bytes per row word of C per 64 inner bits) and the
    matrix cores' rate (2 m k n operations) against the dense peaks (fp4
    10.1 PFLOP/s, int8 5.0 POPS)."""
    import torch
    from paper_1111_6549_amd import gf2ple as G
    from paper_1111_6549_amd import inputs
    ldw = inputs.words(n)
    out = {"ple": []}
    # (update, levels, split, Strassen's split of the fp4 products: 0 default, -1 none)
    cfgs = [(1, 0, 0, 0), (3, 1, 0, 0), (2, 1, 0, 0), (2, 2, 0, 0), (4, 1, 0, 0), (2, 1, 20480, 0), (2, 1, 24576, 0),
            (2, 1, 24576, -1), (2, 1, 28672, 0), (2, 16, 16384, 0)]
    for update, levels, split, psplit in cfgs:
        ws = G.alloc_workspace(G.workspace_bytes(m, n, ldw, update=update, rec_levels=levels, rec_split=split,
                                                 product_split=psplit))
        times = []
        for rep in range(3):
            work.copy_(pristine)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P, Q, rank = G.ple(work, n, ws=ws, update=update, rec_levels=levels, rec_split=split,
                               product_split=psplit)
            torch.cuda.synchronize()
            if rep:
                times.append((time.perf_counter() - t0) * 1000.0)
        pt = {"update": update, "products": {1: "none (Algorithm 2)", 2: "fp4 matrix cores",
                                             3: "Four-Russians tables", 4: "int8 matrix cores"}[update],
              "levels": levels, "split": split or "halves", "ms": round(min(times), 3), "rank": int(rank.item())}
        if update == 2:
            pt["product_split"] = {0: "default (one Strassen level on products of at least 8192 bits a side)",
                                   -1: "none"}[psplit]
        out["ple"].append(pt)
        log_fn("alg3: %s" % json.dumps(pt))
        del ws
    torch.cuda.empty_cache()
    prod = run_products(log_fn)
    out["products"] = prod
    return out


def run_helpers(m, n, A, Qh, r, log_fn):
    """The helpers of the paper's PLE-based reductions on the bench matrix (not
    in the timed step): echelon form and the reduced echelon form from L\\E
    (on the PLE result), and the reduced echelon form of the input in the
    M4RI form."""
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--cpu-cols", type=int, default=4096,
                    help="columns of the oracle's elimination timed on all cores for the CPU baseline")
    ap.add_argument("--cpu-cols-1core", type=int, default=256,
                    help="columns of the oracle's elimination timed on one core")
    ap.add_argument("--no-configs", action="store_true", help="skip the 1024^2 / 16384^2 / 32768x131072 legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-helpers", action="store_true", help="skip timing the echelon / RREF helpers")
    ap.add_argument("--m4-variant", type=int, default=0, help="update schedule 1..8 (0 = library default)")
    ap.add_argument("--m4-blocks", type=int, default=0, help="target blocks per update launch (0 = default)")
    ap.add_argument("--panel-regs", type=int, default=0, help="panel register window 2/4/8 (0 = default)")
    ap.add_argument("--lookahead", type=int, default=0,
                    help="0 = library default, 1 = serial passes, 2 = look-ahead only, 3 = pairs everywhere")
    ap.add_argument("--pair-variant", type=int, default=0, help="fused pair update schedule 1..14 (0 = default)")
    ap.add_argument("--alg", type=int, default=3, choices=(2, 3),
                    help="timed path: 3 = Algorithm 3 with one column split (default), 2 = Algorithm 2 alone "
                         "(the gf2_ple default)")
    ap.add_argument("--no-alg2", action="store_true",
                    help="skip timing Algorithm 2 alone beside the Algorithm 3 path (for profiler runs)")
    ap.add_argument("--product-split", type=int, default=0, choices=(-1, 0, 1),
                    help="Strassen's split of the fp4 products on the timed path (0 = library default)")
    ap.add_argument("--rec-split", type=int, default=0,
                    help="Algorithm 3's left block in columns (a multiple of 64; 0 = 3/8 of n)")
    ap.add_argument("--no-alg3", action="store_true", help="skip Algorithm 3 and the product comparison")
    ap.add_argument("--only-products", action="store_true",
                    help="run only the product comparison (tables, fp4 and int8 matrix cores) and exit")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain measurement")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--batch-cpu-sample", type=int, default=512)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-density", action="store_true", help="skip the 10000^2 density sweep")
    ap.add_argument("--serve-count", type=int, default=3000)
    ap.add_argument("--serve-cpu-sample", type=int, default=40)
    ap.add_argument("--serve-streams", type=int, default=0, help="serving launch streams (0 = library default)")
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
    if args.only_products:
        # the product on its own: the shapes of the comparison and the top
        # product of one Algorithm 3 level on 65536^2 (32768 x 32768 x 32768)
        prod = run_products(log, ((65536, 1024, 65536), (32768, 32768, 32768)))
        print(json.dumps({"metric": "GF(2) product C ^= A B: tables vs fp4 / int8 matrix cores", "products": prod}))
        return
    m = n = args.n
    ldw = inputs.words(n)
    log("generating %dx%d Bernoulli(0.5) seed %d" % (m, n, args.seed))
    A = inputs.bernoulli(m, n, args.seed)
    pristine = torch.from_numpy(A.view(np.int64)).cuda()
    work = torch.empty_like(pristine)
    sched = dict(m4_variant=args.m4_variant, m4_blocks=args.m4_blocks, panel_regs=args.panel_regs,
                 lookahead=args.lookahead, pair_variant=args.pair_variant)
    # Algorithm 3 with one split: the left block of `split` columns and the
    # lower-right block by Algorithm 2, the triangular solve and the Schur
    # product (fp4 matrix cores) between them
    split = (args.rec_split or (3 * n // 8)) // 64 * 64
    use_alg3 = args.alg == 3 and 64 <= split < n
    rec = dict(update=2, rec_levels=1, rec_split=split, product_split=args.product_split) if use_alg3 else {}
    ws = G.alloc_workspace(G.workspace_bytes(m, n, ldw, **rec))
    torch.cuda.synchronize()

    def step():
        work.copy_(pristine)
        return G.ple(work, n, ws=ws, **sched, **rec)

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
    abytes64 = alg_bytes_k64(m, n, Qh, r)
    trsm_bytes = prod_flops = r1 = None
    if use_alg3:
        # the two Algorithm 2 blocks' update launches, the solve's sweeps
        # (rows below each 128-row block, 16 B per row word of the right
        # block) and the product's 2 M K N operations
        import numpy as np
        r1 = int(np.count_nonzero(Qh[:r] < split))
        N = n - split
        kinds_l = G.ple_schedule(m, split, lookahead=args.lookahead)
        kinds_r = G.ple_schedule(m - r1, N, lookahead=args.lookahead)
        abytes = (alg_bytes_m4rm(m, split, Qh[:r1], r1, kinds_l) +
                  alg_bytes_m4rm(m - r1, N, Qh[r1:r] - split, r - r1, kinds_r))
        kinds = kinds_l + kinds_r
        # the solve as the library runs it with fp4 products: with one
        # diagonal block of at most TRSM_BLOCK rows, 128-row blocks swept
        # over the right block's width; with several, the blocks' inverses
        # at once (128-row steps over identities TRSM_BLOCK / 64 words wide,
        # each step's words up to its rows' columns), then per block the
        # product that removes the solved blocks above it (inner size d0)
        # and the product by its inverse.  Sweep bytes: 16 per row word
        # below each 128-row step.
        nwr = (N + 63) // 64
        trsm_bytes = 0
        # each product's 2 M K N operations, and those the matrix cores run
        # by the library's plan for it (seven half-size products when it
        # takes Strassen's split)
        prod_list = [(m - r1, r1)]
        if r1 <= TRSM_BLOCK:
            trsm_bytes = sum(16 * (r1 - b - 128) * nwr for b in range(0, r1, 128) if b + 128 < r1)
        else:
            for d0 in range(0, r1, TRSM_BLOCK):
                d1 = min(r1, d0 + TRSM_BLOCK)
                for b in range(0, d1 - d0, 128):
                    if d0 + b + 128 < d1:
                        trsm_bytes += 16 * (d1 - d0 - b - 128) * min(TRSM_BLOCK // 64, (b + 128) // 64)
                if d0 > 0:
                    prod_list.append((d1 - d0, d0))
                prod_list.append((d1 - d0, d1 - d0))
        prod_flops = sum(2 * M * K * N for M, K in prod_list)
        prod_mfma_flops = 0
        for M, K in prod_list:
            steps_, _ = G.product_plan(M, K, 64 * nwr, args.product_split)
            prod_mfma_flops += sum(2 * b[0][4] * b[0][5] * b[1][4] for kind, b in steps_ if kind == 1)
        trsm_bytes = int(trsm_bytes)
    else:
        kinds = G.ple_schedule(m, n, lookahead=args.lookahead)
        abytes = alg_bytes_m4rm(m, n, Qh, r, kinds)

    roofline = roofline_product = roofline_trsm = None
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
                    and TRAFFIC.get("seed") == args.seed and TRAFFIC.get("split") == (split if use_alg3 else 0)
                    and not args.m4_variant and not args.m4_blocks and not args.pair_variant
                    and not args.lookahead):
                traffic = TRAFFIC["bytes_per_launch"]
            roofline = {
                "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "trailing update (k_m4rm_pair for fused pairs, with the next panel on one wave; "
                          "k_m4rm / k_m4rm_w otherwise)",
                "launches_per_step": launches_per_step,
                "alg_bytes_per_launch": round(bytes_per_launch), "avg_launch_ms": round(avg_ms, 5),
            }
        if use_alg3:
            kp, kt = kernels.get("mfma"), kernels.get("trsm")
            if kp and kp["total_ms"] > 0:
                sec = kp["total_ms"] / args.steps * 1e-3  # every product of a step
                tf = prod_mfma_flops / sec / 1e12
                roofline_product = {"kernel": "k_mfma_gf2_fp4 (the Schur product, %d x %d x %d, and the solve's "
                                              "products: each diagonal block loses the solved blocks above it, "
                                              "then is multiplied by its inverse)" % (m - r1, r1, n - split),
                                    "bound": "mfma", "achieved": round(tf, 1), "peak": FP4_PEAK_TFLOPS,
                                    "unit": "TFLOP/s", "frac": round(tf / FP4_PEAK_TFLOPS, 4),
                                    "launches_per_step": kp["launches"] / args.steps,
                                    "flops_per_step": prod_mfma_flops,
                                    "classical_flops_per_step": prod_flops,
                                    "classical_equivalent_tflops": round(prod_flops / sec / 1e12, 1),
                                    "ms_per_step": round(kp["total_ms"] / args.steps, 3)}
            if kt and kt["total_ms"] > 0:
                gb = trsm_bytes / (kt["total_ms"] / args.steps * 1e-3) / 1e9
                roofline_trsm = {"kernel": "k_trsm_pair sweeps and k_trsm128 block substitutions of the "
                                           "diagonal blocks' inversion (all blocks in each launch), with the "
                                           "identities' set-up", "bound": "hbm",
                                 "achieved": round(gb, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                 "frac": round(gb / HBM_PEAK_GBPS, 4), "alg_bytes_per_step": trsm_bytes,
                                 "ms_per_step": round(kt["total_ms"] / args.steps, 3)}
        log("profiled: %s" % json.dumps(kernels))

    # Algorithm 2 alone on the same matrix in the same run: time and the
    # update kernel's rate (the gf2_ple default, for comparison)
    alg2 = None
    if use_alg3 and not args.no_alg2:
        ws2 = G.alloc_workspace(G.workspace_bytes(m, n, ldw))

        def step2():
            work.copy_(pristine)
            return G.ple(work, n, ws=ws2, **sched)

        step2()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            P2, Q2, rank2 = step2()
        torch.cuda.synchronize()
        ms2 = (time.perf_counter() - t0) * 1000.0 / args.steps
        alg2 = {"ms_per_step": round(ms2, 3), "rank": int(rank2.item())}
        log("Algorithm 2 alone: %d steps, %.3f ms/step" % (args.steps, ms2))
        if not args.no_profile:
            kinds2 = G.ple_schedule(m, n, lookahead=args.lookahead)
            ab2 = alg_bytes_m4rm(m, n, Qh, r, kinds2)
            G.profile_start()
            for i in range(args.steps):
                step2()
            torch.cuda.synchronize()
            k2 = G.profile_stop()
            k = k2.get("m4rm")
            if k and k["total_ms"] > 0:
                lps = k["launches"] / args.steps
                avg = k["total_ms"] / k["launches"]
                ach = ab2 / lps / (avg * 1e-3) / 1e9
                alg2["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                    "frac": round(ach / HBM_PEAK_GBPS, 4), "launches_per_step": lps,
                                    "alg_bytes_per_launch": round(ab2 / lps), "avg_launch_ms": round(avg, 5)}
            alg2["kernels_ms_per_step"] = {kk: round(v["total_ms"] / args.steps, 3) for kk, v in k2.items()}
        del ws2

    alg3 = None
    if not args.no_alg3:
        alg3 = run_alg3(args, m, n, pristine, work, log)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(A, n, Qh, r, args, log)

    configs = None
    if not args.no_configs:
        configs = run_configs(args, log)

    density = None
    if not args.no_density:
        density = run_density(args, log)

    # the helpers (whose M4RI form makes the library's second stream) run
    # before the serving session: its throughput must not depend on that
    del work, pristine, ws
    torch.cuda.empty_cache()
    helpers = None
    if not args.no_helpers:
        helpers = run_helpers(m, n, A, Qh, r, log)
    del A
    batched = None
    if not args.no_batched:
        batched = run_batched(args, log)
    serving = None
    if not args.no_serving:
        serving = run_serving(args, log)

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
                   "m": m, "n": n, "pass_width_K": KW,
                   "algorithm": ("Algorithm 3, one column split at %d: Algorithm 2 on the left block and on the "
                                 "lower-right block, the triangular solve in 128-row blocks between them, the "
                                 "Schur product on the fp4 matrix cores" % split) if use_alg3 else "Algorithm 2",
                   "update": "xor-table",
                   "update_schedule": "pairs of passes: one sweep with 32 nibble tables x 32-word tiles, "
                                      "the next panel inside it; single passes past the last pair",
                   "schedule": dict(sched, **rec)},
        "rank": r,
        "schedule": {"passes": len(kinds), "serial": kinds.count(0), "lookahead": kinds.count(1),
                     "fused_pairs": kinds.count(3)},
        "update_alg_bytes_per_step": abytes,
        "k64_alg_bytes_per_step": abytes64,
        "k64_alg_GBps_whole_ple": round(abytes64 / (ms_per_step * 1e-3) / 1e9, 1),
        "roofline": roofline,
        "roofline_product": roofline_product,
        "roofline_trsm": roofline_trsm,
        "left_rank": r1,
        "alg2_same_run": alg2,
        "cpu_baseline": cpu,
        "configs": configs,
        "helpers": helpers,
        "alg3": alg3,
        "density_sweep": density,
        "batched": batched,
        "serving": serving,
        "kernels_ms_per_step": {k: round(v["total_ms"] / args.steps, 3) for k, v in (kernels or {}).items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
