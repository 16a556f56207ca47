"""CPU check of the panel's kept-row slow search, as a model (Algorithm 1's
pivot search, Section 3.1): the kernel searches only the rows with a
non-zero stripe word, keeps its active rows in position order, and reduces
each group of 64 rows by the pivots when the search reaches it.  This model
follows the same steps and must pick the same pivot, at the same position,
with the same reduced word, as the eager search over every row that
Algorithm 1 describes.  A second model follows the search on several waves
(slots spread over waves, registers and lanes; per column each wave's first
candidates, the smallest over the waves, eager elimination) and must give
the same pivots and, from its special-row list, the same order of the rows
after the pass.  They pin the design; the GPU parity tests pin the kernel
itself."""
import random

import pytest

MASK = (1 << 64) - 1


def above(j):
    return 0 if j >= 63 else ((~0 << (j + 1)) & MASK)


def eager(vals, kp, order=None):
    """Every remaining row, eliminated at once: the definition.  With
    `order`, a list, it receives the first position of the row at each
    position after the pass."""
    rows = list(vals)
    ids = list(range(len(vals)))
    npiv, out = 0, []
    for j in range(kp):
        if npiv >= len(rows):
            break
        f = next((p for p in range(npiv, len(rows)) if (rows[p] >> j) & 1), None)
        if f is None:
            continue
        rows[f], rows[npiv] = rows[npiv], rows[f]
        ids[f], ids[npiv] = ids[npiv], ids[f]
        pv = rows[npiv]
        for p in range(npiv + 1, len(rows)):
            if (rows[p] >> j) & 1:
                rows[p] ^= pv & above(j)
        out.append((j, f, ids[npiv], pv))
        npiv += 1
    if order is not None:
        order[:] = ids
    return out


def kept_lazy(vals, kp):
    """The kernel's form: kept rows only, in slots whose positions never
    change; swaps exchange slot contents, or retire the pivot's slot when a
    zero row sits at the rank position; each 64-slot group is reduced by the
    pivots it has not seen yet (in order) when the search reaches it."""
    kept = [(v, p) for p, v in enumerate(vals) if v]
    nc = len(kept)
    cv = [v for v, _ in kept]
    ci = [p for _, p in kept]
    cp = [p for _, p in kept]
    rg = [0] * ((nc + 63) // 64)
    or_raw = 0
    for v in cv:
        or_raw |= v
    piv, out = [], []
    npiv = head = 0
    or_pe = 0
    for j in range(kp):
        if npiv >= len(vals):
            break
        if not ((or_raw | or_pe) >> j) & 1:
            continue
        h = kf = -1
        s0 = head & ~63
        while s0 < nc and kf < 0:
            g = s0 // 64
            for k in range(s0, min(s0 + 64, nc)):
                for q, fin in piv[rg[g]:]:
                    if (cv[k] >> q) & 1:
                        cv[k] ^= fin & above(q)
            rg[g] = len(piv)
            for k in range(s0, min(s0 + 64, nc)):
                act = cp[k] >= npiv
                if h < 0 and act:
                    h = k
                if act and (cv[k] >> j) & 1:
                    kf = k
                    break
            s0 += 64
        if kf < 0:
            continue
        found, pv, pid = cp[kf], cv[kf], ci[kf]
        if cp[h] == npiv:
            if kf != h:
                cv[h], ci[h], cv[kf], ci[kf] = pv, pid, cv[h], ci[h]
            head = h + 1
        else:
            cp[kf] = -1
            if kf == h:
                head = h + 1
        piv.append((j, pv))
        out.append((j, found, pid, pv))
        or_pe |= pv & above(j)
        npiv += 1
    return out


@pytest.mark.parametrize("seed", range(6))
def test_kept_row_search_matches_eager(seed):
    rng = random.Random(seed)
    for _ in range(60):
        n = rng.choice([1, 63, 64, 65, 257, 700, 1500])
        d = rng.choice([0.001, 0.005, 0.02, 0.08, 0.5])
        zero_heavy = rng.random() < 0.3
        vals = [0 if (zero_heavy and rng.random() < 0.7) else
                sum(1 << b for b in range(64) if rng.random() < d) for _ in range(n)]
        kp = rng.choice([64, 64, 17, 1])
        assert kept_lazy(vals, kp) == eager(vals, kp)


def kept_waves(vals, kp, nw, regs, order):
    """The multi-wave form: slot k lives in register k // (64 nw) of wave
    (k // 64) % nw, lane k % 64; per column every wave finds its first active
    slot and its first active slot with the bit in its own register and lane
    order, the smallest of the waves' win; the swap or the retirement as in
    the one-wave form; every later active slot with the bit is eliminated at
    once.  `order` receives the row order built from the special-row list:
    the pivots, the kept rows that moved, the zero-word rows that moved."""
    kept = [(v, p) for p, v in enumerate(vals) if v]
    nc = len(kept)
    assert nc <= nw * regs * 64
    wd = [v for v, _ in kept]
    cid = [p for _, p in kept]
    cpos = [p for _, p in kept]
    by_wave = [[k for q in range(regs) for k in range((q * nw + w) * 64, (q * nw + w) * 64 + 64) if k < nc]
               for w in range(nw)]
    orv = 0
    for v in wd:
        orv |= v
    out, pid_of = [], []
    dz = {}  # zero-word rows that moved: position now -> first position
    npiv, or_pe = 0, 0
    for j in range(kp):
        if npiv >= len(vals):
            break
        if not ((orv | or_pe) >> j) & 1:
            continue
        posts_a, posts_m = [], []
        for w in range(nw):
            act = [k for k in by_wave[w] if cpos[k] >= npiv]
            posts_a.append(act[0] if act else None)
            m = [k for k in act if (wd[k] >> j) & 1]
            posts_m.append(m[0] if m else None)
        cands = [k for k in posts_m if k is not None]
        if not cands:
            continue
        kf = min(cands)
        h = min(k for k in posts_a if k is not None)
        pv, found, pid = wd[kf], cpos[kf], cid[kf]
        if cpos[h] == npiv:
            if kf != h:
                wd[h], cid[h], wd[kf], cid[kf] = pv, pid, wd[h], cid[h]
        else:
            cpos[kf] = -1
            dz[found] = dz.pop(npiv, npiv)
        pe = pv & above(j)
        for k in range(nc):
            if cpos[k] > npiv and (wd[k] >> j) & 1:
                wd[k] ^= pe
        out.append((j, found, pid, pv))
        pid_of.append(pid)
        or_pe |= pe
        npiv += 1
    # the special-row list applied to the identity order
    order[:] = list(range(len(vals)))
    for l, pid in enumerate(pid_of):
        order[l] = pid
    for k in range(nc):
        if cpos[k] >= npiv and cpos[k] != cid[k]:
            order[cpos[k]] = cid[k]
    for p, first in dz.items():
        order[p] = first
    return out


def kept_waves_nz(vals, kp, nw, regs, order):
    """The multi-wave form with no retirement: when a zero-word row sits at
    the rank position, it moves into the pivot's slot as a word of 0 (its
    first position is that rank position), so the active slots are always
    the range [kthr, nc) and the first of them is kthr; only the first
    active slot with the bit is posted per wave."""
    kept = [(v, p) for p, v in enumerate(vals) if v]
    nc = len(kept)
    assert nc <= nw * regs * 64
    wd = [v for v, _ in kept]
    cid = [p for _, p in kept]
    pos = [p for _, p in kept]  # never changes
    by_wave = [[k for q in range(regs) for k in range((q * nw + w) * 64, (q * nw + w) * 64 + 64) if k < nc]
               for w in range(nw)]
    orv = 0
    for v in wd:
        orv |= v
    out, pid_of = [], []
    npiv, or_pe, kthr = 0, 0, 0
    for j in range(kp):
        if npiv >= len(vals):
            break
        if not ((orv | or_pe) >> j) & 1:
            continue
        posts = []
        for w in range(nw):
            m = [k for k in by_wave[w] if k >= kthr and (wd[k] >> j) & 1]
            posts.append(m[0] if m else None)
        cands = [k for k in posts if k is not None]
        if not cands:
            continue
        kf = min(cands)
        h = kthr
        pv, found, pid = wd[kf], pos[kf], cid[kf]
        if pos[h] == npiv:
            if kf != h:
                wd[h], cid[h], wd[kf], cid[kf] = pv, pid, wd[h], cid[h]
            kthr += 1
        else:
            wd[kf], cid[kf] = 0, npiv
        pe = pv & above(j)
        for k in range(kthr, nc):
            if (wd[k] >> j) & 1:
                wd[k] ^= pe
        out.append((j, found, pid, pv))
        pid_of.append(pid)
        or_pe |= pe
        npiv += 1
    order[:] = list(range(len(vals)))
    for l, pid in enumerate(pid_of):
        order[l] = pid
    for k in range(kthr, nc):
        if cid[k] != pos[k]:
            order[pos[k]] = cid[k]
    return out


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("nw,regs", [(16, 8), (8, 16), (1, 8)])
def test_multi_wave_no_retire_matches_eager(seed, nw, regs):
    rng = random.Random(200 + seed)
    for _ in range(25):
        n = rng.choice([1, 64, 65, 300, 700, 1500])
        d = rng.choice([0.002, 0.01, 0.05, 0.3])
        zero_heavy = rng.random() < 0.4
        vals = [0 if (zero_heavy and rng.random() < 0.7) else
                sum(1 << b for b in range(64) if rng.random() < d) for _ in range(n)]
        if sum(1 for v in vals if v) > nw * regs * 64:
            continue
        kp = rng.choice([64, 64, 23])
        o1, o2 = [], []
        assert kept_waves_nz(vals, kp, nw, regs, o2) == eager(vals, kp, o1)
        assert o2 == o1


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("nw,regs", [(16, 8), (8, 16), (1, 8)])
def test_multi_wave_search_matches_eager(seed, nw, regs):
    rng = random.Random(100 + seed)
    for _ in range(25):
        n = rng.choice([1, 64, 65, 300, 700, 1500])
        d = rng.choice([0.002, 0.01, 0.05, 0.3])
        zero_heavy = rng.random() < 0.4
        vals = [0 if (zero_heavy and rng.random() < 0.7) else
                sum(1 << b for b in range(64) if rng.random() < d) for _ in range(n)]
        if sum(1 for v in vals if v) > nw * regs * 64:
            continue
        kp = rng.choice([64, 64, 23])
        o1, o2 = [], []
        assert kept_waves(vals, kp, nw, regs, o2) == eager(vals, kp, o1)
        assert o2 == o1
