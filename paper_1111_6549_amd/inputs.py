"""Seeded synthetic GF(2) workloads (packed uint64 row words).

Input synthesis only: random bits (``csrc/inputs.c``, xoshiro256** per row),
0/1 integer products for matrices of known rank, and the shapes of the batch
and serving workloads.  No elimination, table or PLE arithmetic lives here;
the HIP library and the CPU oracle both take their inputs from this module
and share nothing else.

Packed format: row-major, ``ldw`` words per row, column j of row i is bit
(j & 63) of word ``A[i, j >> 6]``; bits at columns >= n are zero.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "inputs.c")
_LIB = os.path.join(_HERE, "libgf2inputs.so")
_lib = None

# density 0.05 as the threshold on the top 32 bits of one draw
THRESH_005 = 214748365


def build(force=True):
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, u64, p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        lib.gf2in_bernoulli.argtypes = [p, i64, i64, i64, u64, u64, u64]
        lib.gf2in_raw.argtypes = [p, i64, u64, u64]
        _lib = lib
    return _lib


def words(n):
    """Words per row needed for n columns."""
    return (int(n) + 63) // 64


def density_threshold(p):
    if p == 0.5:
        return 0
    t = int(round(p * 2.0 ** 32))
    if not 0 < t < 2 ** 32:
        raise ValueError("density must be in (0, 1)")
    return t


def bernoulli(m, n, seed, p=0.5, ldw=None, id_base=0, out=None):
    """m x n matrix with i.i.d. Bernoulli(p) entries; row i uses stream id_base + i."""
    ldw = words(n) if ldw is None else int(ldw)
    if out is None:
        out = np.empty((m, ldw), dtype=np.uint64)
    assert out.dtype == np.uint64 and out.shape == (m, ldw) and out.flags["C_CONTIGUOUS"]
    if m > 0 and ldw > 0:
        _load().gf2in_bernoulli(out.ctypes.data_as(ctypes.c_void_p), m, n, ldw,
                                seed & (2 ** 64 - 1), id_base, density_threshold(p))
    return out


def raw(count, seed, stream_id):
    out = np.empty(count, dtype=np.uint64)
    if count:
        _load().gf2in_raw(out.ctypes.data_as(ctypes.c_void_p), count, seed & (2 ** 64 - 1), stream_id)
    return out


def unpack(A, n):
    """Packed (m, ldw) uint64 -> (m, n) uint8 0/1."""
    A = np.ascontiguousarray(A)
    b = np.unpackbits(A.view(np.uint8), axis=1, bitorder="little")
    return b[:, :n]


def pack(bits, ldw=None):
    """(m, n) 0/1 array -> packed (m, ldw) uint64."""
    bits = np.asarray(bits, dtype=np.uint8)
    m, n = bits.shape
    ldw = words(n) if ldw is None else int(ldw)
    padded = np.zeros((m, ldw * 64), dtype=np.uint8)
    padded[:, :n] = bits
    return np.packbits(padded, axis=1, bitorder="little").view(np.uint64).reshape(m, ldw)


def _product_mod2(Xb, Yb, device=None):
    """0/1 integer product X @ Y reduced mod 2 (exact in float32 for k < 2^24)."""
    if device is None or str(device) == "cpu":
        prod = np.matmul(Xb.astype(np.float32), Yb.astype(np.float32))
        return (prod.astype(np.int64) & 1).astype(np.uint8)
    import torch
    X = torch.from_numpy(Xb.astype(np.float32)).to(device)
    Y = torch.from_numpy(Yb.astype(np.float32)).to(device).contiguous()
    prod = torch.matmul(X, Y)
    out = (prod.to(torch.int64) & 1).to(torch.uint8).cpu().numpy()
    return out


def _invertible(rho, seed, tag):
    """Random invertible rho x rho matrix: unit lower times unit upper (mod 2)."""
    Lb = unpack(bernoulli(rho, rho, seed, id_base=tag), rho)
    Ub = unpack(bernoulli(rho, rho, seed, id_base=tag + (1 << 40)), rho)
    Lb = np.tril(Lb, -1)
    Ub = np.triu(Ub, 1)
    np.fill_diagonal(Lb, 1)
    np.fill_diagonal(Ub, 1)
    return _product_mod2(Lb, Ub)


def _permutation(size, seed, tag):
    keys = raw(size, seed, tag)
    return np.argsort(keys, kind="stable")


def known_rank_factors(m, n, rho, seed_x, seed_y):
    """0/1 factors X (m x rho) and Y (rho x n) of full rank rho.

    Uniform i.i.d. bits when both margins m - rho and n - rho are at least 64
    (then each factor is rank deficient with probability below 2^-64).
    Otherwise, so that the rank is exact by construction, X is a row-permuted
    [M; R] and Y a column-permuted [M' | R'] with M, M' products of random
    unit lower and unit upper triangular matrices and R, R' uniform.
    """
    if not 0 <= rho <= min(m, n):
        raise ValueError("rank must be in [0, min(m, n)]")
    if rho == 0:
        return np.zeros((m, 0), np.uint8), np.zeros((0, n), np.uint8)
    if m - rho >= 64 and n - rho >= 64:
        Xb = unpack(bernoulli(m, rho, seed_x), rho)
        Yb = unpack(bernoulli(rho, n, seed_y), n)
        return Xb, Yb
    M = _invertible(rho, seed_x, 1 << 44)
    R = unpack(bernoulli(m - rho, rho, seed_x, id_base=1 << 45), rho) if m > rho else np.zeros((0, rho), np.uint8)
    Xb = np.concatenate([M, R], axis=0)[_permutation(m, seed_x, 1 << 46)]
    M2 = _invertible(rho, seed_y, 1 << 44)
    R2 = unpack(bernoulli(rho, n - rho, seed_y, id_base=1 << 45), n - rho) if n > rho else np.zeros((rho, 0), np.uint8)
    Yb = np.concatenate([M2, R2], axis=1)[:, _permutation(n, seed_y, 1 << 46)]
    return Xb, Yb


def known_rank(m, n, rho, seed_x, seed_y, ldw=None, device=None):
    """Packed m x n matrix X * Y of rank exactly rho (see known_rank_factors)."""
    Xb, Yb = known_rank_factors(m, n, rho, seed_x, seed_y)
    if rho == 0:
        return np.zeros((m, words(n) if ldw is None else ldw), np.uint64)
    return pack(_product_mod2(Xb, Yb, device), ldw)


# ---------------------------------------------------------------------------
# Workload recipes (shapes and seeds of the benchmark configurations)
# ---------------------------------------------------------------------------

def batch_shapes(count=4096, seed=7, lo=64, hi=2048):
    """Shapes of the uneven batch: m, n ~ U{lo..hi}; every 4th (i % 4 == 3)
    matrix is a known-rank product with rho ~ U{ceil(m/4) .. min(m, n)}
    (rho = n when ceil(m/4) > n).  Returns a list of dicts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ms = rng.integers(lo, hi + 1, size=count)
    ns = rng.integers(lo, hi + 1, size=count)
    u = rng.random(count)
    out = []
    for i in range(count):
        m, n = int(ms[i]), int(ns[i])
        d = {"m": m, "n": n, "kind": "bernoulli", "rank": None}
        if i % 4 == 3:
            lo_r = -(-m // 4)
            hi_r = min(m, n)
            rho = n if lo_r > n else lo_r + int(u[i] * (hi_r - lo_r + 1))
            rho = min(rho, hi_r)
            d["kind"] = "known_rank"
            d["rank"] = rho
        out.append(d)
    return out


def batch_matrix(shape, seed, index, device=None):
    """Packed matrix `index` of a batch (deterministic per (seed, index))."""
    m, n = shape["m"], shape["n"]
    sub = (seed << 20) ^ (index * 0x100000001B3)
    if shape["kind"] == "known_rank":
        return known_rank(m, n, shape["rank"], sub ^ 0xA5A5, sub ^ 0x5A5A, device=device)
    return bernoulli(m, n, sub)


def serving_requests(count, seed=8, lo=128, hi=16384, rate=None):
    """Request stream: side s = round(exp(U(ln lo, ln hi))), square or s x ceil(s/2)
    with probability 1/2 each, density 0.5 or 0.05 with probability 1/2 each,
    Poisson arrivals at `rate` per second (None: all at time 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
    rect = rng.random(count) < 0.5
    dens = np.where(rng.random(count) < 0.5, 0.5, 0.05)
    if rate:
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    else:
        arrivals = np.zeros(count)
    reqs = []
    for i in range(count):
        m = int(s[i])
        n = int(-(-m // 2)) if rect[i] else m
        reqs.append({"m": m, "n": n, "p": float(dens[i]), "seed": (seed << 24) + i, "t": float(arrivals[i])})
    return reqs
