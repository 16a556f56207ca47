"""GPU parity: the HIP library (through the C ABI) against the CPU oracle,
bit for bit on (rank, P, Q, L\\E), on seeded inputs that span several tiles,
ragged tails, both pivot-search paths, sparse, rank-deficient, known-rank,
empty and degenerate matrices."""
import numpy as np
import pytest
import torch

from paper_1111_6549_amd import gf2ple as G
from paper_1111_6549_amd import inputs
from tests import helpers as H
from tests.gpu_util import assert_same_ple, gpu_ple, oracle_ple, say, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [
    (1, 1), (1, 64), (64, 1), (63, 63), (64, 64), (65, 65), (100, 70), (70, 100), (127, 129),
    (257, 300), (300, 257), (511, 513), (513, 511), (600, 64), (1000, 1), (1, 1000),
    (130, 2000), (2000, 130), (640, 1100),
]


@pytest.mark.parametrize("m,n", SHAPES)
def test_parity_uniform(m, n):
    say("parity uniform", m, n)
    A = inputs.bernoulli(m, n, 100 + m * 7 + n)
    assert_same_ple(gpu_ple(A, n), oracle_ple(A, n), "%dx%d" % (m, n))


def test_parity_1024_seed1():
    say("parity 1024x1024 seed 1")
    A = inputs.bernoulli(1024, 1024, 1)
    g = gpu_ple(A, 1024)
    assert_same_ple(g, oracle_ple(A, 1024), "1024^2")
    H.check_ple(H.unpack(A, 1024), H.unpack(g[3], 1024), g[0], g[1], g[2])


@pytest.mark.parametrize("m,n,p", [(500, 500, 0.05), (700, 700, 0.01), (1000, 1000, 0.002), (300, 900, 0.05),
                                   (900, 300, 0.01), (2000, 2000, 0.0005)])
def test_parity_sparse(m, n, p):
    say("parity sparse", m, n, p)
    A = inputs.bernoulli(m, n, 7 * m + n, p=p)
    assert_same_ple(gpu_ple(A, n), oracle_ple(A, n), "%dx%d p=%g" % (m, n, p))


DENSITY_POINTS = (0.1, 0.2, 0.5, 1.0, 2.0, 3.0, 5.0, 8.0, 12.0, 20.0)


@pytest.mark.parametrize("x,seed", [(x, 9 + i) for i, x in enumerate(DENSITY_POINTS)])
def test_parity_density_10000(x, seed):
    """Every point of the 10000 x 10000 sparse sweep (x non-zero entries per
    row on average), with the seeds the sweep in bench.py uses (9 + index)."""
    say("parity 10000^2 density", x)
    A = inputs.bernoulli(10000, 10000, seed, p=x / 10000)
    assert_same_ple(gpu_ple(A, 10000), oracle_ple(A, 10000), "10000^2 x=%g" % x)


def test_parity_sparse_tall():
    """30000 x 1500 with about 10 non-zero entries per row: the first stripes
    keep more than 9216 rows with a non-zero stripe word, beyond the panel's
    LDS, so the slow search runs on its workspace copy."""
    say("parity sparse tall 30000x1500")
    A = inputs.bernoulli(30000, 1500, 31, p=10 / 1500)
    assert_same_ple(gpu_ple(A, 1500), oracle_ple(A, 1500), "30000x1500 sparse")


def test_parity_slow_search_forms():
    """24000 x 3072 whose 256-column blocks cycle through 0.0003, 0.005 and
    0.02 non-zero entries per bit: the slow searches of its stripes keep from
    a few hundred rows (handed to the one-wave search) to a few thousand (the
    multi-wave search) and beyond 8192 (its fall-back), in the standalone
    panels and in the pair updates' panel blocks."""
    m, n = 24000, 3072
    say("parity slow-search forms", m, n)
    dens = (0.0003, 0.005, 0.02)
    A = np.ascontiguousarray(np.concatenate(
        [inputs.bernoulli(m, 256, 40 + b, p=dens[b % 3]) for b in range(n // 256)], axis=1))
    assert A.shape == (m, inputs.words(n))
    assert_same_ple(gpu_ple(A, n), oracle_ple(A, n), "24000x3072 banded densities")


@pytest.mark.parametrize("m,n,rho", [(600, 600, 300), (1000, 700, 650), (700, 1000, 700), (800, 800, 800),
                                     (3000, 300, 50), (8000, 300, 100), (256, 2048, 200)])
def test_parity_known_rank(m, n, rho):
    say("parity known rank", m, n, rho)
    A = inputs.known_rank(m, n, rho, 11 + m, 13 + n)
    g = gpu_ple(A, n)
    assert g[0] == rho
    assert_same_ple(g, oracle_ple(A, n), "%dx%d rank %d" % (m, n, rho))


def test_parity_degenerate():
    for m, n in [(300, 300), (65, 200)]:
        say("zero matrix", m, n)
        A = np.zeros((m, inputs.words(n)), np.uint64)
        g = gpu_ple(A, n)
        assert g[0] == 0
        assert_same_ple(g, oracle_ple(A, n), "zero")
    say("identity and reversed identity")
    for rev in (False, True):
        bits = np.eye(200, dtype=np.uint8)
        if rev:
            bits = bits[::-1].copy()
        A = H.pack(bits)
        assert_same_ple(gpu_ple(A, 200), oracle_ple(A, 200), "eye rev=%s" % rev)
    say("all-ones")
    A = H.pack(np.ones((150, 170), np.uint8))
    assert_same_ple(gpu_ple(A, 170), oracle_ple(A, 170), "ones")
    say("padding words")
    A = inputs.bernoulli(100, 100, 5, ldw=5)
    assert_same_ple(gpu_ple(A, 100), oracle_ple(A, 100), "ldw 5")


def test_empty_shapes():
    for m, n in [(0, 10), (10, 0), (0, 0)]:
        say("empty", m, n)
        A = np.zeros((m, inputs.words(n)), np.uint64)
        t = torch.zeros((m, inputs.words(n)), dtype=torch.int64, device="cuda")
        P, Q, rank = G.ple(t, n)
        torch.cuda.synchronize()
        assert int(rank.item()) == 0
        assert list(P.cpu().numpy()) == list(range(m))
        assert Q.numel() == 0


def test_paper_examples_on_gpu():
    blocks = dict(H.read_golden("perm_example.txt"))
    mat = np.array(blocks["matrix"], dtype=np.uint8)
    r, P, Q, out = gpu_ple(H.pack(mat), 5)
    assert r == 5 and list(P) == blocks["P"]
    for key, val in H.read_golden("postprocess_example.txt"):
        if key == "case":
            case = np.array(val, dtype=np.uint8)
        else:
            r, P, Q, out = gpu_ple(H.pack(case), 8)
            assert list(H.unpack(out, 8)[3, :3]) == val


@pytest.mark.parametrize("m,n,seed,rho", [(16384, 16384, 2, None), (16384, 16384, 3, 12000)])
def test_parity_16384(m, n, seed, rho):
    say("parity 16384^2 seed", seed, "rank", rho)
    if rho is None:
        A = inputs.bernoulli(m, n, seed)
    else:
        A = inputs.known_rank(m, n, rho, seed, seed + 1, device="cuda")
    g = gpu_ple(A, n)
    if rho is not None:
        assert g[0] == rho
    say("  gpu done, rank", g[0])
    assert_same_ple(g, oracle_ple(A, n), "16384^2")


# --- the other calls ---------------------------------------------------------

@pytest.mark.parametrize("m,k,n", [(1, 1, 1), (100, 64, 100), (257, 130, 1000), (1000, 200, 64), (64, 1, 513),
                                   (3000, 64, 3000)])
def test_addmul_parity(m, k, n):
    say("addmul", m, k, n)
    import oracle
    C = inputs.bernoulli(m, n, 1 + m)
    A = inputs.bernoulli(m, k, 2 + k)
    B = inputs.bernoulli(k, n, 3 + n)
    want = C.copy()
    oracle.addmul(want, A, B, k, n)
    tC = to_dev(C)
    G.addmul(tC, to_dev(A), to_dev(B), k, n)
    assert np.array_equal(to_host(tC), want)


def test_make_table_parity():
    import oracle
    f3 = dict(H.read_golden("fig3_m4ri.txt"))
    piv = H.pack(np.array(f3["pivots"], np.uint8))
    T = to_host(G.make_table(to_dev(piv), 3, 8))
    assert np.array_equal(H.unpack(T, 8), np.array(f3["table"], np.uint8))
    for k, n in [(1, 5), (4, 130), (8, 1000)]:
        rows = inputs.bernoulli(k, n, 40 + k)
        T = to_host(G.make_table(to_dev(rows), k, n))
        assert np.array_equal(T, oracle.make_table(rows, k))


@pytest.mark.parametrize("m,n,kind", [(300, 500, "u"), (1000, 1000, "u"), (700, 400, "r"), (129, 2000, "u"),
                                      (2000, 700, "r"), (600, 600, "s"), (4096, 4096, "u"), (3000, 2500, "r")])
def test_echelon_and_rref_parity(m, n, kind):
    say("echelon/rref", m, n, kind)
    import oracle
    if kind == "u":
        A = inputs.bernoulli(m, n, 21 + m)
    elif kind == "r":
        A = inputs.known_rank(m, n, min(m, n) // 2, 5, 6)
    else:
        A = inputs.bernoulli(m, n, 22 + m, p=0.01)
    # echelon
    t = to_dev(A)
    P, Q, rank = G.ple(t, n)
    G.echelon_from_ple(t, n, rank)
    B = A.copy()
    r, _, _ = oracle.ple(B, n)
    oracle.echelon_from_ple(B, n, r)
    assert np.array_equal(to_host(t), B)
    # rref via the combined call
    t = to_dev(A)
    P, Q, rank = G.rref(t, n)
    R, r2, _ = oracle.rref(A, n)
    assert int(rank.item()) == r2
    assert np.array_equal(to_host(t), R)


@pytest.mark.parametrize("m,n,kind", [(300, 500, "u"), (1000, 1000, "u"), (700, 400, "r"), (129, 2000, "u"),
                                      (2000, 700, "r"), (600, 600, "s"), (4096, 4096, "u"), (3000, 2500, "r"),
                                      (1, 1, "u"), (64, 64, "u"), (65, 130, "r"), (8192, 8192, "u"),
                                      (3000, 9000, "u"), (9000, 3000, "r")])
def test_m4ri_rref_parity(m, n, kind):
    """The M4RI form (every block eliminated from all rows) against the
    oracle's RREF, which is unique; Q against its pivot columns."""
    say("m4ri rref", m, n, kind)
    import oracle
    if kind == "u":
        A = inputs.bernoulli(m, n, 41 + m)
    elif kind == "r":
        A = inputs.known_rank(m, n, max(1, min(m, n) // 2), 7, 8)
    else:
        A = inputs.bernoulli(m, n, 42 + m, p=0.01)
    t = to_dev(A)
    Q, rank = G.m4ri_rref(t, n)
    R, r2, Qo = oracle.rref(A, n)
    assert int(rank.item()) == r2
    assert np.array_equal(to_host(t), R)
    assert np.array_equal(Q.cpu().numpy()[:r2], np.asarray(Qo)[:r2])


def test_check_padding():
    A = inputs.bernoulli(50, 70, 3)
    t = to_dev(A)
    assert G.check_padding(t, 70) == 0
    A2 = A.copy()
    A2[7, 1] |= np.uint64(1) << np.uint64(20)
    assert G.check_padding(to_dev(A2), 70) == 6
    with pytest.raises(G.GF2Error):
        G.ple(to_dev(A2), 70, check_padding=True)


def test_check_padding_concurrent_streams():
    """Padding scans from two host threads on two streams at once: each
    reports its own matrix (the scan's device flag is not shared between
    concurrent calls)."""
    import threading
    say("check_padding from two threads")
    clean = to_dev(inputs.bernoulli(4000, 70, 8))
    dirty_h = inputs.bernoulli(4000, 70, 9)
    dirty_h[3999, 1] |= np.uint64(1) << np.uint64(63)
    dirty = to_dev(dirty_h)
    torch.cuda.synchronize()
    results = {"clean": [], "dirty": []}

    def worker(name, t):
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            for _ in range(50):
                results[name].append(G.check_padding(t, 70))

    ths = [threading.Thread(target=worker, args=("clean", clean)), threading.Thread(target=worker, args=("dirty", dirty))]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    assert results["clean"] == [0] * 50
    assert results["dirty"] == [6] * 50


@pytest.mark.parametrize("variant", list(range(0, 13)))
def test_schedule_invariance(variant):
    """Every update schedule (tile width, threads, unroll, grid size) gives
    the same bits."""
    say("schedule variant", variant)
    m, n = 1500, 1300
    A = inputs.bernoulli(m, n, 77)
    o = oracle_ple(A, n)
    for blocks in (0, 37, 4096):
        assert_same_ple(gpu_ple(A, n, m4_variant=variant, m4_blocks=blocks), o, "variant %d" % variant)
    C = inputs.bernoulli(700, 900, 1)
    Am = inputs.bernoulli(700, 150, 2)
    Bm = inputs.bernoulli(150, 900, 3)
    import oracle
    want = C.copy()
    oracle.addmul(want, Am, Bm, 150, 900)
    tC = to_dev(C)
    G.addmul(tC, to_dev(Am), to_dev(Bm), 150, 900, m4_variant=variant)
    assert np.array_equal(to_host(tC), want)


@pytest.mark.parametrize("m,n,kind", [(1500, 1300, "u"), (3000, 300, "r"), (8000, 300, "r"), (900, 900, "s"),
                                      (700, 2000, "u")])
def test_panel_modes(m, n, kind):
    """Every register window of the panel's pivot search gives the same bits
    (the smaller windows fall back to the all-rows search more often)."""
    say("panel modes", m, n, kind)
    if kind == "u":
        A = inputs.bernoulli(m, n, 5 + m)
    elif kind == "r":
        A = inputs.known_rank(m, n, min(m, n) // 5, 3, 4)
    else:
        A = inputs.bernoulli(m, n, 6 + m, p=0.01)
    o = oracle_ple(A, n)
    for regs in (0, 2, 4, 8):
        assert_same_ple(gpu_ple(A, n, panel_regs=regs), o, "regs=%d" % regs)


@pytest.mark.parametrize("m,n,kind", [(1500, 1300, "u"), (3000, 300, "r"), (8000, 300, "r"), (900, 900, "s"),
                                      (700, 2000, "u"), (300, 5000, "u"), (2100, 2100, "r")])
def test_lookahead_modes(m, n, kind):
    """The look-ahead (next stripe updated first, next panel on a second
    stream beside the update) and the fused pairs of passes (one trailing
    update for two passes) give the same bits as the serial pass loop,
    on full-rank, rank-deficient (all-rows panel search) and sparse inputs,
    and on wide matrices whose rank saturates before the last pass."""
    say("lookahead modes", m, n, kind)
    if kind == "u":
        A = inputs.bernoulli(m, n, 15 + m)
    elif kind == "r":
        A = inputs.known_rank(m, n, min(m, n) // 3, 5, 6)
    else:
        A = inputs.bernoulli(m, n, 16 + m, p=0.01)
    o = oracle_ple(A, n)
    for mode in (0, 1, 2, 3):
        for regs in (0, 8):
            assert_same_ple(gpu_ple(A, n, lookahead=mode, panel_regs=regs), o, "lookahead=%d regs=%d" % (mode, regs))


def test_lookahead_16384_seed2():
    """Default and forced look-ahead on the 16384^2 input equal the serial
    pass loop bit for bit."""
    say("lookahead 16384^2")
    A = inputs.bernoulli(16384, 16384, 2)
    serial = gpu_ple(A, 16384, lookahead=1)
    for mode in (0, 2, 3):
        assert_same_ple(gpu_ple(A, 16384, lookahead=mode), serial, "lookahead=%d" % mode)


@pytest.mark.parametrize("variant", list(range(0, 15)))
def test_pair_variants(variant):
    """Every schedule of the fused pair update (threads, rows in flight,
    reads per group, coefficient prefetch; the next panel inside the same
    launch, beside the sweep or in a block of its own) gives the oracle's
    bits, with pairs forced on every pass, on full-rank, rank-deficient and
    ragged (n not a multiple of the tile) inputs."""
    say("pair variant", variant)
    cases = [(1500, 1300, "u"), (2100, 2100, "r"), (700, 2000, "u"), (3000, 1111, "s")]
    for m, n, kind in cases:
        if kind == "u":
            A = inputs.bernoulli(m, n, 25 + m)
        elif kind == "r":
            A = inputs.known_rank(m, n, min(m, n) // 3, 7, 8)
        else:
            A = inputs.bernoulli(m, n, 26 + m, p=0.02)
        o = oracle_ple(A, n)
        for mode in (0, 3):
            assert_same_ple(gpu_ple(A, n, lookahead=mode, pair_variant=variant), o,
                            "%dx%d %s lookahead=%d pair_variant=%d" % (m, n, kind, mode, variant))


# --- Algorithm 3 (block-recursive PLE, update = 2 / 3) -----------------------

def _hstack_bits(left, nl, right, nr):
    """[left | right] as one packed matrix (nl + nr columns)."""
    return H.pack(np.concatenate([H.unpack(left, nl), H.unpack(right, nr)], axis=1))


def _alg3_case(kind, m, n):
    n1 = (n // 2 + 63) // 64 * 64  # the recursion's first split
    if kind == "u":
        return inputs.bernoulli(m, n, 500 + m + n)
    if kind == "s":
        return inputs.bernoulli(m, n, 501 + m + n, p=3.0 / n)
    if kind == "r":
        return inputs.known_rank(m, n, min(m, n) // 3, 23 + m, 29 + n)
    if kind == "deficient_left":
        # left block of rank n1 / 2, random right block: the right block's L
        # bits move left across the split
        left = inputs.known_rank(m, n1, n1 // 2, 31 + m, 37 + n)
        right = inputs.bernoulli(m, n - n1, 502 + m)
        return _hstack_bits(left, n1, right, n - n1)
    if kind == "zero_left":
        right = inputs.bernoulli(m, n - n1, 503 + m)
        return _hstack_bits(np.zeros((m, inputs.words(n1)), np.uint64), n1, right, n - n1)
    raise ValueError(kind)


ALG3_CASES = [(1000, 1000, "u"), (300, 2000, "u"), (2000, 300, "u"), (1500, 1300, "u"), (2000, 2000, "s"),
              (1200, 1100, "r"), (1000, 1000, "deficient_left"), (700, 1500, "deficient_left"),
              (1500, 700, "deficient_left"), (900, 1000, "zero_left"), (65, 130, "u"), (64, 65, "u"),
              (3000, 200, "r")]


@pytest.mark.parametrize("update", [2, 3])
@pytest.mark.parametrize("m,n,kind", ALG3_CASES)
def test_alg3_parity(m, n, kind, update):
    """One level of Algorithm 3 (column split in halves, TRSM, product on the
    fp4 matrix cores (2) or the tables (3), PLE of the lower right block, P, Q
    and L combined) gives the oracle's (rank, P, Q, L\\E) bit for bit."""
    say("alg3", update, m, n, kind)
    A = _alg3_case(kind, m, n)
    assert_same_ple(gpu_ple(A, n, update=update), oracle_ple(A, n), "alg3 u%d %dx%d %s" % (update, m, n, kind))


@pytest.mark.parametrize("update", [2, 3, 4])
@pytest.mark.parametrize("m,n,kind,levels", [(3000, 2500, "u", 2), (2500, 3000, "deficient_left", 3),
                                             (4096, 4096, "u", 3), (2000, 2000, "s", 4), (8192, 8192, "u", 1),
                                             (12000, 12000, "u", 1)])
def test_alg3_levels_parity(m, n, kind, levels, update):
    """Several levels of Algorithm 3 (each half recursed again) against the
    oracle, with fp4 (2) and int8 (4) matrix-core products and table products
    (3); 8192^2 takes the matrix-core path for its products of 512 inner bits
    and more; 12000^2 (left rank 6016) solves in two diagonal blocks, the
    first removed from the second by a product."""
    say("alg3 levels", update, m, n, kind, levels)
    A = _alg3_case(kind, m, n)
    assert_same_ple(gpu_ple(A, n, update=update, rec_levels=levels), oracle_ple(A, n),
                    "alg3 u%d %dx%d %s levels %d" % (update, m, n, kind, levels))


@pytest.mark.parametrize("psplit", [1, -1])
@pytest.mark.parametrize("m,n,kind,levels,split", [(3000, 2500, "u", 2, 0), (2500, 3000, "deficient_left", 3, 0),
                                                   (4096, 4096, "u", 3, 0), (2000, 2000, "s", 4, 0),
                                                   (1200, 1100, "r", 2, 0), (1500, 4000, "zero_left", 16, 768),
                                                   (12000, 11000, "u", 1, 5120), (12000, 12000, "u", 1, 0),
                                                   (9000, 7000, "deficient_left", 1, 0)])
def test_alg3_product_split_parity(m, n, kind, levels, split, psplit):
    """Algorithm 3 with fp4 products, each by one level of Strassen's split
    (psplit 1: ten block sums, seven half-size products into one or two
    blocks of the result) or by one product (-1), against the oracle."""
    say("alg3 product split", psplit, m, n, kind, levels, split)
    A = _alg3_case(kind, m, n)
    assert_same_ple(gpu_ple(A, n, update=2, rec_levels=levels, rec_split=split, product_split=psplit),
                    oracle_ple(A, n), "alg3 %dx%d %s levels %d split %d psplit %d" % (m, n, kind, levels, split, psplit))


@pytest.mark.parametrize("update", [2, 3, 4])
@pytest.mark.parametrize("m,n,kind,levels,split", [(3000, 2500, "u", 16, 512), (2500, 3000, "deficient_left", 16, 640),
                                                   (4096, 4096, "u", 3, 1024), (2000, 2000, "s", 16, 256),
                                                   (1500, 4000, "zero_left", 16, 768), (6000, 6000, "u", 16, 1536),
                                                   (1200, 1100, "r", 2, 320), (12000, 11000, "u", 1, 5120)])
def test_alg3_strips_parity(m, n, kind, levels, split, update):
    """Algorithm 3 with left strips of `split` columns (each a leaf), the
    splits going on in the right block while levels remain, against the
    oracle; products on the fp4 (2) or int8 (4) matrix cores or the tables
    (3)."""
    say("alg3 strips", update, m, n, kind, levels, split)
    A = _alg3_case(kind, m, n)
    assert_same_ple(gpu_ple(A, n, update=update, rec_levels=levels, rec_split=split), oracle_ple(A, n),
                    "alg3 u%d %dx%d %s levels %d split %d" % (update, m, n, kind, levels, split))
