"""The C-ABI library loads on the CPU and exports every symbol the public
header declares; argument checks that return before any GPU work."""
import ctypes
import os
import re

import pytest

from paper_1111_6549_amd import gf2ple as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "gf2ple.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gf2_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = G.load()
    names = header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(G.EXPORTS) == sorted(names)


def test_version_and_status_strings():
    assert G.version().startswith("gf2ple")
    lib = G.load()
    for code in range(8):
        assert lib.gf2_status_str(code)
    assert lib.gf2_status_str(0).decode() == "ok"


def test_workspace_sizes():
    lib = G.load()
    o = G.Opts()
    assert lib.gf2_ple_workspace_bytes(-1, 10, 1, ctypes.byref(o)) == 0
    assert lib.gf2_ple_workspace_bytes(10, 65, 1, ctypes.byref(o)) == 0  # ldw too small
    a = lib.gf2_ple_workspace_bytes(1024, 1024, 16, None)
    b = lib.gf2_ple_workspace_bytes(2048, 1024, 16, None)
    assert 0 < a < b
    assert lib.gf2_rref_full_workspace_bytes(100, 100, 2, None) >= lib.gf2_rref_workspace_bytes(100, 100, 2)


def test_argument_errors_before_launch():
    lib = G.load()
    nul = ctypes.c_void_p(0)
    # negative sizes, ldw too small, NULL rank: EINVAL without touching the GPU
    assert lib.gf2_ple(nul, -1, 5, 1, nul, nul, nul, nul, 0, None, nul) == 1
    assert lib.gf2_ple(nul, 5, 200, 2, nul, nul, nul, nul, 0, None, nul) == 1
    assert lib.gf2_ple(nul, 5, 5, 1, nul, nul, nul, nul, 0, None, nul) == 1
    bad = G.Opts()
    bad.update = 7
    assert lib.gf2_addmul(nul, 1, nul, 1, nul, 1, 1, 1, 1, nul, 0, ctypes.byref(bad), nul) == 1
    assert lib.gf2_make_table(nul, 1, 0, 10, nul, 1, nul) == 1
    assert lib.gf2_make_table(nul, 1, 9, 10, nul, 1, nul) == 1
    assert lib.gf2_echelon_from_ple(nul, 3, 3, 1, nul, nul) == 1
    # M4RI RREF: the same checks, then the workspace size (fake aligned
    # addresses are never dereferenced: every check precedes the first launch)
    fake = ctypes.c_void_p(1 << 20)
    assert lib.gf2_m4ri_rref(fake, -1, 5, 1, fake, fake, fake, 1 << 20, nul) == 1
    assert lib.gf2_m4ri_rref(fake, 5, 200, 2, fake, fake, fake, 1 << 20, nul) == 1
    assert lib.gf2_m4ri_rref(fake, 5, 5, 1, fake, nul, fake, 1 << 20, nul) == 1
    assert lib.gf2_m4ri_rref(fake, 5, 5, 1, nul, fake, fake, 1 << 20, nul) == 1
    assert lib.gf2_m4ri_rref(fake, 5, 5, 1, fake, fake, ctypes.c_void_p((1 << 20) + 8), 1 << 20, nul) == 1
    need = lib.gf2_m4ri_rref_workspace_bytes(5, 5, 1)
    assert need > 0 and lib.gf2_m4ri_rref_workspace_bytes(5, 65, 1) == 0
    assert lib.gf2_m4ri_rref(fake, 5, 5, 1, fake, fake, fake, need - 1, nul) == 2
    assert lib.gf2_rref_from_ple(fake, 5, 5, 1, fake, fake, fake, 0, nul) == 2


def test_batch_plan_rejects_bad_descriptors():
    """Descriptor checks of gf2_batch_plan_create return GF2_EINVAL before
    any device call."""
    lib = G.load()
    descs, aw, pl, ql = G.batch_layout([(10, 100), (20, 30)])
    end = descs[1]["a_off"] + descs[1]["m"] * descs[1]["ldw"]

    def create(ds, arena_words, p_len, q_len, config=0):
        arr = (G.Desc * len(ds))(*[G.Desc(d["a_off"], d["m"], d["n"], d["ldw"], d["p_off"], d["q_off"]) for d in ds])
        o = G.BatchOpts()
        o.config = config
        h = ctypes.c_void_p(0)
        return lib.gf2_batch_plan_create(arr, len(ds), arena_words, p_len, q_len, ctypes.byref(o), ctypes.byref(h))

    assert create(descs, end - 1, pl, ql) == 1  # second matrix overruns the arena
    assert create(descs, aw, pl - 1, ql) == 1   # P arena too short
    assert create(descs, aw, pl, ql - 1) == 1   # Q arena too short
    bad = [dict(d) for d in descs]
    bad[0]["ldw"] = 1  # 100 columns need 2 words
    assert create(bad, aw, pl, ql) == 1
    bad = [dict(d) for d in descs]
    bad[1]["m"] = -1
    assert create(bad, aw, pl, ql) == 1
    assert create(descs, aw, pl, ql, config=G.batch_num_configs() + 1) == 1
    assert G.batch_num_configs() >= 4
    assert G.batch_config_name(1) and G.batch_config_name(0) == ""


def test_serve_create_rejects_bad_options():
    """gf2_serve_create checks its options before touching the device."""
    lib = G.load()
    for field, value in (("streams", 17), ("streams", -1), ("small_max_dim", 5000), ("budget_bytes", -5),
                         ("max_batch", -2)):
        o = G.ServeOpts()
        setattr(o, field, value)
        h = ctypes.c_void_p(0)
        assert lib.gf2_serve_create(ctypes.byref(o), ctypes.byref(h)) == 1, field
        assert not h.value
    assert lib.gf2_serve_create(None, None) == 1


def test_pass_schedule():
    """The pass loop's schedule (host only): fused pairs while rows remain
    below the stripe, serial passes otherwise; every pair is a first pass
    followed by a second."""
    k = G.ple_schedule(65536, 65536)
    assert len(k) == 1024
    assert k[:1022] == [2, 3] * 511 and k[1022:] == [0, 0]
    assert set(G.ple_schedule(65536, 65536, lookahead=1)) == {0}
    k3 = G.ple_schedule(65536, 65536, lookahead=3)
    assert k3[:1022] == [2, 3] * 511 and k3[1022:] == [1, 0]
    k2 = G.ple_schedule(4096, 4096, lookahead=2)
    assert set(k2[:-1]) == {1} and k2[-1] == 0
    # wide: rows run out at pass 15 (15 * 64 < 1000 <= 16 * 64); the passes
    # past it are serial, where the loop can stop once the rank reaches m
    kw = G.ple_schedule(1000, 64 * 40)
    assert kw[:16] == [2, 3] * 8 and set(kw[16:]) == {0}
    for ks in (k, k3, kw, G.ple_schedule(300, 5000), G.ple_schedule(2100, 1300)):
        for i, v in enumerate(ks):
            if v == 2:
                assert ks[i + 1] == 3
            if v == 3:
                assert i > 0 and ks[i - 1] == 2
    assert G.ple_schedule(0, 0) == []
    with pytest.raises(G.GF2Error):
        G.ple_schedule(10, 10, lookahead=4)


def test_schedule_options_checked_before_launch():
    """Out-of-range schedule options return EINVAL before any device work
    (host buffers stand in for the device pointers; nothing is launched)."""
    import numpy as np
    lib = G.load()
    m = n = 128
    ldw = 2
    A = np.zeros((m, ldw), dtype=np.uint64)
    P = np.zeros(m, dtype=np.int64)
    Q = np.zeros(m, dtype=np.int64)
    rank = np.zeros(1, dtype=np.int64)
    ws = np.zeros(lib.gf2_ple_workspace_bytes(m, n, ldw, None) // 8 + 64, dtype=np.uint64)
    ws_ptr = (ws.ctypes.data + 255) // 256 * 256
    p = lambda a: ctypes.c_void_p(a.ctypes.data)
    for field, value in (("pair_variant", 99), ("pair_variant", -1), ("lookahead", 4), ("panel_regs", 3),
                         ("update", 5), ("update", -1), ("rec_levels", 17), ("rec_levels", -1),
                         ("rec_split", -64), ("rec_split", 100), ("pair_variant", 15), ("product_split", 2),
                         ("product_split", -2)):
        o = G.Opts()
        setattr(o, field, value)
        st = lib.gf2_ple(p(A), m, n, ldw, p(P), p(Q), p(rank), ctypes.c_void_p(ws_ptr), ws.nbytes - 256,
                         ctypes.byref(o), ctypes.c_void_p(0))
        assert st == 1, (field, value, st)


def test_noalloc_checks_before_any_device_call():
    """gf2_ple_noalloc: argument errors, check_padding and a workspace beyond
    its static array are refused before any device call."""
    lib = G.load()
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)  # aligned, never dereferenced on these paths
    limit = int(lib.gf2_ple_noalloc_max_workspace())
    assert limit == 16 << 20
    assert lib.gf2_ple_noalloc(nul, -1, 5, 1, nul, nul, nul, None, nul) == 1
    assert lib.gf2_ple_noalloc(fake, 5, 200, 2, fake, fake, fake, None, nul) == 1
    o = G.Opts()
    o.check_padding = 1
    assert lib.gf2_ple_noalloc(fake, 5, 5, 1, fake, fake, fake, ctypes.byref(o), nul) == 1
    m, n = 1_000_000, 64
    assert lib.gf2_ple_workspace_bytes(m, n, 1, None) > limit
    assert lib.gf2_ple_noalloc(fake, m, n, 1, fake, fake, fake, None, nul) == 2


def test_recursive_and_product_workspaces():
    """The Algorithm 3 schedules (update 2 and 3) need the pass loop's
    workspace plus their own (sub-ranks; for the matrix-core products the bit
    transpose of the largest product's right operand); the matrix-core
    gf2_addmul needs the bit transpose of B, the table product nothing.  Too
    small a workspace is refused before any device call."""
    lib = G.load()
    m = n = 4096
    ldw = 64
    base = lib.gf2_ple_workspace_bytes(m, n, ldw, None)
    o2, o3 = G.Opts(), G.Opts()
    o2.update, o3.update = 2, 3
    w2 = lib.gf2_ple_workspace_bytes(m, n, ldw, ctypes.byref(o2))
    w3 = lib.gf2_ple_workspace_bytes(m, n, ldw, ctypes.byref(o3))
    assert base < w3 < w2
    # the top product: 2048 inner bits x 2048 columns, bit-transposed
    assert w2 - w3 >= 2048 * 2048 // 8
    # left strips of 1024 columns: the first product is 1024 inner bits x
    # 3072 columns; a strip as wide as the matrix is no split at all
    o2.rec_split = 1024
    w2s = lib.gf2_ple_workspace_bytes(m, n, ldw, ctypes.byref(o2))
    assert w2s - w3 >= 1024 * 3072 // 8 and w2s < w2
    o2.rec_split = 4096
    assert lib.gf2_ple_workspace_bytes(m, n, ldw, ctypes.byref(o2)) == w3
    o2.rec_split = 0
    fake = ctypes.c_void_p(1 << 20)
    nul = ctypes.c_void_p(0)
    assert lib.gf2_ple(fake, m, n, ldw, fake, fake, fake, fake, w2 - 1, ctypes.byref(o2), nul) == 2
    assert lib.gf2_ple(fake, m, n, ldw, fake, fake, fake, fake, w3 - 1, ctypes.byref(o3), nul) == 2
    o1 = G.Opts()
    o1.update = 1
    assert lib.gf2_addmul_workspace_bytes(100, 300, 1000, ctypes.byref(o1)) == 0
    need = lib.gf2_addmul_workspace_bytes(100, 300, 1000, ctypes.byref(o2))
    assert need == 16 * 64 * 5 * 8
    assert lib.gf2_addmul(fake, 16, fake, 5, fake, 16, 100, 300, 1000, fake, need - 1, ctypes.byref(o2), nul) == 2
    assert lib.gf2_addmul(fake, 16, fake, 5, fake, 16, 100, 300, 1000, nul, 0, ctypes.byref(o2), nul) == 1
    # the no-allocation call takes no recursive schedule
    assert lib.gf2_ple_noalloc(fake, m, n, ldw, fake, fake, fake, ctypes.byref(o2), nul) == 1


def _header_struct_fields(name):
    """(type, field, array length) of a typedef struct in include/gf2ple.h, in order."""
    text = open(os.path.join(os.path.dirname(__file__), "..", "include", "gf2ple.h")).read()
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        for nm in names.split(","):
            m = re.match(r"(\w+)(\[(\d+)\])?$", nm.strip())
            assert m, decl
            out.append((ctype, m.group(1), int(m.group(3)) if m.group(3) else None))
    return out


@pytest.mark.parametrize("cname,pyname", [("gf2_ple_opts", "Opts"), ("gf2_desc", "Desc"),
                                          ("gf2_batch_opts", "BatchOpts"), ("gf2_batch_class", "BatchClass"),
                                          ("gf2_serve_opts", "ServeOpts")])
def test_binding_structs_match_header(cname, pyname):
    """The ctypes structures of the binding list the header's fields in the
    header's order with the same widths."""
    width = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double}
    want = _header_struct_fields(cname)
    got = getattr(G, pyname)._fields_
    assert [f for _, f, _ in want] == [f for f, _ in got]
    for (ctype, f, count), (_, pytype) in zip(want, got):
        exp = width[ctype] * count if count else width[ctype]
        assert ctypes.sizeof(pytype) == ctypes.sizeof(exp), f
