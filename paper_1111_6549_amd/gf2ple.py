"""Thin ctypes binding of libgf2ple.so (include/gf2ple.h).

Only argument marshalling happens here: device memory and the current stream
come from PyTorch, every step of the computation runs in the library's HIP
kernels.  There is no CPU fallback: if the library is not built, or no GPU is
present, the calls raise.

Packed matrices are torch tensors of shape (m, ldw) with dtype int64 or
uint64 on a CUDA (HIP) device; column j of row i is bit (j & 63) of
element [i, j >> 6].
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgf2ple.so")
_lib = None

STATUS = {0: "GF2_OK", 1: "GF2_EINVAL", 2: "GF2_EWORKSPACE", 3: "GF2_ENOMEM", 4: "GF2_EBUDGET",
          5: "GF2_EHIP", 6: "GF2_EPADDING", 7: "GF2_EBUSY"}

# every symbol include/gf2ple.h declares
EXPORTS = [
    "gf2_version", "gf2_status_str", "gf2_ple_workspace_bytes", "gf2_ple", "gf2_ple_schedule", "gf2_product_plan",
    "gf2_echelon_from_ple",
    "gf2_rref_workspace_bytes", "gf2_rref_from_ple", "gf2_rref_full_workspace_bytes", "gf2_rref",
    "gf2_m4ri_rref_workspace_bytes", "gf2_m4ri_rref",
    "gf2_addmul_workspace_bytes", "gf2_addmul", "gf2_make_table", "gf2_check_padding", "gf2_profile_start", "gf2_profile_stop",
    "gf2_batch_plan_create", "gf2_batch_workspace_bytes", "gf2_ple_batched", "gf2_batch_plan_info",
    "gf2_batch_plan_destroy", "gf2_batch_num_configs", "gf2_batch_config_name",
    "gf2_serve_create", "gf2_serve_submit", "gf2_serve_poll", "gf2_serve_wait", "gf2_serve_fetch",
    "gf2_serve_release", "gf2_serve_stats_get", "gf2_serve_destroy",
    "gf2_ple_noalloc_max_workspace", "gf2_ple_noalloc",
]


class GF2Error(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s failed: %s (%s)" % (what, STATUS.get(status, status), _status_text(status)))


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("check_padding", ctypes.c_int32), ("update", ctypes.c_int32), ("rec_levels", ctypes.c_int32),
                ("m4_variant", ctypes.c_int32), ("m4_blocks", ctypes.c_int32), ("panel_regs", ctypes.c_int32),
                ("lookahead", ctypes.c_int32), ("pair_variant", ctypes.c_int32), ("rec_split", ctypes.c_int32),
                ("product_split", ctypes.c_int32)]


class PlanBlock(ctypes.Structure):
    _fields_ = [("buf", ctypes.c_int64), ("row0", ctypes.c_int64), ("word0", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("rows", ctypes.c_int64), ("bits", ctypes.c_int64)]


class PlanStep(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int64), ("b", PlanBlock * 4)]


class Desc(ctypes.Structure):
    _fields_ = [("a_off", ctypes.c_int64), ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("ldw", ctypes.c_int64),
                ("p_off", ctypes.c_int64), ("q_off", ctypes.c_int64)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("autotune", ctypes.c_int32), ("config", ctypes.c_int32), ("no_graph", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


class BatchClass(ctypes.Structure):
    _fields_ = [("max_dim", ctypes.c_int64), ("count", ctypes.c_int64), ("config", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("tuned_ms", ctypes.c_double)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("streams", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("small_max_dim", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class ServeInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("ldw", ctypes.c_int64), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "failed", "queued", "running",
                                              "launches_batched", "launches_single", "bytes_in_use", "bytes_peak",
                                              "budget_bytes")] + [("now", ctypes.c_double)]


def load():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libgf2ple.so is not built (run __graft_entry__.build() or "
                           "python -m paper_1111_6549_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    i64, i32, p, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
    st = ctypes.c_int
    sig = {
        "gf2_version": (ctypes.c_char_p, []),
        "gf2_status_str": (ctypes.c_char_p, [st]),
        "gf2_ple_workspace_bytes": (sz, [i64, i64, i64, p]),
        "gf2_ple": (st, [p, i64, i64, i64, p, p, p, p, sz, p, p]),
        "gf2_echelon_from_ple": (st, [p, i64, i64, i64, p, p]),
        "gf2_ple_schedule": (i64, [i64, i64, p, p, i64]),
        "gf2_product_plan": (i64, [i64, i64, i64, ctypes.c_int32, i64, i64, i64, p, i64, p]),
        "gf2_rref_workspace_bytes": (sz, [i64, i64, i64]),
        "gf2_rref_from_ple": (st, [p, i64, i64, i64, p, p, p, sz, p]),
        "gf2_rref_full_workspace_bytes": (sz, [i64, i64, i64, p]),
        "gf2_rref": (st, [p, i64, i64, i64, p, p, p, p, sz, p, p]),
        "gf2_m4ri_rref_workspace_bytes": (sz, [i64, i64, i64]),
        "gf2_m4ri_rref": (st, [p, i64, i64, i64, p, p, p, sz, p]),
        "gf2_addmul_workspace_bytes": (sz, [i64, i64, i64, p]),
        "gf2_addmul": (st, [p, i64, p, i64, p, i64, i64, i64, i64, p, sz, p, p]),
        "gf2_make_table": (st, [p, i64, i32, i64, p, i64, p]),
        "gf2_check_padding": (st, [p, i64, i64, i64, p]),
        "gf2_profile_start": (st, []),
        "gf2_profile_stop": (st, [p, i32, p]),
        "gf2_batch_plan_create": (st, [p, i64, i64, i64, i64, p, p]),
        "gf2_batch_workspace_bytes": (sz, [p]),
        "gf2_ple_batched": (st, [p, p, p, p, p, p, sz, p]),
        "gf2_batch_plan_info": (st, [p, p, i32, p]),
        "gf2_batch_plan_destroy": (st, [p]),
        "gf2_batch_num_configs": (i32, []),
        "gf2_batch_config_name": (ctypes.c_char_p, [i32]),
        "gf2_serve_create": (st, [p, p]),
        "gf2_serve_submit": (st, [p, p, i32, i64, i64, i64, p]),
        "gf2_serve_poll": (st, [p, i64, p]),
        "gf2_serve_wait": (st, [p, i64, p]),
        "gf2_serve_fetch": (st, [p, i64, p, i64, p, p, p, i32]),
        "gf2_serve_release": (st, [p, i64]),
        "gf2_serve_stats_get": (st, [p, p]),
        "gf2_serve_destroy": (st, [p]),
        "gf2_ple_noalloc_max_workspace": (sz, []),
        "gf2_ple_noalloc": (st, [p, i64, i64, i64, p, p, p, p, p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _status_text(status):
    try:
        return load().gf2_status_str(status).decode()
    except Exception:  # library missing while formatting an error
        return "?"


def _check(status, what):
    if status != 0:
        raise GF2Error(status, what)


def version():
    return load().gf2_version().decode()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _packed(t, name, whole_rows=False):
    """Check a packed operand.  whole_rows: the call works on whole rows of
    ldw words in place (the PLE family), so the tensor's rows must be its
    memory rows (no view of a column block)."""
    if not isinstance(t, torch.Tensor) or t.dim() != 2 or t.dtype not in (torch.int64, torch.uint64):
        raise TypeError("%s must be a 2-D int64/uint64 tensor of packed rows" % name)
    if not t.is_cuda:
        raise ValueError("%s must be on the GPU" % name)
    if t.numel() and t.stride(1) != 1:
        raise ValueError("%s rows must be contiguous" % name)
    if t.numel() and t.shape[0] > 1 and t.stride(0) < t.shape[1]:
        raise ValueError("%s rows overlap" % name)
    if whole_rows and t.numel() and t.shape[0] > 1 and t.stride(0) != t.shape[1]:
        raise ValueError("%s must be contiguous (the call works on whole rows of ldw words)" % name)
    return t


def _ld(t):
    """Row stride in words: the leading dimension the C ABI takes."""
    return t.stride(0) if t.shape[0] > 1 else t.shape[1]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def _opts(update=0, check_padding=False, rec_levels=0, m4_variant=0, m4_blocks=0, panel_regs=0, lookahead=0,
          pair_variant=0, rec_split=0, product_split=0):
    o = Opts()
    o.rec_split = int(rec_split)
    o.product_split = int(product_split)
    o.lookahead = int(lookahead)
    o.pair_variant = int(pair_variant)
    o.check_padding = 1 if check_padding else 0
    o.update = int(update)
    o.rec_levels = int(rec_levels)
    o.m4_variant = int(m4_variant)
    o.m4_blocks = int(m4_blocks)
    o.panel_regs = int(panel_regs)
    return o


def workspace_bytes(m, n, ldw, update=0, rec_levels=0, rec_split=0, product_split=0):
    o = _opts(update, rec_levels=rec_levels, rec_split=rec_split, product_split=product_split)
    return int(load().gf2_ple_workspace_bytes(m, n, ldw, ctypes.byref(o)))


def alloc_workspace(nbytes, device=None):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device or "cuda")


def ple(A, n, ws=None, update=0, check_padding=False, m4_variant=0, m4_blocks=0, panel_regs=0, lookahead=0,
        pair_variant=0, rec_levels=0, rec_split=0, product_split=0):
    """In-place PLE of the packed (m, ldw) tensor A with n columns.

    Returns (P, Q, rank) as device tensors (int64 [m], int64 [min(m, n)],
    int64 [1]).  A holds the clean L\\E afterwards."""
    A = _packed(A, "A", whole_rows=True)
    m, ldw = A.shape
    lib = load()
    o = _opts(update, check_padding, rec_levels=rec_levels, m4_variant=m4_variant, m4_blocks=m4_blocks,
              panel_regs=panel_regs, lookahead=lookahead, pair_variant=pair_variant, rec_split=rec_split,
              product_split=product_split)
    need = int(lib.gf2_ple_workspace_bytes(m, n, ldw, ctypes.byref(o)))
    if need == 0 and (m or n):
        raise GF2Error(1, "gf2_ple_workspace_bytes")
    if ws is None:
        ws = alloc_workspace(need, A.device)
    P = torch.empty(m, dtype=torch.int64, device=A.device)
    Q = torch.empty(min(m, n), dtype=torch.int64, device=A.device)
    rank = torch.empty(1, dtype=torch.int64, device=A.device)
    _check(lib.gf2_ple(_ptr(A), m, n, ldw, _ptr(P), _ptr(Q), _ptr(rank), _ptr(ws), ws.numel(),
                       ctypes.byref(o), _stream()), "gf2_ple")
    return P, Q, rank


def ple_noalloc(A, n, lookahead=0, panel_regs=0):
    """In-place PLE of the packed (m, ldw) tensor A through gf2_ple_noalloc
    (the library's static device workspace instead of a caller buffer).
    Returns (P, Q, rank) as device tensors."""
    A = _packed(A, "A", whole_rows=True)
    m, ldw = A.shape
    o = _opts(panel_regs=panel_regs, lookahead=lookahead)
    P = torch.empty(m, dtype=torch.int64, device=A.device)
    Q = torch.empty(min(m, n), dtype=torch.int64, device=A.device)
    rank = torch.empty(1, dtype=torch.int64, device=A.device)
    _check(load().gf2_ple_noalloc(_ptr(A), m, n, ldw, _ptr(P), _ptr(Q), _ptr(rank), ctypes.byref(o), _stream()),
           "gf2_ple_noalloc")
    return P, Q, rank


def product_plan(m, k, n, split=0, lda=0, ldbt=0, ldc=0):
    """The steps by which Algorithm 3 adds an m x k x n product on the fp4
    matrix cores (gf2_product_plan): (steps, workspace words), each step
    (kind, [(buf, row0, word0, ld, rows, bits)] * 4)."""
    steps = (PlanStep * 17)()
    ws = ctypes.c_int64(0)
    ns = int(load().gf2_product_plan(m, k, n, split, lda, ldbt, ldc, steps, 17, ctypes.byref(ws)))
    if ns < 0:
        raise GF2Error(1, "gf2_product_plan")
    out = []
    for i in range(ns):
        st = steps[i]
        out.append((int(st.kind), [(b.buf, b.row0, b.word0, b.ld, b.rows, b.bits) for b in st.b]))
    return out, int(ws.value)


def ple_schedule(m, n, lookahead=0):
    """Per-pass kinds of gf2_ple's schedule (0 serial, 1 look-ahead, 2/3 the
    first/second pass of a fused pair)."""
    o = _opts(lookahead=lookahead)
    np_ = int(load().gf2_ple_schedule(m, n, ctypes.byref(o), None, 0))
    if np_ < 0:
        raise GF2Error(1, "gf2_ple_schedule")
    arr = (ctypes.c_int32 * max(np_, 1))()
    load().gf2_ple_schedule(m, n, ctypes.byref(o), arr, np_)
    return [int(arr[i]) for i in range(np_)]


def echelon_from_ple(A, n, rank):
    A = _packed(A, "A", whole_rows=True)
    m, ldw = A.shape
    _check(load().gf2_echelon_from_ple(_ptr(A), m, n, ldw, _ptr(rank), _stream()), "gf2_echelon_from_ple")


def rref_from_ple(A, n, Q, rank, ws=None):
    A = _packed(A, "A", whole_rows=True)
    m, ldw = A.shape
    lib = load()
    need = int(lib.gf2_rref_workspace_bytes(m, n, ldw))
    if ws is None:
        ws = alloc_workspace(need, A.device)
    _check(lib.gf2_rref_from_ple(_ptr(A), m, n, ldw, _ptr(Q), _ptr(rank), _ptr(ws), ws.numel(), _stream()),
           "gf2_rref_from_ple")


def rref(A, n, ws=None, update=0):
    """In-place RREF (via PLE).  Returns (P, Q, rank)."""
    A = _packed(A, "A", whole_rows=True)
    m, ldw = A.shape
    lib = load()
    o = _opts(update)
    need = int(lib.gf2_rref_full_workspace_bytes(m, n, ldw, ctypes.byref(o)))
    if ws is None:
        ws = alloc_workspace(need, A.device)
    P = torch.empty(m, dtype=torch.int64, device=A.device)
    Q = torch.empty(min(m, n), dtype=torch.int64, device=A.device)
    rank = torch.empty(1, dtype=torch.int64, device=A.device)
    _check(lib.gf2_rref(_ptr(A), m, n, ldw, _ptr(P), _ptr(Q), _ptr(rank), _ptr(ws), ws.numel(), ctypes.byref(o),
                        _stream()), "gf2_rref")
    return P, Q, rank


def m4ri_rref(A, n, ws=None):
    """In-place RREF in the M4RI form.  Returns (Q, rank)."""
    A = _packed(A, "A", whole_rows=True)
    m, ldw = A.shape
    lib = load()
    need = int(lib.gf2_m4ri_rref_workspace_bytes(m, n, ldw))
    if ws is None:
        ws = alloc_workspace(need, A.device)
    Q = torch.empty(max(min(m, n), 1), dtype=torch.int64, device=A.device)
    rank = torch.empty(1, dtype=torch.int64, device=A.device)
    _check(lib.gf2_m4ri_rref(_ptr(A), m, n, ldw, _ptr(Q), _ptr(rank), _ptr(ws), ws.numel(), _stream()),
           "gf2_m4ri_rref")
    return Q, rank


def addmul(C, A, B, k, n, update=0, m4_variant=0, m4_blocks=0):
    """C ^= A * B over GF(2); A is m x k, B is k x n, all packed on the GPU.
    Each may be a view of a column block of a wider matrix (rows contiguous,
    its row stride passed as the leading dimension)."""
    C, A, B = _packed(C, "C"), _packed(A, "A"), _packed(B, "B")
    m = C.shape[0]
    o = _opts(update, m4_variant=m4_variant, m4_blocks=m4_blocks)
    lib = load()
    need = int(lib.gf2_addmul_workspace_bytes(m, k, n, ctypes.byref(o)))
    ws = alloc_workspace(need, C.device) if need else None
    _check(lib.gf2_addmul(_ptr(C), _ld(C), _ptr(A), _ld(A), _ptr(B), _ld(B), m, k, n, _ptr(ws),
                          ws.numel() if ws is not None else 0, ctypes.byref(o), _stream()), "gf2_addmul")


def make_table(rows, k, n, T=None):
    """All 2^k sums of the k packed rows; index bit k-1-t selects row t."""
    rows = _packed(rows, "rows")
    if T is None:
        T = torch.empty((1 << k, rows.shape[1]), dtype=rows.dtype, device=rows.device)
    _check(load().gf2_make_table(_ptr(rows), _ld(rows), k, n, _ptr(T), _ld(T), _stream()), "gf2_make_table")
    return T


def check_padding(A, n):
    A = _packed(A, "A", whole_rows=True)
    m, ldw = A.shape
    return int(load().gf2_check_padding(_ptr(A), m, n, ldw, _stream()))


def profile_start():
    _check(load().gf2_profile_start(), "gf2_profile_start")


def profile_stop():
    """Per-kernel event timings since profile_start(): {name: dict}."""
    out = (KernelTime * 16)()
    cnt = ctypes.c_int32(0)
    _check(load().gf2_profile_stop(out, 16, ctypes.byref(cnt)), "gf2_profile_stop")
    res = {}
    for i in range(min(cnt.value, 16)):
        k = out[i]
        res[k.name.decode()] = {"launches": int(k.launches), "total_ms": k.total_ms, "min_ms": k.min_ms,
                                "max_ms": k.max_ms}
    return res


# ---------------------------------------------------------------------------
# Batched PLE
# ---------------------------------------------------------------------------
ARENA_ALIGN_WORDS = 32  # 256-byte aligned matrices in the arena


def batch_layout(shapes):
    """Arena layout for a list of (m, n) or (m, n, ldw): returns
    (descs as a list of dicts, arena_words, p_len, q_len)."""
    descs = []
    a = p = q = 0
    for sh in shapes:
        m, n = int(sh[0]), int(sh[1])
        ldw = int(sh[2]) if len(sh) > 2 else (n + 63) // 64
        descs.append({"a_off": a, "m": m, "n": n, "ldw": ldw, "p_off": p, "q_off": q})
        a += -(-(m * ldw) // ARENA_ALIGN_WORDS) * ARENA_ALIGN_WORDS
        p += m
        q += min(m, n)
    return descs, a, p, q


def batch_num_configs():
    return int(load().gf2_batch_num_configs())


def batch_config_name(i):
    return load().gf2_batch_config_name(int(i)).decode()


class BatchPlan:
    """A batched-PLE plan over fixed shapes (gf2_batch_plan_*)."""

    def __init__(self, descs, arena_words, p_len, q_len, autotune=False, config=0, graph=True):
        lib = load()
        arr = (Desc * max(len(descs), 1))()
        for i, d in enumerate(descs):
            arr[i] = Desc(d["a_off"], d["m"], d["n"], d["ldw"], d["p_off"], d["q_off"])
        o = BatchOpts()
        o.autotune = 1 if autotune else 0
        o.config = int(config)
        o.no_graph = 0 if graph else 1
        self._h = ctypes.c_void_p(0)
        self.count = len(descs)
        _check(lib.gf2_batch_plan_create(arr, len(descs), int(arena_words), int(p_len), int(q_len), ctypes.byref(o),
                                         ctypes.byref(self._h)), "gf2_batch_plan_create")

    def workspace_bytes(self):
        return int(load().gf2_batch_workspace_bytes(self._h))

    def run(self, arena, P, Q, ranks, ws):
        """Decompose every matrix of `arena` (flat int64/uint64 device tensor) in place."""
        for t, nm in ((arena, "arena"), (P, "P"), (Q, "Q"), (ranks, "ranks"), (ws, "ws")):
            if not isinstance(t, torch.Tensor) or not t.is_cuda:
                raise ValueError("%s must be a device tensor" % nm)
        _check(load().gf2_ple_batched(self._h, _ptr(arena), _ptr(P), _ptr(Q), _ptr(ranks), _ptr(ws), ws.numel(),
                                      _stream()), "gf2_ple_batched")

    def info(self):
        out = (BatchClass * 16)()
        cnt = ctypes.c_int32(0)
        _check(load().gf2_batch_plan_info(self._h, out, 16, ctypes.byref(cnt)), "gf2_batch_plan_info")
        return [{"max_dim": int(c.max_dim), "count": int(c.count), "config": int(c.config),
                 "config_name": batch_config_name(c.config), "grid": int(c.grid), "tuned_ms": c.tuned_ms}
                for c in out[:min(cnt.value, 16)]]

    def close(self):
        if self._h and self._h.value:
            load().gf2_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Serving session
# ---------------------------------------------------------------------------
REQ_STATES = {0: "queued", 1: "running", 2: "done", 3: "failed"}


def _info_dict(i):
    return {"state": REQ_STATES.get(i.state, i.state), "status": int(i.status), "m": int(i.m), "n": int(i.n),
            "ldw": int(i.ldw), "t_submit": i.t_submit, "t_admit": i.t_admit, "t_done": i.t_done}


class ServeSession:
    """gf2_serve_*: submit packed matrices, poll/wait, fetch results."""

    def __init__(self, budget_bytes=0, streams=0, max_batch=0, small_max_dim=0):
        o = ServeOpts()
        o.budget_bytes = int(budget_bytes)
        o.streams = int(streams)
        o.max_batch = int(max_batch)
        o.small_max_dim = int(small_max_dim)
        self._h = ctypes.c_void_p(0)
        self._keep = {}  # device inputs, referenced until their request is done or failed
        _check(load().gf2_serve_create(ctypes.byref(o), ctypes.byref(self._h)), "gf2_serve_create")

    def submit(self, A, n):
        """A: packed (m, ldw) numpy uint64 array (host) or device tensor."""
        t = ctypes.c_int64(0)
        if isinstance(A, torch.Tensor):
            A = _packed(A, "A")
            m, ldw = A.shape
            if A.numel() and A.stride(0) != ldw:
                raise ValueError("A must be contiguous")
            # the session's copy of A is not ordered after this stream
            torch.cuda.current_stream(A.device).synchronize()
            _check(load().gf2_serve_submit(self._h, _ptr(A), 1, m, n, ldw, ctypes.byref(t)), "gf2_serve_submit")
            self._keep[t.value] = A
        else:
            import numpy as np
            A = np.ascontiguousarray(A, dtype=np.uint64)
            m, ldw = A.shape
            ptr = A.ctypes.data_as(ctypes.c_void_p) if A.size else ctypes.c_void_p(0)
            _check(load().gf2_serve_submit(self._h, ptr, 0, m, n, ldw, ctypes.byref(t)), "gf2_serve_submit")
        return t.value

    def poll(self, ticket):
        i = ServeInfo()
        _check(load().gf2_serve_poll(self._h, ticket, ctypes.byref(i)), "gf2_serve_poll")
        if i.state in (2, 3):  # done or failed: the session has read A
            self._keep.pop(ticket, None)
        return _info_dict(i)

    def wait(self, ticket):
        i = ServeInfo()
        _check(load().gf2_serve_wait(self._h, ticket, ctypes.byref(i)), "gf2_serve_wait")
        self._keep.pop(ticket, None)
        return _info_dict(i)

    def fetch(self, ticket, m, n, ldw=None):
        """Copy a finished request to host numpy arrays and release it:
        returns (rank, P, Q, L\\E)."""
        import numpy as np
        ldw = ldw or (n + 63) // 64
        LE = np.zeros((m, ldw), dtype=np.uint64)
        P = np.zeros(m, dtype=np.int64)
        Q = np.zeros(min(m, n), dtype=np.int64)
        r = np.zeros(1, dtype=np.int64)
        cp = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a.size else ctypes.c_void_p(0)
        _check(load().gf2_serve_fetch(self._h, ticket, cp(LE), ldw, cp(P), cp(Q), cp(r), 0), "gf2_serve_fetch")
        self._keep.pop(ticket, None)
        return int(r[0]), P, Q, LE

    def fetch_device(self, ticket, LE, P, Q, rank):
        """Copy a finished request into device tensors and release it."""
        _check(load().gf2_serve_fetch(self._h, ticket, _ptr(LE), LE.shape[1] if LE is not None else 0, _ptr(P),
                                      _ptr(Q), _ptr(rank), 1), "gf2_serve_fetch")
        self._keep.pop(ticket, None)

    def release(self, ticket):
        _check(load().gf2_serve_release(self._h, ticket), "gf2_serve_release")
        self._keep.pop(ticket, None)

    def stats(self):
        st = ServeStats()
        _check(load().gf2_serve_stats_get(self._h, ctypes.byref(st)), "gf2_serve_stats_get")
        return {k: getattr(st, k) for k, _ in ServeStats._fields_}

    def close(self):
        if self._h and self._h.value:
            load().gf2_serve_destroy(self._h)
            self._h = ctypes.c_void_p(0)
        self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
