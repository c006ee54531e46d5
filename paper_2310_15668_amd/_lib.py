"""ctypes binding of libmochy.so: the C ABI of include/mochy.h, same names.

Argument marshalling only.  Every step of the computation runs in the HIP
library; if the library is not built this module raises, it never falls
back to anything else.
"""
from __future__ import annotations

import ctypes
import weakref
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmochy.so")

MOCHY_OK = 0
STATUS = {0: "MOCHY_OK", -1: "MOCHY_EINVAL", -2: "MOCHY_EDUP", -3: "MOCHY_ERANGE",
          -4: "MOCHY_ENOMEM", -5: "MOCHY_EDEVICE", -6: "MOCHY_EUNSUPPORTED"}
MOCHY_DEDUP = 1
MOCHY_CANONICALIZE = 2
MOCHY_LG_FREE = 4
MOCHY_H26 = 1
MOCHY_H431 = 2
MOCHY_WHICH_ALL = 3
MOCHY_OPT_GROUPS = 1
MOCHY_OPT_APLUS_ROWS = 2
MOCHY_OPT_MEMO_BUDGET = 3
MOCHY_OPT_MEMO_ALL = 4
MOCHY_OPT_MEMO_POOL = 5
MOCHY_OPT_GROUP_CAPACITY = 6
MOCHY_OPT_BATCH_LAUNCH = 7
MOCHY_OPT_PAIR_BLOCKS = 8
MOCHY_OPT_CACHE_BYTES = 9
MOCHY_OPT_TEST_FAULTS = 10
NUM_H, NUM_3H = 26, 431
MAX_EDGE = 32

# every symbol include/mochy.h declares
EXPORTED = ("mochy_ctx_create", "mochy_ctx_destroy", "mochy_last_error", "mochy_project",
            "mochy_graph_free", "mochy_count_exact", "mochy_count_exact_range",
            "mochy_count_sampled", "mochy_profile", "mochy_motif_pattern", "mochy_parent_motif",
            "mochy_graph_stats", "mochy_phase_ms", "mochy_memo_stats", "mochy_ctx_set_option",
            "mochy_count_sampled_edges", "mochy_hyperedge_profiles", "mochy_exact_stats",
            "mochy_calibrate_valu", "mochy_count_exact_range_noalloc")
NOALLOC_SCRATCH = 64 << 20
NUM_EXACT_STATS = 12
EXACT_STATS = ("rows_grouped", "groups", "groups_above", "group_pairs_full", "group_pairs_open",
               "rows_regrouped", "max_hash_parts", "light_pairs", "fix_scanned", "fix_centres",
               "fix_changed", "profile_batches")
NUM_PHASES = 12
PHASES = ("upload", "transpose", "lg_degree", "lg_rows", "records", "exact_sched", "exact_pairs",
          "exact_correct", "sample_draw", "sample_enum", "profile_cp", "exact_fix_kernel")


class MochyError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


class CSR(ctypes.Structure):
    _fields_ = [("num_nodes", ctypes.c_int64), ("num_edges", ctypes.c_int64),
                ("edge_ptr", ctypes.c_void_p), ("edge_nodes", ctypes.c_void_p),
                ("on_device", ctypes.c_int32)]


_lib = None


def lib():
    """Load libmochy.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2310_15668_amd.build")
    # One HIP runtime per process: torch ships its own libamdhip64 (soname
    # libamdhip64.so.7) and asks for it by an unversioned name, so if it is
    # loaded after us a second runtime comes up and cannot open the device.
    # Loading torch first makes our libamdhip64.so.7 dependency resolve to the
    # runtime torch already loaded.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    L.mochy_ctx_create.argtypes = [ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.mochy_ctx_create.restype = ctypes.c_int
    L.mochy_ctx_destroy.argtypes = [vp]
    L.mochy_ctx_destroy.restype = None
    L.mochy_last_error.argtypes = [vp]
    L.mochy_last_error.restype = ctypes.c_char_p
    L.mochy_project.argtypes = [vp, ctypes.POINTER(CSR), u32, ctypes.POINTER(vp), ctypes.POINTER(i64)]
    L.mochy_project.restype = ctypes.c_int
    L.mochy_graph_free.argtypes = [vp]
    L.mochy_graph_free.restype = None
    L.mochy_count_exact.argtypes = [vp, vp, u32, vp, vp]
    L.mochy_count_exact.restype = ctypes.c_int
    L.mochy_count_exact_range.argtypes = [vp, vp, i64, i64, u32, vp, vp]
    L.mochy_count_exact_range.restype = ctypes.c_int
    L.mochy_count_exact_range_noalloc.argtypes = [vp, vp, i64, i64, u32, vp, vp]
    L.mochy_count_exact_range_noalloc.restype = ctypes.c_int
    L.mochy_count_sampled.argtypes = [vp, vp, i64, u64, i64, u32, vp, vp, vp, vp]
    L.mochy_count_sampled.restype = ctypes.c_int
    L.mochy_profile.argtypes = [vp, i32, ctypes.POINTER(CSR), ctypes.c_double, u32, vp, vp, vp, vp, vp]
    L.mochy_profile.restype = ctypes.c_int
    L.mochy_motif_pattern.argtypes = [i32, u32, ctypes.POINTER(ctypes.c_uint8)]
    L.mochy_motif_pattern.restype = ctypes.c_int
    L.mochy_parent_motif.argtypes = [i32]
    L.mochy_parent_motif.restype = i32
    L.mochy_graph_stats.argtypes = [vp, vp, vp]
    L.mochy_graph_stats.restype = ctypes.c_int
    L.mochy_phase_ms.argtypes = [vp, vp]
    L.mochy_phase_ms.restype = ctypes.c_int
    L.mochy_memo_stats.argtypes = [vp, vp]
    L.mochy_memo_stats.restype = ctypes.c_int
    L.mochy_exact_stats.argtypes = [vp, vp]
    L.mochy_exact_stats.restype = ctypes.c_int
    L.mochy_calibrate_valu.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    L.mochy_calibrate_valu.restype = ctypes.c_int
    L.mochy_count_sampled_edges.argtypes = [vp, vp, i64, u64, i64, vp, vp, vp, vp]
    L.mochy_count_sampled_edges.restype = ctypes.c_int
    L.mochy_hyperedge_profiles.argtypes = [vp, vp, i64, i64, vp, vp]
    L.mochy_hyperedge_profiles.restype = ctypes.c_int
    L.mochy_ctx_set_option.argtypes = [vp, i32, i64]
    L.mochy_ctx_set_option.restype = ctypes.c_int
    _lib = L
    return L


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def motif_pattern(motif_id: int, kind: int):
    out = (ctypes.c_uint8 * 7)()
    st = lib().mochy_motif_pattern(int(motif_id), int(kind), out)
    if st != MOCHY_OK:
        raise MochyError(st, f"motif id {motif_id} kind {kind}")
    return tuple(out)


def parent_motif(id3: int) -> int:
    return int(lib().mochy_parent_motif(int(id3)))


class Context:
    """mochy_ctx on one device; ``stream`` is a hipStream_t handle (int) or None."""

    def __init__(self, device: int = 0, stream=None):
        h = ctypes.c_void_p()
        st = lib().mochy_ctx_create(int(device), ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
        if st != MOCHY_OK:
            raise MochyError(st, "mochy_ctx_create")
        self.handle = h
        self._graphs = weakref.WeakSet()  # graphs projected on this context

    def close(self):
        if self.handle:
            for g in list(self._graphs):  # a graph may not outlive its context
                g.close()
            lib().mochy_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_option(self, option: int, value: int):
        """mochy_ctx_set_option (e.g. MOCHY_OPT_GROUPS, 0 or 1)."""
        self.check(lib().mochy_ctx_set_option(self.handle, int(option), int(value)),
                   "mochy_ctx_set_option")

    def check(self, st, what):
        if st != MOCHY_OK:
            msg = lib().mochy_last_error(self.handle)
            raise MochyError(st, f"{what}: {msg.decode() if msg else ''}")


def make_csr(edge_ptr, edge_nodes, num_nodes, keep):
    """A CSR struct from numpy arrays (host) or torch tensors (device)."""
    if hasattr(edge_ptr, "data_ptr"):  # torch tensor
        if str(edge_ptr.dtype) != "torch.int64" or str(edge_nodes.dtype) != "torch.int32":
            raise TypeError("edge_ptr must be int64 and edge_nodes int32")
        if not (edge_ptr.is_contiguous() and edge_nodes.is_contiguous()):
            raise ValueError("CSR tensors must be contiguous")
        on_dev = 1 if edge_ptr.is_cuda else 0
        if on_dev != (1 if edge_nodes.is_cuda else 0):
            raise ValueError("edge_ptr and edge_nodes must live on the same side")
        keep.extend([edge_ptr, edge_nodes])
        return CSR(int(num_nodes), int(edge_ptr.numel() - 1), edge_ptr.data_ptr(),
                   edge_nodes.data_ptr() if edge_nodes.numel() else None, on_dev)
    p = np.ascontiguousarray(edge_ptr, dtype=np.int64)
    n = np.ascontiguousarray(edge_nodes, dtype=np.int32)
    keep.extend([p, n])
    return CSR(int(num_nodes), int(p.size - 1), p.ctypes.data, n.ctypes.data if n.size else None, 0)


class Graph:
    """mochy_graph: the device-resident projection of one hypergraph."""

    def __init__(self, ctx: Context, edge_ptr, edge_nodes, num_nodes, flags: int = 0):
        keep = []
        c = make_csr(edge_ptr, edge_nodes, num_nodes, keep)
        h = ctypes.c_void_p()
        w = ctypes.c_int64()
        ctx.check(lib().mochy_project(ctx.handle, ctypes.byref(c), int(flags), ctypes.byref(h), ctypes.byref(w)),
                  "mochy_project")
        self.ctx, self.handle, self.num_hyperwedges = ctx, h, int(w.value)
        self.num_edges = int(c.num_edges)
        ctx._graphs.add(self)

    def close(self):
        if self.handle:
            lib().mochy_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mochy_project(ctx, edge_ptr, edge_nodes, num_nodes, flags=0) -> Graph:
    return Graph(ctx, edge_ptr, edge_nodes, num_nodes, flags)


def _outs(which, n, dtype):
    """An output array for a selected kind, None for one not selected."""
    return np.zeros(n, dtype=dtype) if which else None


def mochy_count_exact(ctx: Context, g: Graph, which: int = MOCHY_WHICH_ALL):
    """(counts26, counts431); an entry is None when ``which`` does not select it."""
    c26 = _outs(which & MOCHY_H26, NUM_H, np.int64)
    c431 = _outs(which & MOCHY_H431, NUM_3H, np.int64)
    ctx.check(lib().mochy_count_exact(ctx.handle, g.handle, int(which), _ptr(c26), _ptr(c431)),
              "mochy_count_exact")
    return c26, c431


def mochy_count_exact_range(ctx: Context, g: Graph, c0: int, c1: int, which: int = MOCHY_WHICH_ALL):
    c26 = _outs(which & MOCHY_H26, NUM_H, np.int64)
    c431 = _outs(which & MOCHY_H431, NUM_3H, np.int64)
    ctx.check(lib().mochy_count_exact_range(ctx.handle, g.handle, int(c0), int(c1), int(which), _ptr(c26),
                                            _ptr(c431)), "mochy_count_exact_range")
    return c26, c431


def mochy_count_exact_range_noalloc(ctx: Context, g: Graph, c0: int, c1: int,
                                    which: int = MOCHY_WHICH_ALL):
    """mochy_count_exact_range without device allocation (static scratch array)."""
    c26 = _outs(which & MOCHY_H26, NUM_H, np.int64)
    c431 = _outs(which & MOCHY_H431, NUM_3H, np.int64)
    ctx.check(lib().mochy_count_exact_range_noalloc(ctx.handle, g.handle, int(c0), int(c1), int(which),
                                                    _ptr(c26), _ptr(c431)), "mochy_count_exact_range_noalloc")
    return c26, c431


def mochy_count_sampled(ctx: Context, g: Graph, r: int, seed: int, sample_begin: int = 0,
                        which: int = MOCHY_WHICH_ALL):
    raw26 = _outs(which & MOCHY_H26, NUM_H, np.int64)
    est26 = _outs(which & MOCHY_H26, NUM_H, np.float64)
    raw431 = _outs(which & MOCHY_H431, NUM_3H, np.int64)
    est431 = _outs(which & MOCHY_H431, NUM_3H, np.float64)
    ctx.check(lib().mochy_count_sampled(ctx.handle, g.handle, int(r), ctypes.c_uint64(seed & (2 ** 64 - 1)),
                                        int(sample_begin), int(which), _ptr(raw26), _ptr(est26),
                                        _ptr(raw431), _ptr(est431)), "mochy_count_sampled")
    return raw26, est26, raw431, est431


def mochy_count_sampled_edges(ctx: Context, g: Graph, s: int, seed: int, sample_begin: int = 0):
    """MoCHy-A: (raw26, est26, raw431, est431) of s hyperedge samples."""
    raw26 = np.zeros(NUM_H, dtype=np.int64)
    est26 = np.zeros(NUM_H, dtype=np.float64)
    raw431 = np.zeros(NUM_3H, dtype=np.int64)
    est431 = np.zeros(NUM_3H, dtype=np.float64)
    ctx.check(lib().mochy_count_sampled_edges(ctx.handle, g.handle, int(s), ctypes.c_uint64(seed & (2 ** 64 - 1)),
                                              int(sample_begin), _ptr(raw26), _ptr(est26), _ptr(raw431),
                                              _ptr(est431)), "mochy_count_sampled_edges")
    return raw26, est26, raw431, est431


def mochy_hyperedge_profiles(ctx: Context, g: Graph, e_begin: int = 0, e_end: int | None = None,
                             with_431: bool = True):
    """(hp26 [n, 26], hp431 [n, 431] or None) for hyperedges [e_begin, e_end)."""
    e_end = g.num_edges if e_end is None else int(e_end)
    n = max(0, e_end - int(e_begin))
    hp26 = np.zeros((n, NUM_H), dtype=np.int64)
    hp431 = np.zeros((n, NUM_3H), dtype=np.int64) if with_431 else None
    ctx.check(lib().mochy_hyperedge_profiles(ctx.handle, g.handle, int(e_begin), int(e_end), _ptr(hp26),
                                             _ptr(hp431) if hp431 is not None else None),
              "mochy_hyperedge_profiles")
    return hp26, hp431


def mochy_profile(ctx: Context, graphs, eps: float = 1.0, which: int = MOCHY_WHICH_ALL):
    """graphs: list of (edge_ptr, edge_nodes, num_nodes); graphs[0] is the hypergraph.
    Returns (counts [n, 457], sig26, cp26, sig431, cp431); the significance and
    CP of a kind ``which`` does not select are None and its count columns 0."""
    keep = []
    arr = (CSR * len(graphs))(*[make_csr(p, n, v, keep) for (p, n, v) in graphs])
    counts = np.zeros((len(graphs), NUM_H + NUM_3H), dtype=np.int64)
    sig26, cp26 = _outs(which & MOCHY_H26, NUM_H, np.float64), _outs(which & MOCHY_H26, NUM_H, np.float64)
    sig431 = _outs(which & MOCHY_H431, NUM_3H, np.float64)
    cp431 = _outs(which & MOCHY_H431, NUM_3H, np.float64)
    ctx.check(lib().mochy_profile(ctx.handle, len(graphs), arr, float(eps), int(which), _ptr(counts),
                                  _ptr(sig26), _ptr(cp26), _ptr(sig431), _ptr(cp431)), "mochy_profile")
    return counts, sig26, cp26, sig431, cp431


def mochy_graph_stats(ctx: Context, g: Graph) -> dict:
    out = np.zeros(8, dtype=np.int64)
    ctx.check(lib().mochy_graph_stats(ctx.handle, g.handle, _ptr(out)), "mochy_graph_stats")
    keys = ("num_edges", "num_nodes", "nnz", "hyperwedges", "max_line_degree", "candidates",
            "candidate_min_size_sum", "sum_deg_sq")
    return {k: int(v) for k, v in zip(keys, out)}


def mochy_exact_stats(ctx: Context) -> dict:
    """What the last exact counting call did (groups, group pairs, correction work)."""
    out = np.zeros(NUM_EXACT_STATS, dtype=np.int64)
    ctx.check(lib().mochy_exact_stats(ctx.handle, _ptr(out)), "mochy_exact_stats")
    return {k: int(v) for k, v in zip(EXACT_STATS, out)}


def mochy_calibrate_valu(ctx: Context, iters: int) -> tuple:
    """(milliseconds, lane operations) of the integer VALU calibration launch."""
    ms = ctypes.c_double()
    ops = ctypes.c_int64()
    ctx.check(lib().mochy_calibrate_valu(ctx.handle, int(iters), ctypes.byref(ms), ctypes.byref(ops)),
              "mochy_calibrate_valu")
    return float(ms.value), int(ops.value)


def mochy_memo_stats(ctx: Context) -> dict:
    """Key memos of the last on-the-fly MoCHy-A+ call."""
    out = np.zeros(5, dtype=np.int64)
    ctx.check(lib().mochy_memo_stats(ctx.handle, _ptr(out)), "mochy_memo_stats")
    return {"samples": int(out[0]), "memo_samples": int(out[1]), "memo_keys": int(out[2]),
            "arena_bytes": int(out[3]), "memo_walk": int(out[4])}


def mochy_phase_ms(ctx: Context) -> dict:
    out = np.zeros(NUM_PHASES, dtype=np.float64)
    ctx.check(lib().mochy_phase_ms(ctx.handle, _ptr(out)), "mochy_phase_ms")
    return {k: float(v) for k, v in zip(PHASES, out)}
