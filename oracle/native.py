"""ctypes front of the C++ oracle (oracle/mochy_oracle.cpp).

Test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import patterns

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "mochy_oracle.cpp")
LIB = os.path.join(_HERE, "libmochy_oracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def build() -> str:
    """Compile the oracle with g++ (plain -O2, no fused multiply-add)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-o", LIB + ".tmp", SRC]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    L = ctypes.CDLL(LIB)
    L.orc_abi_version.restype = ctypes.c_int
    L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.orc_region_cards.argtypes = [_i64p, _i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _i64p]
    L.orc_classify.argtypes = [_i64p, ctypes.c_int, _i32p]
    L.orc_classify.restype = ctypes.c_int
    L.orc_bruteforce.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int, _i32p, _i64p, ctypes.c_int]
    L.orc_line_graph_degrees.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _i64p, ctypes.c_int]
    L.orc_line_graph_degrees.restype = ctypes.c_int64
    L.orc_mochy_e.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, ctypes.c_int64,
                              ctypes.c_int64, ctypes.c_int, _i32p, _i64p, ctypes.c_int]
    L.orc_mochy_e_centers.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _i64p, ctypes.c_int64,
                                      ctypes.c_int, _i32p, _i64p, ctypes.c_int]
    L.orc_candidates.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, ctypes.c_int64, ctypes.c_int64]
    L.orc_candidates.restype = ctypes.c_int64
    L.orc_line_graph_triangles.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, ctypes.c_int]
    L.orc_line_graph_triangles.restype = ctypes.c_int64
    L.orc_aplus_raw.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, ctypes.c_int64,
                                ctypes.c_int64, ctypes.c_uint64, _i64p, _i64p, ctypes.c_int, _i32p,
                                _i64p, ctypes.c_int]
    L.orc_mochy_a_raw.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_uint64, _i64p, ctypes.c_int, _i32p, _i64p,
                                  ctypes.c_int]
    L.orc_mochy_a_raw.restype = ctypes.c_int64
    L.orc_hyperedge_profiles.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_int, _i32p, _i64p, ctypes.c_int]
    L.orc_wedge_prefix.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _i64p, ctypes.c_int]
    L.orc_wedge_prefix.restype = ctypes.c_int64
    L.orc_aplus_raw.restype = ctypes.c_int64
    _lib = L
    return L


def _p(a, t):
    return a.ctypes.data_as(t)


def _threads(n):
    return int(n) if n else (os.cpu_count() or 1)


def _csr(h):
    ptr = np.ascontiguousarray(h.edge_ptr, dtype=np.int64)
    nodes = np.ascontiguousarray(h.edge_nodes, dtype=np.int32)
    return ptr, nodes


def _table():
    return np.ascontiguousarray(patterns.canonical_code_to_id3(), dtype=np.int32)


def philox4x32_10(ctr, key):
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, _u32p), _p(k, _u32p), _p(out, _u32p))
    return [int(x) for x in out]


def region_cards(h, i, j, k):
    ptr, nodes = _csr(h)
    out = np.zeros(7, dtype=np.int64)
    lib().orc_region_cards(_p(ptr, _i64p), _p(nodes, _i32p), i, j, k, _p(out, _i64p))
    return out.tolist()


def classify(card, theta=1):
    c = np.array(card, dtype=np.int64)
    t = _table()
    return int(lib().orc_classify(_p(c, _i64p), int(theta), _p(t, _i32p)))


def fold26(c3):
    """26 h-motif counts from 432 3h-slots (slot 0 = invalid patterns)."""
    parent = patterns.id3_to_id26()
    out = np.zeros(27, dtype=np.int64)
    np.add.at(out, parent[1:], c3[1:])
    return out[1:]


def bruteforce(h, theta=1, nthreads=None):
    """(counts26, counts431, invalid) over all C(|E|,3) triples."""
    ptr, nodes = _csr(h)
    out = np.zeros(432, dtype=np.int64)
    t = _table()
    lib().orc_bruteforce(h.num_edges, _p(ptr, _i64p), _p(nodes, _i32p), int(theta), _p(t, _i32p),
                         _p(out, _i64p), _threads(nthreads))
    return fold26(out), out[1:].copy(), int(out[0])


def mochy_e(h, c0=0, c1=None, theta=1, nthreads=None):
    """(counts26, counts431, invalid) of plain MoCHy-E restricted to centres [c0, c1)."""
    ptr, nodes = _csr(h)
    c1 = h.num_edges if c1 is None else c1
    out = np.zeros(432, dtype=np.int64)
    t = _table()
    lib().orc_mochy_e(h.num_edges, h.num_nodes, _p(ptr, _i64p), _p(nodes, _i32p), int(c0), int(c1),
                      int(theta), _p(t, _i32p), _p(out, _i64p), _threads(nthreads))
    return fold26(out), out[1:].copy(), int(out[0])


def mochy_e_centers(h, centers, theta=1, nthreads=None):
    """(counts26, counts431, invalid) of plain MoCHy-E over an explicit centre list."""
    ptr, nodes = _csr(h)
    c = np.ascontiguousarray(centers, dtype=np.int64)
    out = np.zeros(432, dtype=np.int64)
    t = _table()
    lib().orc_mochy_e_centers(h.num_edges, h.num_nodes, _p(ptr, _i64p), _p(nodes, _i32p), _p(c, _i64p),
                              int(c.size), int(theta), _p(t, _i32p), _p(out, _i64p), _threads(nthreads))
    return fold26(out), out[1:].copy(), int(out[0])


def line_graph_degrees(h, nthreads=None):
    ptr, nodes = _csr(h)
    deg = np.zeros(h.num_edges, dtype=np.int64)
    w = lib().orc_line_graph_degrees(h.num_edges, h.num_nodes, _p(ptr, _i64p), _p(nodes, _i32p),
                                     _p(deg, _i64p), _threads(nthreads))
    return deg, int(w)


def line_graph_triangles(h, nthreads=None):
    ptr, nodes = _csr(h)
    return int(lib().orc_line_graph_triangles(h.num_edges, h.num_nodes, _p(ptr, _i64p),
                                              _p(nodes, _i32p), _threads(nthreads)))


def wedge_prefix(h, nthreads=None):
    """(up_ptr int64[|E|+1], |wedges|): the hyperwedge order used for sampling."""
    ptr, nodes = _csr(h)
    up = np.zeros(h.num_edges + 1, dtype=np.int64)
    w = lib().orc_wedge_prefix(h.num_edges, h.num_nodes, _p(ptr, _i64p), _p(nodes, _i32p),
                               _p(up, _i64p), _threads(nthreads))
    return up, int(w)


def aplus_raw(h, r=None, seed=0, n0=0, indices=None, theta=1, nthreads=None, up_ptr=None):
    """(raw26, raw431, invalid, |wedges|) of MoCHy-A+ samples n in [n0, n0 + r).

    With ``indices`` the samples use those hyperwedge indices instead of Philox.
    ``up_ptr`` (from :func:`wedge_prefix`) skips recomputing the hyperwedge order.
    """
    ptr, nodes = _csr(h)
    out = np.zeros(432, dtype=np.int64)
    t = _table()
    if indices is not None:
        idx = np.ascontiguousarray(indices, dtype=np.int64)
        n0, n1, ip = 0, idx.size, _p(idx, _i64p)
    else:
        n1, ip = n0 + int(r), None
    up = None
    if up_ptr is not None:
        up = np.ascontiguousarray(up_ptr, dtype=np.int64)
        assert up.size == h.num_edges + 1
    w = lib().orc_aplus_raw(h.num_edges, h.num_nodes, _p(ptr, _i64p), _p(nodes, _i32p), int(n0),
                            int(n1), ctypes.c_uint64(seed & (2 ** 64 - 1)), ip,
                            _p(up, _i64p) if up is not None else None, int(theta),
                            _p(t, _i32p), _p(out, _i64p), _threads(nthreads))
    return fold26(out), out[1:].copy(), int(out[0]), int(w)


def mochy_a_raw(h, s=None, seed=0, n0=0, indices=None, theta=1, nthreads=None):
    """(raw26, raw431, invalid, |E|) of MoCHy-A samples n in [n0, n0 + s).

    With ``indices`` the samples are those hyperedges instead of Philox draws.
    """
    ptr, nodes = _csr(h)
    out = np.zeros(432, dtype=np.int64)
    t = _table()
    if indices is not None:
        idx = np.ascontiguousarray(indices, dtype=np.int64)
        n0, n1, ip = 0, idx.size, _p(idx, _i64p)
    else:
        n1, ip = n0 + int(s), None
    e = lib().orc_mochy_a_raw(h.num_edges, h.num_nodes, _p(ptr, _i64p), _p(nodes, _i32p), int(n0),
                              int(n1), ctypes.c_uint64(seed & (2 ** 64 - 1)), ip, int(theta),
                              _p(t, _i32p), _p(out, _i64p), _threads(nthreads))
    return fold26(out), out[1:].copy(), int(out[0]), int(e)


def hyperedge_profiles(h, c0=0, c1=None, theta=1, nthreads=None):
    """(hp26 [n, 26], hp431 [n, 431], invalid [n]) for hyperedges [c0, c1): the
    instances of each motif containing each hyperedge."""
    ptr, nodes = _csr(h)
    c1 = h.num_edges if c1 is None else c1
    if not 0 <= c0 <= c1 <= h.num_edges:
        raise ValueError(f"hyperedge range [{c0}, {c1}) outside [0, {h.num_edges}]")
    n = c1 - c0
    out = np.zeros((n, 432), dtype=np.int64)
    t = _table()
    lib().orc_hyperedge_profiles(h.num_edges, h.num_nodes, _p(ptr, _i64p), _p(nodes, _i32p), int(c0),
                                 int(c1), int(theta), _p(t, _i32p), _p(out, _i64p), _threads(nthreads))
    hp26 = np.array([fold26(row) for row in out]) if n else np.zeros((0, 26), dtype=np.int64)
    return hp26, out[:, 1:].copy(), out[:, 0].copy()
