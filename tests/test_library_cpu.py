"""Host-side checks of the HIP library that need no GPU.

The library must load, export every function include/mochy.h declares, and
its own pattern tables (built independently of the oracle) must describe the
same 26 h-motifs and 431 3h-motifs as the oracle's.
"""
import ctypes
import os
import re

import pytest

from oracle import patterns as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mochy.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mochy_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("mochy_project", "mochy_count_exact", "mochy_count_sampled", "mochy_profile"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2310_15668_amd import _lib
    lib = _lib.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(_lib.EXPORTED)


def test_pattern_tables_agree_with_oracle():
    from paper_2310_15668_amd import _lib
    for i, p in enumerate(P.hmotif_table()):
        assert _lib.motif_pattern(i + 1, 2) == tuple(p)
    for i, (p, parent) in enumerate(P.tmotif_table()):
        assert _lib.motif_pattern(i + 1, 3) == tuple(p)
        assert _lib.parent_motif(i + 1) == parent


def test_pattern_lookup_rejects_bad_ids():
    from paper_2310_15668_amd import _lib
    for bad in ((0, 2), (27, 2), (432, 3), (5, 4)):
        with pytest.raises(_lib.MochyError):
            _lib.motif_pattern(*bad)
    assert _lib.parent_motif(0) == 0 and _lib.parent_motif(432) == 0


def test_no_context_without_gpu_is_an_error_not_a_crash():
    from paper_2310_15668_amd import _lib
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = _lib.lib().mochy_ctx_create(0, None, ctypes.byref(h))
    assert st != 0
