"""The C-ABI library loads and exports every entry point include/lfdpr.h
declares (no compute calls: these run without a GPU)."""
import ctypes
import os

import pytest

from paper_2601_19901_amd import lfdpr


def test_header_declares_the_boundary():
    syms = lfdpr.declared_symbols()
    for name in ["lfdpr_create", "lfdpr_destroy", "lfdpr_scene_upload", "lfdpr_set_views", "lfdpr_set_lens",
                 "lfdpr_render_frame", "lfdpr_reconstruct", "lfdpr_angular_filter", "lfdpr_get_stats"]:
        assert name in syms


def test_library_exports_every_declared_symbol():
    if not os.path.exists(lfdpr.LIB_PATH):
        pytest.skip("liblfdpr.so not built")
    L = ctypes.CDLL(lfdpr.LIB_PATH)
    missing = [s for s in lfdpr.declared_symbols() if not hasattr(L, s)]
    assert not missing, missing
    lib = lfdpr.lib()
    assert lib.lfdpr_abi_version() == 6
    assert lib.lfdpr_strerror(-3) == b"point capacity exceeded"
    assert lib.lfdpr_strerror(12345) == b"unknown status"
    assert lib.lfdpr_destroy(None) == 0
    assert lib.lfdpr_last_error(None) == b"null context"


def test_binding_signatures_match_header():
    """Every binding's argument count equals the header prototype's."""
    arity = lfdpr.declared_arity()
    sigs = lfdpr.signatures()
    assert set(arity) == set(lfdpr.declared_symbols())
    assert set(sigs) == set(arity), set(sigs) ^ set(arity)
    bad = {n: (len(sigs[n][0]), arity[n]) for n in arity if len(sigs[n][0]) != arity[n]}
    assert not bad, bad
