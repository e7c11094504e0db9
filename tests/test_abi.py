"""The C-ABI library loads and exports every function include/kfx.h declares
(no compute calls: no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2002_06295_amd", "libkfx.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kfx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kfx_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["kfx_create", "kfx_destroy", "kfx_last_error", "kfx_load_layers", "kfx_bin_hits",
              "kfx_seed_states", "kfx_step_compat", "kfx_build_tracks", "kfx_fit_tracks",
              "kfx_fit_tracks_backward", "kfx_find_duplicates", "kfx_mask_hits", "kfx_cluster_strips"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkfx.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkfx.so not built")
def test_binding_matches_header():
    from paper_2002_06295_amd import kfx
    assert sorted(kfx.EXPORTED) == sorted(n for n in declared_functions() if n in kfx.EXPORTED)
    assert set(kfx.EXPORTED) == set(declared_functions())


def test_null_context_calls_fail_cleanly():
    if not os.path.exists(LIB):
        pytest.skip("libkfx.so not built")
    lib = ctypes.CDLL(LIB)
    lib.kfx_last_error.restype = ctypes.c_char_p
    lib.kfx_last_error.argtypes = [ctypes.c_void_p]
    assert lib.kfx_last_error(None) == b"null context"
    lib.kfx_load_layers.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int]
    assert lib.kfx_load_layers(None, None, 0, 0.0, 0, 0) == -1
    lib.kfx_destroy.argtypes = [ctypes.c_void_p]
    lib.kfx_destroy(None)
    lib.kfx_create.argtypes = [ctypes.c_int, ctypes.c_void_p]
    assert lib.kfx_create(0, None) == -1
    # the entry points after building reject a NULL context before any
    # device call
    lib.kfx_find_duplicates.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int32] * 5 + [ctypes.c_void_p] * 2
    assert lib.kfx_find_duplicates(None, None, 0, 1, 0, 1, 2, None, None) == -1
    lib.kfx_mask_hits.argtypes = ([ctypes.c_void_p] * 2 + [ctypes.c_int32] * 2 + [ctypes.c_void_p, ctypes.c_int32,
                                  ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                  ctypes.c_void_p])
    assert lib.kfx_mask_hits(None, None, 0, 1, None, 8, 3.0, None, None, 0, None) == -1
    lib.kfx_cluster_strips.argtypes = [ctypes.c_void_p] * 6
    assert lib.kfx_cluster_strips(None, None, None, None, None, None) == -1
