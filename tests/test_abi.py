"""The C-ABI library loads and exports every symbol include/mc.h declares.

These run without a GPU: no call here reaches a kernel.
"""
import ctypes
import os
import re

import pytest

import paper_2106_08150_amd as mc
from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "mc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["mc_db_create", "mc_db_add_targets", "mc_db_set_taxonomy", "mc_classify"]:
        assert required in names
    assert set(names) == set(mc.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(mc.LIB_PATH):
        pytest.skip("libmc.so not built")
    lib = ctypes.CDLL(mc.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_argument_errors_without_device():
    if not os.path.exists(mc.LIB_PATH):
        pytest.skip("libmc.so not built")
    L = mc.lib()
    assert L.mc_last_error() is not None
    # invalid parameters are rejected before any device work
    for args in [(0, 128, 16, 254), (17, 128, 16, 254), (16, 15, 1, 1), (16, 128, 0, 254),
                 (16, 128, 65, 254), (16, 128, 16, 0), (16, 128, 16, 65536), (16, 300, 16, 1),
                 (4, 6, 4, 1)]:
        assert not L.mc_db_create(*args)
        assert b"invalid" in L.mc_last_error()
    assert L.mc_db_destroy(None) == mc.MC_OK
    assert L.mc_release_cached_memory() == mc.MC_OK   # nothing kept: no device call
    opts = mc.QueryOpts(4, 4, 0, 0, 0)
    assert L.mc_classify_ex(None, None, None, 1, ctypes.byref(opts), None, None, None) == \
        mc.MC_ERR_INVALID_ARG
    assert L.mc_db_set_taxonomy(None, None, 0) == mc.MC_ERR_INVALID_ARG
    assert L.mc_db_add_targets(None, None, None, None, 0) == mc.MC_ERR_INVALID_ARG


def test_binding_raises_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setattr(mc, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(mc, "_lib", None)
    with pytest.raises(ImportError):
        mc.lib()
