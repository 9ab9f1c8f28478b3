"""The C-ABI library loads and exports every function include/qscatter.h
declares (no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qscatter.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(qs_[a-z_0-9]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def _lib_path():
    from paper_2308_09348_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libqscatter.so not built")
    return _lib.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ("qs_create", "qs_destroy", "qs_forward", "qs_radiation_eval", "qs_sync_status",
              "qs_strerror", "qs_last_error", "qs_abi_version"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    for n in _declared_functions():
        assert hasattr(lib, n), n


def test_binding_covers_the_exports():
    from paper_2308_09348_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared_functions()


def test_abi_version_and_strerror():
    from paper_2308_09348_amd import _lib
    L = _lib.lib()
    assert L.qs_abi_version() == 1
    assert L.qs_strerror(0) == b"ok"
    assert L.qs_strerror(1) == b"invalid argument"
    assert L.qs_strerror(99) == b"unknown status"


def test_struct_layouts_match_header():
    from paper_2308_09348_amd import _lib
    # sizes follow from the header's field lists (8-byte aligned doubles)
    assert ctypes.sizeof(_lib.Laser) == 8 * 4 + 4 * 2 + 8 * 3 + 4 * 2
    assert ctypes.sizeof(_lib.Beam) == 8 * 5 + 4 * 2
    assert ctypes.sizeof(_lib.Numerics) == 8 + 4 * 2 + 8 * 2 + 4 * 4 + 8 * 3 + 4 * 2
    assert ctypes.sizeof(_lib.Bins) == 4 * 4 + 8 * 4
    assert ctypes.sizeof(_lib.Outputs) == 8 * 8
    assert ctypes.sizeof(_lib.NodeGrid) == 4 * 2 + 8 * 2
    assert ctypes.sizeof(_lib.Tuning) == 4 * 4 + 8 * 2
    assert ctypes.sizeof(_lib.GradOutputs) == 8 * 6


def test_null_context_is_rejected_without_a_device():
    from paper_2308_09348_amd import _lib
    L = _lib.lib()
    assert L.qs_forward(None, None, None, None, None, None, None) == _lib.QS_EINVAL
    assert L.qs_forward_factorised(None, None, None, None, None, None, None,
                                   None) == _lib.QS_EINVAL
    assert L.qs_create(None, 0) == _lib.QS_EINVAL
    assert L.qs_tune(None, 1, None, None, None, None, None, None, None, None) == _lib.QS_EINVAL
    assert L.qs_set_graphs(None, 1) == _lib.QS_EINVAL
    L.qs_destroy(None)
