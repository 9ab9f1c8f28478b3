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
    assert L.qs_abi_version() == 3
    assert L.qs_strerror(0) == b"ok"
    assert L.qs_strerror(1) == b"invalid argument"
    assert L.qs_strerror(99) == b"unknown status"


# binding struct -> C struct name in the header
STRUCTS = {"Laser": "qs_laser", "Beam": "qs_beam", "Numerics": "qs_numerics", "Bins": "qs_bins",
           "Outputs": "qs_outputs", "NodeGrid": "qs_node_grid", "Tuning": "qs_tuning",
           "GradOutputs": "qs_grad_outputs", "PhotonBins": "qs_photon_bins",
           "PhotonOutputs": "qs_photon_outputs"}


def test_struct_layouts_match_header(tmp_path):
    """Every binding struct has the size, field names and field offsets that
    a C compiler gives the header's struct (gcc on the host)."""
    import shutil
    import subprocess
    from paper_2308_09348_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "qscatter.h"',
             "int main(void) {"]
    for py, c in STRUCTS.items():
        lines.append(f'  printf("{py} size %zu\\n", sizeof({c}));')
        for name, _ in getattr(_lib, py)._fields_:
            lines.append(f'  printf("{py} {name} %zu\\n", offsetof({c}, {name}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        py, name, v = line.split()
        got[(py, name)] = int(v)
    for py in STRUCTS:
        cls = getattr(_lib, py)
        assert ctypes.sizeof(cls) == got[(py, "size")], py
        for name, _ in cls._fields_:
            assert getattr(cls, name).offset == got[(py, name)], (py, name)


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


def test_library_was_built_from_these_sources():
    from paper_2308_09348_amd import _lib
    _lib_path()
    bid = _lib.check_build()
    assert len(bid) == 64 and int(bid, 16) >= 0
