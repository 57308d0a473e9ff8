"""The C ABI library loads and exports every function include/tpc.h declares
(no device calls: these run without a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tpc.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpc_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_hot_path_calls():
    names = declared()
    for n in ("tpc_build_grid", "tpc_find_neighbours", "tpc_construct_tracklets",
              "tpc_select_tracks", "tpc_refit", "tpc_refit_adjoint", "tpc_track_batch"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1905_05515_amd import _lib
    if not os.path.exists(_lib.SO):
        from paper_1905_05515_amd import build
        build.build()
    L = _lib.lib()
    for n in declared():
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.SO], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (tpc_[a-z_0-9]+)", out))
    assert set(declared()) <= exported
    assert L.tpc_status_string(2) == b"output capacity exceeded"


def test_binding_has_no_fallback():
    """The binding refuses to run when the library is absent."""
    from paper_1905_05515_amd import _lib
    saved, saved_so = _lib._lib, _lib.SO
    try:
        _lib._lib = None
        _lib.SO = os.path.join(ROOT, "does-not-exist.so")
        with pytest.raises(ImportError):
            _lib.lib()
    finally:
        _lib._lib, _lib.SO = saved, saved_so


def test_binding_modules_import_and_declare_every_export():
    """The Python binding imports on a machine without a GPU, and every
    symbol the header declares has a ctypes signature."""
    import re as _re
    from paper_1905_05515_amd import _lib, api, autograd  # noqa: F401
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "tpc.h")).read()
    declared = set(_re.findall(r"^(?:int|const char\*)\s+(tpc_\w+)\(", hdr, _re.M))
    assert declared and declared <= set(_lib.EXPORTS), declared - set(_lib.EXPORTS)
