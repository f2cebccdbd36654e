"""The C-ABI library loads and exports every entry point include/ltsim.h declares (CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ltsim.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lts_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lts_context_create", "lts_set_response", "lts_plan", "lts_simulate", "lts_simulate_batch",
                 "lts_stage_quench_drift", "lts_stage_electronics", "lts_status_str", "lts_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2212_09807_amd import ltsim
    if not os.path.exists(ltsim.LIB_PATH):
        pytest.skip("libltsim.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(ltsim.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(ltsim.EXPORTS) <= set(declared_functions())
    lib.lts_status_str.restype = ctypes.c_char_p
    assert lib.lts_status_str(2) == b"output capacity too small"
    lib.lts_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.lts_version()


def test_binding_struct_layouts_match_header_field_order():
    from paper_2212_09807_amd import ltsim, workloads as W
    for dc, st in ((W.Physics, ltsim.lts_physics), (W.Readout, ltsim.lts_readout),
                   (W.Electronics, ltsim.lts_electronics), (W.Light, ltsim.lts_light_params)):
        assert [f for f, _ in st._fields_] == [f.name for f in __import__("dataclasses").fields(dc)]


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2212_09807_amd import ltsim
    monkeypatch.setattr(ltsim, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(ltsim, "_LIB", None)
    with pytest.raises(ltsim.LtsimError):
        ltsim.lib()
