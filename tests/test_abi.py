"""The C-ABI library loads and exports every entry point include/kc.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

from paper_1211_6193_amd import kc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "kc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kc_[a-z_]+)\s*\(", text)))


def test_header_declares_binding_exports():
    assert _declared() == sorted(kc.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(kc.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_loads_signatures():
    lib = kc.load_library()
    assert lib.kc_report_records.restype is ctypes.c_uint64
    # report accessors are null-safe
    assert lib.kc_report_records(None) == 0
    n = ctypes.c_uint64(7)
    assert lib.kc_report_races(None, ctypes.byref(n)) is None and n.value == 0
