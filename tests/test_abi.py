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


def test_new_report_accessor_is_null_safe():
    lib = kc.load_library()
    n = ctypes.c_uint64(7)
    assert lib.kc_report_race_sites(None, ctypes.byref(n)) is None and n.value == 0


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof / offsetof of the ABI structs, compiled from include/kc.h with
    gcc, against the binding's ctypes structures."""
    import subprocess
    src = tmp_path / "layout.c"
    fields = {"kc_job": ["launches", "n_launches", "dev_mem", "n_words", "tag", "streams", "deps", "n_deps",
                         "allocs", "n_allocs", "items", "n_items"],
              "kc_item": ["kind", "stream", "ref", "flags", "dst", "src", "words", "value", "pad"],
              "kc_launch_desc": ["prog", "grid", "block", "shmem_bytes", "params", "n_params"],
              "kc_dep": ["before", "after"], "kc_region": ["base", "words"], "kc_race_site": ["w_pc", "o_pc"]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{os.path.join(ROOT, "include", "kc.h")}"',
             "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0; }")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-o", str(exe), str(src)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    py = {"kc_job": kc.JobDesc, "kc_launch_desc": kc.LaunchDesc, "kc_dep": kc.Dep, "kc_region": kc.Region,
          "kc_item": kc.ItemDesc}
    for st, cls in py.items():
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f in fields[st]:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)
    assert int(got["kc_race_site"]) == kc.SITE_DTYPE.itemsize
