"""Build libkc.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkc.so")
SOURCES = ["kc_interp.hip", "kc_sort.hip", "kc_check.hip", "kc_jit.hip", "kc_runtime.hip"]
ARCH = os.environ.get("KC_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
]


EMBED = [("kc_jit_internal_h", "kc_internal.h"), ("kc_jit_device_h", "kc_device.h")]


def write_embedded(bdir: str) -> None:
    """The device headers as string constants, for run-time compilation of the
    program-specialised kernels (kc_jit.hip includes the generated file)."""
    out = []
    for name, header in EMBED:
        text = open(os.path.join(CSRC, header)).read()
        if ")KCJIT\"" in text:
            raise RuntimeError(f"{header} contains the raw-string delimiter")
        out.append(f'static const char *const {name} = R"KCJIT({text})KCJIT";\n')
    path = os.path.join(bdir, "kc_jit_src.inc")
    new = "".join(out)
    if not os.path.exists(path) or open(path).read() != new:
        with open(path, "w") as f:
            f.write(new)


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source to an object, then link the shared library."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    write_embedded(bdir)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = ["hipcc", *FLAGS, "-I", bdir, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _reap(procs)
    _reap(procs)
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-lhiprtc", "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def _reap(procs):
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip())
        if p.returncode != 0:
            failed.append((src, text))
        elif text:
            print(f"[{src}]\n{text}", file=sys.stderr)
    procs.clear()
    if failed:
        for src, text in failed:
            print(f"[{src}] FAILED\n{text}", file=sys.stderr)
        raise RuntimeError("hipcc failed: " + ", ".join(s for s, _ in failed))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
