"""Build the hsolve shared library (HIP for gfx950) in-tree.

    python -m paper_1611_03189_amd.build          # -> paper_1611_03189_amd/libhsolve.so

Every HIP source under csrc/ is compiled by hipcc for gfx950 with packed-FP32 instructions
disabled, then linked into one shared library exporting the C ABI of include/hsolve.h.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libhsolve.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn and os.environ.get("HSOLVE_BUILD_VERBOSE"):
        print(warn, file=sys.stderr)
    return obj


def hip_runtime() -> list[str]:
    """Link arguments for the HIP runtime.

    Inside a PyTorch-ROCm installation the library links the runtime that PyTorch ships, so
    that one process holds a single HIP runtime (shared default stream, valid torch stream
    handles, ordered with torch's work). Without PyTorch (or with HSOLVE_HIP_RUNTIME=rocm)
    it links /opt/rocm's runtime.
    """
    if os.environ.get("HSOLVE_HIP_RUNTIME", "torch") == "torch":
        try:
            import importlib.util
            spec = importlib.util.find_spec("torch")
            if spec and spec.origin:
                tlib = os.path.join(os.path.dirname(spec.origin), "lib")
                rt = os.path.join(tlib, "libamdhip64.so")
                if os.path.exists(rt):
                    return [rt, f"-Wl,-rpath,{tlib}"]
        except Exception:
            pass
    return ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    cmd = [clang, "-shared", "-fPIC", "-o", tmp, *objs, *hip_runtime()]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
