"""Build libhjr.so (the gfx950 HIP library) in-tree with hipcc.

    python -m paper_1903_07715_amd.build        # or: from paper_1903_07715_amd.build import build

Every HIP source is compiled for gfx950 only, with packed FP32 instructions disabled
(-target-feature -packed-fp32-ops) and floating-point contraction only within one expression
(-ffp-contract=on: an a * b + c written in one expression becomes a fused multiply-add, nothing
across statements does), so the rounding of the arithmetic the kernel variants share is fixed by
the source and every variant produces the same bits; linked into paper_1903_07715_amd/libhjr.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhjr.so")
SOURCES = ["hjr_kernels.hip", "hjr_control.hip", "hjr_api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libhjr)")


def flags() -> list:
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-function",
            "-ffp-contract=on", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def source_hash() -> str:
    """Hash of everything the library is built from: every file under csrc/, the public header
    and the compiler flags.  Compiled into the library (hjr_build_id) so a stale build can be
    told from a current one."""
    import hashlib

    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        path = os.path.join(CSRC, name)
        if os.path.isfile(path) and name.endswith((".hip", ".hpp", ".h")):
            h.update(name.encode())
            with open(path, "rb") as f:
                h.update(f.read())
    with open(os.path.join(ROOT, "include", "hjr.h"), "rb") as f:
        h.update(f.read())
    h.update(" ".join(flags()).replace(ROOT, "").encode())
    return h.hexdigest()[:16]


def _compile(src: str, obj: str, extra=()) -> None:
    cmd = [hipcc()] + flags() + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the GPU target feature; that warning is expected
    err = "\n".join(ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every HIP source and link libhjr.so (or `out`).  Always recompiles."""
    objdir = os.path.join(HERE, "_build", os.path.basename(out))
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    extra = [f"-D{d}" for d in defines] + [f'-DHJR_SOURCE_HASH="{source_hash()}"']
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], extra), zip(SOURCES, objs)))
    tmp = out + f".tmp{os.getpid()}"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link of libhjr.so failed:\n" + r.stderr)
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
