"""Build the HIP library libadg.so for gfx950 (in-tree, no JIT cache).

    python -m paper_2404_03399_amd.build

build_asan.py builds a variant with the host code under AddressSanitizer.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libadg.so")
# (source, extra defines): the fused step is compiled once per integrator so
# that its many instantiations build in parallel
# kernel arguments preloaded into SGPRs (gfx950): the fused step reaches its
# first HBM load one scalar load earlier
PRELOAD = ["-mllvm", "-amdgpu-kernarg-preload-count=16"]
UNITS = [("adg_fused.hip", ["-DADG_RK=0"] + PRELOAD), ("adg_fused.hip", ["-DADG_RK=1"] + PRELOAD),
         ("adg_fused.hip", ["-DADG_RK=2"] + PRELOAD), ("adg_fused.hip", ["-DADG_RK=3"] + PRELOAD),
         ("adg_fused.hip", ["-DADG_RK=4"] + PRELOAD),
         ("adg_adjoint.hip", []), ("adg_kernels.hip", []), ("adg_api.hip", [])]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags() -> list:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # packed FP32 instructions stay off (only FP64 math here; belt and braces)
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
        f"-I{INCLUDE}", f"-I{CSRC}",
    ]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stdout}\n{res.stderr}")
    if verbose and res.stderr.strip():
        print(res.stderr, file=sys.stderr)


def source_hash() -> str:
    """Hash of the library's sources (every file under csrc/ and include/),
    compiled into the library as adg_build_id(); the binding compares the two
    and refuses a library built from other sources."""
    import hashlib
    h = hashlib.sha256()
    for d in (CSRC, INCLUDE):
        for name in sorted(os.listdir(d)):
            path = os.path.join(d, name)
            if os.path.isfile(path):
                h.update(name.encode() + b"\0")
                with open(path, "rb") as fh:
                    h.update(fh.read())
    return h.hexdigest()[:24]


def build(verbose: bool = False, jobs: int = 0, extra=(), libdir: str = LIBDIR) -> str:
    """Compile every unit to an object (in parallel), then link libdir/libadg.so
    (extra: more compiler options for every unit)."""
    from concurrent.futures import ThreadPoolExecutor
    lib = os.path.join(libdir, "libadg.so")
    objdir = os.path.join(libdir, "obj")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    extra = list(extra)
    ident = [f'-DADG_SOURCE_HASH="{source_hash()}"']
    objs, cmds = [], []
    for src, defs in UNITS:
        tag = "".join(d.split("=")[-1] for d in defs if d.startswith("-D"))
        if src == "adg_api.hip":
            defs = defs + ident
        obj = os.path.join(objdir, os.path.splitext(src)[0] + (f"_{tag}" if tag else "") + ".o")
        objs.append(obj)
        cmds.append([cc] + flags() + extra + defs + ["-c", os.path.join(CSRC, src), "-o", obj])
    jobs = jobs or max(1, min(len(cmds), (os.cpu_count() or 2) - 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = lib + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
