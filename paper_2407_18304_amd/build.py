"""Build the HIP libraries in-tree with hipcc for gfx950.

    libmgrhd.so        the source-update kernels and the C ABI of include/mgrhd.h
    libmgrhd_synth.so  the seeded synthetic-input generator (test/bench inputs)
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
ARCH = os.environ.get("MGRHD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep loop-invariant FP64 constants (polynomial and exp coefficients) out of
    # registers across the persistent loop: rematerialising them is cheaper
    "-mllvm", "-disable-machine-licm",
    "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"),
]

LIBS = {
    "libmgrhd.so": ["source_update.hip", "source_update_tdep.hip", "source_update_full.hip",
                    "source_update_tdep_full.hip", "batch.hip", "mlp.hip", "imex.hip",
                    "transport1d.hip"],
    "libmgrhd_synth.so": ["synth.hip"],
}


def hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


def _headers_mtime() -> float:
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".inc"))]
    heads.append(os.path.join(ROOT, "include", "mgrhd.h"))
    return max(os.path.getmtime(h) for h in heads)


def build_lib(name: str, verbose: bool = True, force: bool = True) -> str:
    """Compile the library's sources to objects in parallel, then link.
    force=False recompiles only objects older than their source or any
    header of the library (a development shortcut)."""
    srcs = [os.path.join(CSRC, s) for s in LIBS[name]]
    out = os.path.join(PKG, name)
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    hdr = _headers_mtime()
    for src in srcs:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        if (not force and os.path.exists(obj) and
                os.path.getmtime(obj) > max(os.path.getmtime(src), hdr)):
            procs.append((obj, None))
            continue
        cmd = [hipcc(), *HIPCC_FLAGS, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((obj, subprocess.Popen(cmd)))
    failed = [obj for obj, pr in procs if pr is not None and pr.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, f"hipcc ({', '.join(failed)})")
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
           *[obj for obj, _ in procs]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_all(verbose: bool = True, force: bool = True):
    return [build_lib(n, verbose, force) for n in LIBS if all(
        os.path.exists(os.path.join(CSRC, s)) for s in LIBS[n])]


if __name__ == "__main__":
    args = sys.argv[1:]
    force = "--changed" not in args
    names = [a for a in args if not a.startswith("--")] or list(LIBS)
    for n in names:
        build_lib(n, force=force)
