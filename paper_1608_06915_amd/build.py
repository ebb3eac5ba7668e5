"""Compile the HIP library (gfx950) in-tree: paper_1608_06915_amd/libelbm.so."""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libelbm.so")
SOURCES = [os.path.join(CSRC, f) for f in ("kernels.hip", "adjoint.hip", "indicator.hip", "remesh.hip", "elbm.cpp")]
ARCH = os.environ.get("ELBM_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            # packed FP32 instructions are disabled for all device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(os.path.dirname(HERE), "include")]


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link the shared library."""
    with tempfile.TemporaryDirectory(prefix="elbm_build") as tmpdir:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            objs.append(obj)
            procs.append((src, subprocess.Popen([hipcc()] + flags() + ["-c", src, "-o", obj],
                                                stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        errors = []
        for src, p in procs:
            out, err = p.communicate()
            if p.returncode != 0:
                errors.append("hipcc failed on %s:\n%s%s" % (src, out, err))
            elif verbose and err:
                print(err)
        if errors:
            raise RuntimeError("\n".join(errors))
        tmp = LIB + ".tmp%d" % os.getpid()
        res = subprocess.run([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp],
                             capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=False))
