"""Build the HIP libraries in-tree with hipcc for gfx950.

``libmwax.so`` (the correlator: runtime + kernels) lands next to this file and
``libsynth.so`` (the seeded voltage generator) in ``synth/``.  Objects are
compiled in parallel and linked into shared libraries; every call rebuilds.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmwax.so")
SYNTH_SRC = os.path.join(ROOT, "synth", "synth.hip")
SYNTH_LIB = os.path.join(ROOT, "synth", "libsynth.so")

SOURCES = ["runtime.cpp", "batch.cpp", "stream.cpp", "fengine.hip", "fft6400.hip", "xengine.hip", "pack.hip", "weights.hip", "average.hip", "beamform.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC,
        # keep the compiler from emitting packed FP32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
    ]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build(jobs: int | None = None, verbose: bool = False) -> list[str]:
    cc = hipcc()
    jobs = jobs or min(8, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="mwax_build_") as tmp:
        objs = []
        cmds = []
        for src in SOURCES:
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            lang = ["-x", "hip"] if src.endswith(".cpp") else []
            cmds.append([cc, *_flags(), *lang, "-c", os.path.join(CSRC, src), "-o", obj])
            objs.append(obj)
        synth_obj = os.path.join(tmp, "synth.o")
        cmds.append([cc, *_flags(), "-c", SYNTH_SRC, "-o", synth_obj])
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            for r in ex.map(_run, cmds):
                if verbose and r.stderr:
                    print(r.stderr)
        for out, inputs in ((LIB, objs), (SYNTH_LIB, [synth_obj])):
            tmp_out = out + ".tmp"
            _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *inputs, "-o", tmp_out])
            os.replace(tmp_out, out)
    return [LIB, SYNTH_LIB]


if __name__ == "__main__":
    for p in build(verbose=True):
        print(p)
