"""Build the gfx950 shared library ``libpint.so`` in-tree with hipcc.

Usage: ``python -m paper_2007_13125_amd.build`` (or ``build()`` from Python).
The library exports the C ABI declared in ``include/pint.h``.  Each source is
compiled to an object in a temporary folder (in parallel), then linked.
"""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpint.so")

SOURCES = ["pint_forward.hip", "pint_space.hip", "pint_time.hip", "pint_gentime.hip", "pint_seq.hip", "pint_noalloc.hip", "pint_host.cpp"]

# Packed FP32 instructions are disabled for all device code (hipcc -O3 would
# otherwise form v_pk_* FP32 ops from ordinary float code).
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; the HIP toolchain is required to build libpint.so")
    return exe


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    return res.returncode, res.stdout


def build(verbose=False, jobs=None):
    """Compile every HIP source for gfx950 into paper_2007_13125_amd/libpint.so."""
    inc = ["-I", os.path.join(ROOT, "include")]
    with tempfile.TemporaryDirectory(prefix="pint_build_") as tmpd:
        objs, cmds = [], []
        for s in SOURCES:
            o = os.path.join(tmpd, os.path.splitext(s)[0] + ".o")
            objs.append(o)
            cmds.append([hipcc()] + FLAGS + inc + ["-c", os.path.join(CSRC, s), "-o", o])
        jobs = jobs or min(len(cmds), max(1, os.cpu_count() or 1))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(lambda c: _run(c, verbose), cmds))
        for (rc, out), c in zip(results, cmds):
            if rc != 0:
                sys.stderr.write(out)
                raise RuntimeError("hipcc failed: " + " ".join(c))
        tmp = LIB + ".tmp"
        rc, out = _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
        if rc != 0:
            sys.stderr.write(out)
            raise RuntimeError("hipcc failed linking libpint.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
