"""Builds librsv.so for gfx950 from csrc/ with hipcc (no JIT, no torch extension).

    python -m paper_1807_07433_amd.build [--jobs N] [--asm]

Objects go to paper_1807_07433_amd/_build/, the library to
paper_1807_07433_amd/librsv.so.  Every call rebuilds everything.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "librsv.so")
PROBE_LIB = os.path.join(PKG, "libprobe.so")
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-ffp-contract=off",                      # FMAs only where written (fmaf / fma)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    f"-I{INCLUDE}", f"-I{CSRC}",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    out = []
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp")):
            out.append(os.path.join(CSRC, name))
    return out


def _compile(src: str, asm: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *COMMON, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if asm and src.endswith(".hip"):
        s = os.path.join(BUILD, os.path.basename(src) + ".s")
        subprocess.run([hipcc(), *COMMON, "--cuda-device-only", "-S", src, "-o", s],
                       check=True, capture_output=True)
    return obj


def build(jobs: int | None = None, asm: bool = False, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, asm), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources")
    build_probe(verbose)
    return LIB


def build_probe(verbose: bool = True) -> str:
    """libprobe.so: the LDS bandwidth probe that bench.py measures the LDS peak with
    (measurement only; librsv.so does not use it)."""
    src = os.path.join(PKG, "probe", "lds_probe.hip")
    obj = os.path.join(BUILD, "lds_probe.hip.o")
    for cmd in ([hipcc(), *COMMON, "-c", src, "-o", obj],
                [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", obj, "-o", PROBE_LIB + ".tmp"]):
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"probe build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    if verbose:
        print(f"built {PROBE_LIB}")
    return PROBE_LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--asm", action="store_true", help="also write device assembly to _build/")
    a = ap.parse_args(argv)
    build(a.jobs, a.asm)


if __name__ == "__main__":
    sys.exit(main())
