"""Build libhfci.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1811_12378_amd.build [--jobs N] [--debug]

Every translation unit under csrc/ is compiled with hipcc for gfx950 into
_build/, then linked into paper_1811_12378_amd/libhfci.so next to this file.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libhfci.so")
ARCH = "gfx950"

COMMON = [
    "-std=c++17", "-O3", "-fPIC", "-Wall", "-Wno-unused-result",
    "--offload-arch=" + ARCH,
    # keep the compiler from forming packed FP32 instructions on gfx950
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libhfci)")


def sources():
    out = []
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp")):
            out.append(os.path.join(CSRC, name))
    return out


def compile_one(cc, src, extra):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [cc] + COMMON + extra + ["-x", "hip", "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), res.stdout, res.stderr))
    warn = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return obj, warn


def build(jobs: int = 8, debug: bool = False, verbose: bool = False) -> str:
    cc = hipcc()
    os.makedirs(BUILD, exist_ok=True)
    extra = ["-g"] if debug else []
    srcs = sources()
    objs = []
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        futs = {ex.submit(compile_one, cc, s, extra): s for s in srcs}
        for fut in cf.as_completed(futs):
            obj, warn = fut.result()
            objs.append(obj)
            if verbose and warn:
                print(warn, file=sys.stderr)
    tmp = LIB + ".tmp"
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    # rocBLAS: the complex GEMMs of the inner preconditioner's sine transforms;
    # hipFFT: the 3D transforms of the Fourier-spectral operator
    cmd = ([cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + sorted(objs)
           + ["-L" + rocm_lib, "-lrocblas", "-lhipfft", "-Wl,-rpath," + rocm_lib])
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (res.stdout, res.stderr))
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.debug, a.verbose))


if __name__ == "__main__":
    main()
