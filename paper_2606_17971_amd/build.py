"""Compile the HIP library libadef2.so for gfx950 (in-tree).

The library is split into translation units that compile in parallel: the
host runtime with the setup kernels (adef2.hip), the per-instance iteration
kernels once per vector type / panel type / tile height (iter_inst.hip with
-D defines) and the tile-major iteration kernels (iter_bt.hip).  Objects go
to _build/ next to this file; the shared library is linked in place.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libadef2.so")
BUILD = os.path.join(HERE, "_build")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wno-unused-value", "-Wno-unused-result",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

# (object name, source, extra defines)
UNITS = [("adef2", "adef2.hip", [])]
for v, m, tag in (("double", "double", "dd"), ("double", "float", "df"), ("float", "float", "ff")):
    for rpt in (1, 2):
        UNITS.append((f"iter_{tag}_r{rpt}", "iter_inst.hip",
                      [f"-DITER_V={v}", f"-DITER_M={m}", f"-DITER_RPT={rpt}"]))
UNITS.append(("iter_bt", "iter_bt.hip", []))


def _compile(hipcc: str, unit):
    name, src, defs = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [hipcc, *FLAGS, *defs, "-c", "-o", obj, os.path.join(CSRC, src)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    return name, obj, res


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda u: _compile(hipcc, u), UNITS))
    failed = [(n, r) for n, _, r in results if r.returncode != 0]
    for n, r in failed:
        sys.stderr.write(f"--- {n}\n{r.stdout}{r.stderr}")
    if failed:
        raise RuntimeError(f"hipcc failed for {[n for n, _ in failed]}")
    if verbose:
        for n, _, r in results:
            sys.stderr.write(r.stderr)
    tmp = OUT + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[o for _, o, _ in results]]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"link failed ({res.returncode}) building {OUT}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
