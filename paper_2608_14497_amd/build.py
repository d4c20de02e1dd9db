"""Build libhdconv.so (gfx950) from csrc/ with hipcc, in parallel.

The line and column kernels are templates on the FFT length; each
(precision, log2 m) instantiation is compiled as its own object so the build
spreads over all cores.  ``python -m paper_2608_14497_amd.build`` or
``build()`` always recompiles every object (no cache), then links.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhdconv.so")

ARCH = os.environ.get("HDC_OFFLOAD_ARCH", "gfx950")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: all FP32 math is scalar/vector-lane code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
LINE_MAX_LOGM = {"float": 12, "double": 11}
COL_MAX_LOGM = 10


def _units():
    units = []
    for t in ("float", "double"):
        for lm in range(LINE_MAX_LOGM[t] + 1):
            # long lines: one object per block cap (their register-heavy instantiations dominate the build)
            for kg in (0, 1):
                if lm >= 10:
                    for pm in (0, 1, 2, 4):
                        units.append((f"line_{t}_{lm}_{kg}_{pm}", "hdc_line.hip",
                                      [f"-DHDC_T={t}", f"-DHDC_LOGM={lm}", f"-DHDC_KG={kg}", f"-DHDC_PMAX={pm}"]))
                else:
                    units.append((f"line_{t}_{lm}_{kg}", "hdc_line.hip",
                                  [f"-DHDC_T={t}", f"-DHDC_LOGM={lm}", f"-DHDC_KG={kg}"]))
            units.append((f"line_{t}_{lm}_2", "hdc_line.hip", [f"-DHDC_T={t}", f"-DHDC_LOGM={lm}", "-DHDC_KG=2"]))
        for lm in range(COL_MAX_LOGM + 1):
            units.append((f"col_{t}_{lm}", "hdc_col.hip", [f"-DHDC_T={t}", f"-DHDC_LOGM={lm}"]))
        for lm in range(LINE_MAX_LOGM[t] + 1):
            units.append((f"cs_{t}_{lm}", "hdc_cs.hip", [f"-DHDC_T={t}", f"-DHDC_LOGM={lm}"]))
    units.append(("misc", "hdc_col.hip", ["-DHDC_MISC=1"]))
    units.append(("noalloc", "hdc_noalloc.hip", []))
    units.append(("host", "hdc_host.hip", []))
    return units


def _compile(unit):
    name, src, defs = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC, *FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{' '.join(cmd)}\n{r.stderr[-4000:]}")
    return obj, time.time() - t0


def build(jobs: int | None = None, verbose: bool = True) -> str:
    """Compile every HIP object for gfx950 and link libhdconv.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = _units()
    # longest units first (large FFT lengths)
    def _cost(u):
        parts = u[0].split("_")
        return -int(parts[2]) if len(parts) > 2 and parts[2].isdigit() else (-int(parts[-1]) if parts[-1].isdigit() else 0)

    units.sort(key=_cost)
    t0 = time.time()
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, dt in ex.map(_compile, units):
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"[hdconv] built {LIB} from {len(objs)} objects in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    build(jobs=int(sys.argv[1]) if len(sys.argv) > 1 else None)
