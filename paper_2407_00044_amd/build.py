"""Build libstreamk.so (the HIP kernels and the C ABI) for gfx950.

Every (input type, A layout, B layout) triple is one compilation of
csrc/sk_inst.hip; the host library csrc/sk_api.hip is another, and the
operand-packing transpose csrc/sk_transpose.hip a third.  The units
are compiled in parallel with hipcc and linked into a shared library next to
this file, where the Python binding loads it.

Flags: -O3 for gfx950 only; packed-FP32 instruction forms are disabled for
all device code (the kernels' FP32 arithmetic is written scalar and must not
be fused into packed pairs).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libstreamk.so")
BUILD = os.path.join(ROOT, "_build")

ARCH = "gfx950"
DTYPES = {0: "f32", 1: "f16", 2: "bf16", 3: "e4m3", 4: "mx8", 5: "mx4", 6: "mx6", 7: "mx6e3m2",
          8: "mx8e5m2", 9: "e5m2"}
LAYOUTS = {0: "r", 1: "c"}

COMMON = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-I" + os.path.join(ROOT, "include"),
          "-Rpass-analysis=kernel-resource-usage"]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _units():
    units = [("sk_api", os.path.join(CSRC, "sk_api.hip"), []),
             ("sk_transpose", os.path.join(CSRC, "sk_transpose.hip"), [])]
    for dt, dn in DTYPES.items():
        for la, an in LAYOUTS.items():
            for lb, bn in LAYOUTS.items():
                if 4 <= dt <= 8 and (la, lb) != (0, 1):
                    continue   # MX formats: K-contiguous operands only
                units.append((f"sk_inst_{dn}_{an}{bn}", os.path.join(CSRC, "sk_inst.hip"),
                              [f"-DSK_DT={dt}", f"-DSK_LA={la}", f"-DSK_LB={lb}"]))
    return units


def _compile(unit, verbose):
    name, src, defs = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [_hipcc()] + COMMON + defs + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{r.stderr}")
    with open(os.path.join(BUILD, name + ".resources.txt"), "w") as f:
        f.write(r.stderr)
    return obj


def build(verbose: bool = False, jobs: int = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), _units()))
    tmp = OUT + ".tmp"
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
