"""Build libcsi.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcsi.so")
SPECIES = tuple(int(s) for s in os.environ.get("CSI_SPECIES", "2,3,5,11,16,20,32").split(","))
# temperature models compiled per species count (the seeded synthetic mechanisms are one-temperature)
MODELS = {16: (1,), 20: (1,), 32: (1,)}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I" + CSRC, "-Wno-unused-result"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    return cmd


def _stale(src, obj, deps):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in [src, *deps])


def build(jobs: int = 8, verbose: bool = False, force: bool = True) -> str:
    """Compile every unit (force=True) or only the stale ones, then link."""
    os.makedirs(BUILD, exist_ok=True)
    with open(os.path.join(BUILD, "species.txt"), "w") as f:
        f.write(",".join(map(str, SPECIES)))
    units = [(os.path.join(CSRC, "csi_api.hip"), os.path.join(BUILD, "csi_api.o"), [])]
    for ns in SPECIES:
        for nt in MODELS.get(ns, (1, 2)):
            units.append((os.path.join(CSRC, "csi_inst.hip"), os.path.join(BUILD, f"csi_inst_{ns}_{nt}.o"),
                          [f"-DCSI_NS={ns}", f"-DCSI_NT={nt}"]))
    extra = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip") and f not in ("csi_api.hip", "csi_inst.hip"))
    for f in extra:
        units.append((os.path.join(CSRC, f), os.path.join(BUILD, f[:-4] + ".o"), []))
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "csi.h"))
    cmds = [[HIPCC, *FLAGS, *d, "-c", src, "-o", obj] for src, obj, d in units
            if force or _stale(src, obj, deps)]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for c in ex.map(_run, cmds):
            if verbose:
                print(" ".join(c))
    objs = [obj for _, obj, _ in units]
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", LIB + ".tmp", *objs])
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, force="--force" in sys.argv))
