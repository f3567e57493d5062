"""Build libjfnk.so (HIP, gfx950) in place: ``python -m paper_2605_13378_amd.build``.

Each translation unit under csrc/ is compiled by hipcc in parallel, then
linked into ``paper_2605_13378_amd/libjfnk.so``.  The per-operator kernels
(stencil and single-workgroup solve) are one translation unit per
(operator, precision) pair, compiled from ``stencil_inst.hip`` with the pair
given as macros, so that the expensive instantiations spread over all cores.
Packed-FP32 instructions are disabled for all device code.

``--incremental`` recompiles only the units whose object is older than one of
the files it depends on (hipcc's dependency lists); the default rebuilds all.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libjfnk.so")
ARCH = os.environ.get("JFNK_OFFLOAD_ARCH", "gfx950")

# (object name, source, macro definitions)
UNITS = [(os.path.splitext(s)[0], s, []) for s in
         ["solver.hip", "serving.hip", "kernels_f64.hip", "kernels_f32.hip", "kernels_f16.hip"]]
OPS = ["Burgers1DOp", "Burgers2DOp", "GrayScottOp", "KerrOp", "RD2DOp", "SuOlsonOp", "SuOlsonPYOp", "MaxwellTEOp",
       "MaxwellTECslpOp", "KerrCslpOp"]
for _t, _vt, _tag in (("double", "double", "f64"), ("float", "float", "f32"), ("float", "__half", "f16")):
    for _op in OPS:
        _fused = 1 if (_t == _vt and not _op.endswith("CslpOp")) else 0
        UNITS.append((f"stencil_{_tag}_{_op}", "stencil_inst.hip",
                      [f"-DJFNK_OP={_op}", f"-DJFNK_T={_t}", f"-DJFNK_VT={_vt}", f"-DJFNK_FUSED={_fused}"]))


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-Wall",
        "-Wno-unused-function",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE,
        "-I", CSRC,
    ]


def _up_to_date(obj: str, dep: str) -> bool:
    if not (os.path.exists(obj) and os.path.exists(dep)):
        return False
    t = os.path.getmtime(obj)
    with open(dep) as f:
        text = f.read().replace("\\\n", " ")
    files = text.split(":", 1)[1].split() if ":" in text else []
    return all(os.path.exists(p) and os.path.getmtime(p) <= t for p in files)


def _compile(unit, extra: list[str], incremental: bool) -> str:
    name, src, defs = unit
    obj = os.path.join(BUILD, name + ".o")
    dep = os.path.join(BUILD, name + ".d")
    if incremental and _up_to_date(obj, dep):
        return obj
    cmd = [hipcc(), *common_flags(), *defs, *extra, "-MD", "-MF", dep, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{res.stdout}\n{res.stderr}")
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if err and os.environ.get("JFNK_BUILD_VERBOSE"):
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = False, extra: list[str] | None = None, incremental: bool = False) -> str:
    """Compile every unit and link libjfnk.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    extra = list(extra or [])
    # the largest units first, so that the pool ends together
    order = sorted(UNITS, key=lambda u: (not u[0].startswith("stencil"), u[0]))
    with ThreadPoolExecutor(max_workers=max(1, min(len(order), os.cpu_count() or 4))) as ex:
        objs = list(ex.map(lambda u: _compile(u, extra, incremental), order))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    args = sys.argv[1:]
    inc = "--incremental" in args
    build(verbose=True, extra=[a for a in args if a != "--incremental"], incremental=inc)
