"""Build the HIP library libsap.so for gfx950 (in-tree, next to this file).

The host runtime and the K-independent kernels form one translation unit
(csrc/sap_api.hip), the batched engine another (csrc/sap_batch.hip); the
kernels templated on the projection width K are compiled once per K = 1..16
from csrc/sap_kinst.hip.  The units compile in
parallel to objects under _build/ and are linked into one shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

HERE = Path(__file__).resolve().parent
CSRC = HERE / "csrc"
LIB = HERE / "libsap.so"
OBJ = HERE / "_build"
ARCH = os.environ.get("SAP_OFFLOAD_ARCH", "gfx950")
KMAX = 16

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # arithmetic exactly as written: the rescoring kernel recomputes coarse
    # values and must reproduce the pass bit for bit
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def sources() -> list[Path]:
    return sorted(CSRC.glob("*")) + [HERE.parent / "include" / "sap.h"]


def _units() -> list[tuple[Path, list[str], Path]]:
    units = [(CSRC / "sap_api.hip", [], OBJ / "sap_api.o"),
             (CSRC / "sap_batch.hip", [], OBJ / "sap_batch.o")]
    for k in range(1, KMAX + 1):
        units.append((CSRC / "sap_kinst.hip", [f"-DSAP_K={k}"], OBJ / f"sap_k{k}.o"))
    return units


def _compile(hipcc: str, src: Path, defs: list[str], out: Path, verbose: bool) -> tuple[Path, str]:
    cmd = [hipcc, *HIPCC_FLAGS, *defs, "-c", "-o", str(out), str(src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        return out, res.stdout + res.stderr
    return out, ""


def build(verbose: bool = False, jobs: int | None = None) -> Path:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    OBJ.mkdir(exist_ok=True)
    units = _units()
    jobs = jobs or max(1, min(len(units), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda u: _compile(hipcc, u[0], u[1], u[2], verbose), units))
    errors = [(o, e) for o, e in results if e]
    if errors:
        for o, e in errors:
            sys.stderr.write(f"--- {o.name}\n{e}\n")
        raise RuntimeError(f"hipcc failed on {len(errors)} unit(s) building {LIB.name}")
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *[str(u[2]) for u in units]]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"linking {LIB.name} failed ({res.returncode})")
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not LIB.exists():
        return True
    t = LIB.stat().st_mtime
    return any(p.stat().st_mtime > t for p in sources())


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
