"""Build libomerf.so (the C-ABI ray marcher) for gfx950 with hipcc, in-tree.

Usage: python -m paper_2404_09531_amd.build [--asm DIR]
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["api.hip", "march_fwd.hip", "march_bwd.hip", "mlp.hip", "bake.hip", "order.hip"]
LIB = os.path.join(HERE, "libomerf.so")
# measurement-only calibration kernels (not part of the C ABI)
CALIB_SOURCES = ["calib.hip"]
CALIB_LIB = os.path.join(HERE, "libomcalib.so")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # code object v5: loadable by the HIP runtime that ships with torch
    "-mcode-object-version=5",
    # no packed-FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # float atomics as native global_atomic_add_f32 (device memory is coarse-grained)
    "-munsafe-fp-atomics",
    "-I", os.path.join(ROOT, "include"),
]


def check_no_scratch(src: str, remarks: str) -> None:
    """Refuse kernels that spill to scratch memory.  The shipped kernels keep
    every live value in registers; a build whose register allocation spills
    (e.g. after a change that raises register pressure) is rejected rather
    than shipped, so its cross-lane code always runs on unspilled registers."""
    name = None
    for line in remarks.splitlines():
        if "Function Name:" in line:
            name = line.split("Function Name:")[1].split("[")[0].strip()
        elif "ScratchSize [bytes/lane]:" in line:
            size = int(line.split("ScratchSize [bytes/lane]:")[1].split("[")[0])
            if size != 0:
                raise RuntimeError(f"{src}: kernel {name} uses {size} bytes/lane of scratch (register spills)")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def build(asm_dir: str | None = None, verbose: bool = False, out: str | None = None,
          defines: tuple = ()) -> str:
    """Compile every source to an object, then link the shared library
    (to `out`, default the in-tree libomerf.so) with extra -D `defines`."""
    obj_dir = os.path.join(ROOT, "_build", "_".join(defines) or "default")
    os.makedirs(obj_dir, exist_ok=True)
    cc = hipcc()

    def compile_one(src: str) -> str:
        obj = os.path.join(obj_dir, src.replace(".hip", ".o"))
        cmd = [cc, *FLAGS, *[f"-D{x}" for x in defines], "-Rpass-analysis=kernel-resource-usage", "-c",
               os.path.join(CSRC, src), "-o", obj]
        if asm_dir:
            os.makedirs(asm_dir, exist_ok=True)
            cmd += ["-save-temps=obj"]
            cmd[cmd.index("-o") + 1] = os.path.join(asm_dir, src.replace(".hip", ".o"))
            obj = cmd[cmd.index("-o") + 1]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{res.stderr}")
        check_no_scratch(src, res.stderr)
        if verbose and res.stderr.strip():
            print(res.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(len(SOURCES) + len(CALIB_SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES + CALIB_SOURCES))

    def link(objects, lib):
        os.makedirs(os.path.dirname(lib), exist_ok=True)
        tmp = lib + ".tmp"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objects, "-o", tmp]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed:\n{res.stderr}")
        os.replace(tmp, lib)

    lib = out or LIB
    link(objs[:len(SOURCES)], lib)
    if out is None:
        link(objs[len(SOURCES):], CALIB_LIB)
    return lib


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--asm", default=None, help="also keep the gfx950 assembly in this directory")
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    print(build(a.asm, a.v))


def ensure_built() -> str:
    """Build the library if it is not there yet; return its path."""
    if not os.path.exists(LIB):
        build()
    return LIB
