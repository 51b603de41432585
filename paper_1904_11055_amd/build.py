"""Builds libpolyspec.so (HIP kernels for gfx950 + the C ABI) in place.

Usage: python -m paper_1904_11055_amd.build  (or build() from Python).

After compiling, every device code object is disassembled and the build fails if
it holds a packed float32 instruction (v_pk_add_f32, v_pk_mul_f32, v_pk_fma_f32):
the kernels are meant to use plain float32 VALU instructions only.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpolyspec.so")
SOURCES = ["fft.hip", "contract_tiles_lo.hip", "contract_tiles_hi.hip", "contract_j3.hip", "reduce.hip",
           "adjoint.hip", "adjoint_fp32.hip", "adjoint_bf16.hip", "adjoint_fp16.hip", "util.hip", "plan.cpp"]
ARCH = "gfx950"
ROCM_LLVM = "/opt/rocm/llvm/bin"
PACKED_F32 = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _flags() -> list[str]:
    # -packed-fp32-ops turns off the packed float32 instructions in the gfx950 device
    # pass; the host (x86) pass does not know the feature and warns that it ignores
    # it, which is harmless.  check_no_packed_f32() verifies the device code.
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(os.path.dirname(HERE), "include")]


def check_no_packed_f32(obj: str) -> list[str]:
    """Packed float32 instructions found in the gfx950 code object of a compiled .o."""
    tools = [os.path.join(ROCM_LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-objdump")]
    if not all(os.path.exists(t) for t in tools):
        raise RuntimeError("llvm-objcopy, clang-offload-bundler and llvm-objdump are needed for the code check")
    objcopy, bundler, objdump = tools
    with tempfile.TemporaryDirectory() as td:
        fatbin = os.path.join(td, "fatbin")
        dev = os.path.join(td, "dev.co")
        r = subprocess.run([objcopy, f"--dump-section=.hip_fatbin={fatbin}", obj, os.path.join(td, "o")],
                           capture_output=True, text=True)
        if r.returncode != 0:       # no device code in this object (host-only source)
            return []
        subprocess.run([bundler, "--unbundle", "--type=o", f"--input={fatbin}",
                        f"--targets=hipv4-amdgcn-amd-amdhsa--{ARCH}", f"--output={dev}"],
                       check=True, capture_output=True)
        dis = subprocess.run([objdump, "-d", dev], check=True, capture_output=True, text=True).stdout
    return sorted({m.group(0) for m in PACKED_F32.finditer(dis)})


def _newest_header() -> float:
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    heads.append(os.path.join(os.path.dirname(HERE), "include", "polyspec.h"))
    return max(os.path.getmtime(h) for h in heads)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compiles every source (or, with incremental=True, those newer than their object)."""
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    newest_header = _newest_header()

    def compile_one(src: str) -> str:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        if incremental and os.path.exists(obj):
            t = os.path.getmtime(obj)
            if t > os.path.getmtime(os.path.join(CSRC, src)) and t > newest_header:
                return obj
        cmd = [hipcc, *_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
        if verbose:
            sys.stderr.write(" ".join(cmd) + "\n")
        found = check_no_packed_f32(obj)
        if found:
            raise RuntimeError(f"{src}: device code holds packed float32 instructions {found}")
        return obj

    workers = max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
