"""Build libttnn.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

    python -m paper_2412_06111_amd.build          # or build() from Python

Objects go to paper_2412_06111_amd/_build/, the library to
paper_2412_06111_amd/libttnn.so.  Always recompiles every source.
"""

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libttnn.so")
INCLUDE = os.path.join(os.path.dirname(PKG), "include")

ARCH = "gfx950"
COMMON = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result", "-Wno-unknown-pragmas",
    f"-I{INCLUDE}",
]
# sources whose floating-point results must not depend on FMA contraction
NO_CONTRACT = {"drm.hip"}
# per-source extra flags: the fused kernels keep their accumulator arrays in registers
# (LDS is reserved for the staged operands)
EXTRA = {"fused.hip": ["-mllvm", "-disable-promote-alloca-to-lds"]}


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src):
    name = os.path.basename(src)
    obj = os.path.join(OUT_DIR, name + ".o")
    flags = list(COMMON)
    if name in NO_CONTRACT:
        flags.append("-ffp-contract=off")
    flags += EXTRA.get(name, [])
    if name.endswith(".hip"):
        cmd = [_hipcc(), "-x", "hip", *flags, "-c", src, "-o", obj]
    else:
        cmd = [_hipcc(), *flags, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        results = list(ex.map(_compile, srcs))
    objs = [o for o, _ in results]
    if verbose:
        for _, warn in results:
            if warn.strip():
                print(warn, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
