"""Build ``libbsi.so`` (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled in parallel, then linked into one shared library
next to this file.  Flags:
  --offload-arch=gfx950        MI355X only
  -ffp-contract=off            no implicit FMA contraction: the kernels spell out
                               every fmaf, so one routine gives the same bits
                               wherever it is inlined
  -Xclang -target-feature -Xclang -packed-fp32-ops
                               no packed-FP32 instructions
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libbsi.so")
# host-only checker of the kernels' index arithmetic (CPU tests), linked to libbsi
CHECK_LIB = os.path.join(HERE, "libbsi_check.so")
CHECK_SRC = "index_check.cpp"
OBJDIR = os.path.join(ROOT, "_build", "obj")

SOURCES = ["lut.hip", "forward.hip", "lerp.hip", "adjoint.hip", "warp.hip", "fused.hip", "general.hip", "batch.hip", "noalloc.hip", "abi.cpp"]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-I" + INCLUDE, "-I" + CSRC,
]


def _compile(src):
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC] + CFLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature: harmless
    noise = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, "\n".join(noise)))
    return obj, noise


def build(verbose: bool = False) -> str:
    """Compile every source and link libbsi.so; returns the library path."""
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        results = list(ex.map(_compile, SOURCES))
    if verbose:
        for obj, noise in results:
            for line in noise:
                print(line, file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    build_checker()
    return LIB


def build_checker() -> str:
    """Compile the host-side index checker against the freshly linked libbsi.so."""
    tmp = CHECK_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-x", "hip"] + CFLAGS + ["-shared", os.path.join(CSRC, CHECK_SRC), "-L" + HERE, "-lbsi",
                                           "-Wl,-rpath,$ORIGIN", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        noise = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        raise RuntimeError("index checker build failed:\n" + "\n".join(noise))
    os.replace(tmp, CHECK_LIB)
    return CHECK_LIB


if __name__ == "__main__":
    print(build(verbose=True))
