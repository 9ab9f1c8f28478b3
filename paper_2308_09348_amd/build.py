"""Build the HIP library libqscatter.so for gfx950, in-tree.

Each source is compiled to an object of its own (in parallel, in a temporary
directory) with the common flags plus its entry in SOURCE_FLAGS, then the
objects are linked into the library."""
import concurrent.futures
import hashlib
import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libqscatter.so")
SOURCES = ["csrc/qs_kernels.hip", "csrc/qs_tables.hip", "csrc/qs_adjoint.hip", "csrc/qs_photon.hip",
           "csrc/qs_factor.hip", "csrc/qs_api.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # no packed FP32 instructions (hipcc would otherwise form them from float code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]

# The tangent kernels' step loop runs about 7% faster under the instruction-
# level-parallelism scheduling strategy than under the default occupancy one
# (the same instructions in another order; measured on the differentiation
# workload's tape pass).
SOURCE_FLAGS = {
    "csrc/qs_adjoint.hip": ["-mllvm", "--amdgpu-sched-strategy=max-ilp"],
}


def source_id(extra_flags=()):
    """SHA-256 (hex) of everything the library is built from: each source
    and header under csrc/, the C-ABI header and the compiler flags.  The
    build stamps it into the library (qs_build_id), so a loaded library can
    be matched against the checked-out sources."""
    h = hashlib.sha256()
    csrc = os.path.join(PKG, "csrc")
    files = sorted(os.path.join("csrc", f) for f in os.listdir(csrc)
                   if f.endswith((".hip", ".h")))
    for rel in files + [os.path.join("..", "include", "qscatter.h")]:
        h.update(rel.encode() + b"\0")
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    flags = HIPCC_FLAGS + sorted(f"{k}:{' '.join(v)}" for k, v in SOURCE_FLAGS.items())
    h.update(" ".join(flags + list(extra_flags)).encode())
    return h.hexdigest()


def build(verbose=False, extra_flags=()):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(PKG, "csrc")]
    stamp = ['-DQS_BUILD_ID="' + source_id(extra_flags) + '"']
    with tempfile.TemporaryDirectory(prefix="qs_build_") as tmp:
        def compile_one(src):
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            cmd = ([hipcc] + HIPCC_FLAGS + SOURCE_FLAGS.get(src, []) + list(extra_flags) + inc +
                   (stamp if src == "csrc/qs_api.hip" else []) +
                   ["-c", os.path.join(PKG, src), "-o", obj])
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)
            return obj
        with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(SOURCES), 6)) as ex:
            objs = list(ex.map(compile_one, SOURCES))
        cmd = [hipcc, "-shared", "--offload-arch=gfx950", "-fPIC"] + objs + ["-o", LIB + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
