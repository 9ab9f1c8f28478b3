"""Build the FP64 CPU oracle (test infrastructure only) into oracle/libqso.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libqso.so")


FLAGS = ["-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-Wall",
         "-Wextra"]


def build(verbose=False, source=None, lib=None, extra_flags=()):
    """Compile qso.cpp (or `source`, a copy of it) into oracle/libqso.so (or
    `lib`)."""
    source = source or os.path.join(HERE, "qso.cpp")
    lib = lib or LIB
    cmd = ["g++"] + FLAGS + ["-I" + HERE] + list(extra_flags) + [source, "-o", lib + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
