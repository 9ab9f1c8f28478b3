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


SAN_LIB = os.path.join(HERE, "libqso_san.so")
# AddressSanitizer and UndefinedBehaviorSanitizer, any report fatal: the
# sanitized oracle runs the CPU pins with the ASan runtime preloaded
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-g"]


def build_sanitized(verbose=False):
    """The oracle built under ASan + UBSan into oracle/libqso_san.so."""
    return build(verbose=verbose, lib=SAN_LIB, extra_flags=SAN_FLAGS)


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
