"""Build the HIP library liblbm_axi.so for gfx950 (in-tree)."""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "liblbm_axi.so")
SOURCES = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 vector ops stay off: the compiler may not form them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


SAN_OUT = os.path.join(HERE, "liblbm_axi_hostsan.so")


def build(verbose=False):
    cmd = ["hipcc", *FLAGS, "-o", OUT + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


def build_host_sanitized(verbose=False):
    """The library with its host code (argument checks, layouts, the C ABI)
    built with AddressSanitizer and UndefinedBehaviorSanitizer, for the CPU
    sanitizer test; the device code is built as usual.  Rebuilt only when a
    source is newer than the library."""
    newest = max(os.path.getmtime(f) for f in SOURCES + glob.glob(os.path.join(HERE, "csrc", "*.hpp")) +
                 glob.glob(os.path.join(HERE, "..", "include", "*.h")))
    if os.path.exists(SAN_OUT) and os.path.getmtime(SAN_OUT) > newest:
        return SAN_OUT
    cmd = ["hipcc", *FLAGS, "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-o", SAN_OUT + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SAN_OUT + ".tmp", SAN_OUT)
    return SAN_OUT


if __name__ == "__main__":
    build(verbose=True)
