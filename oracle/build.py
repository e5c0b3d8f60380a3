"""Build the CPU oracle shared libraries (real and complex-step builds).

Test infrastructure only: the oracle is compiled with plain gcc, without
fast-math and without floating-point contraction, so every operation is the
one written in the source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_axi_oracle.c")
FLAGS = ["-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared"]
OUTPUTS = {
    "liboracle.so": [],
    "liboracle_complex.so": ["-DORACLE_COMPLEX"],
}


# AddressSanitizer + UndefinedBehaviorSanitizer builds for the CPU sanitizer
# test (clang, whose shared sanitizer runtime the HIP host code shares)
SAN_CC = "/opt/rocm/llvm/bin/clang"
SAN_FLAGS = ["-O1", "-g", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
             "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-shared-libsan"]


def build(verbose=False, sanitize=False):
    for name, extra in OUTPUTS.items():
        out = os.path.join(HERE, name.replace(".so", "_san.so") if sanitize else name)
        if sanitize:
            cmd = [SAN_CC, *SAN_FLAGS, *extra, "-o", out + ".tmp", SRC, "-lm"]
        else:
            cmd = ["gcc", *FLAGS, *extra, "-o", out + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(verbose=True)
