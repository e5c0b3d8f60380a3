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


def build(verbose=False):
    for name, extra in OUTPUTS.items():
        out = os.path.join(HERE, name)
        cmd = ["gcc", *FLAGS, *extra, "-o", out + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(verbose=True)
