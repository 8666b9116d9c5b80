"""Build the CPU oracle (test infrastructure) with gcc.

Two shared libraries come from the single C source: ``liboracle.so`` (double)
and ``liboracle_cs.so`` (double complex, for complex-step derivatives).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIBS = {"liboracle.so": [], "liboracle_cs.so": ["-DORC_COMPLEX"]}


def build(verbose: bool = False) -> None:
    for name, extra in LIBS.items():
        out = os.path.join(HERE, name)
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               *extra, "-o", out + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(verbose=True)
