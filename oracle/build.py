"""Build the CPU oracle (test infrastructure) with gcc.

Two shared libraries come from the single C source: ``liboracle.so`` (double)
and ``liboracle_cs.so`` (double complex, for complex-step derivatives).

``build(outdir, sanitize=True)`` writes both with AddressSanitizer and
UndefinedBehaviorSanitizer instead (every finding fatal); they load only in
a process that has gcc's ASan runtime preloaded, and the oracle's loader
takes them from ``outdir`` when ``ORACLE_LIB_DIR`` names it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIBS = {"liboracle.so": [], "liboracle_cs.so": ["-DORC_COMPLEX"]}


SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=all"]


def build(verbose: bool = False, outdir: str = HERE, sanitize: bool = False) -> None:
    for name, extra in LIBS.items():
        out = os.path.join(outdir, name)
        opt = SANITIZE if sanitize else ["-O2"]
        cmd = ["gcc", *opt, "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               *extra, "-o", out + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(verbose=True)
