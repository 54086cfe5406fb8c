"""Build the FP64 CPU oracle (test infrastructure) into oracle/libcm_oracle.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cm_oracle.c")
LIB = os.path.join(HERE, "libcm_oracle.so")


def compile_lib(src: str, out: str, verbose: bool = False) -> str:
    """Compile one oracle source file into a shared library at ``out``."""
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-Werror",
           "-I", HERE, src, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    return compile_lib(SRC, LIB, verbose)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
