"""Compile the oracle's C sources into oracle/liboracle.so (gcc, -O2, no FP contraction)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["orc_fem.c", "orc_amg.c", "orc_solve.c", "orc_api.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False, src_dir=HERE, out=LIB):
    """Build the library from the sources in src_dir (default: this
    directory) into out."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-o", out + ".tmp"]
    cmd += [os.path.join(src_dir, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
