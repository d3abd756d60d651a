"""Build the oracle's C sources into ``oracle/liboracle.so`` with gcc.

Test infrastructure only (the oracle checks the HIP library; the library never
loads it).  ``python oracle/build.py`` or ``oracle.build.build()``.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["pic_oracle.c", "qed_oracle.c"]
LIB = os.path.join(HERE, "liboracle.so")


OMP_SOURCES = ["pic_oracle.c", "omp_push.c"]
OMP_LIB = os.path.join(HERE, "liboracle_omp.so")


def build_omp(verbose: bool = False) -> str:
    """The parallel driver of the benchmark's CPU baseline (the oracle's own
    particle step on every host thread, -O3 -fopenmp, same IEEE arithmetic:
    no contraction, no fast-math)."""
    srcs = [os.path.join(HERE, s) for s in OMP_SOURCES]
    tmp = OMP_LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, OMP_LIB)
    return OMP_LIB


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    build_omp(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
