"""Compile the CPU oracle (host C, gcc, no FMA contraction).

oracle/liboracle.so      the oracle the tests check against: sequential, -O2.
oracle/liboracle_omp.so  a timing build of the same source with -O3 -fopenmp
                         (row and element loops in parallel, per-thread
                         compensated dot partials), used only for the
                         all-cores CPU baseline of the benchmark.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")


def _gcc(out, flags, verbose):
    cmd = ["gcc", *flags, "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    out = _gcc(os.path.join(HERE, "liboracle.so"), ["-O2"], verbose)
    _gcc(os.path.join(HERE, "liboracle_omp.so"), ["-O3", "-fopenmp"], verbose)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
