"""Build the CPU oracle (plain C, gcc) into oracle/liboracle.so.

TEST INFRASTRUCTURE ONLY.  The oracle is single-threaded and compiled without
floating-point contraction; only the exhaustive pin loops (pins.c) use OpenMP.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    objs = []
    for src, extra in (("oracle.c", []), ("pins.c", ["-fopenmp"])):
        obj = os.path.join(HERE, src[:-2] + ".o")
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-Wall",
               "-Wextra", "-Wno-unused-parameter", *extra, "-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-shared", "-fopenmp", *objs, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
