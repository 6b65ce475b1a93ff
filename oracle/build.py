"""Compile liboracle.so (the serial FP64 oracle) with gcc.  Test infrastructure only."""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    out = os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    # -O2 without -ffast-math: IEEE evaluation order is kept (Neumaier sums rely on it)
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_native(out: str, verbose: bool = False) -> str:
    """The same oracle compiled for the host it runs on (-O3 -march=native), for timing
    the CPU baseline; -ffp-contract=off keeps every product and sum separately rounded,
    as in the portable build."""
    src = os.path.join(_HERE, "oracle.c")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-march=native", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-o", tmp, src,
           "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
