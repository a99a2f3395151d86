"""Builds the oracle's shared library with gcc (test infrastructure only)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(HERE, "liboracle.so")


def build_oracle(verbose: bool = False) -> str:
    src = os.path.join(HERE, "glint_oracle.c")
    out = library_path()
    tmp = out + ".tmp"
    # -ffp-contract=off: every float/double expression is rounded as written
    # (the float gating thresholds must round exactly as the paper's FP32).
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_oracle(verbose=True))
