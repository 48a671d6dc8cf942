"""Compile the C oracle into ``oracle/liboracle.so`` with gcc.

Test infrastructure: the oracle is built beside the product so the checker
exists wherever the tests run; building it is not using it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "gb_oracle.c"), os.path.join(HERE, "gb_oracle_wide.c")]
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", OUT + ".tmp"] + SRCS
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
