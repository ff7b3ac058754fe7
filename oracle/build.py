"""Build the CPU oracle shared library (test infrastructure)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))

# -ffp-contract=off: no fused multiply-add, every product is rounded on its own
# (IEEE round-to-nearest-even for each operation as written).
CMD = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
       "-Wall", "-o", os.path.join(HERE, "liboracle.so"), os.path.join(HERE, "cg_oracle.cpp")]


def build():
    subprocess.run(CMD, check=True, cwd=HERE)
    return os.path.join(HERE, "liboracle.so")


if __name__ == "__main__":
    print(build())
