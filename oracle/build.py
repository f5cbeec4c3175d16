"""Compile the C oracle (``ray_oracle.c``) into ``liboracle_ray.so`` with gcc.

Test infrastructure only (see the package docstring).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ray_oracle.c")
LIB = os.path.join(HERE, "liboracle_ray.so")


def build(force=False):
    """Compile the oracle if the library is missing or older than its source."""
    if (not force and os.path.exists(LIB)
            and os.path.getmtime(LIB) >= os.path.getmtime(SRC)):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared",
           "-ffp-contract=off", "-o", tmp, SRC, "-lm", "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


COUNT_SRC = os.path.join(HERE, "opcount.cpp")
COUNT_LIB = os.path.join(HERE, "liboracle_count.so")


def build_count(force=False):
    """Compile the operation-counting build of the oracle (opcount.cpp, which
    compiles ray_oracle.c as C++ with a counting number type)."""
    newest = max(os.path.getmtime(SRC), os.path.getmtime(COUNT_SRC))
    if not force and os.path.exists(COUNT_LIB) and os.path.getmtime(COUNT_LIB) >= newest:
        return COUNT_LIB
    tmp = COUNT_LIB + ".tmp%d" % os.getpid()
    cmd = ["g++", "-O2", "-std=c++17", "-D_GNU_SOURCE", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", tmp, COUNT_SRC, "-lm", "-lpthread"]
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(tmp, COUNT_LIB)
    return COUNT_LIB


if __name__ == "__main__":
    print(build(force=True))
    print(build_count(force=True))
