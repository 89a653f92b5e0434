"""Build the oracle's shared library with the host C compiler.

Test infrastructure: compiled so that tests, the smoke check and the
benchmark's CPU baseline can load it; the product never links it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libcdef_oracle.so")
CFLAGS = ["-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared"]


def build(extra_flags=(), out=LIB):
    src = os.path.join(HERE, "cdef_oracle.c")
    cmd = ["gcc", *CFLAGS, *extra_flags, src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())
