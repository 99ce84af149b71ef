"""Build step for the CPU oracle (test infrastructure; plain gcc, no GPU code)."""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def lib_path():
    return os.path.join(_HERE, "liboracle.so")


def build():
    """Compile tc_oracle.c with separate multiply/add roundings and OpenMP."""
    src = os.path.join(_HERE, "tc_oracle.c")
    out = lib_path()
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", src, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
