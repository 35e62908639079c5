"""Compiles the C oracle (test infrastructure) into ``oracle/liboracle.so`` with gcc.

No FMA contraction and no fast-math, so the oracle's rounding follows its source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")


def library_path():
    return os.path.join(HERE, "liboracle.so")


def build_oracle(force=True):
    out = library_path()
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out
