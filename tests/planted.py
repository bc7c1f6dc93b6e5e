"""Copies of the oracle with one planted mistake, for showing that a pin fails
when the oracle is wrong.  The mistake is a text substitution in a temporary
copy of the oracle's C source, compiled on the CPU and swapped in for the
duration of a `with` block; the oracle's own sources and library are not
touched."""
import contextlib
import os
import subprocess
import tempfile

import oracle


@contextlib.contextmanager
def planted(old, new):
    src = open(oracle.SRC_PATH).read()
    assert src.count(old) == 1, f"planted mistake: pattern not unique in the oracle source: {old!r}"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "planted.c")
        with open(c, "w") as f:
            f.write(src.replace(old, new))
        so = os.path.join(d, "libplanted.so")
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", so, c, "-lm"])
        saved = oracle._lib
        oracle._lib = oracle.load_library(so)
        try:
            yield
        finally:
            oracle._lib = saved
