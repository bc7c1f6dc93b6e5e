"""The shared library loads without a GPU and exports every function that
include/cpic.h declares; the Python binding refuses to run without it."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cpic.h")
LIB = os.path.join(ROOT, "paper_2303_05599_amd", "libcpic.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cpic_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2303_05599_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (cpic_\w+)", out))
    assert set(names) <= exported


def test_error_message_without_context(lib):
    lib.cpic_last_error.restype = ctypes.c_char_p
    lib.cpic_last_error.argtypes = [ctypes.c_void_p]
    assert isinstance(lib.cpic_last_error(None), bytes)


def test_parameter_validation_needs_no_gpu():
    """cpic_create rejects bad parameters before touching the device."""
    import paper_2303_05599_amd as cp
    for bad in (dict(N=100), dict(N=32, L_fm=-1.0), dict(N=32, precision=7), dict(N=2)):
        with pytest.raises(cp.CpicError) as e:
            cp.Context(bad, None, stream=None)
        assert e.value.status == -1
    # particle records are addressed with 32-bit offsets: the count is bounded
    # so that they stay below 2 GiB (19 reals per particle)
    for prec, limit in ((cp.FP64, 2**31 // 152), (cp.FP32, 2**31 // 76)):
        for n in (limit + 1, 2**40, -1):
            with pytest.raises(cp.CpicError) as e:
                cp.Context(dict(N=32, precision=prec), dict(n=n, mass_GeV=1.0), stream=None)
            assert e.value.status == -1 and "particle count" in str(e.value)


def test_struct_layout_matches_header(tmp_path):
    """Offsets and sizes of the parameter structs as the C compiler lays them out."""
    import paper_2303_05599_amd as cp
    probe = tmp_path / "probe.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "cpic.h"', "int main(void){"]
    for cname, py in (("cpic_glasma_params", cp.GlasmaParams), ("cpic_particle_params", cp.ParticleParams),
                     ("cpic_jet_params", cp.JetParams)):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    probe.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        name, field, val = line.split()
        got[(name, field)] = int(val)
    for cname, py in (("cpic_glasma_params", cp.GlasmaParams), ("cpic_particle_params", cp.ParticleParams),
                     ("cpic_jet_params", cp.JetParams)):
        assert got[(cname, "size")] == ctypes.sizeof(py)
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
