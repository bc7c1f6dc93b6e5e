"""Pins of the oracle's SU(3) algebra against values the paper prints
(Tables I and II, the initial colour vectors, the Casimirs, the running
coupling) and against library routines (scipy's matrix exponential)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def golden_tables():
    f = np.zeros((8, 8, 8))
    d = np.zeros((8, 8, 8))
    for line in open(os.path.join(GOLD, "su3_structure_constants.txt")):
        if line.startswith("#") or not line.strip():
            continue
        kind, a, b, c, v = line.split()[:5]
        a, b, c, v = int(a) - 1, int(b) - 1, int(c) - 1, float(v)
        import itertools
        for perm in itertools.permutations((0, 1, 2)):
            idx = tuple((a, b, c)[k] for k in perm)
            if kind == "f":
                sign = 1 if perm in ((0, 1, 2), (1, 2, 0), (2, 0, 1)) else -1
                f[idx] = sign * v
            else:
                d[idx] = v
    return f, d


def paper_values():
    return json.load(open(os.path.join(GOLD, "paper_values.json")))


def test_generators_reproduce_tables_I_and_II():
    """[T^a,T^b] = i f_abc T^c and {T^a,T^b} = delta_ab/3 + d_abc T^c with
    the printed tables (Appendix B.1)."""
    T = [oracle.generator(a) for a in range(8)]
    f_ref, d_ref = golden_tables()
    for a in range(8):
        for b in range(8):
            assert np.trace(T[a] @ T[b]) == pytest.approx(0.5 * (a == b), abs=1e-15)
            for c in range(8):
                fabc = (-2j * np.trace((T[a] @ T[b] - T[b] @ T[a]) @ T[c])).real
                dabc = (2 * np.trace((T[a] @ T[b] + T[b] @ T[a]) @ T[c])).real
                assert fabc == pytest.approx(f_ref[a, b, c], abs=1e-14)
                assert dabc == pytest.approx(d_ref[a, b, c], abs=1e-14)


def test_proj_is_the_generator_part():
    """Proj[exp(i eps X)] = eps X + O(eps^3): the reading of [.]_ah; exp from scipy."""
    rng = np.random.default_rng(1)
    T = [oracle.generator(a) for a in range(8)]
    for eps in (1e-2, 1e-3):
        x = rng.normal(size=8)
        X = sum(x[a] * T[a] for a in range(8))
        M = scipy.linalg.expm(1j * eps * X)
        p = oracle.proj(M)
        assert np.max(np.abs(p - eps * x)) < 5 * eps ** 3 * np.max(np.abs(x)) ** 3
    # Proj of a Hermitian matrix is zero, of the identity too
    H = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
    H = H + H.conj().T
    assert np.max(np.abs(oracle.proj(H))) < 1e-15


@pytest.mark.parametrize("scale", [1e-4, 0.05, 0.7, 3.0, 12.0])
def test_exponential_matches_scipy(scale):
    rng = np.random.default_rng(int(scale * 1000))
    T = [oracle.generator(a) for a in range(8)]
    for _ in range(5):
        x = rng.normal(size=8)
        X = sum(x[a] * T[a] for a in range(8))
        ref = scipy.linalg.expm(1j * scale * X)
        got = oracle.expi(x, scale)
        assert np.max(np.abs(got - ref)) < 1e-14 * max(1.0, scale)
        assert np.max(np.abs(got @ got.conj().T - np.eye(3))) < 1e-14 * max(1.0, scale)
        assert abs(np.linalg.det(got) - 1) < 1e-14 * max(1.0, scale)


def test_initial_colour_vectors_and_casimirs():
    """Q_0 as printed ([eq:initq0], 6 significant digits) and the exact classical
    Casimirs q2(F)=4, q3(F)=10/3, q2(A)=24, q3(A)=0; q3 also evaluated with the
    printed d table, independently of the oracle's 4 Tr Q^3."""
    pv = paper_values()
    _, d = golden_tables()
    for rep, key, q2ref, q3ref in ((0, "q0_fundamental", 4.0, 10.0 / 3.0), (1, "q0_adjoint", 24.0, 0.0)):
        q = oracle.q0(rep)
        assert np.max(np.abs(q - np.array(pv[key]["value"]))) < 0.5e-5
        q2, q3 = oracle.casimirs(q)
        assert q2 == pytest.approx(q2ref, abs=1e-14)
        assert q3 == pytest.approx(q3ref, abs=1e-14)
        assert np.einsum("abc,a,b,c->", d, q, q, q) == pytest.approx(q3ref, abs=1e-13)
    c = pv["casimirs"]
    assert c["q2_F"] == 4.0 and c["q3_F_num"] / c["q3_F_den"] == pytest.approx(10 / 3)


def test_classical_casimir_formulas():
    """q2 = D_R C2 and q3 = D_R C3 for SU(3) ([eq:q23c23]) give the printed values."""
    Nc = 3
    q2F, q3F = (Nc ** 2 - 1) / 2, (Nc ** 2 - 4) * (Nc ** 2 - 1) / (4 * Nc)
    q2A = Nc * (Nc ** 2 - 1)
    assert (q2F, q3F, q2A) == (4.0, 10.0 / 3.0, 24)
    C2F, C2A = (Nc ** 2 - 1) / (2 * Nc), Nc
    assert (q2A / 8) / (q2F / 3) == pytest.approx(C2A / C2F)
    pv = paper_values()["casimir_scaling"]
    assert q2A / q2F == pv["raw_A_over_F"]
    assert C2A / C2F == pv["div_DR_A_over_F"]


def test_running_coupling_sec_VII_A():
    pv = paper_values()["running_coupling"]
    a = oracle.alpha_s(pv["Qs_GeV"], pv["nf"], pv["lambda_qcd_GeV"])
    assert a == pytest.approx(pv["alpha_s"], abs=5e-4)
    assert math.sqrt(4 * math.pi * a) == pytest.approx(pv["g"], abs=5e-3)
