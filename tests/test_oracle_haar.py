"""Colour charges sampled with the Haar measure (Sec. IV.B): the n-point
functions of [eq:qnpointfct_main] hold, and every sample keeps the classical
Casimirs of its representation."""
import numpy as np
import pytest

import oracle
from test_oracle_algebra import golden_tables

TR = {0: 0.5, 1: 3.0}
AR = {0: 1.0, 1: 0.0}


@pytest.mark.parametrize("rep", [0, 1])
def test_haar_npoint_functions(rep):
    n = 200_000
    P = oracle.particles_init(16, n, 1234 + rep, 0.0, 0.0, True, rep)
    Q = P[:, 6:14]
    _, d = golden_tables()
    q2 = np.sum(Q * Q, 1)
    q3 = np.einsum("abc,na,nb,nc->n", d, Q, Q, Q)
    q2ref, q3ref = oracle.casimirs(oracle.q0(rep))
    assert np.max(np.abs(q2 - q2ref)) < 1e-12
    assert np.max(np.abs(q3 - q3ref)) < 1e-11
    # one-point function: zero
    se = np.sqrt(q2ref / 8 / n)
    assert np.all(np.abs(Q.mean(0)) < 5 * se)
    # two-point function: T_R delta_ab
    C2 = Q.T @ Q / n
    target = TR[rep] * np.eye(8)
    se2 = np.sqrt(np.mean((Q[:, :, None] * Q[:, None, :] - C2) ** 2, axis=0) / n)
    assert np.all(np.abs(C2 - target) < 5 * se2 + 1e-12)
    # three-point function: (A_R/4) d_abc
    C3 = np.einsum("na,nb,nc->abc", Q, Q, Q) / n
    X = np.einsum("na,nb,nc->nabc", Q[:20000], Q[:20000], Q[:20000])
    se3 = X.std(0) / np.sqrt(n)
    assert np.all(np.abs(C3 - AR[rep] / 4 * d) < 6 * se3 + 1e-12)


def test_particle_positions_and_momenta():
    N, n = 32, 50_000
    P = oracle.particles_init(N, n, 99, 0.1, 0.3, True, 0)
    for col in (0, 1):
        assert P[:, col].min() >= 0 and P[:, col].max() < N
        assert abs(P[:, col].mean() - N / 2) < 5 * N / np.sqrt(12 * n)
    pt = np.hypot(P[:, 3], P[:, 4])
    assert np.allclose(pt, P[:, 19], atol=1e-15)
    assert pt.min() >= 0.1 and pt.max() < 0.3
    assert abs(P[:, 3].mean()) < 5 * 0.3 / np.sqrt(n)
    assert np.all(P[:, 2] == 0) and np.all(P[:, 5] == 0)
    assert np.array_equal(P[:, 14], np.floor(P[:, 0] + 0.5) % N)
