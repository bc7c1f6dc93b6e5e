"""Pins of the oracle's alternative colour update (Sec. III.B): the charge
follows dQ/dt = i[Q, A_x v_x + A_y v_y + phi v_eta] with a A_i = -i log U_i
at the link midpoints, stepped by explicit Euler.

  * the matrix logarithm against scipy's logm and against the oracle's own
    exponential (round trip);
  * closed forms of the Euler recursion for commuting (Abelian) links and
    scalar: the transverse part (sign, nearest-midpoint link, velocity) and
    the rapidity part (phi at the grid point, v_eta = p^eta / p^tau);
  * explicit Euler on a rotation grows |Q|^2 by dt^2 |[Q, M]|^2 per step, so
    the Casimir drift at fixed tau is first order in dt (the CPIC rotation
    keeps it at rounding level);
  * the paper's cross-check: both colour updates give the same broadening
    within the ensemble's statistical error.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import inputs
import oracle

PCOL = {c: k for k, c in enumerate(oracle.COLUMNS)}


def comps(X):
    return np.array([2 * np.trace(oracle.generator(a) @ X).real for a in range(8)])


@pytest.mark.parametrize("eps", [0.05, 0.6, 1.5, 2.5])
def test_link_generator_against_scipy_logm(eps):
    rng = np.random.default_rng(int(eps * 100))
    for U in inputs.su3_near_identity(rng, (20,), eps):
        got = oracle.link_generator(U)
        want = comps(-1j * scipy.linalg.logm(U))
        assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, np.max(np.abs(want)))
        # exp(i a) = U up to a centre element: the principal logarithm of a
        # far-from-identity link can carry a trace 2 pi k / 3 that the
        # traceless generator drops (it commutes with every charge)
        Z = oracle.expi(got) @ U.conj().T
        w = Z[0, 0]
        assert np.max(np.abs(Z - w * np.eye(3))) < 1e-12 and abs(w ** 3 - 1) < 1e-12


def frozen_state(N):
    return oracle.empty_state(N)


def step_particles(N, n, n_form, dt, mhat, st, P, mode):
    E = np.ascontiguousarray(st["E"])
    pi = np.ascontiguousarray(st["pi"])
    return oracle.lib().orc_particles_step(N, n, n_form, dt, mhat, 0, mode, oracle._ptr(st["U"]),
                                           oracle._ptr(st["phi"]), oracle._ptr(E), oracle._ptr(E),
                                           oracle._ptr(pi), oracle._ptr(pi), P.shape[0], oracle._ptr(P), None)


def one_particle(N, x, y, px, py, q):
    P = np.zeros((1, oracle.NCOL))
    P[0, PCOL["x"]], P[0, PCOL["y"]] = x, y
    P[0, PCOL["px"]], P[0, PCOL["py"]] = px, py
    P[0, PCOL["cx"]], P[0, PCOL["cy"]] = math.floor(x + 0.5) % N, math.floor(y + 0.5) % N
    P[0, PCOL["Q1"]:PCOL["Q1"] + 8] = q
    return P


@pytest.mark.parametrize("axis,p,x0", [(0, 0.7, 0.3), (0, -0.45, 4.8), (1, 0.55, 2.7), (1, -0.6, 0.2)])
def test_transverse_euler_closed_form(axis, p, x0):
    """Links along `axis` exp(i alpha(s) T3) that depend only on the coordinate
    s along it (no plaquette, no field), Q_0 = T1, motion along the axis:
    each Euler step multiplies q1 + i q2 by 1 + i dt alpha(floor(s_n)) v."""
    N, dt, mhat, steps, n_form = 6, 0.125, 0.3, 60, 2
    st = frozen_state(N)
    alpha = np.array([0.3, -1.1, 0.8, 2.0, -0.4, 0.6])
    for k in range(N):
        Uk = np.diag(np.exp(1j * alpha[k] * np.array([0.5, -0.5, 0.0])))
        if axis == 0:
            st["U"][0, :, k] = Uk
        else:
            st["U"][1, k, :] = Uk
    q = np.zeros(8)
    q[0] = 1.0
    other = 2.3 if axis == 0 else 3.6   # the other coordinate: NGP and floor differ
    P = one_particle(N, x0, other, p, 0.0, q) if axis == 0 else one_particle(N, other, x0, 0.0, p, q)
    v = p / math.sqrt(p * p + mhat * mhat)
    z, s_ = 1.0 + 0j, x0
    for n in range(n_form, n_form + steps):
        assert step_particles(N, n, n_form, dt, mhat, st, P, 1) == 0
        z *= 1 + 1j * dt * alpha[math.floor(s_) % N] * v
        s_ = (s_ + dt * v) % N
    Q = P[0, PCOL["Q1"]:PCOL["Q1"] + 8]
    assert abs(Q[0] - z.real) < 1e-13 and abs(Q[1] - z.imag) < 1e-13
    assert np.max(np.abs(Q[2:])) < 1e-15
    assert abs(P[0, PCOL["x" if axis == 0 else "y"]] - s_) < 1e-12


def test_rapidity_euler_closed_form():
    """phi = f T3 at every site, trivial links, Q_0 = T1, p^eta != 0: each
    Euler step multiplies q1 + i q2 by 1 + i dt f p^eta_n / p^tau_n, with the
    particle's own p^eta_n, p^tau_n (which relax without fields)."""
    N, dt, mhat, f = 5, 0.125, 0.4, 0.9
    st = frozen_state(N)
    st["phi"][:, :, 2] = f
    q = np.zeros(8)
    q[0] = 1.0
    P = one_particle(N, 1.2, 3.1, 0.2, 0.1, q)
    P[0, PCOL["peta"]] = 0.8
    z = 1.0 + 0j
    for n in range(3, 40):
        t = n * dt
        px, py, pe = P[0, PCOL["px"]], P[0, PCOL["py"]], P[0, PCOL["peta"]]
        ptau = math.sqrt(px * px + py * py + (t * pe) ** 2 + mhat * mhat)
        z *= 1 + 1j * dt * f * pe / ptau
        assert step_particles(N, n, 3, dt, mhat, st, P, 1) == 0
    Q = P[0, PCOL["Q1"]:PCOL["Q1"] + 8]
    assert abs(Q[0] - z.real) < 1e-13 and abs(Q[1] - z.imag) < 1e-13
    assert abs(z) > 1.0001  # the Euler growth is visible


def casimir_drift(dt, color, tau=1.0):
    N = 12
    st = oracle.mv_initial_condition(N, 6.0 * N / 32, 2.0, 0.2, 10.0, 1, 17)
    P = oracle.particles_init(N, 200, 18, 0.2, 0.6, True, 0)
    r = oracle.Run(N, dt, st, P, mhat=0.3, n_form=1, color=color)
    for _ in range(int(round(tau / dt))):
        r.step()
    assert r.errors == 0
    q2 = np.sum(r.P[:, PCOL["Q1"]:PCOL["Q1"] + 8] ** 2, axis=1)
    q20 = float(np.dot(oracle.q0(0), oracle.q0(0)))
    return float(np.mean(q2 / q20 - 1)), float(np.max(np.abs(q2 / q20 - 1)))


def test_casimir_drift_is_first_order_in_dt():
    """On this coarse lattice (g^2 mu a = 1.9) the links are far from 1 and the
    drift is 20 % after one lattice time unit at dt = a/8; it halves with dt
    (measured ratios 1.96 and 2.01 for dt = a/8, a/16, a/32)."""
    m1, _ = casimir_drift(0.125, "log")
    m2, _ = casimir_drift(0.0625, "log")
    m3, _ = casimir_drift(0.03125, "log")
    assert m1 > 0 and m2 > 0 and m3 > 0  # Euler on a rotation only grows |Q|
    assert 1.8 < m1 / m2 < 2.2 and 1.8 < m2 / m3 < 2.2
    _, c = casimir_drift(0.125, "cpic")
    assert c < 1e-12


def test_both_colour_updates_give_the_same_broadening():
    """16^2 MV event, 1500 charm-like quarks with p_T up to 2 (hat units),
    dt = a/16: <dp_T^2> and <dp_L^2> of the two colour updates agree within
    four standard errors of their per-particle difference."""
    N, dt = 16, 0.0625
    st = oracle.mv_initial_condition(N, 6.0 * N / 32, 2.0, 0.2, 10.0, 1, 23)
    P = oracle.particles_init(N, 1500, 24, 0.0, 2.0, True, 0)
    runs = {}
    for color in ("cpic", "log"):
        r = oracle.Run(N, dt, st, P, mhat=0.4, n_form=2, color=color)
        for _ in range(96):
            r.step()
        runs[color] = r
    pt0 = P[:, PCOL["pt0"]] ** 2
    dT = {c: r.P[:, PCOL["px"]] ** 2 + r.P[:, PCOL["py"]] ** 2 - pt0 for c, r in runs.items()}
    d = dT["log"] - dT["cpic"]
    assert abs(d.mean()) < 4 * d.std() / math.sqrt(len(d))
    assert abs(d.mean()) < 0.1 * abs(dT["cpic"].mean())
