"""Pins of the oracle's field leapfrog (Sec. II.A) against brute force,
closed forms and exact invariants:
  * the kick forces are minus the gradient of one lattice Hamiltonian
    (central finite differences on a 4x4 lattice);
  * Abelian and free-scalar configurations with closed-form forces, the
    commutator term checked with the printed f_abc table;
  * the Gauss constraint is conserved; links stay unitary with unit determinant;
  * the update commutes with lattice gauge transformations;
  * in frozen-time mode the energy error scales as dt^2;
  * the one-nucleus initial condition is pure gauge and stays at zero energy.
"""
import math

import numpy as np
import pytest

import inputs
import oracle
from test_oracle_algebra import golden_tables


def comps(X, T):
    return np.array([2 * np.trace(T[a] @ X).real for a in range(8)])


def mat(x, T):
    return sum(x[a] * T[a] for a in range(8))


def total_energy(N, t, st):
    return oracle.energy(N, t, st["U"], st["phi"], st["E"], st["pi"]).sum()


def test_forces_are_minus_gradient_of_hamiltonian_4x4():
    N, t, h = 4, 1.3, 1e-5
    st = inputs.random_state(N, 7, eps_link=0.6, phi_scale=0.5)
    T = [oracle.generator(a) for a in range(8)]
    FE, Fp = oracle.forces(N, t, st["U"], st["phi"])
    scaleE = np.max(np.abs(FE))
    for i in range(2):
        for y in range(N):
            for x in range(N):
                for a in range(8):
                    Hs = []
                    for sgn in (+1, -1):
                        s2 = {k: v.copy() for k, v in st.items()}
                        s2["U"][i, y, x] = oracle.expi(np.eye(8)[a], sgn * h) @ st["U"][i, y, x]
                        Hs.append(total_energy(N, t, s2))
                    dH = (Hs[0] - Hs[1]) / (2 * h)
                    assert abs(FE[i, y, x, a] + dH) < 1e-8 * scaleE, (i, y, x, a)
    scaleP = np.max(np.abs(Fp))
    for y in range(N):
        for x in range(N):
            for a in range(8):
                Hs = []
                for sgn in (+1, -1):
                    s2 = {k: v.copy() for k, v in st.items()}
                    s2["phi"][y, x, a] += sgn * h
                    Hs.append(total_energy(N, t, s2))
                dH = (Hs[0] - Hs[1]) / (2 * h)
                assert abs(Fp[y, x, a] + dH) < 1e-8 * scaleP


def test_abelian_plaquette_force_closed_form():
    """U_1(x) = exp(i theta(x) T^3), U_2 = 1, phi = 0: the plaquettes are
    exp(i dtheta T^3) with Proj^3 = 2 sin(dtheta/2)."""
    N, t = 6, 0.7
    rng = np.random.default_rng(3)
    theta = rng.uniform(-1, 1, (N, N))   # [y, x]
    st = oracle.empty_state(N)
    for y in range(N):
        for x in range(N):
            z = np.zeros(8); z[2] = theta[y, x]
            st["U"][0, y, x] = oracle.expi(z)
    FE, Fp = oracle.forces(N, t, st["U"], st["phi"])
    for y in range(N):
        for x in range(N):
            yp, ym, xm = (y + 1) % N, (y - 1) % N, (x - 1) % N
            f1 = -t * (2 * math.sin((theta[y, x] - theta[yp, x]) / 2) + 2 * math.sin((theta[y, x] - theta[ym, x]) / 2))
            f2 = -t * (2 * math.sin((theta[yp, x] - theta[y, x]) / 2)
                       + 2 * math.sin((theta[y, xm] - theta[yp, xm]) / 2))
            e1 = np.zeros(8); e1[2] = f1
            e2 = np.zeros(8); e2[2] = f2
            assert np.allclose(FE[0, y, x], e1, atol=1e-14)
            assert np.allclose(FE[1, y, x], e2, atol=1e-14)
    assert np.max(np.abs(Fp)) == 0


def test_free_scalar_forces_closed_form():
    """U = 1: pi force = lattice Laplacian of phi / t, E force = (1/t) i[phi(x+i), phi(x)]
    with (i[A,B])^c = -f_abc A^a B^b from the printed Table I."""
    N, t = 5, 0.9
    f, _ = golden_tables()
    rng = np.random.default_rng(4)
    st = oracle.empty_state(N)
    st["phi"] = rng.normal(size=(N, N, 8))
    FE, Fp = oracle.forces(N, t, st["U"], st["phi"])
    ph = st["phi"]
    lap = (np.roll(ph, 1, 0) + np.roll(ph, -1, 0) + np.roll(ph, 1, 1) + np.roll(ph, -1, 1) - 4 * ph) / t
    assert np.allclose(Fp, lap, atol=1e-13)
    for i, axis in ((0, 1), (1, 0)):
        fwd = np.roll(ph, -1, axis)
        ref = -np.einsum("abc,yxa,yxb->yxc", f, fwd, ph) / t
        assert np.allclose(FE[i], ref, atol=1e-13)


def test_gauss_law_conserved_random_state():
    N, dt = 8, 0.125
    st = inputs.random_state(N, 11, eps_link=0.5)
    G0 = oracle.gauss(N, st["U"], st["phi"], st["E"], st["pi"])
    assert np.max(np.abs(G0)) > 0.1          # a generic state violates Gauss ...
    for n in range(1, 31):                    # ... and the update keeps G fixed
        oracle.field_step(N, n, dt, st)
        G = oracle.gauss(N, st["U"], st["phi"], st["E"], st["pi"])
        assert np.max(np.abs(G - G0)) < 1e-12


def test_mv_event_gauss_unitarity():
    N = 16
    st = oracle.mv_initial_condition(N, 6.0 * N / 64, 2.0, 0.2, 10.0, 2, 21)
    for n in range(200):
        oracle.field_step(N, n, 0.125, st)
    G = oracle.gauss(N, st["U"], st["phi"], st["E"], st["pi"])
    assert np.max(np.abs(st["E"])) > 1e-2
    assert np.max(np.abs(G)) < 1e-12
    mu, md = oracle.unitarity(N, st["U"])
    assert mu < 1e-13 and md < 1e-13


def apply_gauge(st, V, T):
    N = st["phi"].shape[0]
    out = {k: v.copy() for k, v in st.items()}
    Vd = np.conj(np.swapaxes(V, -1, -2))
    Vx1 = np.roll(V, -1, axis=1)      # V(x + e1)
    Vx2 = np.roll(V, -1, axis=0)      # V(x + e2)
    out["U"][0] = V @ st["U"][0] @ np.conj(np.swapaxes(Vx1, -1, -2))
    out["U"][1] = V @ st["U"][1] @ np.conj(np.swapaxes(Vx2, -1, -2))
    for key in ("phi", "pi"):
        for y in range(N):
            for x in range(N):
                out[key][y, x] = comps(V[y, x] @ mat(st[key][y, x], T) @ Vd[y, x], T)
    for i in range(2):
        for y in range(N):
            for x in range(N):
                out["E"][i, y, x] = comps(V[y, x] @ mat(st["E"][i, y, x], T) @ Vd[y, x], T)
    return out


def test_gauge_covariance_fields_and_particles():
    N, dt, steps = 6, 0.125, 12
    T = [oracle.generator(a) for a in range(8)]
    st = inputs.random_state(N, 5, eps_link=0.4)
    V = inputs.haar_su3(np.random.default_rng(6), (N, N))
    gst = apply_gauge(st, V, T)
    P = inputs.random_particles(64, N, 8, p_scale=0.8)
    gP = P.copy()
    for p in range(P.shape[0]):
        cx, cy = int(P[p, 14]), int(P[p, 15])
        gP[p, 6:14] = comps(V[cy, cx] @ mat(P[p, 6:14], T) @ V[cy, cx].conj().T, T)
    runs = []
    for s, parts in ((st, P), (gst, gP)):
        r = oracle.Run(N, dt, s, parts, mhat=0.3, n_form=1, n0=1)
        for _ in range(steps):
            r.step()
        runs.append(r)
    a, b = runs
    assert a.errors == 0 and b.errors == 0
    expect = apply_gauge(a.st, V, T)
    for key in ("U", "phi", "E", "pi"):
        assert np.max(np.abs(expect[key] - b.st[key])) < 1e-11, key
    # positions, momenta, cells and rapidity are gauge invariant
    assert np.max(np.abs(a.P[:, :6] - b.P[:, :6])) < 1e-11
    assert np.array_equal(a.P[:, 14:16], b.P[:, 14:16])
    for p in range(P.shape[0]):
        cx, cy = int(a.P[p, 14]), int(a.P[p, 15])
        q = comps(V[cy, cx] @ mat(a.P[p, 6:14], T) @ V[cy, cx].conj().T, T)
        assert np.max(np.abs(q - b.P[p, 6:14])) < 1e-11


def frozen_energy_drift(dt, total=2.0, t_fixed=1.0):
    N = 6
    st = inputs.random_state(N, 13, eps_link=0.25, e_scale=0.1, phi_scale=0.15, pi_scale=0.1)
    Hs = []
    E_prev, pi_prev = st["E"].copy(), st["pi"].copy()
    U_prev, phi_prev = st["U"].copy(), st["phi"].copy()
    for n in range(int(round(total / dt))):
        oracle.field_step(N, n, dt, st, t_fixed=t_fixed)
        Eav = np.ascontiguousarray(0.5 * (E_prev + st["E"]))
        piav = np.ascontiguousarray(0.5 * (pi_prev + st["pi"]))
        Hs.append(oracle.energy(N, t_fixed, U_prev, phi_prev, Eav, piav).sum())
        E_prev, pi_prev = st["E"].copy(), st["pi"].copy()
        U_prev, phi_prev = st["U"].copy(), st["phi"].copy()
    Hs = np.array(Hs)
    return np.max(np.abs(Hs - Hs[0])), Hs[0]


def test_energy_error_scales_as_dt_squared_frozen_time():
    d1, H0 = frozen_energy_drift(0.1)
    d2, _ = frozen_energy_drift(0.05)
    d3, _ = frozen_energy_drift(0.025)
    assert d1 < 1e-2 * H0
    assert 3.5 < d1 / d2 < 4.5 and 3.5 < d2 / d3 < 4.5


def test_one_nucleus_limit_is_pure_gauge():
    N = 12
    st = oracle.mv_initial_condition(N, 6.0 * N / 64, 2.0, 0.2, 10.0, 2, 4, rho_scale_B=0.0,
                                     keep_nuclei=True)
    assert np.max(np.abs(st["U"] - st["UA"])) < 1e-13
    assert np.max(np.abs(st["pi"])) < 1e-14
    Ufree = st["UA"]
    for y in range(N):
        for x in range(N):
            P12 = Ufree[0, y, x] @ Ufree[1, y, (x + 1) % N] @ Ufree[0, (y + 1) % N, x].conj().T @ Ufree[1, y, x].conj().T
            assert np.max(np.abs(P12 - np.eye(3))) < 1e-13
    P = oracle.particles_init(N, 200, 3, 0.2, 0.2, True, 0)
    r = oracle.Run(N, 0.125, st, P, mhat=0.5, n_form=0)
    for n in range(40):
        r.step()
        H = oracle.energy(N, r.n * 0.125, r.st["U"], r.st["phi"], r.st["E"], r.st["pi"]).sum()
        assert abs(H) < 1e-12
    assert np.max(np.abs(r.P[:, 3:6] - P[:, 3:6])) < 1e-13
