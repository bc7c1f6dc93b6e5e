"""Pins of the SU(2) oracle (the SU(2) variant of Sec. II.A, III.B and IV.A).

  * the generators are the Pauli matrices over two and the exponential has
    the closed form cos(|x|/2) + i sin(|x|/2) x.sigma/|x|;
  * the kick forces are minus the gradient of the lattice Hamiltonian
    (central finite differences on a 4x4 lattice);
  * the Gauss residual is conserved from a random state; an MV event keeps
    it at rounding and its links unitary;
  * the update commutes with lattice gauge transformations;
  * frozen-time energy error scales as dt^2;
  * the tau = 0 links solve the initial-link condition; with one nucleus they
    are its pure-gauge links and pi(0) = 0;
  * Darboux charges: |Q|^2 = q2 exactly, <Q^a> = 0, <Q^a Q^b> = q2/3 delta^ab;
  * static limit and Casimir scaling: adjoint over fundamental broadening is
    q2(A)/q2(F) = 4, i.e. 8/3 after the division by D_R of Sec. VII.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import su2

SIG = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]


def su2_random(rng, shape, eps):
    """exp(i eps x.sigma/2) with Gaussian x (scipy expm)."""
    x = rng.normal(size=shape + (3,))
    H = np.einsum("...a,aij->...ij", x, np.array(SIG)) / 2
    out = np.zeros(shape + (2, 2), complex)
    for idx in np.ndindex(*shape):
        out[idx] = scipy.linalg.expm(1j * eps * H[idx])
    return out


def random_state(N, seed, eps=0.5, scale=0.3):
    rng = np.random.default_rng(seed)
    st = su2.empty_state(N)
    st["U"] = su2_random(rng, (2, N, N), eps)
    st["phi"] = scale * rng.normal(size=(N, N, 3))
    st["E"] = scale * rng.normal(size=(2, N, N, 3))
    st["pi"] = scale * rng.normal(size=(N, N, 3))
    return st


def comps(X):
    return np.array([np.trace(SIG[a] @ X).real for a in range(3)])


def mat(x):
    return sum(x[a] * SIG[a] / 2 for a in range(3))


def test_generators_and_exponential_closed_form():
    for a in range(3):
        assert np.allclose(su2.generator(a), SIG[a] / 2)
    rng = np.random.default_rng(1)
    for _ in range(20):
        x = rng.normal(size=3) * 1.7
        r = np.linalg.norm(x)
        want = math.cos(r / 2) * np.eye(2) + 1j * math.sin(r / 2) * sum(x[a] * SIG[a] for a in range(3)) / r
        assert np.max(np.abs(su2.expi(x) - want)) < 1e-14
        # Proj of exp(i x.T) = 2 sin(|x|/2) x/|x|
        assert np.allclose(su2.proj(want), 2 * math.sin(r / 2) * x / r, atol=1e-14)


def energy_total(N, t, st):
    return su2.energy(N, t, st["U"], st["phi"], st["E"], st["pi"]).sum()


def test_forces_are_minus_gradient_of_hamiltonian_4x4():
    N, t, h = 4, 1.1, 1e-5
    st = random_state(N, 2, eps=0.8, scale=0.5)
    FE, Fp = su2.forces(N, t, st["U"], st["phi"])
    sE, sP = np.max(np.abs(FE)), np.max(np.abs(Fp))
    for i in range(2):
        for y in range(N):
            for x in range(N):
                for a in range(3):
                    Hs = []
                    for sgn in (+1, -1):
                        s2 = {k: v.copy() for k, v in st.items()}
                        s2["U"][i, y, x] = su2.expi(np.eye(3)[a], sgn * h) @ st["U"][i, y, x]
                        Hs.append(energy_total(N, t, s2))
                    assert abs(FE[i, y, x, a] + (Hs[0] - Hs[1]) / (2 * h)) < 1e-8 * sE
    for y in range(N):
        for x in range(N):
            for a in range(3):
                Hs = []
                for sgn in (+1, -1):
                    s2 = {k: v.copy() for k, v in st.items()}
                    s2["phi"][y, x, a] += sgn * h
                    Hs.append(energy_total(N, t, s2))
                assert abs(Fp[y, x, a] + (Hs[0] - Hs[1]) / (2 * h)) < 1e-8 * sP


def test_gauss_law_conserved_random_state():
    N = 8
    st = random_state(N, 3)
    G0 = su2.gauss(N, st["U"], st["phi"], st["E"], st["pi"])
    assert np.max(np.abs(G0)) > 0.1
    for n in range(1, 31):
        su2.field_step(N, n, 0.125, st)
        assert np.max(np.abs(su2.gauss(N, st["U"], st["phi"], st["E"], st["pi"]) - G0)) < 1e-12


def test_mv_event_gauss_and_unitarity():
    N = 16
    st = su2.mv_initial_condition(N, 3.0, 2.0, 0.2, 10.0, 2, 5)
    for n in range(100):
        su2.field_step(N, n, 0.125, st)
    assert np.max(np.abs(st["E"])) > 0.1
    assert np.max(np.abs(su2.gauss(N, st["U"], st["phi"], st["E"], st["pi"]))) < 1e-12
    U = st["U"].reshape(-1, 2, 2)
    assert np.max(np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - np.eye(2))) < 1e-13
    assert np.max(np.abs(np.linalg.det(U) - 1)) < 1e-13


def apply_gauge(st, Vg):
    out = {k: v.copy() for k, v in st.items()}
    Vd = np.conj(np.swapaxes(Vg, -1, -2))
    for i, ax in ((0, 1), (1, 0)):
        out["U"][i] = Vg @ st["U"][i] @ np.conj(np.swapaxes(np.roll(Vg, -1, axis=ax), -1, -2))
    N = st["phi"].shape[0]
    for y in range(N):
        for x in range(N):
            for key in ("phi", "pi"):
                out[key][y, x] = comps(Vg[y, x] @ mat(st[key][y, x]) @ Vd[y, x])
            for i in range(2):
                out["E"][i, y, x] = comps(Vg[y, x] @ mat(st["E"][i, y, x]) @ Vd[y, x])
    return out


def test_gauge_covariance_fields_and_particles():
    N, dt, steps = 6, 0.125, 12
    st = random_state(N, 4, eps=0.6)
    Vg = su2_random(np.random.default_rng(5), (N, N), 2.0)
    gst = apply_gauge(st, Vg)
    rng = np.random.default_rng(6)
    P = np.zeros((40, oracle.NCOL))
    P[:, 0:2] = rng.uniform(0, N, (40, 2))
    P[:, 3:5] = rng.normal(0, 0.8, (40, 2))
    P[:, 6:9] = rng.normal(size=(40, 3))
    P[:, 14:16] = np.floor(P[:, 0:2] + 0.5) % N
    gP = P.copy()
    for p in range(40):
        cx, cy = int(P[p, 14]), int(P[p, 15])
        gP[p, 6:9] = comps(Vg[cy, cx] @ mat(P[p, 6:9]) @ Vg[cy, cx].conj().T)
    runs = []
    for s, parts in ((st, P), (gst, gP)):
        r = su2.Run(N, dt, s, parts, mhat=0.3, n_form=1, n0=1)
        for _ in range(steps):
            r.step()
        runs.append(r)
    a, b = runs
    assert a.errors == 0 and b.errors == 0
    want = apply_gauge(a.st, Vg)
    for key in ("U", "phi", "E", "pi"):
        assert np.max(np.abs(want[key] - b.st[key])) < 1e-11, key
    assert np.max(np.abs(a.P[:, :6] - b.P[:, :6])) < 1e-11
    for p in range(40):
        cx, cy = int(a.P[p, 14]), int(a.P[p, 15])
        q = comps(Vg[cy, cx] @ mat(a.P[p, 6:9]) @ Vg[cy, cx].conj().T)
        assert np.max(np.abs(q - b.P[p, 6:9])) < 1e-11


def frozen_drift(dt, total=2.0, t_fixed=1.0):
    N = 6
    st = random_state(N, 7, eps=0.3, scale=0.1)
    Hs, E_prev, pi_prev = [], st["E"].copy(), st["pi"].copy()
    U_prev, phi_prev = st["U"].copy(), st["phi"].copy()
    for n in range(int(round(total / dt))):
        su2.field_step(N, n, dt, st, t_fixed=t_fixed)
        Eav = np.ascontiguousarray(0.5 * (E_prev + st["E"]))
        piav = np.ascontiguousarray(0.5 * (pi_prev + st["pi"]))
        Hs.append(su2.energy(N, t_fixed, U_prev, phi_prev, Eav, piav).sum())
        E_prev, pi_prev, U_prev, phi_prev = st["E"].copy(), st["pi"].copy(), st["U"].copy(), st["phi"].copy()
    Hs = np.array(Hs)
    return np.max(np.abs(Hs - Hs[0]))


def test_energy_error_scales_as_dt_squared_frozen_time():
    d1, d2, d3 = frozen_drift(0.1), frozen_drift(0.05), frozen_drift(0.025)
    assert 3.0 < d1 / d2 < 5.0 and 3.0 < d2 / d3 < 5.0


def test_initial_links_solve_the_condition_and_one_nucleus_limit():
    N = 12
    st = su2.mv_initial_condition(N, 2.5, 2.0, 0.2, 10.0, 3, 8, keep_nuclei=True)
    UA, UB, U = st["UA"], st["UB"], st["U"]
    W = UA + UB
    M = W @ (np.eye(2) + np.conj(np.swapaxes(U, -1, -2)))
    A = (M - np.conj(np.swapaxes(M, -1, -2))) / 2
    A = A - np.trace(A, axis1=-2, axis2=-1)[..., None, None] / 2 * np.eye(2)
    assert np.max(np.abs(A)) < 1e-13
    Uf = U.reshape(-1, 2, 2)
    assert np.max(np.abs(Uf @ np.conj(np.swapaxes(Uf, -1, -2)) - np.eye(2))) < 1e-14
    one = su2.mv_initial_condition(N, 2.5, 2.0, 0.2, 10.0, 3, 8, rho_scale_B=0.0, keep_nuclei=True)
    assert np.max(np.abs(one["U"] - one["UA"])) < 1e-13
    assert np.max(np.abs(one["pi"])) < 1e-13


def test_darboux_charges():
    for rep, q2 in ((0, 1.5), (1, 6.0)):
        assert su2.q2(rep) == q2
        P = su2.particles_init(8, 20000, 9, 0.0, 0.0, True, rep)
        Q = P[:, 6:9]
        assert np.max(np.abs(np.sum(Q ** 2, axis=1) - q2)) < 1e-12
        assert np.max(np.abs(P[:, 9:14])) == 0
        n = len(Q)
        assert np.all(np.abs(Q.mean(axis=0)) < 5 * math.sqrt(q2 / 3 / n))
        C = Q.T @ Q / n
        # var of Q_a Q_b for a point uniform on the sphere of radius J: q2^2/15 (a != b), 4 q2^2/45 (a = b)
        for a in range(3):
            for b in range(3):
                want = q2 / 3 if a == b else 0.0
                sd = q2 * math.sqrt((4 / 45 if a == b else 1 / 15) / n)
                assert abs(C[a, b] - want) < 5 * sd


def static_run(rep, N=16, steps=40):
    st = su2.mv_initial_condition(N, 3.0, 2.0, 0.2, 10.0, 2, 12)
    P = su2.particles_init(N, 3000, 13, 0.0, 0.0, True, rep)
    r = su2.Run(N, 0.125, st, P, mhat=math.inf, n_form=0)
    S = np.zeros((N * N, 3, 3))
    for n in range(steps):
        U, phi, Eo, po = r.st["U"].copy(), r.st["phi"].copy(), r.st["E"].copy(), r.st["pi"].copy()
        r.step()
        for s in range(N * N):
            f = su2.particle_fields(N, n, 0.125, s, U, phi, Eo, r.st["E"], po, r.st["pi"])
            S[s] += 0.125 * f[:3]
    return r, P, S


def test_static_limit_and_casimir_scaling():
    rF, PF, S = static_run(0)
    rA, PA, _ = static_run(1)
    N = 16
    sites = (PF[:, 15] * N + PF[:, 14]).astype(int)
    pred = np.einsum("na,nka->nk", PF[:, 6:9], S[sites])
    assert np.max(np.abs(rF.P[:, 3:6] - pred)) < 1e-12 * np.max(np.abs(pred))
    assert np.array_equal(PF[:, :2], PA[:, :2])
    base = np.sum(S[sites, :2] ** 2, axis=(1, 2))
    xF = np.sum(rF.P[:, 3:5] ** 2, 1) / base
    xA = np.sum(rA.P[:, 3:5] ** 2, 1) / base
    ratio = xA.mean() / xF.mean()
    err = ratio * np.hypot(xA.std() / xA.mean(), xF.std() / xF.mean()) / math.sqrt(len(xA))
    assert abs(ratio - 4.0) < 5 * err
    assert abs(ratio * 2 / 3 - 8 / 3) < 5 * err * 2 / 3


def test_clover_magnetic_field_uniform_flux():
    """U_1(x, y) = exp(i theta y T^3), U_2 = 1, theta = 4 pi / N: every
    counter-clockwise plaquette is exp(-i theta T^3), so B_eta^3 = 2 sin(theta/2)."""
    N = 8
    theta = 4 * math.pi / N
    st = su2.empty_state(N)
    for y in range(N):
        st["U"][0, y, :] = su2.expi([0.0, 0.0, theta * y])
    z, zs = np.zeros((2, N, N, 3)), np.zeros((N, N, 3))
    for s in (0, 9, 63):
        f = su2.particle_fields(N, 3, 0.125, s, st["U"], zs, z, z, zs, zs)
        assert np.allclose(f[5], [0.0, 0.0, 2 * math.sin(theta / 2)], atol=1e-14)


def test_colour_rotation_known_links():
    N, dt = 6, 0.125
    rng = np.random.default_rng(2)
    st = su2.empty_state(N)
    st["U"] = su2_random(rng, (2, N, N), 2.5)
    z2, z1 = np.zeros((2, N, N, 3)), np.zeros((N, N, 3))
    Q = rng.normal(size=3)

    def one(x_prev, y_prev, x_new, y_new):
        P = np.zeros((1, oracle.NCOL))
        P[0, 0], P[0, 1] = x_new, y_new
        P[0, 6:9] = Q
        P[0, 14], P[0, 15] = x_prev, y_prev
        P[0, 17] = 1.0
        assert su2.lib().orc2_particles_step(N, 4, 1, dt, 1e9, 0, oracle._ptr(st["U"]), oracle._ptr(z1),
                                             oracle._ptr(z2), oracle._ptr(z2), oracle._ptr(z1), oracle._ptr(z1), 1,
                                             oracle._ptr(P)) == 0
        return P[0, 6:9]

    U1, U2, Qm = st["U"][0], st["U"][1], mat(Q)
    assert np.allclose(one(2, 3, 3.2, 3.0), comps(U1[3, 2].conj().T @ Qm @ U1[3, 2]), atol=1e-13)
    assert np.allclose(one(0, 1, 5.4, 1.0), comps(U1[1, 5] @ Qm @ U1[1, 5].conj().T), atol=1e-13)
    assert np.allclose(one(4, 4, 4.0, 5.1), comps(U2[4, 4].conj().T @ Qm @ U2[4, 4]), atol=1e-13)
    W = U1[1, 1] @ U2[1, 2]
    assert np.allclose(one(1, 1, 2.1, 1.9), comps(W.conj().T @ Qm @ W), atol=1e-13)
