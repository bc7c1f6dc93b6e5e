"""Pins of the oracle's particle push (Sec. III.B):
  * the lattice E/B interpolations in closed form on trivial links;
  * the CPIC colour rotation with known links, one axis and both axes;
  * Casimir conservation of the rotation over many steps [eq:q2_main], [eq:q3_main];
  * the magnetic force does no work: |p_T|^2 grows by exactly dt^2 b^2 |v|^2
    per Euler step in a uniform Abelian B_eta;
  * static (infinite-mass) limit [eq:mombroadhqs]: per particle the momentum is
    the summed Q.E, and over the ensemble <dp^2> = T_F <|sum E dt|^2>;
  * Casimir scaling of the static broadening, adjoint/fundamental = 6
    ([eq:diffcasscaling]);
  * a very heavy dynamical particle reproduces the static p_z, which fixes the
    p^eta equation of [eq:wonginmilne] together with the lab-frame p^z.
"""
import math

import numpy as np
import pytest

import inputs
import oracle


def comps(X, T):
    return np.array([2 * np.trace(T[a] @ X).real for a in range(8)])


def mat(x, T):
    return sum(x[a] * T[a] for a in range(8))


def test_field_interpolation_trivial_links():
    N, n, dt = 7, 5, 0.125
    t = n * dt
    rng = np.random.default_rng(1)
    st = oracle.empty_state(N)
    phi = rng.normal(size=(N, N, 8))
    Eo, En = rng.normal(size=(2, N, N, 8)), rng.normal(size=(2, N, N, 8))
    po, pn = rng.normal(size=(N, N, 8)), rng.normal(size=(N, N, 8))
    for (y, x) in ((0, 0), (3, 6), (6, 2)):
        f = oracle.particle_fields(N, n, dt, y * N + x, st["U"], phi, Eo, En, po, pn)
        xm, ym, xp, yp = (x - 1) % N, (y - 1) % N, (x + 1) % N, (y + 1) % N
        assert np.allclose(f[0], (En[0, y, x] + Eo[0, y, x] + En[0, y, xm] + Eo[0, y, xm]) / (4 * t), atol=1e-14)
        assert np.allclose(f[1], (En[1, y, x] + Eo[1, y, x] + En[1, ym, x] + Eo[1, ym, x]) / (4 * t), atol=1e-14)
        assert np.allclose(f[2], 0.5 * (pn[y, x] + po[y, x]), atol=1e-14)
        assert np.allclose(f[3], -(phi[yp, x] - phi[ym, x]) / (2 * t), atol=1e-14)
        assert np.allclose(f[4], (phi[y, xp] - phi[y, xm]) / (2 * t), atol=1e-14)
        assert np.max(np.abs(f[5])) < 1e-15


def uniform_flux_links(N, k=1):
    """U_1(x, y) = exp(i theta y T^3), U_2 = 1 with theta = 4 pi k / N: every
    counter-clockwise plaquette is exp(-i theta T^3), so B_eta^3 = 2 sin(theta/2)."""
    theta = 4 * math.pi * k / N
    st = oracle.empty_state(N)
    for y in range(N):
        z = np.zeros(8); z[2] = theta * y
        st["U"][0, y, :] = oracle.expi(z)
    return st, theta


def test_clover_magnetic_field_uniform_flux():
    N = 8
    st, theta = uniform_flux_links(N)
    z = np.zeros((2, N, N, 8)); zs = np.zeros((N, N, 8))
    for s in (0, 9, 63):
        f = oracle.particle_fields(N, 3, 0.125, s, st["U"], zs, z, z, zs, zs)
        ref = np.zeros(8); ref[2] = 2 * math.sin(theta / 2)
        assert np.allclose(f[5], ref, atol=1e-14)


def test_colour_rotation_known_links():
    N, dt = 6, 0.125
    T = [oracle.generator(a) for a in range(8)]
    rng = np.random.default_rng(2)
    st = oracle.empty_state(N)
    st["U"] = np.ascontiguousarray(inputs.haar_su3(rng, (2, N, N)))
    z2, z1 = np.zeros((2, N, N, 8)), np.zeros((N, N, 8))
    Q = rng.normal(size=8)

    def one(x_prev, y_prev, x_new, y_new):
        P = np.zeros((1, 20))
        P[0, 0], P[0, 1] = x_new, y_new
        P[0, 6:14] = Q
        P[0, 14], P[0, 15] = x_prev, y_prev
        P[0, 17] = 1.0
        err = oracle.lib().orc_particles_step(N, 4, 1, dt, 1e9, 0, 0, oracle._ptr(st["U"]), oracle._ptr(z1),
                                              oracle._ptr(z2), oracle._ptr(z2), oracle._ptr(z1), oracle._ptr(z1),
                                              1, oracle._ptr(P), None)
        assert err == 0
        return P[0, 6:14]

    U1, U2 = st["U"][0], st["U"][1]
    Qm = mat(Q, T)
    # +x from (2,3) to (3,3): Q <- U_1(c)^+ Q U_1(c)
    assert np.allclose(one(2, 3, 3.2, 3.0), comps(U1[3, 2].conj().T @ Qm @ U1[3, 2], T), atol=1e-13)
    # -x across the periodic edge from (0,1) to (5,1): Q <- U_1(c-1) Q U_1(c-1)^+
    assert np.allclose(one(0, 1, 5.4, 1.0), comps(U1[1, 5] @ Qm @ U1[1, 5].conj().T, T), atol=1e-13)
    # +y
    assert np.allclose(one(4, 4, 4.0, 5.1), comps(U2[4, 4].conj().T @ Qm @ U2[4, 4], T), atol=1e-13)
    # both axes: x first, then y from the intermediate cell
    W = U1[1, 1] @ U2[1, 2]
    assert np.allclose(one(1, 1, 2.1, 1.9), comps(W.conj().T @ Qm @ W, T), atol=1e-13)
    # a jump of two cells is reported
    P = np.zeros((1, 20)); P[0, 0] = 4.0; P[0, 14] = 2; P[0, 17] = 1
    assert oracle.lib().orc_particles_step(N, 4, 1, dt, 1.0, 0, 0, oracle._ptr(st["U"]), oracle._ptr(z1),
                                           oracle._ptr(z2), oracle._ptr(z2), oracle._ptr(z1), oracle._ptr(z1),
                                           1, oracle._ptr(P), None) == 1


def test_casimirs_conserved_by_rotation_many_steps():
    N, dt = 16, 0.125
    st = oracle.mv_initial_condition(N, 6.0 * N / 64, 2.0, 0.2, 10.0, 2, 31)
    P = oracle.particles_init(N, 300, 32, 0.6, 0.6, True, 0)
    q2_0, q3_0 = oracle.casimirs(P[0, 6:14])
    r = oracle.Run(N, dt, st, P, mhat=0.05, n_form=2)
    for _ in range(600):
        r.step()
    assert r.errors == 0
    moved = np.sum(np.abs(r.P[:, 0] - P[:, 0]) > 2)
    assert moved > 100                                        # many cell crossings happened
    assert np.max(np.abs(r.P[:, 2])) > 1e-3                   # and eta rotations
    # the rotation is exact for exactly unitary links; after 600 leapfrog steps
    # the links carry ~1e-14 unitarity error and each particle crossed ~75
    # cells, which bounds the drift well below 1e-11 (a wrong rotation is O(1))
    assert oracle.unitarity(N, r.st["U"])[0] < 1e-13
    for p in range(P.shape[0]):
        q2, q3 = oracle.casimirs(r.P[p, 6:14])
        assert abs(q2 - q2_0) < 1e-11 and abs(q3 - q3_0) < 1e-11


def test_magnetic_force_does_no_work():
    N, dt, n = 16, 0.125, 6
    st, theta = uniform_flux_links(N)
    z2, z1 = np.zeros((2, N, N, 8)), np.zeros((N, N, 8))
    P = oracle.particles_init(N, 50, 5, 0.4, 0.4, True, 0)
    for step in range(40):
        before = P.copy()
        oracle.lib().orc_particles_step(N, n + step, n, dt, 0.3, 0, 0, oracle._ptr(st["U"]), oracle._ptr(z1),
                                        oracle._ptr(z2), oracle._ptr(z2), oracle._ptr(z1), oracle._ptr(z1),
                                        P.shape[0], oracle._ptr(P), None)
        b = before[:, 8] * 2 * math.sin(theta / 2)           # Q^3 is unchanged by diagonal links
        ptau = np.sqrt(before[:, 3] ** 2 + before[:, 4] ** 2 + 0.3 ** 2)
        v2 = (before[:, 3] ** 2 + before[:, 4] ** 2) / ptau ** 2
        growth = P[:, 3] ** 2 + P[:, 4] ** 2 - (before[:, 3] ** 2 + before[:, 4] ** 2)
        assert np.allclose(growth, dt ** 2 * b ** 2 * v2, rtol=1e-9, atol=1e-16)
        assert np.all(P[:, 5] == 0)


def static_run(rep, N=16, n_part=20000, steps=24, seed_f=1, seed_p=2):
    dt = 0.125
    st = oracle.mv_initial_condition(N, 6.0 * N / 32, 2.0, 0.2, 10.0, 1, seed_f)
    P = oracle.particles_init(N, n_part, seed_p, 0.0, 0.0, True, rep)
    r = oracle.Run(N, dt, st, P, mhat=math.inf, n_form=0)
    S = np.zeros((N * N, 3, 8))
    for n in range(steps):
        U_n, phi_n = r.st["U"].copy(), r.st["phi"].copy()
        Eo, po = r.st["E"].copy(), r.st["pi"].copy()
        r.step()
        for s in range(N * N):
            f = oracle.particle_fields(N, n, dt, s, U_n, phi_n, Eo, r.st["E"], po, r.st["pi"])
            S[s] += dt * f[:3]
    return r, P, S


def test_static_limit_equals_electric_correlator():
    r, P, S = static_run(0)
    N = 16
    sites = (P[:, 15] * N + P[:, 14]).astype(int)
    Q = P[:, 6:14]
    pred = np.einsum("na,nka->nk", Q, S[sites])
    assert np.max(np.abs(r.P[:, 3:6] - pred)) < 1e-12 * np.max(np.abs(pred))
    # ensemble: <(Q.S)^2> = T_F <|S|^2> over the same positions (Q-sampling error only)
    for k in range(3):
        x = pred[:, k] ** 2
        y = 0.5 * np.sum(S[sites, k] ** 2, axis=1)
        d = x - y
        assert abs(d.mean()) < 5 * d.std() / np.sqrt(len(d))
    obs = r.observe()
    assert obs[0] == pytest.approx(np.sum(pred[:, 0] ** 2 + pred[:, 1] ** 2), rel=1e-12)
    assert obs[1] == pytest.approx(np.sum(pred[:, 2] ** 2), rel=1e-12)


def test_casimir_scaling_static():
    rF, PF, S = static_run(0)
    rA, PA, _ = static_run(1)
    assert np.array_equal(PF[:, :2], PA[:, :2])
    N = 16
    sites = (PF[:, 15] * N + PF[:, 14]).astype(int)
    base = np.sum(S[sites, :2] ** 2, axis=(1, 2))          # |S_x|^2 + |S_y|^2 per particle
    xF = np.sum(rF.P[:, 3:5] ** 2, 1) / base
    xA = np.sum(rA.P[:, 3:5] ** 2, 1) / base
    ratio = xA.mean() / xF.mean()
    err = ratio * np.hypot(xA.std() / xA.mean(), xF.std() / xF.mean()) / np.sqrt(len(xA))
    assert abs(ratio - 6.0) < 5 * err
    assert abs(ratio * 3 / 8 - 2.25) < 5 * err * 3 / 8


def test_heavy_dynamical_particle_reproduces_static_pz():
    N, dt = 12, 0.125
    st = oracle.mv_initial_condition(N, 6.0 * N / 32, 2.0, 0.2, 10.0, 1, 7)
    P = oracle.particles_init(N, 64, 8, 0.0, 0.0, True, 0)
    rs = oracle.Run(N, dt, st, P, mhat=math.inf, n_form=4)
    rd = oracle.Run(N, dt, st, P, mhat=1e7, n_form=4)
    for _ in range(60):
        rs.step(); rd.step()
    t = rd.n * dt
    pe, eta = rd.P[:, 5], rd.P[:, 2]
    ptau = np.sqrt(rd.P[:, 3] ** 2 + rd.P[:, 4] ** 2 + (t * pe) ** 2 + 1e14)
    pz_dyn = ptau * np.sinh(eta) + t * pe * np.cosh(eta)
    pz_sta = rs.P[:, 5]
    scale = np.sqrt(np.mean(pz_sta ** 2))
    assert np.max(np.abs(pz_dyn - pz_sta)) < 0.05 * scale
    assert np.max(np.abs(rd.P[:, 3:5] - rs.P[:, 3:5])) < 1e-5 * scale
