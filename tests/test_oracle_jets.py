"""Pins of the oracle's light-like jet limit (Sec. V.B, [eq:mombroadjets]).

  * the particle solver in the limit p^x -> infinity gives, per particle,
    dp_i = Q_0 . F_i with F the transported force integral of the same path
    (the paper's Fig. 3b comparison, here exact for x and y; the z component
    agrees up to the Euler discretisation of p^eta and its omission at
    t = 0);
  * the ensemble mean over charges is q2/8 |F_i|^2 ([eq:qnpointfct_main]);
  * gauge covariance: F of every path transforms with the gauge
    transformation at its starting cell, so |F_i|^2 is invariant;
  * closed forms for Abelian (commuting) configurations: the force
    combinations f_y = E_y - B_eta and f_z = E_eta + B_y, the cell schedule
    of the path, the stride weights, and the transport W f W^+ of a field
    that does not commute with the Wilson line.
"""
import math

import numpy as np
import pytest

import inputs
import oracle
from test_oracle_fields import apply_gauge, comps, mat


def light_like_run(N, steps, x_off, pT=1e7, n_form=0):
    """Particles on the jet paths (one per site, row offset 0.2 so that the
    nearest grid point is the path's row) with p^x = pT along +x."""
    dt = 0.125
    st = oracle.mv_initial_condition(N, 6.0 * N / 32, 2.0, 0.2, 10.0, 1, 7)
    P = oracle.particles_init(N, N * N, 8, 0.0, 0.0, True, 0)
    ys, xs = np.divmod(np.arange(N * N), N)
    P[:, 0] = xs + x_off
    P[:, 1] = ys + 0.2
    P[:, 3], P[:, 4] = pT, 0.0
    P[:, 14], P[:, 15] = np.floor(P[:, 0] + 0.5) % N, np.floor(P[:, 1] + 0.5) % N
    P[:, 17], P[:, 18], P[:, 19] = 1.0, 0.0, 0.0
    jets = oracle.Jets(N, dt, n_form, x_off, 1)
    r = oracle.Run(N, dt, st, P, mhat=1e-3, n_form=n_form, jets=jets)
    for _ in range(steps):
        r.step()
    return st, P, r, jets


def lab_pz(r):
    t = r.n * r.dt
    px, py, pe, eta = r.P[:, 3], r.P[:, 4], r.P[:, 5], r.P[:, 2]
    ptau = np.sqrt(px ** 2 + py ** 2 + (t * pe) ** 2 + r.mhat ** 2)
    return ptau * np.sinh(eta) + t * pe * np.cosh(eta)


# start offsets that are not multiples of dt: the particles' nearest grid
# points then never sit on a tie that their speed (1 - 1e-14) resolves
# differently from the paths' exact speed of light
@pytest.mark.parametrize("x_off", [0.3, 0.55])
def test_light_like_particles_match_the_correlator(x_off):
    N, steps = 12, 64
    st, P0, r, jets = light_like_run(N, steps, x_off)
    assert r.errors == 0
    F = jets.F.reshape(N * N, 3, 8)
    Q0 = P0[:, 6:14]
    pred = np.einsum("na,nka->nk", Q0, F)
    dpx, dpy = r.P[:, 3] - P0[:, 3], r.P[:, 4] - P0[:, 4]
    for got, ref in ((dpx, pred[:, 0]), (dpy, pred[:, 1])):
        rms = np.sqrt(np.mean(ref ** 2))
        assert rms > 0.1
        # p^x = 1e7 resolves momentum changes to ~2e-9; the transverse velocity
        # and rapidity left over at finite energy are ~1e-7
        assert np.max(np.abs(got - ref)) < 1e-5 * rms
    # z: the solver leaves out the p^eta force at t = 0, so compare with the
    # correlator without its t_0 term; the rest differs by the Euler
    # discretisation of p^z = t p^eta, O(dt^2/t) per step
    j0 = oracle.Jets(N, 0.125, 0, x_off, 1)
    oracle.Run(N, 0.125, st, None, jets=j0).step()
    ref = pred[:, 2] - np.einsum("na,na->n", Q0, j0.F.reshape(N * N, 3, 8)[:, 2])
    rms = np.sqrt(np.mean(ref ** 2))
    assert np.max(np.abs(lab_pz(r) - ref)) < 0.02 * rms
    # the t_0 term is what the correlator adds (the integral starts at 0)
    assert np.max(np.abs(lab_pz(r) - pred[:, 2])) > 0.1 * rms


def test_ensemble_mean_over_charges():
    """<dp_i^2> over the Haar-distributed charges = q2/8 |F_i|^2 per path."""
    N, steps = 12, 32
    _, P0, r, jets = light_like_run(N, steps, 0.3)
    F = jets.F.reshape(N * N, 3, 8)
    q2 = float(np.dot(oracle.q0(0), oracle.q0(0)))
    for k, got in ((0, r.P[:, 3] - P0[:, 3]), (1, r.P[:, 4] - P0[:, 4])):
        d = got ** 2 - q2 / 8 * np.sum(F[:, k] ** 2, axis=1)
        assert abs(d.mean()) < 5 * d.std() / math.sqrt(len(d))
    obs = jets.observe(0)
    assert obs[0] == pytest.approx(q2 / 8 * np.mean(np.sum(F[:, 0] ** 2, axis=1)), rel=1e-14)


def test_gauge_covariance():
    N, dt, steps, x_off, n_form = 6, 0.125, 30, 0.45, 2
    T = [oracle.generator(a) for a in range(8)]
    st = inputs.random_state(N, 31, eps_link=0.4)
    V = inputs.haar_su3(np.random.default_rng(32), (N, N))
    out = []
    for s in (st, apply_gauge(st, V, T)):
        j = oracle.Jets(N, dt, n_form, x_off, 1)
        r = oracle.Run(N, dt, s, None, n0=1, jets=j)
        for _ in range(steps):
            r.step()
        out.append(j)
    a, b = out
    k0 = math.floor(x_off + 0.5)
    assert np.max(np.abs(a.F)) > 0.1
    for y in range(N):
        for i in range(N):
            Vs = V[y, (i + k0) % N]
            for c in range(3):
                want = comps(Vs @ mat(a.F[y, i, c], T) @ Vs.conj().T, T)
                assert np.max(np.abs(want - b.F[y, i, c])) < 1e-11
    assert np.allclose(a.observe(1), b.observe(1), rtol=1e-11)


def frozen_abelian_run(st, N, n_form, steps, x_off, stride, dt=0.125):
    j = oracle.Jets(N, dt, n_form, x_off, stride)
    for n in range(n_form, n_form + steps):
        j.step(n, st["U"], st["phi"], st["E"], st["E"], st["pi"], st["pi"])
    return j


def cells_and_weights(N, n_form, steps, x_off, stride, dt):
    """(step n, cell offset k(m), weight) of every evaluated step."""
    out = []
    for m in range(steps):
        if m % stride == 0:
            out.append((n_form + m, math.floor(x_off + m * dt + 0.5), stride * dt))
    return out


@pytest.mark.parametrize("n_form,x_off,stride", [(0, 0.0, 1), (3, 0.6, 1), (0, 0.25, 8), (5, 0.9, 3)])
def test_abelian_closed_forms(n_form, x_off, stride):
    """Commuting T3/T8 fields with trivial x links: no transport.
    U_y(x) = exp(i gamma(x) T3) gives B_eta(x) = -[sin(eps(x)/2) + sin(eps(x-1)/2)] T3
    with eps(x) = gamma(x+1) - gamma(x) (each clover leaf has Proj = 2 sin(eps/2) T3);
    phi = A sin(2 pi x/N) T8 gives B_y = (phi(x+1) - phi(x-1)) / (2t); pi = p0 T3."""
    N, dt, steps = 8, 0.125, 40
    st = oracle.empty_state(N)
    x = np.arange(N)
    gamma = 0.7 * np.sin(2 * np.pi * x / N) + 0.2 * np.cos(4 * np.pi * x / N)
    for y in range(N):
        for xx in range(N):
            st["U"][1, y, xx] = np.diag(np.exp(1j * gamma[xx] * np.array([0.5, -0.5, 0.0])))
    A, p0 = 0.8, 0.37
    st["phi"][:, :, 7] = A * np.sin(2 * np.pi * x / N)[None, :]
    st["pi"][:, :, 2] = p0
    j = frozen_abelian_run(st, N, n_form, steps, x_off, stride, dt)
    eps = np.roll(gamma, -1) - gamma
    beta = -(np.sin(eps / 2) + np.sin(np.roll(eps, 1) / 2))
    for i in (0, 3, 7):
        Fy, Fz = np.zeros(8), np.zeros(8)
        for n, k, w in cells_and_weights(N, n_form, steps, x_off, stride, dt):
            c = (i + k) % N
            Fy[2] -= w * beta[c]
            Fz[2] += w * p0
            if n > 0:
                Fz[7] += w * A * (np.sin(2 * np.pi * (c + 1) / N) - np.sin(2 * np.pi * (c - 1) / N)) / (2 * n * dt)
        for y in (0, 5):
            assert np.max(np.abs(j.F[y, i, 0])) < 1e-14
            assert np.allclose(j.F[y, i, 1], Fy, atol=1e-13)
            assert np.allclose(j.F[y, i, 2], Fz, atol=1e-13)


@pytest.mark.parametrize("x_off,stride", [(0.0, 1), (0.7, 2)])
def test_transport_of_a_non_commuting_field(x_off, stride):
    """x links exp(i alpha(x) T3), every other field zero except pi = p0 T1:
    after crossing cells c_0 .. c_{k-1} the Wilson line is exp(i theta T3),
    theta = sum alpha(c_j), and W T1 W^+ = cos(theta) T1 - sin(theta) T2."""
    N, dt, steps, n_form = 6, 0.125, 50, 1
    st = oracle.empty_state(N)
    alpha = np.array([0.3, -1.1, 0.8, 2.0, -0.4, 0.6])
    for y in range(N):
        for xx in range(N):
            st["U"][0, y, xx] = np.diag(np.exp(1j * alpha[xx] * np.array([0.5, -0.5, 0.0])))
    p0 = 0.9
    st["pi"][:, :, 0] = p0
    j = frozen_abelian_run(st, N, n_form, steps, x_off, stride, dt)
    for i in range(N):
        F = np.zeros(8)
        k0 = math.floor(x_off + 0.5)
        for n, k, w in cells_and_weights(N, n_form, steps, x_off, stride, dt):
            theta = sum(alpha[(i + kk) % N] for kk in range(k0, k))
            F[0] += w * p0 * math.cos(theta)
            F[1] -= w * p0 * math.sin(theta)
        assert np.allclose(j.F[2, i, 2], F, atol=1e-13)
        assert np.max(np.abs(j.F[2, i, :2])) < 1e-14
