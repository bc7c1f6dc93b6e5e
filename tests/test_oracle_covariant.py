"""Pins of the oracle against the covariant form of the equations, independent
of the component equations it implements:

  * the particle push against the covariant Wong equation of Appendix A
    ([eq:wongmompropertime]): the field strength tensor F_{mu nu} is assembled
    from the definitions of [eq:glasmafields_main] (E_i = F_{tau i},
    E_eta = F_{tau eta}/tau, B_eta = -F_xy) with F_{eta j} = -D_j A_eta taken
    directly from the scalar field, with no epsilon_ij and no B_x, B_y; the
    force (g/T_R) Tr(Q F_{nu mu}) p^mu / p^tau is contracted with the Milne
    metric and turned into dp^nu/dtau by the covariant derivatives printed in
    Appendix A.  This fixes the signs and indices of the B_x and B_y terms
    (v_L != 0) and of the temporal component [eq:ptaueq];
  * the leapfrog's time arguments (kick at t_n, drift at t_{n+1/2}) through the
    energy balance of a physical (expanding) run: H(t_1) - H(t_0) minus the
    trapezoid integral of dH/dt = (K_L + V_B - K_T - V_phi)/t must vanish as
    dt^2 for a second-order scheme;
  * the temporal constraint (Appendix D): p^tau integrated from [eq:ptaueq]
    against [eq:ptau] in closed form for a free particle in the expanding
    frame, and their percent-level difference in an MV event, shrinking at
    first order in dt.

Each pin is shown to fail on a copy of the oracle with a planted mistake.
"""
import math

import numpy as np
import pytest

import inputs
import oracle
from planted import planted


def gell_mann_generators():
    """T^a = lambda^a / 2, the Gell-Mann matrices (Appendix B.1), written out here."""
    l = np.zeros((8, 3, 3), np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7] = np.diag([1, 1, -2]) / math.sqrt(3)
    return l / 2


T = gell_mann_generators()


def to_mat(x):
    return np.einsum("a,aij->ij", x, T)


def comps(X):
    """x^a = 2 Re Tr(T^a X) of a Hermitian X."""
    return np.array([2 * np.trace(T[a] @ X).real for a in range(8)])


def proj(M):
    """Hermitian traceless generator part of M: x^a = 2 Im Tr(T^a M)."""
    return np.array([2 * np.trace(T[a] @ M).imag for a in range(8)])


def field_strength(N, t, y, x, U, phi, E_old, E_new, pi_old, pi_new):
    """F_{mu nu} at site (y, x), lower indices in the order (tau, x, y, eta), as
    8-component algebra vectors in hat units (F_{tau i}, F_xy scaled by g a^2,
    F_{tau eta}, F_{eta j} by g a)."""
    def at(dy, dx):
        return (y + dy) % N, (x + dx) % N
    F = np.zeros((4, 4, 8))
    steps = ((0, 1), (1, 0))  # (dy, dx) of e_x, e_y
    for i, (dy, dx) in enumerate(steps):
        # E_i = F_{tau i}: the second-order interpolation of Sec. III.B
        yb, xb = at(-dy, -dx)
        Ub = U[i, yb, xb]
        s = to_mat(E_old[i, y, x] + E_new[i, y, x]) + Ub.conj().T @ to_mat(E_old[i, yb, xb] + E_new[i, yb, xb]) @ Ub
        F[0, 1 + i] = comps(s) / (4 * t)
        # F_{eta j} = -D_j A_eta, central covariant difference of phi = g A_eta
        # (stored as F_{j eta} = -F_{eta j})
        yf, xf = at(dy, dx)
        fwd = U[i, y, x] @ to_mat(phi[yf, xf]) @ U[i, y, x].conj().T
        bwd = Ub.conj().T @ to_mat(phi[yb, xb]) @ Ub
        F[1 + i, 3] = comps(fwd - bwd) / 2
    # E_eta = F_{tau eta} / tau
    F[0, 3] = t * 0.5 * (pi_old[y, x] + pi_new[y, x])
    # B_eta = -F_xy, B_eta = -(1/4) Proj of the clover of counter-clockwise plaquettes
    U1, U2 = U[0], U[1]
    d = lambda M: M.conj().T  # noqa: E731
    c = (y, x)
    xp, yp, xm, ym = at(0, 1), at(1, 0), at(0, -1), at(-1, 0)
    xmyp, xpym, xmym = at(1, -1), at(-1, 1), at(-1, -1)
    leaves = (U1[c] @ U2[xp] @ d(U1[yp]) @ d(U2[c]),
              U2[c] @ d(U1[xmyp]) @ d(U2[xm]) @ U1[xm],
              d(U1[xm]) @ d(U2[xmym]) @ U1[xmym] @ U2[ym],
              d(U2[ym]) @ U1[ym] @ U2[xpym] @ d(U1[c]))
    F[1, 2] = 0.25 * proj(sum(leaves))
    for m in range(4):
        for n in range(m):
            F[m, n] = -F[n, m]
    return F


def covariant_rates(F, Q, t, px, py, pe, mhat):
    """dp^x/dt, dp^y/dt, dp^eta/dt, dp^tau/dt from D p_nu/dt = Q.F_{nu mu} p^mu/p^tau
    with the Milne covariant derivatives of Appendix A:
      D p_tau = dp^tau + t (p^eta)^2/p^tau,  D p_i = -dp^i,  D p_eta = -t^2 dp^eta - 2 t p^eta."""
    ptau = math.sqrt(px * px + py * py + (t * pe) ** 2 + mhat * mhat)
    pu = np.array([ptau, px, py, pe])
    K = np.array([sum(np.dot(Q, F[nu, mu]) * pu[mu] for mu in range(4)) / ptau for nu in range(4)])
    return -K[1], -K[2], -(K[3] + 2 * t * pe) / t ** 2, K[0] - t * pe * pe / ptau


def check_push_against_covariant_force(links):
    N, n, dt, mhat = 8, 6, 0.125, 0.7
    t = n * dt
    rng = np.random.default_rng(11)
    st = inputs.random_state(N, 12, eps_link=0.5, e_scale=0.3, phi_scale=0.3, pi_scale=0.3)
    if links == "trivial":
        st["U"] = oracle.empty_state(N)["U"]
    Eo = rng.normal(0, 0.3, (2, N, N, 8))
    po = rng.normal(0, 0.3, (N, N, 8))
    m = 24
    P = np.zeros((m, oracle.NCOL))
    cells = rng.integers(0, N, (m, 2))
    P[:, 0] = cells[:, 0] + rng.uniform(-0.4, 0.4, m)
    P[:, 1] = cells[:, 1] + rng.uniform(-0.4, 0.4, m)
    P[:, 0] %= N
    P[:, 1] %= N
    P[:, 3:5] = rng.normal(0, 0.6, (m, 2))
    P[:, 5] = rng.normal(0, 0.5, m) / t          # v_L = t p^eta / p^tau of order one
    P[:, 6:14] = rng.normal(0, 1.0, (m, 8))
    P[:, 14] = np.floor(P[:, 0] + 0.5) % N
    P[:, 15] = np.floor(P[:, 1] + 0.5) % N
    P0 = P.copy()
    ptau = np.zeros(m)
    # formation step: no colour rotation, the force acts on the charges as given
    err = oracle.lib().orc_particles_step(N, n, n, dt, mhat, 0, 0, oracle._ptr(st["U"]), oracle._ptr(st["phi"]),
                                          oracle._ptr(Eo), oracle._ptr(st["E"]), oracle._ptr(po),
                                          oracle._ptr(st["pi"]), m, oracle._ptr(P), oracle._ptr(ptau))
    assert err == 0
    worst = 0.0
    for k in range(m):
        x, y = int(P0[k, 14]), int(P0[k, 15])
        F = field_strength(N, t, y, x, st["U"], st["phi"], Eo, st["E"], po, st["pi"])
        rates = covariant_rates(F, P0[k, 6:14], t, *P0[k, 3:6], mhat)
        ptau0 = math.sqrt(P0[k, 3] ** 2 + P0[k, 4] ** 2 + (t * P0[k, 5]) ** 2 + mhat ** 2)
        got = ((P[k, 3] - P0[k, 3]) / dt, (P[k, 4] - P0[k, 4]) / dt, (P[k, 5] - P0[k, 5]) / dt,
               (ptau[k] - ptau0) / dt)
        scale = max(abs(r) for r in rates)
        worst = max(worst, max(abs(g - r) for g, r in zip(got, rates)) / scale)
    return worst


@pytest.mark.parametrize("links", ["trivial", "random"])
def test_push_follows_the_covariant_wong_force(links):
    assert check_push_against_covariant_force(links) < 1e-12


@pytest.mark.parametrize("old,new", [
    # B_x with the opposite sign (epsilon_ij dropped)
    ("for (int a = 0; a < 8; a++) out[24 + a] = -b[a] / (2.0 * t);",
     "for (int a = 0; a < 8; a++) out[24 + a] = b[a] / (2.0 * t);"),
    # B_y with the opposite sign
    ("for (int a = 0; a < 8; a++) out[32 + a] = b[a] / (2.0 * t);",
     "for (int a = 0; a < 8; a++) out[32 + a] = -b[a] / (2.0 * t);"),
    # B_x from the derivative along x (the index repeated as printed)
    ("mat_to_alg(m_sub(phi_fwd(U, phi, N, 1, s), phi_bwd(U, phi, N, 1, s)), b);",
     "mat_to_alg(m_sub(phi_fwd(U, phi, N, 0, s), phi_bwd(U, phi, N, 0, s)), b);"),
    # the Christoffel term of the temporal equation dropped
    ("ptau_ode[p] = pt + dt * (-t * pe * pe + ee * t * pe + e1 * px + e2 * py) / pt;",
     "ptau_ode[p] = pt + dt * (ee * t * pe + e1 * px + e2 * py) / pt;"),
])
def test_covariant_force_pin_catches_planted_mistakes(old, new):
    with planted(old, new):
        assert check_push_against_covariant_force("random") > 1e-3


# --------------------------------------------------------------------------- energy balance
def energy_balance_residual(N, st0, t0, t1, dt):
    """H(t1) - H(t0) - trapezoid sum of dH/dt over the leapfrog run from t0 to t1
    (state st0 at integer time t0; momenta set half a step back with the kick
    forces; energies at integer times with the momenta kicked half a step)."""
    n0, n1 = round(t0 / dt), round(t1 / dt)
    st = {k: st0[k].copy() for k in ("U", "phi", "E", "pi")}
    FE, Fp = oracle.forces(N, t0, st["U"], st["phi"])
    st["E"] -= 0.5 * dt * FE
    st["pi"] -= 0.5 * dt * Fp

    def h_and_rate(n):
        t = n * dt
        FE, Fp = oracle.forces(N, t, st["U"], st["phi"])
        KT, KL, VB, VP = oracle.energy(N, t, st["U"], st["phi"], st["E"] + 0.5 * dt * FE, st["pi"] + 0.5 * dt * Fp)
        # H = (1/t) K_T' + t K_L' + t V_B' + (1/t) V_phi' in its explicit t: dH/dt = partial_t H
        return KT + KL + VB + VP, (KL + VB - KT - VP) / t

    H0, r0 = h_and_rate(n0)
    integral = 0.0
    for n in range(n0, n1):
        oracle.field_step(N, n, dt, st)
        H1, r1 = h_and_rate(n + 1)
        integral += 0.5 * dt * (r0 + r1)
        r0 = r1
    return H1 - H0 - integral, H0


def glasma_state_at(N, t0_steps=32, dt=1 / 16):
    st = oracle.mv_initial_condition(N, 6.0 * N / 64, 2.0, 0.2, 10.0, 2, 5)
    run = oracle.Run(N, dt, st)
    for _ in range(t0_steps):
        run.step()
    t0 = run.n * dt
    FE, Fp = oracle.forces(N, t0, run.st["U"], run.st["phi"])
    s0 = {k: run.st[k].copy() for k in ("U", "phi")}
    s0["E"] = run.st["E"] + 0.5 * dt * FE
    s0["pi"] = run.st["pi"] + 0.5 * dt * Fp
    return s0, t0


def energy_balance_ratios(N=12):
    s0, t0 = glasma_state_at(N)
    R = [energy_balance_residual(N, s0, t0, t0 + 2.0, dt)[0] for dt in (1 / 8, 1 / 16, 1 / 32)]
    return R[0] / R[1], R[1] / R[2], R


def test_energy_balance_of_the_expanding_run_is_second_order():
    r1, r2, R = energy_balance_ratios()
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, R


@pytest.mark.parametrize("old,new", [
    # drift at t_n instead of t_{n+1/2}
    ("double th = t_fixed > 0 ? t_fixed : (n + 0.5) * dt;", "double th = t_fixed > 0 ? t_fixed : n * dt;"),
    # kick at t_{n+1/2} instead of t_n
    ("double t = t_fixed > 0 ? t_fixed : n * dt;\n    double th",
     "double t = t_fixed > 0 ? t_fixed : (n + 0.5) * dt;\n    double th"),
])
def test_energy_balance_pin_catches_planted_time_arguments(old, new):
    with planted(old, new):
        r1, r2, R = energy_balance_ratios()
        assert not (3.6 < r1 < 4.4 and 3.8 < r2 < 4.2), R


# --------------------------------------------------------------------------- temporal constraint
def free_particle_ptau(dt, t0=1.0, t1=4.0, mhat=0.3, px=0.4, py=-0.2, pe=0.5):
    """A particle without fields from t0: p^eta(t) = p^eta(t0) (t0/t)^2
    solves [eq:wonginmilne], p_T is constant, and [eq:ptau] gives p^tau(t) in
    closed form; returns the errors of the integrated and constraint p^tau."""
    N = 8
    st = oracle.empty_state(N)
    z2, z1 = np.zeros((2, N, N, 8)), np.zeros((N, N, 8))
    P = np.zeros((1, oracle.NCOL))
    P[0, 0], P[0, 1] = 3.0, 4.0
    P[0, 3], P[0, 4], P[0, 5] = px, py, pe
    P[0, 6] = 1.0
    P[0, 14], P[0, 15] = 3, 4
    ptau = np.zeros(1)
    n0, n1 = round(t0 / dt), round(t1 / dt)
    for n in range(n0, n1):
        oracle.lib().orc_particles_step(N, n, n0, dt, mhat, 0, 0, oracle._ptr(st["U"]), oracle._ptr(z1),
                                        oracle._ptr(z2), oracle._ptr(z2), oracle._ptr(z1), oracle._ptr(z1), 1,
                                        oracle._ptr(P), oracle._ptr(ptau))
    exact = math.sqrt(px * px + py * py + (pe * t0 * t0 / t1) ** 2 + mhat * mhat)
    constraint = math.sqrt(P[0, 3] ** 2 + P[0, 4] ** 2 + (t1 * P[0, 5]) ** 2 + mhat * mhat)
    return ptau[0] - exact, constraint - exact, exact


def test_temporal_equation_matches_the_free_particle_closed_form():
    errs = [free_particle_ptau(dt) for dt in (1 / 8, 1 / 16, 1 / 32, 1 / 64)]
    for ode, con, exact in errs:
        assert abs(ode) < 0.05 * exact and abs(con) < 0.05 * exact
    # both are first order in dt (explicit Euler)
    for k in range(3):
        assert 1.7 < errs[k][0] / errs[k + 1][0] < 2.3
        assert 1.7 < errs[k][1] / errs[k + 1][1] < 2.3


def test_free_particle_pin_catches_a_planted_mistake():
    with planted("ptau_ode[p] = pt + dt * (-t * pe * pe + ee * t * pe + e1 * px + e2 * py) / pt;",
                 "ptau_ode[p] = pt + dt * (-pe * pe + ee * t * pe + e1 * px + e2 * py) / pt;"):
        errs = [free_particle_ptau(dt)[0] for dt in (1 / 16, 1 / 32, 1 / 64)]
        assert not (1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3), errs


def glasma_ptau_difference(dt, N=16, steps_fm=0.6):
    """Mean and maximum of |p^tau(ODE) - p^tau(constraint)| / p^tau for charm-like
    quarks (m = 1.27 GeV, p_T = 1 GeV) in an MV event, from 0.1 fm/c."""
    L = 6.0 * N / 64
    a = oracle.lattice_spacing(L, N)
    st = oracle.mv_initial_condition(N, L, 2.0, 0.2, 10.0, 2, 41)
    P = oracle.particles_init(N, 200, 42, 1.0 * a, 1.0 * a, True, 0)
    afm = L / N
    n_form = math.ceil(0.1 / (dt * afm) - 1e-9)
    run = oracle.Run(N, dt, st, P, mhat=1.27 * a, n_form=n_form)
    for _ in range(n_form + round(steps_fm / (dt * afm))):
        run.step()
    c = run.ptau_constraint()
    rel = np.abs(run.ptau_ode - c) / c
    return rel.mean(), rel.max()


def test_temporal_constraint_holds_at_the_percent_level_in_glasma():
    m8, x8 = glasma_ptau_difference(1 / 8)
    m16, x16 = glasma_ptau_difference(1 / 16)
    # the two p^tau differ at the percent level and converge at first order
    assert m8 < 0.05 and x8 < 0.2
    assert 1.5 < m8 / m16 < 2.6
