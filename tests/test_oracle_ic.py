"""Pins of the oracle's MV initial condition (Sec. II, II.A):
  * Poisson solve: (-Laplacian + m^2) alpha equals the kept charge modes
    (lattice Laplacian applied independently with numpy);
  * the pure-gauge nucleus links have unit plaquettes;
  * the tau = 0 links solve the initial-link condition, checked directly;
  * weak-field limit: Proj U -> alpha_A + alpha_B and
    pi -> -i sum_i [alpha^i_A, alpha^i_B] [eq:Glasmainitcond] with the
    relative error shrinking linearly with g^2 mu a.
"""
import numpy as np
import pytest

import oracle
from test_oracle_algebra import golden_tables


def test_poisson_residual_and_cuts():
    N, mhat, uvhat = 32, 0.19, 1.4
    rho = oracle.mv_charges(N, 3, 0, 0, 1.0)
    K = oracle.poisson_kernel(N, mhat, uvhat)
    alpha = oracle.poisson_solve(rho, K)
    lap = (np.roll(alpha, 1, 0) + np.roll(alpha, -1, 0) + np.roll(alpha, 1, 1) + np.roll(alpha, -1, 1)
           - 4 * alpha)
    lhs = -lap + mhat ** 2 * alpha
    keep = (K != 0).astype(float)
    rho_kept = np.real(np.fft.ifft2(np.fft.fft2(rho, axes=(0, 1)) * keep[:, :, None], axes=(0, 1)))
    assert np.max(np.abs(lhs - rho_kept)) < 1e-12 * np.max(np.abs(rho))
    # the zero mode and every mode above the cut are removed
    k = np.fft.fftfreq(N) * N
    kk = (2 * np.pi / N) * np.hypot(k[:, None], k[None, :])
    assert K[0, 0] == 0 and np.all(K[kk > uvhat] == 0) and np.all(K[(kk <= uvhat) & (kk > 0)] > 0)
    assert abs(alpha.mean(axis=(0, 1))).max() < 1e-14


def test_pure_gauge_links_have_unit_plaquettes():
    N = 16
    UA = oracle.nucleus_links(N, 9, 0, 3, 0.8, 0.08, 0.0)
    for y in range(N):
        for x in range(N):
            P12 = UA[0, y, x] @ UA[1, y, (x + 1) % N] @ UA[0, (y + 1) % N, x].conj().T @ UA[1, y, x].conj().T
            assert np.max(np.abs(P12 - np.eye(3))) < 1e-13


def test_initial_links_solve_the_condition_strong_field():
    """g^2 mu a = 1.9 (32^2 at L = 6 fm, the coarse configuration)."""
    N = 32
    a = oracle.lattice_spacing(6.0, N)
    st = oracle.mv_initial_condition(N, 6.0, 2.0, 0.2, 10.0, 1, 1, keep_nuclei=True)
    UA, UB, U = st["UA"], st["UB"], st["U"]
    W = UA + UB
    Ud = np.conj(np.swapaxes(U, -1, -2))
    M = W @ (np.eye(3) + Ud)
    A = 0.5 * (M - np.conj(np.swapaxes(M, -1, -2)))
    A = A - (np.trace(A, axis1=-2, axis2=-1) / 3)[..., None, None] * np.eye(3)
    assert np.max(np.abs(A)) < 1e-13
    assert np.max(np.abs(U @ Ud - np.eye(3))) < 1e-14
    assert np.max(np.abs(np.linalg.det(U) - 1)) < 1e-14
    assert st["newton_iters"] <= 50
    assert 2.0 * a == pytest.approx(1.900399, abs=1e-6)


def weak_field_errors(eps, N=12, seed=5):
    f, _ = golden_tables()
    UA = oracle.nucleus_links(N, seed, 0, 1, eps, 0.1, 0.0)
    UB = oracle.nucleus_links(N, seed, 1, 1, eps, 0.1, 0.0)
    U, _ = oracle.glasma_links(N, UA, UB)
    pi = oracle.pi0(N, UA, UB, U)
    aA = np.array([[[oracle.proj(UA[i, y, x]) for x in range(N)] for y in range(N)] for i in range(2)])
    aB = np.array([[[oracle.proj(UB[i, y, x]) for x in range(N)] for y in range(N)] for i in range(2)])
    aU = np.array([[[oracle.proj(U[i, y, x]) for x in range(N)] for y in range(N)] for i in range(2)])
    err_links = np.max(np.abs(aU - (aA + aB))) / np.max(np.abs(aA + aB))
    comm = np.einsum("abc,iyxa,iyxb->iyxc", f, aA, aB)          # (-i[A,B])^c = f_abc A^a B^b
    ref = 0.5 * (comm[0] + np.roll(comm[0], 1, axis=1) + comm[1] + np.roll(comm[1], 1, axis=0))
    err_pi = np.max(np.abs(pi - ref)) / np.max(np.abs(ref))
    return err_links, err_pi


def test_weak_field_limit_of_initial_condition():
    l1, p1 = weak_field_errors(1e-2)
    l2, p2 = weak_field_errors(1e-3)
    assert l1 < 0.05 and p1 < 0.05
    assert l2 < l1 / 5 and p2 < p1 / 5
