"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module holds none of the method's arithmetic: it only draws random
unitary matrices, random real vectors and random gauge transformations with
numpy/scipy, so that both implementations can be started from the same
state.  Nothing here is imported by the oracle or by the product library.
"""
import numpy as np
import scipy.stats


def _hermitian_traceless(rng, shape):
    A = rng.normal(size=shape + (3, 3)) + 1j * rng.normal(size=shape + (3, 3))
    H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1) / 3.0
    H = H - tr[..., None, None] * np.eye(3)
    return H


def su3_near_identity(rng, shape, eps):
    """exp(i eps H) with H random Hermitian traceless (numpy eigh)."""
    H = _hermitian_traceless(rng, shape)
    w, V = np.linalg.eigh(H)
    return np.einsum("...ij,...j,...kj->...ik", V, np.exp(1j * eps * w), np.conj(V))


def haar_su3(rng, shape):
    """Haar-random SU(3) matrices (scipy unitary_group, determinant phase removed)."""
    n = int(np.prod(shape)) if shape else 1
    U = scipy.stats.unitary_group.rvs(3, size=n, random_state=rng).reshape(shape + (3, 3))
    det = np.linalg.det(U)
    return U / (det ** (1.0 / 3.0))[..., None, None]


def random_state(N, seed, eps_link=0.3, e_scale=0.2, phi_scale=0.2, pi_scale=0.2):
    """Random lattice state in hat units: links near the identity, algebra
    fields Gaussian.  Not a Glasma state (no Gauss law), only a test input."""
    rng = np.random.default_rng(seed)
    return {
        "U": np.ascontiguousarray(su3_near_identity(rng, (2, N, N), eps_link)),
        "phi": rng.normal(0, phi_scale, (N, N, 8)),
        "E": rng.normal(0, e_scale, (2, N, N, 8)),
        "pi": rng.normal(0, pi_scale, (N, N, 8)),
    }


def random_particles(n, N, seed, p_scale=0.3, q_scale=1.0):
    """Random particle records (columns as in the oracle): positions in
    [0,N), small momenta, random colour vectors, cells consistent with the
    nearest grid point, initial direction along x."""
    rng = np.random.default_rng(seed)
    P = np.zeros((n, 20))
    P[:, 0] = rng.uniform(0, N, n)
    P[:, 1] = rng.uniform(0, N, n)
    P[:, 2] = rng.normal(0, 0.01, n)
    P[:, 3] = rng.normal(0, p_scale, n)
    P[:, 4] = rng.normal(0, p_scale, n)
    P[:, 5] = rng.normal(0, 0.01, n)
    P[:, 6:14] = rng.normal(0, q_scale, (n, 8))
    P[:, 14] = np.floor(P[:, 0] + 0.5) % N
    P[:, 15] = np.floor(P[:, 1] + 0.5) % N
    P[:, 16] = rng.normal(0, 0.001, n)
    P[:, 17] = 1.0
    P[:, 18] = 0.0
    P[:, 19] = np.hypot(P[:, 3], P[:, 4])
    return P
