"""SU(2) variant of the FP64 CPU oracle (cpic_oracle_su2.c).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.  The same readings as
the SU(3) oracle with 2x2 links and three colour components (T^a = sigma^a/2);
the MV Poisson solve is the same numpy FFT; the tau = 0 links have the
closed-form SU(2) solution of the SU(3) oracle's condition; charges are drawn
from the Darboux parametrisation of Sec. IV.A.  Particle records keep the 20
columns of the SU(3) oracle with Q^1..Q^3 in columns 6..8.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import NCOL, _ptr, lattice_spacing, poisson_kernel, lib as _lib, particles_observe

_sig_done = False


def lib():
    global _sig_done
    L = _lib()
    if not _sig_done:
        d, i, u64, p = ctypes.c_double, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p
        sig = {
            "orc2_forces": (None, [i, d, p, p, p, p]),
            "orc2_field_step": (None, [i, i, d, d, p, p, p, p]),
            "orc2_energy": (None, [i, d, p, p, p, p, p]),
            "orc2_gauss": (None, [i, p, p, p, p, p]),
            "orc2_mv_charges": (None, [i, u64, i, i, d, p]),
            "orc2_wilson_mult": (None, [i, p, p]),
            "orc2_pure_gauge": (None, [i, p, p]),
            "orc2_links": (None, [i, p, p, p]),
            "orc2_pi0": (None, [i, p, p, p, p]),
            "orc2_q2": (d, [i]),
            "orc2_particles_init": (None, [i, i, u64, d, d, i, i, p]),
            "orc2_particle_fields": (None, [i, i, d, i, p, p, p, p, p, p, p]),
            "orc2_particles_step": (i, [i, i, i, d, d, i, p, p, p, p, p, p, i, p]),
            "orc2_generator": (None, [i, p]),
            "orc2_expi": (None, [p, d, p]),
            "orc2_proj": (None, [p, p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _sig_done = True
    return L


def empty_state(N: int) -> dict:
    U = np.zeros((2, N, N, 2, 2), np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = 1.0
    return {"U": U, "phi": np.zeros((N, N, 3)), "E": np.zeros((2, N, N, 3)), "pi": np.zeros((N, N, 3))}


def generator(a: int) -> np.ndarray:
    out = np.zeros((2, 2), np.complex128)
    lib().orc2_generator(a, _ptr(out))
    return out


def expi(x, scale=1.0) -> np.ndarray:
    out = np.zeros((2, 2), np.complex128)
    lib().orc2_expi(_ptr(np.ascontiguousarray(x, np.float64)), scale, _ptr(out))
    return out


def proj(M) -> np.ndarray:
    out = np.zeros(3)
    lib().orc2_proj(_ptr(np.ascontiguousarray(M, np.complex128)), _ptr(out))
    return out


def q2(rep: int) -> float:
    return lib().orc2_q2(rep)


def forces(N, t, U, phi):
    FE, Fp = np.zeros((2, N, N, 3)), np.zeros((N, N, 3))
    lib().orc2_forces(N, t, _ptr(U), _ptr(phi), _ptr(FE), _ptr(Fp))
    return FE, Fp


def field_step(N, n, dt, st, t_fixed=0.0):
    lib().orc2_field_step(N, n, dt, t_fixed, _ptr(st["U"]), _ptr(st["phi"]), _ptr(st["E"]), _ptr(st["pi"]))


def energy(N, t, U, phi, E, pi):
    out = np.zeros(4)
    lib().orc2_energy(N, t, _ptr(U), _ptr(phi), _ptr(E), _ptr(pi), _ptr(out))
    return out


def gauss(N, U, phi, E, pi):
    G = np.zeros((N, N, 3))
    lib().orc2_gauss(N, _ptr(U), _ptr(phi), _ptr(E), _ptr(pi), _ptr(G))
    return G


def mv_charges(N, seed, nucleus, sheet, sigma):
    rho = np.zeros((N, N, 3))
    lib().orc2_mv_charges(N, seed, nucleus, sheet, sigma, _ptr(rho))
    return rho


def nucleus_links(N, seed, nucleus, n_sheets, g2mua, mhat, uvhat, rho_scale=1.0):
    K = poisson_kernel(N, mhat, uvhat)
    sigma = rho_scale * g2mua / math.sqrt(n_sheets)
    Vdag = np.zeros((N, N, 2, 2), np.complex128)
    Vdag[..., 0, 0] = Vdag[..., 1, 1] = 1.0
    for n in range(n_sheets):
        rho = mv_charges(N, seed, nucleus, n, sigma)
        alpha = np.ascontiguousarray(np.real(np.fft.ifft2(np.fft.fft2(rho, axes=(0, 1)) * K[:, :, None],
                                                          axes=(0, 1))))
        lib().orc2_wilson_mult(N, _ptr(alpha), _ptr(Vdag))
    UX = np.zeros((2, N, N, 2, 2), np.complex128)
    lib().orc2_pure_gauge(N, _ptr(Vdag), _ptr(UX))
    return UX


def mv_initial_condition(N, L_fm, g2mu_GeV, m_ir_GeV, uv_GeV, n_sheets, seed, rho_scale_B=1.0, keep_nuclei=False):
    a = lattice_spacing(L_fm, N)
    g2mua, mhat, uvhat = g2mu_GeV * a, m_ir_GeV * a, uv_GeV * a
    UA = nucleus_links(N, seed, 0, n_sheets, g2mua, mhat, uvhat)
    UB = nucleus_links(N, seed, 1, n_sheets, g2mua, mhat, uvhat, rho_scale=rho_scale_B)
    U = np.zeros_like(UA)
    lib().orc2_links(N, _ptr(UA), _ptr(UB), _ptr(U))
    st = empty_state(N)
    st["U"] = U
    pi = np.zeros((N, N, 3))
    lib().orc2_pi0(N, _ptr(UA), _ptr(UB), _ptr(U), _ptr(pi))
    st["pi"] = pi
    if keep_nuclei:
        st["UA"], st["UB"] = UA, UB
    return st


def particles_init(N, n, seed, pt_min_hat, pt_max_hat, azimuth_uniform=True, rep=0):
    P = np.zeros((n, NCOL))
    if n:
        lib().orc2_particles_init(N, n, seed, pt_min_hat, pt_max_hat, int(azimuth_uniform), rep, _ptr(P))
    return P


def particle_fields(N, n, dt, site, U, phi, E_old, E_new, pi_old, pi_new):
    out = np.zeros((6, 3))
    lib().orc2_particle_fields(N, n, dt, site, _ptr(U), _ptr(phi), _ptr(E_old), _ptr(E_new), _ptr(pi_old),
                               _ptr(pi_new), _ptr(out))
    return out


class Run:
    """SU(2) field leapfrog and particle push, as oracle.Run."""

    def __init__(self, N, dt, state, particles=None, mhat=math.inf, n_form=0, n0=0):
        self.N, self.dt, self.n = N, dt, n0
        self.st = {k: np.ascontiguousarray(state[k]).copy() for k in ("U", "phi", "E", "pi")}
        self.P = None if particles is None else np.ascontiguousarray(particles).copy()
        self.is_static = math.isinf(mhat)
        self.mhat = 0.0 if self.is_static else float(mhat)
        self.n_form = n_form
        self.errors = 0

    def step(self):
        N, n, st = self.N, self.n, self.st
        push = self.P is not None and self.P.shape[0] > 0 and n >= self.n_form
        if push:
            U_n, phi_n = st["U"].copy(), st["phi"].copy()
            E_old, pi_old = st["E"].copy(), st["pi"].copy()
        field_step(N, n, self.dt, st)
        if push:
            self.errors += lib().orc2_particles_step(
                N, n, self.n_form, self.dt, self.mhat, int(self.is_static), _ptr(U_n), _ptr(phi_n),
                _ptr(E_old), _ptr(st["E"]), _ptr(pi_old), _ptr(st["pi"]), self.P.shape[0], _ptr(self.P))
        self.n += 1

    def observe(self):
        return particles_observe(self.n * self.dt, self.mhat, self.is_static, self.P)
