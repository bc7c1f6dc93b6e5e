"""FP64 CPU oracle for the colored particle-in-cell (CPIC) hot path of
arXiv:2303.05599.

TEST INFRASTRUCTURE ONLY: this package is imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``,
never by the product library.  It shares no code with the HIP path.

The per-site and per-particle arithmetic lives in ``cpic_oracle.c`` (plain C,
double precision, written for readability); this module adds the parts that
are plainer in numpy: the FFT Poisson solve of the MV initial condition
(Sec. II.A, where the paper names an FFT), unit conversion, and the loop
that interleaves the field leapfrog with the particle push.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpic_oracle.so")
SRC_PATH = os.path.join(HERE, "cpic_oracle.c")
SRC_PATHS = [SRC_PATH, os.path.join(HERE, "cpic_oracle_su2.c")]
HBARC_GEV_FM = 0.1973269804
NCOL = 20  # particle record columns (see COLUMNS)
COLUMNS = ["x", "y", "eta", "px", "py", "peta"] + [f"Q{a}" for a in range(1, 9)] + [
    "cx", "cy", "deta", "ux0", "uy0", "pt0"]


def build(force: bool = False) -> str:
    """Compile the oracle's C part (gcc, -O2, OpenMP, IEEE double)."""
    newest = max(os.path.getmtime(p) for p in SRC_PATHS)
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < newest:
        tmp = LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, *SRC_PATHS, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = load_library(LIB_PATH)
    return _lib


def load_library(path):
    """A compiled copy of the oracle's C part with its argument types set
    (the oracle's own library, or a copy the tests build from modified
    sources to show that a pin catches a planted mistake)."""
    L = ctypes.CDLL(path)
    d, i, u64, p = ctypes.c_double, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p
    sig = {
        "orc_forces": (None, [i, d, p, p, p, p]),
        "orc_kick": (None, [i, d, d, p, p, p, p]),
        "orc_drift": (None, [i, d, d, p, p, p, p]),
        "orc_field_step": (None, [i, i, d, d, p, p, p, p]),
        "orc_energy": (None, [i, d, p, p, p, p, p]),
        "orc_gauss": (None, [i, p, p, p, p, p]),
        "orc_unitarity": (None, [i, p, p]),
        "orc_philox": (None, [p, p, p]),
        "orc_mv_charges": (None, [i, u64, i, i, d, p]),
        "orc_wilson_mult": (None, [i, p, p]),
        "orc_pure_gauge": (None, [i, p, p]),
        "orc_kv_links": (i, [i, p, p, p, d, i, p]),
        "orc_pi0": (None, [i, p, p, p, p]),
        "orc_q0": (None, [i, p]),
        "orc_casimirs": (None, [p, p, p]),
        "orc_particles_init": (None, [i, i, u64, d, d, i, i, p]),
        "orc_particle_fields": (None, [i, i, d, i, p, p, p, p, p, p, p]),
        "orc_particles_step": (i, [i, i, i, d, d, i, i, p, p, p, p, p, p, i, p, p]),
        "orc_link_generator": (None, [p, p]),
        "orc_particles_observe": (None, [d, d, i, i, p, p]),
        "orc_jet_step": (None, [i, i, i, d, d, i, p, p, p, p, p, p, p, p]),
        "orc_generator": (None, [i, p]),
        "orc_proj": (None, [p, p]),
        "orc_expi": (None, [p, d, p]),
        "orc_set_threads": (None, [i]),
        "orc_max_threads": (i, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def set_threads(n: int) -> int:
    """Run the oracle's parallel loops on n OpenMP threads; returns the previous count."""
    prev = lib().orc_max_threads()
    lib().orc_set_threads(int(n))
    return prev


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------
# state containers (hat units)
# ----------------------------------------------------------------------------
def empty_state(N: int) -> dict:
    """U: (2,N,N,3,3) complex128 identity links; phi, pi: (N,N,8); E: (2,N,N,8)."""
    U = np.zeros((2, N, N, 3, 3), np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return {"U": U, "phi": np.zeros((N, N, 8)), "E": np.zeros((2, N, N, 8)),
            "pi": np.zeros((N, N, 8))}


def forces(N, t, U, phi):
    FE = np.zeros((2, N, N, 8))
    Fp = np.zeros((N, N, 8))
    lib().orc_forces(N, t, _ptr(U), _ptr(phi), _ptr(FE), _ptr(Fp))
    return FE, Fp


def energy(N, t, U, phi, E, pi):
    out = np.zeros(4)
    lib().orc_energy(N, t, _ptr(U), _ptr(phi), _ptr(E), _ptr(pi), _ptr(out))
    return out


def gauss(N, U, phi, E, pi):
    G = np.zeros((N, N, 8))
    lib().orc_gauss(N, _ptr(U), _ptr(phi), _ptr(E), _ptr(pi), _ptr(G))
    return G


def unitarity(N, U):
    out = np.zeros(2)
    lib().orc_unitarity(N, _ptr(U), _ptr(out))
    return out


def field_step(N, n, dt, st, t_fixed=0.0):
    """Leapfrog step n -> n+1 in place on st (U, phi at n -> n+1; E, pi at n-1/2 -> n+1/2)."""
    lib().orc_field_step(N, n, dt, t_fixed, _ptr(st["U"]), _ptr(st["phi"]), _ptr(st["E"]), _ptr(st["pi"]))


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint64)
    k = np.ascontiguousarray(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def generator(a: int) -> np.ndarray:
    out = np.zeros((3, 3), np.complex128)
    lib().orc_generator(a, _ptr(out))
    return out


def proj(M) -> np.ndarray:
    M = np.ascontiguousarray(M, np.complex128)
    out = np.zeros(8)
    lib().orc_proj(_ptr(M), _ptr(out))
    return out


def expi(x, scale=1.0) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    out = np.zeros((3, 3), np.complex128)
    lib().orc_expi(_ptr(x), scale, _ptr(out))
    return out


def q0(rep: int) -> np.ndarray:
    out = np.zeros(8)
    lib().orc_q0(rep, _ptr(out))
    return out


def casimirs(Q) -> tuple:
    Q = np.ascontiguousarray(Q, np.float64)
    q2, q3 = ctypes.c_double(), ctypes.c_double()
    lib().orc_casimirs(_ptr(Q), ctypes.byref(q2), ctypes.byref(q3))
    return q2.value, q3.value


# ----------------------------------------------------------------------------
# units (Sec. VII.A parameters; hbar c converts fm to 1/GeV)
# ----------------------------------------------------------------------------
def lattice_spacing(L_fm: float, N: int) -> float:
    """a in 1/GeV."""
    return (L_fm / N) / HBARC_GEV_FM


def alpha_s(Qs_GeV=2.0, nf=3, lam_qcd=0.2):
    """One-loop running coupling of Sec. VII.A."""
    return 1.0 / ((33 - 3 * nf) / (12 * math.pi) * math.log(Qs_GeV ** 2 / lam_qcd ** 2))


# ----------------------------------------------------------------------------
# MV initial condition (Sec. II, II.A)
# ----------------------------------------------------------------------------
def poisson_kernel(N: int, mhat: float, uvhat: float) -> np.ndarray:
    """K(k) = 1/(khat^2 + m^2) with the lattice khat^2 = 4 sum_i sin^2(pi k_i/N),
    K(0) = 0, and K = 0 above the UV cut |k| = (2 pi/N) |k~| > Lambda (k~ signed).
    uvhat <= 0 disables the UV cut."""
    k = np.arange(N)
    ks = np.where(k > N // 2, k - N, k).astype(np.float64)
    s2 = np.sin(np.pi * k / N) ** 2
    khat2 = 4.0 * (s2[:, None] + s2[None, :])
    K = 1.0 / (khat2 + mhat * mhat)
    K[0, 0] = 0.0
    if uvhat > 0:
        kc = (2 * np.pi / N) * np.sqrt(ks[:, None] ** 2 + ks[None, :] ** 2)
        K[kc > uvhat] = 0.0
    return K


def poisson_solve(rho: np.ndarray, K: np.ndarray) -> np.ndarray:
    """alpha = IFFT[FFT[rho] K] per colour; rho shape (N,N,8) -> real (N,N,8)."""
    f = np.fft.fft2(rho, axes=(0, 1))
    return np.ascontiguousarray(np.real(np.fft.ifft2(f * K[:, :, None], axes=(0, 1))))


def mv_charges(N, seed, nucleus, sheet, sigma):
    rho = np.zeros((N, N, 8))
    lib().orc_mv_charges(N, seed, nucleus, sheet, sigma, _ptr(rho))
    return rho


def nucleus_links(N, seed, nucleus, n_sheets, g2mua, mhat, uvhat, rho_scale=1.0):
    """Pure-gauge links U^X_i of one nucleus: sheets of Gaussian charge, Poisson
    solve, Wilson line V^+ = prod_n exp(-i alpha_n), U^X_i(x) = V(x) V(x+i)^+."""
    K = poisson_kernel(N, mhat, uvhat)
    sigma = rho_scale * g2mua / math.sqrt(n_sheets)
    Vdag = np.zeros((N, N, 3, 3), np.complex128)
    Vdag[..., 0, 0] = Vdag[..., 1, 1] = Vdag[..., 2, 2] = 1.0
    for n in range(n_sheets):
        alpha = poisson_solve(mv_charges(N, seed, nucleus, n, sigma), K)
        lib().orc_wilson_mult(N, _ptr(alpha), _ptr(Vdag))
    UX = np.zeros((2, N, N, 3, 3), np.complex128)
    lib().orc_pure_gauge(N, _ptr(Vdag), _ptr(UX))
    return UX


def glasma_links(N, UA, UB, tol=1e-14, maxit=50):
    U = np.zeros_like(UA)
    it = ctypes.c_int()
    fails = lib().orc_kv_links(N, _ptr(UA), _ptr(UB), _ptr(U), tol, maxit, ctypes.byref(it))
    if fails:
        raise RuntimeError(f"initial-link Newton solve failed on {fails} links")
    return U, it.value


def pi0(N, UA, UB, U):
    pi = np.zeros((N, N, 8))
    lib().orc_pi0(N, _ptr(UA), _ptr(UB), _ptr(U), _ptr(pi))
    return pi


def mv_initial_condition(N, L_fm, g2mu_GeV, m_ir_GeV, uv_GeV, n_sheets, seed, rho_scale_B=1.0,
                         keep_nuclei=False):
    """Glasma state at tau = 0 in hat units: U, phi = 0, E = 0, pi(0).
    rho_scale_B = 0 gives the one-nucleus limit."""
    a = lattice_spacing(L_fm, N)
    g2mua, mhat, uvhat = g2mu_GeV * a, m_ir_GeV * a, uv_GeV * a
    UA = nucleus_links(N, seed, 0, n_sheets, g2mua, mhat, uvhat)
    UB = nucleus_links(N, seed, 1, n_sheets, g2mua, mhat, uvhat, rho_scale=rho_scale_B)
    U, iters = glasma_links(N, UA, UB)
    st = empty_state(N)
    st["U"] = U
    st["pi"] = pi0(N, UA, UB, U)
    st["newton_iters"] = iters
    if keep_nuclei:
        st["UA"], st["UB"] = UA, UB
    return st


# ----------------------------------------------------------------------------
# particles (Sec. III.B, IV.B)
# ----------------------------------------------------------------------------
def particles_init(N, n, seed, pt_min_hat, pt_max_hat, azimuth_uniform=True, rep=0):
    P = np.zeros((n, NCOL))
    if n:
        lib().orc_particles_init(N, n, seed, pt_min_hat, pt_max_hat, int(azimuth_uniform), rep, _ptr(P))
    return P


def link_generator(U) -> np.ndarray:
    """Components a^a of -i log U (principal matrix logarithm), U = exp(i a^a T^a)."""
    out = np.zeros(8)
    lib().orc_link_generator(_ptr(np.ascontiguousarray(U, np.complex128)), _ptr(out))
    return out


def particle_fields(N, n, dt, site, U, phi, E_old, E_new, pi_old, pi_new):
    out = np.zeros((6, 8))
    lib().orc_particle_fields(N, n, dt, site, _ptr(U), _ptr(phi), _ptr(E_old), _ptr(E_new),
                              _ptr(pi_old), _ptr(pi_new), _ptr(out))
    return out


def particles_observe(t, mhat, is_static, P):
    out = np.zeros(4)
    lib().orc_particles_observe(t, mhat, int(is_static), P.shape[0], _ptr(P), _ptr(out))
    return out


def transport_coefficients(tau_form, tau, broadening):
    """Instantaneous transport coefficients and anisotropies from a sampled
    broadening series ([eq:kappalt], [eq:qhati], the heavy-quark anisotropy
    <dp_L^2>/<dp_T^2> and the jet anisotropy [eq:jetanisotropy]).

    tau: (k,) sample times; broadening: (k, 4) the means <dp_T^2>, <dp_L^2>,
    <dp_par^2>, <dp_perp^2> at those times (par / perp: along / across the
    initial transverse direction, x / y for jets launched along x, whose
    longitudinal component is <dp_z^2> = <dp_L^2>).  Every <dp^2> vanishes at
    the formation time tau_form, which opens the series.  The derivative
    d<dp^2>/dtau of each component is taken between consecutive points, at the
    midpoint (the central difference: exact there for a quadratic series).

    Returns (k, 8): tau_mid, kappa_T, kappa_L, qhat_par, qhat_perp (the
    derivatives of the four means over [tau_{k-1}, tau_k], tau_{-1} = tau_form),
    tau_k, <dp_L^2>/<dp_T^2>, <dp_L^2>/<dp_perp^2>."""
    tau = np.asarray(tau, dtype=np.float64)
    b = np.asarray(broadening, dtype=np.float64)
    t = np.concatenate([[tau_form], tau])
    v = np.concatenate([np.zeros((1, 4)), b])
    out = np.zeros((len(tau), 8))
    out[:, 0] = 0.5 * (t[1:] + t[:-1])
    out[:, 1:5] = (v[1:] - v[:-1]) / (t[1:] - t[:-1])[:, None]
    out[:, 5] = tau
    with np.errstate(divide="ignore", invalid="ignore"):
        out[:, 6] = b[:, 1] / b[:, 0]
        out[:, 7] = b[:, 1] / b[:, 3]
    return out


class Jets:
    """Light-like jet limit of the momentum broadening (Sec. V.B,
    [eq:mombroadjets]): straight paths along +x at the speed of light, one per
    lattice site, starting at x = site + x_off at step n_form.  W (N,N,3,3) is
    each path's Wilson line, F (N,N,3,8) the accumulated transported force
    sum_n w f~_i(t_n), i = x, y, z (see orc_jet_step for the discretisation)."""

    def __init__(self, N, dt, n_form=0, x_off=0.0, stride=1):
        assert 0 < dt <= 1 and stride >= 1 and 0 <= x_off < 1
        self.N, self.dt, self.n_form, self.x_off, self.stride = N, dt, n_form, float(x_off), int(stride)
        self.W = np.zeros((N, N, 3, 3), np.complex128)
        self.F = np.zeros((N, N, 3, 8))

    def step(self, n, U, phi, E_old, E_new, pi_old, pi_new):
        """Step n with U(n), phi(n), E(n -+ 1/2), pi(n -+ 1/2) (the push's inputs)."""
        lib().orc_jet_step(self.N, n, self.n_form, self.dt, self.x_off, self.stride, _ptr(U), _ptr(phi),
                           _ptr(E_old), _ptr(E_new), _ptr(pi_old), _ptr(pi_new), _ptr(self.W), _ptr(self.F))

    def observe(self, rep=0):
        """<dp_i^2>, i = x, y, z, in hat units for charges of representation rep:
        a charge rotated uniformly over its orbit has <Q^a Q^b> = delta^ab q2 / 8
        ([eq:qnpointfct_main]), so <(Q.F_i)^2> = q2 / 8 |F_i|^2, averaged over
        the paths."""
        q = q0(rep)
        q2 = float(np.dot(q, q))
        return q2 / 8.0 * np.mean(np.sum(self.F ** 2, axis=-1), axis=(0, 1))


class Run:
    """Interleaved field leapfrog and particle push (Sec. II.A and III.B).

    step n: the fields go U(n), phi(n), E(n-1/2), pi(n-1/2) -> U(n+1), phi(n+1),
    E(n+1/2), pi(n+1/2); then, if n >= n_form, the particles are pushed at t_n
    with U(n), phi(n), E(n +- 1/2), pi(n +- 1/2).  mhat = inf selects the static
    branch.  color = "cpic" rotates the charges with the links (Eq. colorrotnum),
    "log" integrates dQ/dt = i[Q, A.v] with A from the matrix logarithm of the
    links (the alternative of Sec. III.B).  An optional Jets object is stepped
    with the same inputs as the push."""

    def __init__(self, N, dt, state, particles=None, mhat=math.inf, n_form=0, n0=0, jets=None, color="cpic"):
        self.N, self.dt, self.n = N, dt, n0
        self.st = {k: np.ascontiguousarray(state[k]).copy() for k in ("U", "phi", "E", "pi")}
        self.P = None if particles is None else np.ascontiguousarray(particles).copy()
        self.is_static = math.isinf(mhat)
        self.mhat = 0.0 if self.is_static else float(mhat)
        self.n_form = n_form
        self.errors = 0
        self.jets = jets
        self.color_mode = {"cpic": 0, "log": 1}[color]
        self.t_field = self.t_push = 0.0   # wall seconds spent in the field step and in the push
        # p^tau from its equation of motion [eq:ptaueq] beside the constraint (moving
        # particles); a run started past formation starts it from the constraint
        self.ptau_ode = None if self.P is None or self.is_static else self.ptau_constraint()

    def step(self):
        N, n, st = self.N, self.n, self.st
        push = self.P is not None and self.P.shape[0] > 0 and n >= self.n_form
        jets = self.jets is not None and n >= self.jets.n_form
        if push or jets:
            U_n, phi_n = st["U"].copy(), st["phi"].copy()
            E_old, pi_old = st["E"].copy(), st["pi"].copy()
        t0 = time.perf_counter()
        field_step(N, n, self.dt, st)
        t1 = time.perf_counter()
        self.t_field += t1 - t0
        if push:
            self.errors += lib().orc_particles_step(
                N, n, self.n_form, self.dt, self.mhat, int(self.is_static), self.color_mode, _ptr(U_n), _ptr(phi_n),
                _ptr(E_old), _ptr(st["E"]), _ptr(pi_old), _ptr(st["pi"]), self.P.shape[0], _ptr(self.P),
                None if self.ptau_ode is None else _ptr(self.ptau_ode))
            self.t_push += time.perf_counter() - t1
        if jets:
            self.jets.step(n, U_n, phi_n, E_old, st["E"], pi_old, st["pi"])
        self.n += 1

    def observe(self):
        """Sums of (dp_T^2, dp_L^2, dp_par^2, dp_perp^2) at t_n in hat units."""
        return particles_observe(self.n * self.dt, self.mhat, self.is_static, self.P)

    def ptau_constraint(self):
        """p^tau of every particle at t_n from the constraint [eq:ptau] (hat units)."""
        t = self.n * self.dt
        P = self.P
        return np.sqrt(P[:, 3] ** 2 + P[:, 4] ** 2 + (t * P[:, 5]) ** 2 + self.mhat ** 2)
