"""Python binding of libcpic (include/cpic.h): the colored particle-in-cell
hot path of arXiv:2303.05599 on MI355X.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  If the compiled library is missing this module raises; there
is no fallback implementation.  PyTorch, when present, only supplies the HIP
stream the library enqueues on.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpic.so")

FP64, FP32 = 0, 1
REP_FUND, REP_ADJ = 0, 1
COLOR_ROTATE, COLOR_LOG = 0, 1
PUSH_GATHER, PUSH_TABLE, PUSH_TILE = 0, 1, 2
STATE_U, STATE_PHI, STATE_E, STATE_PI, STATE_PARTICLES, STATE_STEP, STATE_JET_W, STATE_JET_F, STATE_PTAU = range(9)
ERRORS = {-1: "INVALID", -2: "NOMEM", -3: "HIP", -4: "IC_NEWTON", -5: "NAN", -6: "DRIFT", -7: "CAPACITY",
          -8: "CELL_JUMP", -9: "IO"}


class GlasmaParams(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("L_fm", ctypes.c_double), ("g2mu_GeV", ctypes.c_double),
                ("m_ir_GeV", ctypes.c_double), ("uv_GeV", ctypes.c_double), ("n_sheets", ctypes.c_int32),
                ("dtau_over_a", ctypes.c_double), ("tau_max_fm", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("precision", ctypes.c_int32), ("reunit_every", ctypes.c_int32), ("record_every", ctypes.c_int32),
                ("n_colors", ctypes.c_int32)]


class ParticleParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mass_GeV", ctypes.c_double), ("pT_min_GeV", ctypes.c_double),
                ("pT_max_GeV", ctypes.c_double), ("azimuth_uniform", ctypes.c_int32),
                ("tau_form_fm", ctypes.c_double), ("rep", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("color_update", ctypes.c_int32)]


class JetParams(ctypes.Structure):
    _fields_ = [("x_offset", ctypes.c_double), ("stride", ctypes.c_int32), ("tau_form_fm", ctypes.c_double),
                ("rep", ctypes.c_int32)]


GLASMA_DEFAULTS = dict(N=32, L_fm=6.0, g2mu_GeV=2.0, m_ir_GeV=0.2, uv_GeV=10.0, n_sheets=1, dtau_over_a=0.125,
                       tau_max_fm=1.0, seed=1, precision=FP64, reunit_every=16, record_every=8, n_colors=3)
PARTICLE_DEFAULTS = dict(n=0, mass_GeV=math.inf, pT_min_GeV=0.0, pT_max_GeV=0.0, azimuth_uniform=1,
                         tau_form_fm=0.0, rep=REP_FUND, seed=2, color_update=COLOR_ROTATE)


class CpicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{ERRORS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libcpic.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, d, sz, cp = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_size_t, ctypes.c_char_p)
        pp = ctypes.POINTER(ctypes.c_void_p)
        sigs = {
            "cpic_create": [ctypes.POINTER(GlasmaParams), ctypes.POINTER(ParticleParams), P, pp],
            "cpic_init_mv": [P], "cpic_step": [P, i32], "cpic_evolve": [P, d], "cpic_sync": [P],
            "cpic_current_step": [P, ctypes.POINTER(i64)], "cpic_num_samples": [P, ctypes.POINTER(i32)],
            "cpic_observables": [P, P, P, P, i32], "cpic_observables_full": [P, P, i32],
            "cpic_diagnostics": [P, P], "cpic_get_state": [P, i32, P, sz], "cpic_set_state": [P, i32, P, sz],
            "cpic_save": [P, cp], "cpic_load": [P, cp], "cpic_set_launch": [P, i32, i32, i32, i32, i32],
            "cpic_set_timing": [P, i32], "cpic_set_push_lanes": [P, i32], "cpic_get_launch": [P, P],
            "cpic_set_store_policy": [P, i32],
            "cpic_tune": [P, i32, P, sz],
            "cpic_timing": [P, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(i64), ctypes.POINTER(i64)],
            "cpic_straggler_pushes": [P, ctypes.POINTER(i64)],
            "cpic_set_watchdog": [P, i32, d, d, d],
            "cpic_diagnostics_summary": [P, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(d)],
            "cpic_transport": [P, P, i32, ctypes.POINTER(i32)],
            "cpic_jets_transport": [P, P, i32, ctypes.POINTER(i32)],
            "cpic_batch_create": [i32, ctypes.POINTER(GlasmaParams), ctypes.POINTER(ParticleParams), P, pp],
            "cpic_batch_init_mv": [P], "cpic_batch_run": [P], "cpic_batch_step": [P, i32], "cpic_batch_sync": [P],
            "cpic_batch_tune": [P, i32, P, sz], "cpic_batch_set_launch": [P, i32, i32, i32, i32],
            "cpic_batch_set_group_bytes": [P, i64],
            "cpic_batch_set_lanes": [P, i32],
            "cpic_batch_get_launch": [P, P], "cpic_batch_num_events": [P, ctypes.POINTER(i32)],
            "cpic_batch_current_step": [P, i32, ctypes.POINTER(i64)],
            "cpic_batch_observables": [P, i32, P, i32, ctypes.POINTER(i32)],
            "cpic_batch_get_state": [P, i32, i32, P, sz],
            "cpic_jets_enable": [P, ctypes.POINTER(JetParams)],
            "cpic_set_push_mode": [P, i32], "cpic_get_push_mode": [P, ctypes.POINTER(i32)],
            "cpic_jets_observables": [P, P, i32, ctypes.POINTER(i32)],
            "cpic_jets_timing": [P, ctypes.POINTER(d), ctypes.POINTER(i64)],
            "cpic_field_diagnostics_noalloc": [i32, i32, d, i64, P, P, P],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int32
        for name in ("cpic_last_error", "cpic_batch_last_error"):
            f = getattr(L, name)
            f.argtypes = [P]
            f.restype = ctypes.c_char_p
        L.cpic_destroy.argtypes = [P]
        L.cpic_destroy.restype = None
        L.cpic_batch_destroy.argtypes = [P]
        L.cpic_batch_destroy.restype = None
        _lib = L
    return _lib


def current_stream():
    """The HIP stream torch is using on the current device (None without torch/GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return None


def field_diagnostics_noalloc(precision, N, dtau_over_a, n, fields_dev_ptr, out_dev_ptr, stream=None):
    """cpic_field_diagnostics_noalloc: field diagnostics of a caller-owned device
    buffer set (68 N^2 reals, the library's layout) into 8 doubles of caller-owned
    device memory; asynchronous on `stream` (a raw hipStream_t, default torch's)."""
    L = lib()
    s = current_stream() if stream is None else stream
    st = L.cpic_field_diagnostics_noalloc(precision, N, dtau_over_a, n, ctypes.c_void_p(fields_dev_ptr),
                                          ctypes.c_void_p(out_dev_ptr), s)
    if st:
        raise CpicError(st, L.cpic_last_error(None).decode())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _glasma(params):
    p = dict(GLASMA_DEFAULTS)
    p.update(params or {})
    return GlasmaParams(**p)


def _particles(params):
    p = dict(PARTICLE_DEFAULTS)
    p.update(params or {})
    return ParticleParams(**p)


class Context:
    """One Glasma event with its test particles (cpic_ctx)."""

    def __init__(self, glasma=None, particles=None, stream="torch"):
        L = lib()
        self.gp, self.pp = _glasma(glasma), _particles(particles)
        s = current_stream() if stream == "torch" else stream
        h = ctypes.c_void_p()
        st = L.cpic_create(ctypes.byref(self.gp), ctypes.byref(self.pp), s, ctypes.byref(h))
        if st:
            raise CpicError(st, L.cpic_last_error(None).decode())
        self.h = h
        self.N = self.gp.N
        self.np = self.pp.n

    def _chk(self, st):
        if st:
            raise CpicError(st, lib().cpic_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().cpic_destroy(self.h)
            self.h = None

    def __del__(self):
        if lib is not None:     # None once the interpreter has cleared module globals at exit
            self.close()

    def init_mv(self):
        self._chk(lib().cpic_init_mv(self.h))

    def step(self, n=1):
        self._chk(lib().cpic_step(self.h, n))

    def evolve(self, tau_fm):
        self._chk(lib().cpic_evolve(self.h, tau_fm))

    def sync(self):
        self._chk(lib().cpic_sync(self.h))

    @property
    def n(self):
        v = ctypes.c_int64()
        self._chk(lib().cpic_current_step(self.h, ctypes.byref(v)))
        return v.value

    def num_samples(self):
        v = ctypes.c_int32()
        self._chk(lib().cpic_num_samples(self.h, ctypes.byref(v)))
        return v.value

    def observables(self):
        """(k, 6): tau_fm, <dp_T^2>, <dp_L^2>, <dp_par^2>, <dp_perp^2>, count (GeV^2)."""
        k = self.num_samples()
        out = np.zeros((max(k, 1), 6))
        self._chk(lib().cpic_observables_full(self.h, _ptr(out), k))
        return out[:k]

    def transport(self):
        """(k, 8): tau_mid, kappa_T, kappa_L, qhat_x, qhat_y, tau_k, <dp_L^2>/<dp_T^2>,
        <dp_z^2>/<dp_y^2> (cpic_transport)."""
        k = self.num_samples()
        out = np.zeros((max(k, 1), 8))
        n = ctypes.c_int32()
        self._chk(lib().cpic_transport(self.h, _ptr(out), k, ctypes.byref(n)))
        return out[:n.value]

    def jet_transport(self):
        """(k, 6): tau_mid, qhat_x, qhat_y, qhat_z, tau_k, <dp_z^2>/<dp_y^2> of the light-like paths."""
        n = ctypes.c_int32()
        self._chk(lib().cpic_jets_transport(self.h, None, 1 << 30, ctypes.byref(n)))
        out = np.zeros((max(n.value, 1), 6))
        self._chk(lib().cpic_jets_transport(self.h, _ptr(out), n.value, ctypes.byref(n)))
        return out[:n.value]

    def diagnostics(self):
        out = np.zeros(10)
        self._chk(lib().cpic_diagnostics(self.h, _ptr(out)))
        return out

    def diagnostics_summary(self):
        """(gauss_l2, energy_lat, unitarity_max, casimir_max) (cpic_diagnostics_summary)."""
        v = [ctypes.c_double() for _ in range(4)]
        self._chk(lib().cpic_diagnostics_summary(self.h, *(ctypes.byref(x) for x in v)))
        return tuple(x.value for x in v)

    def _shape(self, which):
        N = self.N
        if self.gp.n_colors == 2:
            return {STATE_U: (2, N, N, 2, 2), STATE_PHI: (N, N, 3), STATE_E: (2, N, N, 3), STATE_PI: (N, N, 3),
                    STATE_PARTICLES: (self.np, 20), STATE_STEP: (1,)}[which]
        return {STATE_U: (2, N, N, 3, 3), STATE_PHI: (N, N, 8), STATE_E: (2, N, N, 8), STATE_PI: (N, N, 8),
                STATE_PARTICLES: (self.np, 20), STATE_STEP: (1,), STATE_JET_W: (N, N, 3, 3),
                STATE_JET_F: (N, N, 3, 8), STATE_PTAU: (self.np, 2)}[which]

    def get_state(self, which):
        dt = (np.complex128 if which in (STATE_U, STATE_JET_W) else
              (np.int64 if which == STATE_STEP else np.float64))
        a = np.zeros(self._shape(which), dt)
        self._chk(lib().cpic_get_state(self.h, which, _ptr(a), a.nbytes))
        return a

    def set_state(self, which, arr):
        dt = (np.complex128 if which in (STATE_U, STATE_JET_W) else
              (np.int64 if which == STATE_STEP else np.float64))
        a = np.ascontiguousarray(np.asarray(arr, dt).reshape(self._shape(which)))
        self._chk(lib().cpic_set_state(self.h, which, _ptr(a), a.nbytes))

    def state(self):
        return {"U": self.get_state(STATE_U), "phi": self.get_state(STATE_PHI), "E": self.get_state(STATE_E),
                "pi": self.get_state(STATE_PI)}

    def load_state(self, st, n=0, particles=None):
        """Install a lattice state (hat units, oracle layout) at step n."""
        self.set_state(STATE_STEP, [n])
        self.set_state(STATE_U, st["U"])
        self.set_state(STATE_PHI, st["phi"])
        self.set_state(STATE_E, st["E"])
        self.set_state(STATE_PI, st["pi"])
        if particles is not None:
            self.set_state(STATE_PARTICLES, particles)

    def save(self, path):
        self._chk(lib().cpic_save(self.h, str(path).encode()))

    def load(self, path):
        self._chk(lib().cpic_load(self.h, str(path).encode()))

    def set_launch(self, bx, by, xcd_remap=1, waves=1, variant=0):
        """Field-kernel launch; variant 0 site-parallel, 1 link-parallel, 2 LDS halo tiles,
        3 two-row-link LDS tiles, 4 the fused step (tile push, PUSH_TILE)."""
        self._chk(lib().cpic_set_launch(self.h, bx, by, xcd_remap, waves, variant))

    def set_watchdog(self, every=64, max_unitarity=1e-8, max_gauss_drift=1e-8, max_casimir_drift=1e-8):
        """Drift watchdog every `every` steps (0: off); breaches raise at the next sync."""
        self._chk(lib().cpic_set_watchdog(self.h, every, max_unitarity, max_gauss_drift, max_casimir_drift))

    def set_store_policy(self, non_temporal):
        """New links and phi of the compressed-tile field update stored non-temporal (1) or not (0)."""
        self._chk(lib().cpic_set_store_policy(self.h, int(non_temporal)))

    def set_push_lanes(self, lanes):
        self._chk(lib().cpic_set_push_lanes(self.h, lanes))

    def set_push_mode(self, mode):
        """PUSH_GATHER (fields per particle), PUSH_TABLE (per-site force table) or
        PUSH_TILE (fused step: fields per tile in the field update's workgroup)."""
        self._chk(lib().cpic_set_push_mode(self.h, mode))

    def push_mode(self):
        v = ctypes.c_int32()
        self._chk(lib().cpic_get_push_mode(self.h, ctypes.byref(v)))
        return v.value

    def get_launch(self):
        out = np.zeros(7, np.int32)
        self._chk(lib().cpic_get_launch(self.h, _ptr(out)))
        return dict(zip(("bx", "by", "xcd_remap", "waves", "push_lanes", "variant", "nt_store"), out.tolist()))

    def tune(self, reps=5):
        """Time the launch candidates on the current state and keep the fastest; returns the report."""
        buf = ctypes.create_string_buffer(16384)
        self._chk(lib().cpic_tune(self.h, reps, buf, len(buf)))
        return buf.value.decode()

    def set_timing(self, enable=True):
        self._chk(lib().cpic_set_timing(self.h, int(enable)))

    def enable_jets(self, x_offset=0.0, stride=1, tau_form_fm=0.0, rep=REP_FUND):
        """Light-like jet limit: one straight path along +x per site (cpic_jets_enable)."""
        jp = JetParams(x_offset=x_offset, stride=stride, tau_form_fm=tau_form_fm, rep=rep)
        self._chk(lib().cpic_jets_enable(self.h, ctypes.byref(jp)))

    def jet_observables(self):
        """(k, 4): tau_fm, <dp_x^2>, <dp_y^2>, <dp_z^2> of the light-like paths (GeV^2)."""
        cap = max(self.num_jet_samples(), 1)
        ns = ctypes.c_int32()
        out = np.zeros((cap, 4))
        self._chk(lib().cpic_jets_observables(self.h, _ptr(out), cap, ctypes.byref(ns)))
        return out[:ns.value]

    def num_jet_samples(self):
        ns = ctypes.c_int32()
        self._chk(lib().cpic_jets_observables(self.h, None, 1 << 30, ctypes.byref(ns)))
        return ns.value

    def jets_timing(self):
        ms, k = ctypes.c_double(), ctypes.c_int64()
        self._chk(lib().cpic_jets_timing(self.h, ctypes.byref(ms), ctypes.byref(k)))
        return {"jets_ms": ms.value, "n_jets": k.value}

    def timing(self):
        f, p = ctypes.c_double(), ctypes.c_double()
        nf, npu = ctypes.c_int64(), ctypes.c_int64()
        self._chk(lib().cpic_timing(self.h, ctypes.byref(f), ctypes.byref(p), ctypes.byref(nf), ctypes.byref(npu)))
        ns = ctypes.c_int64()
        self._chk(lib().cpic_straggler_pushes(self.h, ctypes.byref(ns)))
        return {"field_ms": f.value, "push_ms": p.value, "n_field": nf.value, "n_push": npu.value,
                "straggler_pushes": ns.value}


class Batch:
    """Many events evolved together (cpic_batch)."""

    def __init__(self, glasma_list, particle_list, stream="torch"):
        L = lib()
        n = len(glasma_list)
        self.gps = (GlasmaParams * n)(*[_glasma(g) for g in glasma_list])
        self.pps = (ParticleParams * n)(*[_particles(p) for p in particle_list])
        s = current_stream() if stream == "torch" else stream
        h = ctypes.c_void_p()
        st = L.cpic_batch_create(n, self.gps, self.pps, s, ctypes.byref(h))
        if st:
            raise CpicError(st, L.cpic_batch_last_error(None).decode())
        self.h, self.n_events = h, n

    def _chk(self, st):
        if st:
            raise CpicError(st, lib().cpic_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().cpic_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        if lib is not None:     # None once the interpreter has cleared module globals at exit
            self.close()

    def init_mv(self):
        self._chk(lib().cpic_batch_init_mv(self.h))

    def run(self):
        """Evolve every event to its tau_max (asynchronous)."""
        self._chk(lib().cpic_batch_run(self.h))

    def step(self, k):
        """Advance every unfinished event by up to k steps (asynchronous)."""
        self._chk(lib().cpic_batch_step(self.h, k))

    def n(self, event):
        v = ctypes.c_int64()
        self._chk(lib().cpic_batch_current_step(self.h, event, ctypes.byref(v)))
        return v.value

    def tune(self, reps=5):
        """Time the batched field launch per tile shape; keep the fastest; returns the report."""
        buf = ctypes.create_string_buffer(8192)
        self._chk(lib().cpic_batch_tune(self.h, reps, buf, len(buf)))
        return buf.value.decode()

    def set_launch(self, bx, by, xcd_remap=1, push_lanes=1):
        self._chk(lib().cpic_batch_set_launch(self.h, bx, by, xcd_remap, push_lanes))

    def set_lanes(self, lanes):
        """Launch lanes, 1 to 4: the launch groups dealt to that many concurrent streams (default 2)."""
        self._chk(lib().cpic_batch_set_lanes(self.h, lanes))

    def set_group_bytes(self, nbytes):
        """Working-set budget of one launch group (0: one group for all events)."""
        self._chk(lib().cpic_batch_set_group_bytes(self.h, int(nbytes)))

    def get_launch(self):
        out = np.zeros(4, np.int32)
        self._chk(lib().cpic_batch_get_launch(self.h, _ptr(out)))
        return dict(zip(("bx", "by", "xcd_remap", "push_lanes"), out.tolist()))

    def sync(self):
        self._chk(lib().cpic_batch_sync(self.h))

    def observables(self, event):
        ns = ctypes.c_int32()
        cap = 4096
        out = np.zeros((cap, 6))
        self._chk(lib().cpic_batch_observables(self.h, event, _ptr(out), cap, ctypes.byref(ns)))
        return out[:ns.value]

    def get_state(self, event, which, shape, dtype=np.float64):
        a = np.zeros(shape, dtype)
        self._chk(lib().cpic_batch_get_state(self.h, event, which, _ptr(a), a.nbytes))
        return a
