"""GPU tests of the SU(2) variant (n_colors = 2) against the SU(2) oracle.

  * the MV initial condition (Philox charges, FFT Poisson solve, Wilson lines,
    closed-form tau = 0 links, pi(0)) at 1e-12;
  * the leapfrog from the initial condition and from a random state with all
    fields nonzero, 1e-11 per component over 50 steps (the library holds
    links as quaternions, the oracle as 2x2 matrices);
  * moving and static particles (Darboux charges, CPIC rotation, Euler push),
    cells bit-exact, records at 1e-11, samples at 1e-10;
  * single precision within the FP32 budget; graph replay, eager stepping and
    checkpoint resume bitwise; diagnostics; rejected combinations;
  * at 512^2: Casimir scaling of the static broadening, adjoint over
    fundamental = q2(A)/q2(F) = 4 (8/3 after the division by D_R).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import su2

cp = pytest.importorskip("paper_2303_05599_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-11
DT = 0.125


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    cp.lib()
    yield


def rel_err(a, ref):
    a, ref = np.asarray(a), np.asarray(ref)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2)) if ref.size else 0.0
    den = np.maximum(np.abs(ref), rms)
    den = np.where(den == 0, 1.0, den)
    return float(np.max(np.abs(a - ref) / den)) if a.size else 0.0


def event(N, steps, L=None, precision=cp.FP64, seed=61, n_sheets=2, uv=10.0):
    L = L if L is not None else 6.0 * N / 32
    return dict(N=N, L_fm=L, g2mu_GeV=2.0, m_ir_GeV=0.2, uv_GeV=uv, n_sheets=n_sheets, dtau_over_a=DT,
                tau_max_fm=steps * DT * L / N, seed=seed, precision=precision,
                reunit_every=16 if precision == cp.FP32 else 0, record_every=8, n_colors=2)


def state(ctx):
    return {k: ctx.get_state(w) for k, w in (("U", cp.STATE_U), ("phi", cp.STATE_PHI), ("E", cp.STATE_E),
                                            ("pi", cp.STATE_PI))}


@pytest.mark.parametrize("N,uv", [(12, 10.0), (32, 0.0), (48, 10.0)])
def test_su2_initial_condition(N, uv):
    g = event(N, 10, uv=uv)
    ctx = cp.Context(g, None)
    ctx.init_mv()
    got = state(ctx)
    ref = su2.mv_initial_condition(N, g["L_fm"], 2.0, 0.2, uv, 2, 61)
    for k in ("U", "pi"):
        assert rel_err(got[k], ref[k]) <= 1e-12, k
    assert np.max(np.abs(got["phi"])) == 0 and np.max(np.abs(got["E"])) == 0
    ctx.close()


def test_su2_initial_condition_in_sheet_chunks():
    """230 sheets at 192^2: a full chunk of 227 charge planes and a ragged one
    of 3 (L = 6 fm)."""
    N, ns = 192, 230
    print(f"case SU(2) IC chunks N={N} sheets={ns}", flush=True)
    g = event(N, 10, L=6.0, n_sheets=ns)
    ctx = cp.Context(g, None)
    ctx.init_mv()
    got = state(ctx)
    ref = su2.mv_initial_condition(N, 6.0, 2.0, 0.2, 10.0, ns, 61)
    for k in ("U", "pi"):
        assert rel_err(got[k], ref[k]) <= 1e-12, k
    ctx.close()


def test_su2_leapfrog_from_mv_event():
    N, steps = 36, 50
    g = event(N, steps)
    ctx = cp.Context(g, None)
    ctx.init_mv()
    ctx.evolve(1e9)
    st = su2.mv_initial_condition(N, g["L_fm"], 2.0, 0.2, 10.0, 2, 61)
    for n in range(steps):
        su2.field_step(N, n, DT, st)
    got = state(ctx)
    for k in ("U", "phi", "E", "pi"):
        assert rel_err(got[k], st[k]) <= TOL, (k, rel_err(got[k], st[k]))
    d = ctx.diagnostics()
    assert d[1] < 1e-11 and d[6] < 1e-13
    ctx.close()


def test_su2_leapfrog_from_random_state():
    """All fields nonzero from the first step (phi, E, pi random): set_state
    at step 3, 40 steps."""
    from test_oracle_su2 import random_state
    N = 24
    st = random_state(N, 62, eps=0.7, scale=0.4)
    g = event(N, 43)
    ctx = cp.Context(g, None)
    ctx.load_state(st, n=3)
    ctx.step(40)
    ref = {k: v.copy() for k, v in st.items()}
    for n in range(3, 43):
        su2.field_step(N, n, DT, ref)
    got = state(ctx)
    for k in ("U", "phi", "E", "pi"):
        assert rel_err(got[k], ref[k]) <= TOL, (k, rel_err(got[k], ref[k]))
    ctx.close()


@pytest.mark.parametrize("mass,nf,rep", [(0.5, 2, 0), (math.inf, 0, 1), (2.0, 0, 1)])
def test_su2_particles_against_oracle(mass, nf, rep):
    N, steps, n = 32, 48, 700
    g = event(N, steps, L=4.0)
    a = oracle.lattice_spacing(4.0, N)
    p = dict(n=n, mass_GeV=mass, pT_min_GeV=0.0, pT_max_GeV=2.0 if math.isfinite(mass) else 0.0,
             azimuth_uniform=1, tau_form_fm=nf * DT * 4.0 / N, rep=rep, seed=63)
    print(f"case su2 particles mass={mass} nf={nf} rep={rep}", flush=True)
    ctx = cp.Context(g, p)
    ctx.init_mv()
    P0 = ctx.get_state(cp.STATE_PARTICLES)
    ref0 = su2.particles_init(N, n, 63, 0.0, p["pT_max_GeV"] * a, True, rep)
    assert rel_err(P0, ref0) <= 1e-14
    ctx.evolve(1e9)
    st = su2.mv_initial_condition(N, 4.0, 2.0, 0.2, 10.0, 2, 61)
    run = su2.Run(N, DT, st, ref0, mhat=mass * a if math.isfinite(mass) else math.inf, n_form=nf)
    for _ in range(steps):
        run.step()
    assert run.errors == 0
    got = ctx.get_state(cp.STATE_PARTICLES)
    assert np.array_equal(got[:, 14:16], run.P[:, 14:16])
    assert rel_err(got, run.P) <= TOL, rel_err(got, run.P)
    obs = ctx.observables()
    last = run.observe() / (n * a * a)
    for k in range(4):
        assert abs(obs[-1, 1 + k] - last[k]) <= 1e-10 * abs(last[k]), (k, obs[-1], last)
    d = ctx.diagnostics()
    assert d[8] < 1e-12 and d[9] < 1e-12          # q2 kept by the rotation, q3 = 0
    ctx.close()


@pytest.mark.parametrize("n", [1, 63, 65])
def test_su2_partial_particle_groups(n):
    """Four wavefronts share each group of 64 particles: a lone particle, a
    group one short of full, and a full group with a one-particle tail,
    moving through a 16^2 event for 32 steps against the oracle (cells
    exact, records at 1e-11, the sums at 1e-10)."""
    N, steps = 16, 32
    g = event(N, steps, L=3.0)
    a = oracle.lattice_spacing(3.0, N)
    p = dict(n=n, mass_GeV=0.5, pT_min_GeV=0.0, pT_max_GeV=2.0, azimuth_uniform=1, tau_form_fm=0.0, rep=0, seed=65)
    print(f"case su2 partial groups n={n}", flush=True)
    ctx = cp.Context(g, p)
    ctx.init_mv()
    P0 = ctx.get_state(cp.STATE_PARTICLES)
    ctx.evolve(1e9)
    st = su2.mv_initial_condition(N, 3.0, 2.0, 0.2, 10.0, 2, 61)
    run = su2.Run(N, DT, st, P0, mhat=0.5 * a, n_form=0)
    for _ in range(steps):
        run.step()
    assert run.errors == 0
    got = ctx.get_state(cp.STATE_PARTICLES)
    assert np.array_equal(got[:, 14:16], run.P[:, 14:16])
    assert rel_err(got, run.P) <= TOL, rel_err(got, run.P)
    obs = ctx.observables()
    last = run.observe() / (n * a * a)
    for k in range(4):
        assert abs(obs[-1, 1 + k] - last[k]) <= 1e-10 * abs(last[k]) + 1e-300, (k, obs[-1], last)
    ctx.close()


def test_su2_fp32_against_oracle():
    N, steps, n = 32, 64, 400
    g = event(N, steps, L=4.0, precision=cp.FP32)
    a = oracle.lattice_spacing(4.0, N)
    p = dict(n=n, mass_GeV=1.0, pT_min_GeV=0.5, pT_max_GeV=1.5, azimuth_uniform=1, tau_form_fm=0.0, rep=0,
             seed=64)
    ctx = cp.Context(g, p)
    ctx.init_mv()
    ctx.evolve(1e9)
    st = su2.mv_initial_condition(N, 4.0, 2.0, 0.2, 10.0, 2, 61)
    run = su2.Run(N, DT, st, su2.particles_init(N, n, 64, 0.5 * a, 1.5 * a, True, 0), mhat=a, n_form=0)
    for _ in range(steps):
        run.step()
    got = state(ctx)
    for k in ("U", "phi", "E", "pi"):
        assert rel_err(got[k], run.st[k]) < 2e-3, k
    d = ctx.diagnostics()
    assert d[6] < 1e-5
    gp = ctx.get_state(cp.STATE_PARTICLES)
    ok = np.all(gp[:, 14:16] == run.P[:, 14:16], axis=1)
    assert ok.mean() > 0.99
    assert rel_err(gp[ok][:, 3:9], run.P[ok][:, 3:9]) < 2e-3
    ctx.close()


def test_su2_graph_eager_checkpoint_bitwise(tmp_path):
    N, steps = 48, 70
    g = event(N, steps)
    p = dict(n=500, mass_GeV=1.0, pT_min_GeV=0.0, pT_max_GeV=1.0, azimuth_uniform=1, tau_form_fm=0.0, rep=0,
             seed=65)
    out = []
    for mode in ("graph", "eager", "resume"):
        ctx = cp.Context(g, p)
        ctx.init_mv()
        if mode == "graph":
            ctx.evolve(1e9)
        elif mode == "eager":
            ctx.set_timing(True)
            ctx.step(steps)
            t = ctx.timing()
            assert t["n_field"] == steps and t["n_push"] == steps
        else:
            ctx.step(37)
            ctx.save(tmp_path / "ck2.bin")
            ctx.close()
            ctx = cp.Context(g, p)
            ctx.load(tmp_path / "ck2.bin")
            ctx.evolve(1e9)
        ctx.sync()
        out.append((state(ctx), ctx.get_state(cp.STATE_PARTICLES), ctx.observables()))
        ctx.close()
    for other in out[1:]:
        for k in ("U", "phi", "E", "pi"):
            assert np.array_equal(out[0][0][k], other[0][k])
        assert np.array_equal(out[0][1], other[1])
        assert np.array_equal(out[0][2], other[2])


def test_su2_rejected_combinations():
    g = event(16, 10)
    with pytest.raises(cp.CpicError):
        cp.Context(g, dict(n=10, mass_GeV=1.0, color_update=cp.COLOR_LOG))
    with pytest.raises(cp.CpicError):
        cp.Batch([g], [dict(n=0)])
    ctx = cp.Context(g, None)
    with pytest.raises(cp.CpicError):
        ctx.enable_jets()
    with pytest.raises(cp.CpicError):
        ctx.set_launch(64, 4, 1, 1, 3)
    ctx.init_mv()
    assert "SU(2)" in ctx.tune(1)
    ctx.close()
    # a checkpoint of an SU(2) event does not load into an SU(3) context of the same size
    g3 = dict(g, n_colors=3)
    c2, c3 = cp.Context(g, None), cp.Context(g3, None)
    c2.init_mv()
    import tempfile, os
    path = os.path.join(tempfile.mkdtemp(), "x.bin")
    c2.save(path)
    with pytest.raises(cp.CpicError):
        c3.load(path)
    c2.close()
    c3.close()


def test_su2_casimir_scaling_full_size():
    """512^2, L = 6 fm, 50 sheets, FP64, 1e5 static quarks to 1 fm/c, in the
    fundamental and the adjoint representation.  The same seed gives the same
    positions and Darboux angles, so the adjoint charges are the fundamental
    ones scaled by sqrt(q2(A)/q2(F)) = 2 and the broadening ratio is exactly
    A/F = 4, i.e. 8/3 after the division by D_R (Sec. VII, Fig. 10)."""
    g = dict(N=512, L_fm=6.0, g2mu_GeV=2.0, m_ir_GeV=0.2, uv_GeV=10.0, n_sheets=50, dtau_over_a=DT, tau_max_fm=1.0,
             seed=3, precision=cp.FP64, reunit_every=0, record_every=8, n_colors=2)
    res = {}
    for rep in (0, 1):
        p = dict(n=100_000, mass_GeV=math.inf, pT_min_GeV=0.0, pT_max_GeV=0.0, azimuth_uniform=1, tau_form_fm=0.0,
                 rep=rep, seed=4)
        ctx = cp.Context(g, p)
        ctx.init_mv()
        ctx.evolve(1e9)
        res[rep] = ctx.observables()[-1]
        d = ctx.diagnostics()
        assert d[1] < 1e-10 and d[6] < 1e-12
        ctx.close()
    ratio = res[1][1] / res[0][1]
    print("SU(2) static <dp_T^2> F, A:", res[0][1], res[1][1], "A/F", ratio, "after D_R", ratio * 2 / 3, flush=True)
    assert abs(ratio - 4.0) < 1e-9
    assert abs(ratio * 2 / 3 - 8 / 3) < 1e-9
