"""GPU tests of the batched multi-event path (cpic_batch_*).

The batched kernels run the same per-site and per-particle arithmetic as the
single-event kernels, so with the same particle lanes (which fix the partial
sums of the observables) every event of a batch must equal the same event
evolved alone, bit for bit; one event is also checked against the FP64 oracle.
Events differ in lattice size (ragged tiles), MV scale, particle number and
species, formation time and number of steps, so that events drop out of the
work list at different steps and reorder their particles at different steps.
"""
import math

import numpy as np
import pytest

import oracle

cp = pytest.importorskip("paper_2303_05599_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-11


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


def events(precision, a_fm=0.1):
    """Five uneven events at lattice spacing a_fm: (N, g2mu, steps, particles, mass, pT range,
    formation step)."""
    spec = [(16, 2.0, 70, 300, 1.27, (0.0, 0.0), 3),
            (24, 1.5, 45, 0, None, None, 0),            # no particles
            (32, 2.5, 100, 777, math.inf, (0.0, 0.0), 0),  # static quarks
            (48, 1.8, 37, 1500, 4.18, (0.0, 5.0), 5),   # beauty with p_T spread; ragged 48-site tiles
            (12, 2.2, 64, 64, 0.5, (1.0, 2.0), 1)]
    gl, pl = [], []
    for e, (N, g2mu, steps, n, m, pt, nf) in enumerate(spec):
        gl.append(dict(N=N, L_fm=N * a_fm, g2mu_GeV=g2mu, m_ir_GeV=0.1 * g2mu, uv_GeV=10.0, n_sheets=2,
                       dtau_over_a=0.125, tau_max_fm=steps * 0.125 * a_fm, seed=1000 + e, precision=precision,
                       reunit_every=16, record_every=8))
        if n:
            pl.append(dict(n=n, mass_GeV=m, pT_min_GeV=pt[0], pT_max_GeV=pt[1], azimuth_uniform=1,
                           tau_form_fm=nf * 0.125 * a_fm, rep=0, seed=2000 + e))
        else:
            pl.append(dict(n=0))
    return gl, pl


def alone(g, p, lanes):
    ctx = cp.Context(g, p)
    ctx.init_mv()
    if ctx.np:
        ctx.set_push_mode(cp.PUSH_GATHER)   # the batched push evaluates the fields per particle
        ctx.set_push_lanes(lanes)
    ctx.evolve(1e9)
    ctx.sync()
    return ctx


def assert_event_equal(b, e, ctx):
    N = ctx.N
    shapes = {cp.STATE_U: ((2, N, N, 3, 3), np.complex128), cp.STATE_PHI: ((N, N, 8), np.float64),
              cp.STATE_E: ((2, N, N, 8), np.float64), cp.STATE_PI: ((N, N, 8), np.float64)}
    for which, (shape, dt) in shapes.items():
        assert np.array_equal(b.get_state(e, which, shape, dt), ctx.get_state(which)), (e, which)
    if ctx.np:
        assert np.array_equal(b.get_state(e, cp.STATE_PARTICLES, (ctx.np, 20)), ctx.get_state(cp.STATE_PARTICLES)), e
    assert np.array_equal(b.observables(e), ctx.observables()), e


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_events_alone_bitwise(precision):
    prec = cp.FP64 if precision == "fp64" else cp.FP32
    print(f"case batch precision={precision}", flush=True)
    gl, pl = events(prec)
    b = cp.Batch(gl, pl)
    b.init_mv()
    lanes = b.get_launch()["push_lanes"]
    b.run()
    b.sync()
    for e, (g, p) in enumerate(zip(gl, pl)):
        ctx = alone(g, p, lanes)
        assert b.n(e) == ctx.n
        assert_event_equal(b, e, ctx)
        ctx.close()
    b.close()


def test_batch_event_against_oracle():
    """Event 0 of the FP64 batch (16^2, charm-like, formed at step 3) against the oracle."""
    gl, pl = events(cp.FP64)
    b = cp.Batch(gl, pl)
    b.init_mv()
    b.run()
    b.sync()
    g, p = gl[0], pl[0]
    N, L = g["N"], g["L_fm"]
    a = oracle.lattice_spacing(L, N)
    st = oracle.mv_initial_condition(N, L, g["g2mu_GeV"], g["m_ir_GeV"], g["uv_GeV"], g["n_sheets"], g["seed"])
    P = oracle.particles_init(N, p["n"], p["seed"], 0.0, 0.0, True, 0)
    run = oracle.Run(N, 0.125, st, P, mhat=p["mass_GeV"] * a, n_form=3)
    for _ in range(70):
        run.step()
    assert b.n(0) == 70
    got = {"U": b.get_state(0, cp.STATE_U, (2, N, N, 3, 3), np.complex128),
           "E": b.get_state(0, cp.STATE_E, (2, N, N, 8)), "phi": b.get_state(0, cp.STATE_PHI, (N, N, 8)),
           "pi": b.get_state(0, cp.STATE_PI, (N, N, 8))}
    for k in got:
        assert rel_err(got[k], run.st[k]) <= TOL, k
    gp = b.get_state(0, cp.STATE_PARTICLES, (p["n"], 20))
    assert np.array_equal(gp[:, 14:16], run.P[:, 14:16])
    assert rel_err(gp, run.P) <= TOL
    obs = b.observables(0)
    last = run.observe() / (p["n"] * a * a)
    for c in range(4):
        assert abs(obs[-1, 1 + c] - last[c]) <= TOL * abs(last[c]), (c, obs[-1], last)
    b.close()


def test_batch_stepwise_equals_run_and_tuner_keeps_state():
    """Partial advances (crossing formation, reordering and drop-out steps), a tuned
    tile shape and one run to the end give the same bits as one untuned run."""
    gl, pl = events(cp.FP64)
    a, b = cp.Batch(gl, pl), cp.Batch(gl, pl)
    for x in (a, b):
        x.init_mv()
    a.run()
    for k in (1, 2, 5, 17, 30):
        b.step(k)
    b.sync()
    rep = b.tune(2)
    assert "chosen" in rep
    b.run()
    for x in (a, b):
        x.sync()
    for e, g in enumerate(gl):
        N = g["N"]
        assert a.n(e) == b.n(e)
        for which, shape, dt in ((cp.STATE_U, (2, N, N, 3, 3), np.complex128), (cp.STATE_E, (2, N, N, 8), np.float64)):
            assert np.array_equal(a.get_state(e, which, shape, dt), b.get_state(e, which, shape, dt)), e
        if pl[e].get("n"):
            n = pl[e]["n"]
            assert np.array_equal(a.get_state(e, cp.STATE_PARTICLES, (n, 20)), b.get_state(e, cp.STATE_PARTICLES, (n, 20)))
            assert np.array_equal(a.observables(e), b.observables(e))
    a.close()
    b.close()


def test_batch_rejects_mixed_precision():
    gl, pl = events(cp.FP64)
    gl[1] = dict(gl[1], precision=cp.FP32)
    with pytest.raises(cp.CpicError):
        cp.Batch(gl, pl)


def test_batch_grouping_does_not_change_results():
    """One launch group for all events, one group per event, and the default
    cache-sized groups give identical bits (same push lanes)."""
    gl, pl = events(cp.FP64)
    runs = []
    for budget in (0, 1, None):
        b = cp.Batch(gl, pl)
        if budget is not None:
            b.set_group_bytes(budget)
        lc = b.get_launch()
        b.set_launch(lc["bx"], lc["by"], lc["xcd_remap"], 2)
        b.init_mv()
        b.run()
        b.sync()
        runs.append(b)
    for e, g in enumerate(gl):
        N = g["N"]
        ref = runs[0].get_state(e, cp.STATE_E, (2, N, N, 8))
        for b in runs[1:]:
            assert np.array_equal(b.get_state(e, cp.STATE_E, (2, N, N, 8)), ref), e
            assert np.array_equal(b.observables(e), runs[0].observables(e)), e
    for b in runs:
        b.close()


def test_batch_lanes_do_not_change_results():
    """Two and four launch lanes (the launch groups dealt to concurrent
    streams) against one, with one group per event so that the lanes hold
    several groups: identical bits, also when the batch advances in uneven
    stretches.
    The results are read right after the runs, without a separate wait for
    the second lane (the batch stream orders the reads after it)."""
    print("case batch lanes", flush=True)
    gl, pl = events(cp.FP32)
    runs = []
    for lanes, stepwise in ((1, False), (2, False), (2, True), (4, False)):
        b = cp.Batch(gl, pl)
        b.set_group_bytes(1)
        b.set_lanes(lanes)
        b.init_mv()
        if stepwise:
            for k in (7, 16, 33, 100000):
                b.step(k)
        else:
            b.run()
        runs.append(b)
    for e, g in enumerate(gl):
        N = g["N"]
        ref = runs[0].get_state(e, cp.STATE_E, (2, N, N, 8))
        for b in runs[1:]:
            assert np.array_equal(b.get_state(e, cp.STATE_E, (2, N, N, 8)), ref), e
            assert np.array_equal(b.observables(e), runs[0].observables(e)), e
            if pl[e].get("n", 0):
                assert np.array_equal(b.get_state(e, cp.STATE_PARTICLES, (pl[e]["n"], 20)),
                                      runs[0].get_state(e, cp.STATE_PARTICLES, (pl[e]["n"], 20))), e
    for bad in (0, 5):
        with pytest.raises(cp.CpicError):
            runs[0].set_lanes(bad)
    for b in runs:
        b.close()
