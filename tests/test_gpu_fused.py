"""The fused step (field launch variant 4, push mode PUSH_TILE) through the C
ABI: the field update and the push of every tile's particles in one kernel,
the particles that have left their tile (or exceed one per thread of the
tile) in a second, gathering kernel.

  * against the FP64 oracle at 1e-11 (records, fields), cells exact, sums at
    1e-10, on every tile shape, with moving particles that cross tiles
    between reorderings, dense tiles (more particles than threads) and
    sparse ones, static particles, and particles formed at tau = 0;
  * a particle gets the same fields, bit for bit, whether its tile pushes it
    or the straggler kernel does: runs on different tile shapes (different
    straggler sets) end in identical records, and the field update is the
    compressed-tile kernel's, bit for bit.
"""
import math

import numpy as np
import pytest

import inputs
import oracle

cp = pytest.importorskip("paper_2303_05599_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-11
SHAPES = [(64, 8), (32, 8), (16, 16), (8, 8)]


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


def glasma(N, L, steps, **kw):
    g = dict(N=N, L_fm=L, g2mu_GeV=2.0, m_ir_GeV=0.2, uv_GeV=10.0, n_sheets=1, dtau_over_a=0.125,
             tau_max_fm=steps * (L / N) * 0.125, seed=1, precision=cp.FP64, reunit_every=0, record_every=8)
    g.update(kw)
    return g


def particles(n, mass, N, L, n_form, seed=2, pt=(0.0, 0.0)):
    return dict(n=n, mass_GeV=mass, pT_min_GeV=pt[0], pT_max_GeV=pt[1], azimuth_uniform=1,
                tau_form_fm=n_form * 0.125 * L / N, rep=0, seed=seed)


def random_run(N, L, n, n0, n_form, steps, static, seed, shape=None, mode=None):
    a = oracle.lattice_spacing(L, N)
    mhat = math.inf if static else 0.3
    st = inputs.random_state(N, seed, eps_link=0.4)
    P = inputs.random_particles(n, N, seed + 1, p_scale=0.6)
    ctx = cp.Context(glasma(N, L, n0 + steps), particles(n, math.inf if static else mhat / a, N, L, n_form))
    if shape is not None:
        ctx.set_launch(shape[0], shape[1], 1, 1, 4)
    if mode is not None:
        ctx.set_push_mode(mode)
    ctx.load_state(st, n=n0, particles=P)
    ctx.step(steps)
    ctx.sync()
    return ctx, st, P, mhat


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("n,static", [(3000, False), (300, False), (3000, True)])
def test_fused_against_oracle(shape, n, static):
    """32^2 random state, 50 steps from n0 = 5 with the push formed at n = 3:
    3000 particles (dense: every tile holds more particles than threads) or
    300 (sparse), moving fast enough to cross tiles between reorderings, or
    static.  The 64 x 8 tile is wider than the lattice (ragged)."""
    N, L, n0, n_form, steps = 32, 6.0, 5, 3, 50
    print(f"case fused shape={shape} n={n} static={static}", flush=True)
    ctx, st, P, mhat = random_run(N, L, n, n0, n_form, steps, static, 71, shape)
    assert ctx.push_mode() == cp.PUSH_TILE
    assert ctx.get_launch()["variant"] == 4
    a = oracle.lattice_spacing(L, N)
    run = oracle.Run(N, 0.125, st, P, mhat=mhat, n_form=n_form, n0=n0)
    for _ in range(steps):
        run.step()
    assert run.errors == 0
    got = ctx.get_state(cp.STATE_PARTICLES)
    assert np.array_equal(got[:, 14:16], run.P[:, 14:16])
    assert rel_err(got, run.P) <= TOL
    for k in ("U", "phi", "E", "pi"):
        assert rel_err(ctx.state()[k], run.st[k]) <= TOL, k
    if not static:
        assert rel_err(ctx.get_state(cp.STATE_PTAU)[:, 0], run.ptau_constraint()) <= TOL
    obs = ctx.observables()
    sums = run.observe() / (n * a * a)
    for c in range(4):
        assert abs(obs[-1, 1 + c] - sums[c]) <= 1e-10 * abs(sums[c]), (c, obs[-1], sums)
    ctx.close()


def test_tile_and_straggler_push_agree_bitwise():
    """The same particles on different tile shapes: which particles the
    tiles push and which the straggler kernel pushes differs, the records do
    not (bit for bit); the fields equal those of the compressed-tile kernel
    with the gather push, bit for bit."""
    N, L, n0, n_form, steps, n = 32, 6.0, 5, 3, 40, 3000
    print("case fused bitwise", flush=True)
    runs = []
    for shape in SHAPES:
        ctx, *_ = random_run(N, L, n, n0, n_form, steps, False, 81, shape)
        runs.append((ctx.get_state(cp.STATE_PARTICLES), ctx.state(), ctx.observables()))
        ctx.close()
    gather, *_ = random_run(N, L, n, n0, n_form, steps, False, 81, mode=cp.PUSH_GATHER)
    assert gather.push_mode() == cp.PUSH_GATHER
    fields = gather.state()
    gather.close()
    for recs, st, obs in runs[1:]:
        assert np.array_equal(recs, runs[0][0])
        assert rel_err(obs, runs[0][2]) < 1e-13   # sums over other groups of particles
    for recs, st, obs in runs:
        for k in ("U", "phi", "E", "pi"):
            assert np.array_equal(st[k], fields[k]), k


@pytest.mark.parametrize("shape", [(16, 16), (8, 8)])
def test_fused_formed_at_tau_zero(shape):
    """Particles formed at tau = 0 on a 32^2 MV event: at n = 0 the electric
    fields are E_eta = pi(1/2) only, the magnetic ones the clover; 24 steps
    against the oracle."""
    print(f"case fused tau_form=0 shape={shape}", flush=True)
    N, L, steps = 32, 6.0, 24
    a = oracle.lattice_spacing(L, N)
    g = glasma(N, L, steps, seed=5)
    p = dict(n=700, mass_GeV=2.0, pT_min_GeV=0.5, pT_max_GeV=2.0, azimuth_uniform=1, tau_form_fm=0.0, rep=0, seed=6)
    ctx = cp.Context(g, p)
    ctx.set_launch(shape[0], shape[1], 1, 1, 4)
    ctx.init_mv()
    ctx.step(steps)
    ref = oracle.mv_initial_condition(N, L, 2.0, 0.2, 10.0, 1, 5)
    P = oracle.particles_init(N, 700, 6, 0.5 * a, 2.0 * a, True, 0)
    run = oracle.Run(N, 0.125, ref, P, mhat=2.0 * a, n_form=0)
    for _ in range(steps):
        run.step()
    got = ctx.get_state(cp.STATE_PARTICLES)
    assert np.array_equal(got[:, 14:16], run.P[:, 14:16])
    assert rel_err(got, run.P) <= TOL
    for k in ("U", "phi", "E", "pi"):
        assert rel_err(ctx.state()[k], run.st[k]) <= TOL, k
    ctx.close()


def test_push_modes_switch_and_reorder():
    """Switching from the fused step to the gather push and back (onto
    another tile shape, so the records are reordered by the new tiles before
    the next push step) mid-run: the run agrees with an all-fused one, cells
    exactly, records to rounding (the gather push takes B_eta from the
    plaquette field, another rounding)."""
    print("case fused mode switch", flush=True)
    N, L, n0, n_form, steps, n = 32, 6.0, 5, 3, 48, 2000
    a = oracle.lattice_spacing(L, N)
    ref, st, P, _ = random_run(N, L, n, n0, n_form, steps, False, 91, (16, 16))
    ctx = cp.Context(glasma(N, L, n0 + steps), particles(n, 0.3 / a, N, L, n_form))
    ctx.set_launch(16, 16, 1, 1, 4)
    ctx.load_state(st, n=n0, particles=P)
    ctx.step(10)
    ctx.set_push_mode(cp.PUSH_GATHER)
    assert ctx.push_mode() == cp.PUSH_GATHER
    ctx.step(7)
    ctx.set_push_mode(cp.PUSH_TILE)
    ctx.set_launch(8, 8, 1, 1, 4)
    ctx.step(steps - 17)
    ctx.sync()
    got, want = ctx.get_state(cp.STATE_PARTICLES), ref.get_state(cp.STATE_PARTICLES)
    assert np.array_equal(got[:, 14:16], want[:, 14:16])
    assert rel_err(got, want) <= TOL
    for k in ("U", "phi", "E", "pi"):
        assert np.array_equal(ctx.state()[k], ref.state()[k]), k
    ctx.close()
    ref.close()


def test_fused_mv_event_with_graphs():
    """A 128^2 MV event with 20000 charm-like quarks evolved with the 16-step
    graphs, against the same event stepped eagerly with the gather push: the
    fields bit for bit, the particles to rounding, the sums at 1e-12."""
    print("case fused MV graphs", flush=True)
    N, L = 128, 6.0
    g = glasma(N, L, 150, n_sheets=4, seed=9)
    p = dict(n=20000, mass_GeV=1.27, pT_min_GeV=0.0, pT_max_GeV=2.0, azimuth_uniform=1, tau_form_fm=0.1, rep=0,
             seed=10)
    fused, gather = cp.Context(g, p), cp.Context(g, p)
    fused.set_push_mode(cp.PUSH_TILE)
    gather.set_push_mode(cp.PUSH_GATHER)   # (the default here is the force table: more particles than sites)
    for c in (fused, gather):
        c.init_mv()
    fused.evolve(1e9)
    gather.step(150 - gather.n)
    assert fused.n == gather.n == 150
    for k in ("U", "phi", "E", "pi"):
        assert np.array_equal(fused.state()[k], gather.state()[k]), k
    a, b = fused.get_state(cp.STATE_PARTICLES), gather.get_state(cp.STATE_PARTICLES)
    assert np.array_equal(a[:, 14:16], b[:, 14:16])
    assert rel_err(a, b) <= 1e-11
    oa, ob = fused.observables(), gather.observables()
    assert rel_err(oa, ob) <= 1e-12
    fused.close()
    gather.close()
