"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle
on the same seeded inputs.

Tolerance for double precision: |lib - oracle| <= 1e-11 * max(|oracle|, RMS of
that field) per site and component over the first 50 steps (the agreement the
method's double-precision path is held to; both implementations are exact up
to rounding order).  Integer data (particle cells) must agree exactly.
"""
import ctypes
import math
import os

import numpy as np
import pytest

import inputs
import oracle

cp = pytest.importorskip("paper_2303_05599_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-11
HBARC = oracle.HBARC_GEV_FM


def rel_err(a, ref):
    a, ref = np.asarray(a), np.asarray(ref)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2)) if ref.size else 0.0
    den = np.maximum(np.abs(ref), rms)
    den = np.where(den == 0, 1.0, den)
    return float(np.max(np.abs(a - ref) / den)) if a.size else 0.0


def glasma(N, L=None, steps=60, **kw):
    L = L if L is not None else 6.0 * N / 32
    g = dict(N=N, L_fm=L, g2mu_GeV=2.0, m_ir_GeV=0.2, uv_GeV=10.0, n_sheets=1, dtau_over_a=0.125,
             tau_max_fm=steps * (L / N) * 0.125, seed=1, precision=cp.FP64, reunit_every=0, record_every=8)
    g.update(kw)
    return g


def compare_fields(st, ref, tol=TOL):
    errs = {k: rel_err(st[k], ref[k]) for k in ("U", "phi", "E", "pi")}
    for k, e in errs.items():
        assert e <= tol, (k, e, errs)
    return errs


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    cp.lib()
    yield


LAUNCHES = {"site64x4": (64, 4, 1, 1, 0), "site256x1w2": (256, 1, 0, 2, 0), "link128x1": (128, 1, 1, 1, 1),
            "link32x4w2": (32, 4, 0, 2, 1), "tile64x4": (64, 4, 1, 1, 2), "tile32x8": (32, 8, 0, 1, 2),
            "tile16x8": (16, 8, 1, 1, 2), "tile64x2": (64, 2, 0, 1, 2), "tile32x4": (32, 4, 1, 1, 2),
            "ctile64x4": (64, 4, 1, 1, 3), "ctile32x8": (32, 8, 0, 1, 3), "ctile16x16": (16, 16, 1, 1, 3),
            "ctile32x4": (32, 4, 0, 1, 3), "ctile64x8": (64, 8, 1, 1, 3)}


@pytest.mark.parametrize("N,n0,launch", [(32, 3, "site64x4"), (96, 0, "site64x4"), (48, 1, "site64x4"),
                                         (96, 2, "link128x1"), (48, 1, "link32x4w2"), (32, 5, "site256x1w2"),
                                         (96, 1, "tile64x4"), (48, 2, "tile32x8"), (12, 0, "tile16x8"),
                                         (36, 3, "tile64x2"), (64, 1, "tile32x4"), (96, 2, "ctile64x4"),
                                         (48, 1, "ctile32x8"), (12, 0, "ctile16x16"), (36, 3, "ctile32x4"),
                                         (72, 2, "ctile64x8")])
def test_field_leapfrog_fp64_random_state(N, n0, launch):
    """50 fused kick+drift steps from a random state; N = 96, 48, 36 and 12 leave ragged
    tiles (12 is smaller than the 16 x 8 tile); site-parallel, link-parallel and LDS
    halo-tile decompositions."""
    print(f"case N={N} n0={n0} launch={launch}", flush=True)
    steps = 50
    st = inputs.random_state(N, 100 + N, eps_link=0.4)
    ctx = cp.Context(glasma(N, steps=n0 + steps + 1))
    ctx.set_launch(*LAUNCHES[launch])
    ctx.load_state(st, n=n0)
    ctx.step(steps)
    got = ctx.state()
    ref = {k: v.copy() for k, v in st.items()}
    for n in range(n0, n0 + steps):
        oracle.field_step(N, n, 0.125, ref)
    compare_fields(got, ref)


@pytest.mark.parametrize("N,ns,uv", [(32, 1, 10.0), (48, 3, 4.0), (64, 2, 0.0), (96, 1, 10.0)])
def test_initial_condition_parity(N, ns, uv):
    """Full MV chain: charges, FFT Poisson (radix 2/3/4; 96 = 4 4 2 3 mixes all three), Wilson lines,
    Newton links, pi(0)."""
    print(f"case IC N={N} sheets={ns} uv={uv}", flush=True)
    L = 6.0 * N / 32
    ctx = cp.Context(glasma(N, L, n_sheets=ns, uv_GeV=uv, seed=7))
    ctx.init_mv()
    got = ctx.state()
    ref = oracle.mv_initial_condition(N, L, 2.0, 0.2, uv, ns, 7)
    assert rel_err(got["U"], ref["U"]) < 1e-12
    assert rel_err(got["pi"], ref["pi"]) < 1e-12
    assert np.max(np.abs(got["E"])) == 0 and np.max(np.abs(got["phi"])) == 0


def test_initial_condition_parity_in_sheet_chunks():
    """The sheets of a nucleus go through the FFT Poisson solve in chunks of
    at most 256 MiB of charge planes (113 sheets at 192^2): 120 sheets take
    a full chunk and a ragged one of 7, each Wilson line the product over
    both.  L = 6 fm keeps the links weak enough for the Newton solve."""
    N, ns = 192, 120
    print(f"case IC chunks N={N} sheets={ns}", flush=True)
    ctx = cp.Context(glasma(N, 6.0, n_sheets=ns, uv_GeV=10.0, seed=7))
    ctx.init_mv()
    got = ctx.state()
    ref = oracle.mv_initial_condition(N, 6.0, 2.0, 0.2, 10.0, ns, 7)
    assert rel_err(got["U"], ref["U"]) < 1e-12
    assert rel_err(got["pi"], ref["pi"]) < 1e-12
    ctx.close()


def particle_params(n, mass, N, L, n_form, seed=2, pt=(0.0, 0.0), rep=0):
    a_fm = L / N
    return dict(n=n, mass_GeV=mass, pT_min_GeV=pt[0], pT_max_GeV=pt[1], azimuth_uniform=1,
                tau_form_fm=n_form * 0.125 * a_fm, rep=rep, seed=seed)


def test_particles_init_parity():
    N, L = 32, 6.0
    a = oracle.lattice_spacing(L, N)
    ctx = cp.Context(glasma(N, L), particle_params(5000, 1.27, N, L, 0, seed=9, pt=(0.5, 3.0)))
    ctx.init_mv()
    got = ctx.get_state(cp.STATE_PARTICLES)
    ref = oracle.particles_init(N, 5000, 9, 0.5 * a, 3.0 * a, True, 0)
    assert np.array_equal(got[:, 14:16], ref[:, 14:16])
    assert rel_err(got, ref) < 1e-13


@pytest.mark.parametrize("is_static,lanes", [(False, 1), (False, 2), (False, 4), (True, 1), (True, 2), (True, 4),
                                             (False, "table"), (True, "table")])
def test_particle_push_fp64_random_state(is_static, lanes):
    """Rotation on cell changes (both axes), rapidity Wilson line, E/B interpolation, Euler step,
    with 1, 2 or 4 wavefronts sharing each particle group, or with the fields
    taken from the per-site force table."""
    print(f"case push static={is_static} lanes={lanes}", flush=True)
    N, L, n0, n_form, steps = 32, 6.0, 5, 3, 50
    a = oracle.lattice_spacing(L, N)
    mhat = math.inf if is_static else 0.3
    st = inputs.random_state(N, 41, eps_link=0.4)
    P = inputs.random_particles(3000, N, 42, p_scale=0.6)
    ctx = cp.Context(glasma(N, L, steps=n0 + steps),       # the last step is a sampling step
                     particle_params(3000, math.inf if is_static else mhat / a, N, L, n_form))
    ctx.load_state(st, n=n0, particles=P)
    if lanes == "table":
        ctx.set_push_mode(cp.PUSH_TABLE)
    else:
        ctx.set_push_mode(cp.PUSH_GATHER)
        ctx.set_push_lanes(lanes)
    assert ctx.push_mode() == (cp.PUSH_TABLE if lanes == "table" else cp.PUSH_GATHER)
    ctx.step(steps)
    ctx.sync()
    got = ctx.get_state(cp.STATE_PARTICLES)
    run = oracle.Run(N, 0.125, st, P, mhat=mhat, n_form=n_form, n0=n0)
    for _ in range(steps):
        run.step()
    assert run.errors == 0
    ref = run.P
    flips = np.sum(np.any(got[:, 14:16] != ref[:, 14:16], axis=1))
    assert flips == 0, f"{flips} particles on a different cell"
    assert rel_err(got, ref) <= TOL
    if not is_static:
        # p^tau from the constraint (the integrated p^tau of Appendix D is
        # compared on MV events: in these strong random fields its Euler
        # integration amplifies rounding, 1e-15 at the start -> 5e-9 here)
        pt = ctx.get_state(cp.STATE_PTAU)
        assert rel_err(pt[:, 0], run.ptau_constraint()) <= TOL
    compare_fields(ctx.state(), run.st)
    obs = ctx.observables()
    assert obs[-1, 0] == pytest.approx(run.n * 0.125 * L / N, rel=1e-14)
    sums = run.observe() / (3000 * a * a)
    for c in range(4):
        assert abs(obs[-1, 1 + c] - sums[c]) <= 1e-10 * abs(sums[c]), (c, obs[-1], sums)


@pytest.mark.parametrize("N,launch", [(4, "ctile64x8"), (4, "site64x4"), (4, "tile16x8"), (4, "link128x1"),
                                      (6, "ctile32x4")])
def test_smallest_lattices(N, launch):
    """The smallest lattices (N = 4, 6: every tile shape is larger than the
    lattice, every neighbour wraps): fields and moving particles, which cross
    the periodic boundary often, over 40 steps against the oracle."""
    print(f"case smallest N={N} launch={launch}", flush=True)
    L, n0, steps, n = 0.75 * N / 4, 2, 40, 300
    a = oracle.lattice_spacing(L, N)
    st = inputs.random_state(N, 51 + N, eps_link=0.4)
    P = inputs.random_particles(n, N, 52 + N, p_scale=0.6)
    ctx = cp.Context(glasma(N, L, steps=n0 + steps), particle_params(n, 0.3 / a, N, L, 0))
    ctx.set_launch(*LAUNCHES[launch])
    ctx.load_state(st, n=n0, particles=P)
    ctx.step(steps)
    ctx.sync()
    run = oracle.Run(N, 0.125, st, P, mhat=0.3, n_form=0, n0=n0)
    for _ in range(steps):
        run.step()
    assert run.errors == 0
    got = ctx.get_state(cp.STATE_PARTICLES)
    assert np.array_equal(got[:, 14:16], run.P[:, 14:16])
    assert rel_err(got, run.P) <= TOL
    compare_fields(ctx.state(), run.st)


@pytest.mark.parametrize("n", [1, 63, 65])
def test_partial_particle_groups(n):
    """Four wavefronts share each group of 64 particles, and a single record
    needs no reordering: a lone particle, a group one short of full and a
    full group with a one-particle tail, moving on a 16^2 random state for 40
    steps with the step graphs (reorderings every 16 steps inside them)
    against the oracle; the broadening sums at 1e-10."""
    print(f"case partial groups n={n}", flush=True)
    N, L, n0, steps = 16, 3.0, 2, 40
    a = oracle.lattice_spacing(L, N)
    st = inputs.random_state(N, 55, eps_link=0.4)
    P = inputs.random_particles(n, N, 56, p_scale=0.6)
    ctx = cp.Context(glasma(N, L, steps=n0 + steps), particle_params(n, 0.3 / a, N, L, 0))
    ctx.load_state(st, n=n0, particles=P)
    ctx.evolve(1e9)
    assert ctx.n == n0 + steps
    run = oracle.Run(N, 0.125, st, P, mhat=0.3, n_form=0, n0=n0)
    for _ in range(steps):
        run.step()
    assert run.errors == 0
    got = ctx.get_state(cp.STATE_PARTICLES)
    assert np.array_equal(got[:, 14:16], run.P[:, 14:16])
    assert rel_err(got, run.P) <= TOL
    obs = ctx.observables()
    sums = run.observe() / (n * a * a)
    for c in range(4):
        assert abs(obs[-1, 1 + c] - sums[c]) <= 1e-10 * abs(sums[c]) + 1e-300, (c, obs[-1], sums)
    compare_fields(ctx.state(), run.st)
    ctx.close()


def test_particle_order_does_not_matter():
    """Particles are independent given the fields: the same particles loaded
    in a shuffled order (the library reorders them by cell and hands the
    records back in input order) end in the same records, bit for bit, and
    the broadening sums agree to rounding."""
    N, L, n0, steps, n = 32, 6.0, 4, 40, 3000
    a = oracle.lattice_spacing(L, N)
    st = inputs.random_state(N, 61, eps_link=0.4)
    P = inputs.random_particles(n, N, 62, p_scale=0.6)
    perm = np.random.default_rng(63).permutation(n)
    out = []
    for recs in (P, P[perm]):
        ctx = cp.Context(glasma(N, L, steps=n0 + steps), particle_params(n, 0.3 / a, N, L, 0))
        ctx.load_state(st, n=n0, particles=recs)
        ctx.step(steps)
        ctx.sync()
        out.append((ctx.get_state(cp.STATE_PARTICLES), ctx.observables()))
        ctx.close()
    assert np.array_equal(out[1][0], out[0][0][perm])
    assert rel_err(out[1][1], out[0][1]) < 1e-13


def test_static_limit_config_32():
    """The coarse static configuration: 32^2, L = 6 fm, g^2 mu = 2 GeV, m = 0.2 GeV,
    one sheet, dtau = a/8 to 1 fm/c (43 steps), 1024 static quarks, seeds 1 and 2."""
    N, L = 32, 6.0
    a = oracle.lattice_spacing(L, N)
    g = glasma(N, L, tau_max_fm=1.0, seed=1)
    p = dict(n=1024, mass_GeV=math.inf, pT_min_GeV=0, pT_max_GeV=0, azimuth_uniform=1, tau_form_fm=0.0,
             rep=0, seed=2)
    ctx = cp.Context(g, p)
    ctx.init_mv()
    ctx.evolve(1.0)
    assert ctx.n == 43
    obs = ctx.observables()
    ref = oracle.mv_initial_condition(N, L, 2.0, 0.2, 10.0, 1, 1)
    P = oracle.particles_init(N, 1024, 2, 0.0, 0.0, True, 0)
    run = oracle.Run(N, 0.125, ref, P, mhat=math.inf, n_form=0)
    ref_obs = []
    for n in range(43):
        run.step()
        if (n + 1) % 8 == 0 or n + 1 == 43:
            ref_obs.append([run.n * 0.125 * L / N] + list(run.observe() / (1024 * a * a)))
    ref_obs = np.array(ref_obs)
    assert obs.shape[0] == ref_obs.shape[0] == 6
    assert np.allclose(obs[:, 0], ref_obs[:, 0], rtol=1e-14)
    for c in (1, 2, 3, 4):
        assert rel_err(obs[:, c], ref_obs[:, c]) <= TOL
    assert rel_err(ctx.get_state(cp.STATE_PARTICLES), run.P) <= TOL
    # transport coefficients and anisotropies ([eq:kappalt], the heavy-quark
    # ratio): the library's from its samples against the oracle's definition,
    # on the library's samples (to rounding) and on the oracle's (the sample
    # differences amplify the 1e-11 agreement of the sums)
    tr = ctx.transport()
    assert tr.shape == (6, 8)
    mine = oracle.transport_coefficients(0.0, obs[:, 0], obs[:, 1:5])
    assert np.allclose(tr, mine, rtol=1e-12, atol=0)
    theirs = oracle.transport_coefficients(0.0, ref_obs[:, 0], ref_obs[:, 1:5])
    for c in range(8):
        scale = np.max(np.abs(theirs[:, c]))
        assert np.max(np.abs(tr[:, c] - theirs[:, c])) <= 1e-9 * scale, c
    assert np.all(tr[:, 2] != 0) and np.all(np.isfinite(tr))


@pytest.mark.parametrize("launch", [None, "tile64x4", "link128x1", "ctile32x8"])
def test_full_chain_charm_like_64(launch):
    """Full chain at the paper-scale lattice spacing (a = 6 fm / 512) on a 64^2
    patch: 4 sheets, charm quarks (m = 1.27 GeV, p_T = 0) formed at 0.1 fm/c; the
    field update in each decomposition also writes the magnetic-field pieces
    the push reads."""
    print(f"case full chain launch={launch}", flush=True)
    N, L = 64, 0.75
    a = oracle.lattice_spacing(L, N)
    n_form = math.ceil(0.1 / (0.125 * L / N) - 1e-9)
    steps = n_form + 50
    g = glasma(N, L, n_sheets=4, steps=steps, seed=3)
    p = dict(n=2000, mass_GeV=1.27, pT_min_GeV=0, pT_max_GeV=0, azimuth_uniform=1, tau_form_fm=0.1, rep=0, seed=4)
    ctx = cp.Context(g, p)
    if launch:
        ctx.set_launch(*LAUNCHES[launch])
    ctx.init_mv()
    ctx.evolve(1e9)
    ctx.sync()
    ref = oracle.mv_initial_condition(N, L, 2.0, 0.2, 10.0, 4, 3)
    P = oracle.particles_init(N, 2000, 4, 0.0, 0.0, True, 0)
    run = oracle.Run(N, 0.125, ref, P, mhat=1.27 * a, n_form=n_form)
    for _ in range(steps):
        run.step()
    compare_fields(ctx.state(), run.st)
    got = ctx.get_state(cp.STATE_PARTICLES)
    assert np.array_equal(got[:, 14:16], run.P[:, 14:16])
    assert rel_err(got, run.P) <= TOL
    obs = ctx.observables()
    last = run.observe() / (2000 * a * a)
    for c in range(4):
        assert abs(obs[-1, 1 + c] - last[c]) <= TOL * max(abs(last[c]), 1e-300), (c, obs[-1], last)


@pytest.mark.parametrize("launch", ["site64x4", "tile16x8", "link32x4w2", "ctile16x16"])
def test_particles_formed_at_tau_zero(launch):
    """Dynamic particles formed at tau = 0 (n_form = 0): at n = 0 the kick is
    skipped but the magnetic-field pieces (clover, scalar gradients) must still
    be written for the push; 24 steps on a 32^2 MV event against the oracle."""
    print(f"case tau_form=0 launch={launch}", flush=True)
    N, L, steps = 32, 6.0, 24
    a = oracle.lattice_spacing(L, N)
    g = glasma(N, L, steps=steps, seed=5)
    p = dict(n=700, mass_GeV=2.0, pT_min_GeV=0.5, pT_max_GeV=2.0, azimuth_uniform=1, tau_form_fm=0.0, rep=0, seed=6)
    ctx = cp.Context(g, p)
    ctx.set_launch(*LAUNCHES[launch])
    ctx.init_mv()
    ctx.step(steps)
    ctx.sync()
    ref = oracle.mv_initial_condition(N, L, 2.0, 0.2, 10.0, 1, 5)
    P = oracle.particles_init(N, 700, 6, 0.5 * a, 2.0 * a, True, 0)
    run = oracle.Run(N, 0.125, ref, P, mhat=2.0 * a, n_form=0)
    for _ in range(steps):
        run.step()
    compare_fields(ctx.state(), run.st)
    got = ctx.get_state(cp.STATE_PARTICLES)
    assert np.array_equal(got[:, 14:16], run.P[:, 14:16])
    assert rel_err(got, run.P) <= TOL


def test_graph_replay_equals_eager_bitwise():
    N, L = 32, 6.0
    g = glasma(N, L, steps=80, record_every=4)
    p = particle_params(500, 1.27, N, L, 5, pt=(1.0, 1.0))
    a_ctx, b_ctx = cp.Context(g, p), cp.Context(g, p)
    for c in (a_ctx, b_ctx):
        c.init_mv()
    a_ctx.step(80)
    b_ctx.evolve(1e9)          # graphs of 16 steps
    for k in ("U", "phi", "E", "pi"):
        assert np.array_equal(a_ctx.state()[k], b_ctx.state()[k]), k
    assert np.array_equal(a_ctx.get_state(cp.STATE_PARTICLES), b_ctx.get_state(cp.STATE_PARTICLES))
    assert np.array_equal(a_ctx.observables(), b_ctx.observables())


def test_checkpoint_resume_bitwise(tmp_path):
    N, L = 32, 6.0
    g = glasma(N, L, steps=40, record_every=4)
    p = particle_params(300, 1.27, N, L, 2, pt=(1.0, 1.0))
    full = cp.Context(g, p)
    full.init_mv()
    full.step(40)
    half = cp.Context(g, p)
    half.init_mv()
    half.step(20)
    half.save(tmp_path / "ck.bin")
    resumed = cp.Context(g, p)
    resumed.load(tmp_path / "ck.bin")
    resumed.step(20)
    for k in ("U", "phi", "E", "pi"):
        assert np.array_equal(full.state()[k], resumed.state()[k]), k
    assert np.array_equal(full.get_state(cp.STATE_PARTICLES), resumed.get_state(cp.STATE_PARTICLES))
    assert np.array_equal(full.observables(), resumed.observables())
    # a truncated checkpoint is rejected
    data = (tmp_path / "ck.bin").read_bytes()
    (tmp_path / "bad.bin").write_bytes(data[: len(data) // 2])
    with pytest.raises(cp.CpicError) as e:
        resumed.load(tmp_path / "bad.bin")
    assert e.value.status == -9


def test_diagnostics_match_oracle():
    N, L, n0 = 32, 6.0, 4
    st = inputs.random_state(N, 77, eps_link=0.3)
    ctx = cp.Context(glasma(N, L, steps=20))
    ctx.load_state(st, n=n0)
    d = ctx.diagnostics()
    G = oracle.gauss(N, st["U"], st["phi"], st["E"], st["pi"])
    assert d[0] == pytest.approx(np.sum(G ** 2), rel=1e-12)
    assert d[1] == pytest.approx(np.max(np.sqrt(np.sum(G ** 2, axis=-1))), rel=1e-12)
    t = n0 * 0.125
    FE, Fp = oracle.forces(N, t, st["U"], st["phi"])
    Eav = np.ascontiguousarray(st["E"] + 0.0625 * FE)
    piav = np.ascontiguousarray(st["pi"] + 0.0625 * Fp)
    H = oracle.energy(N, t, st["U"], st["phi"], Eav, piav)
    assert np.allclose(d[2:6], H, rtol=1e-12, atol=1e-12)
    mu, _ = oracle.unitarity(N, st["U"])
    assert d[6] == pytest.approx(mu, rel=1e-3, abs=1e-15)
    # the four-quantity form: the Gauss L2 norm, the summed lattice energy,
    # the unitarity maximum and (without particles) no Casimir drift
    gl2, en, um, cm = ctx.diagnostics_summary()
    assert gl2 == pytest.approx(np.sqrt(np.sum(G ** 2)), rel=1e-12)
    assert en == pytest.approx(np.sum(H), rel=1e-12)
    assert um == d[6] and cm == 0.0


def test_mv_event_invariants_fp64():
    """Gauss law, unitarity and Casimirs on an MV event after 200 steps."""
    N, L = 64, 0.75
    g = glasma(N, L, n_sheets=4, steps=200, seed=5)
    p = dict(n=4000, mass_GeV=0.2, pT_min_GeV=2.0, pT_max_GeV=2.0, azimuth_uniform=1, tau_form_fm=0.0, rep=0, seed=6)
    ctx = cp.Context(g, p)
    ctx.init_mv()
    ctx.evolve(1e9)
    d = ctx.diagnostics()
    assert d[1] < 1e-12          # Gauss
    assert d[6] < 1e-13          # unitarity
    assert d[8] < 1e-11 and d[9] < 1e-11   # Casimirs
    gl2, en, um, cm = ctx.diagnostics_summary()
    assert gl2 == pytest.approx(np.sqrt(d[0]), rel=1e-14) and en == pytest.approx(np.sum(d[2:6]), rel=1e-14)
    assert um == d[6] and cm == max(d[8], d[9])


def test_fp32_against_fp64_oracle():
    """Float storage and update with reunitarisation and charge renormalisation every
    16 steps: error against the double-precision oracle after 64 steps."""
    N, L = 32, 6.0
    a = oracle.lattice_spacing(L, N)
    steps = 64
    g = glasma(N, L, steps=steps, precision=cp.FP32, reunit_every=16, seed=1)
    p = dict(n=4096, mass_GeV=math.inf, pT_min_GeV=0, pT_max_GeV=0, azimuth_uniform=1, tau_form_fm=0.0, rep=0, seed=2)
    ctx = cp.Context(g, p)
    ctx.init_mv()
    ctx.evolve(1e9)
    obs = ctx.observables()
    d = ctx.diagnostics()
    ref = oracle.mv_initial_condition(N, L, 2.0, 0.2, 10.0, 1, 1)
    P = oracle.particles_init(N, 4096, 2, 0.0, 0.0, True, 0)
    run = oracle.Run(N, 0.125, ref, P, mhat=math.inf, n_form=0)
    for _ in range(steps):
        run.step()
    errs = {k: rel_err(ctx.state()[k], run.st[k]) for k in ("U", "phi", "E", "pi")}
    last = run.observe() / (4096 * a * a)
    e_pt = abs(obs[-1, 1] - last[0]) / abs(last[0])
    e_pl = abs(obs[-1, 2] - last[1]) / abs(last[1])
    print(f"FP32 field errors {errs}, <dp_T^2> rel {e_pt:.2e}, <dp_L^2> rel {e_pl:.2e}, unitarity {d[6]:.1e}")
    assert max(errs.values()) < 2e-3
    assert e_pt < 1e-4 and e_pl < 1e-4
    assert d[6] < 1e-5


def test_fp32_dynamic_particles_with_charge_renormalisation():
    """Moving particles in float: rotations, the rapidity Wilson line and the
    renormalisation of Q onto Q0's spectrum every 16 steps, against the double
    oracle after 48 steps (three renormalisations)."""
    N, L, n0, n_form, steps = 32, 6.0, 4, 2, 48
    a = oracle.lattice_spacing(L, N)
    st = inputs.random_state(N, 51, eps_link=0.3, e_scale=0.05, phi_scale=0.05, pi_scale=0.05)
    P = inputs.random_particles(2000, N, 52, p_scale=0.6)
    P[:, 6:14] = oracle.particles_init(N, 2000, 53, 0.0, 0.0, True, 0)[:, 6:14]   # Casimirs of Q0
    ctx = cp.Context(glasma(N, L, steps=n0 + steps, precision=cp.FP32, reunit_every=16),
                     particle_params(2000, 0.3 / a, N, L, n_form))
    ctx.load_state(st, n=n0, particles=P)
    ctx.step(steps)
    d = ctx.diagnostics()
    got = ctx.get_state(cp.STATE_PARTICLES)
    run = oracle.Run(N, 0.125, st, P, mhat=0.3, n_form=n_form, n0=n0)
    for _ in range(steps):
        run.step()
    same = np.all(got[:, 14:16] == run.P[:, 14:16], axis=1)
    assert same.mean() > 0.99                       # float rounding may move a particle across a cell edge
    q_err = np.max(np.abs(got[same, 6:14] - run.P[same, 6:14]))
    p_err = np.max(np.abs(got[same, 3:6] - run.P[same, 3:6])) / np.max(np.abs(run.P[:, 3:6]))
    print(f"FP32 dynamic: cells equal {same.mean():.4f}, max |dQ| {q_err:.2e}, rel |dp| {p_err:.2e}, "
          f"Casimir drift {d[8]:.1e} {d[9]:.1e}")
    assert q_err < 1e-3 and p_err < 1e-3
    assert d[8] < 1e-4 and d[9] < 1e-4


def test_tuner_leaves_state_unchanged():
    N, L = 64, 0.75
    g = glasma(N, L, n_sheets=2, steps=64, seed=9)
    p = dict(n=5000, mass_GeV=1.27, pT_min_GeV=1.0, pT_max_GeV=1.0, azimuth_uniform=1, tau_form_fm=0.0, rep=0, seed=10)
    a_ctx, b_ctx = cp.Context(g, p), cp.Context(g, p)
    for c in (a_ctx, b_ctx):
        c.enable_jets(x_offset=0.3)
        c.init_mv()
        c.step(20)
    before = a_ctx.state()
    rep = a_ctx.tune(2)
    # isolated trials, then whole steps from a saved copy of the state
    assert "best field" in rep and "best push" in rep and "step with field" in rep
    assert rep.strip().splitlines()[-1].startswith("chosen:")
    after = a_ctx.state()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    assert np.array_equal(a_ctx.get_state(cp.STATE_PARTICLES), b_ctx.get_state(cp.STATE_PARTICLES))
    for w in (cp.STATE_JET_W, cp.STATE_JET_F):
        assert np.array_equal(a_ctx.get_state(w), b_ctx.get_state(w))
    a_ctx.step(20)
    b_ctx.step(20)
    # the tuned launch may use another decomposition of the same stencil, whose
    # products associate differently: results agree to rounding
    for k in ("U", "phi", "E", "pi"):
        assert rel_err(a_ctx.state()[k], b_ctx.state()[k]) < 1e-12, k
    assert rel_err(a_ctx.get_state(cp.STATE_PARTICLES), b_ctx.get_state(cp.STATE_PARTICLES)) < 1e-12
    assert rel_err(a_ctx.get_state(cp.STATE_JET_F), b_ctx.get_state(cp.STATE_JET_F)) < 1e-12
    oa, ob = a_ctx.observables(), b_ctx.observables()
    assert oa.shape == ob.shape and rel_err(oa, ob) < 1e-12


def test_force_table_matches_gather_push():
    """A dense ensemble (4 particles per site) in the three push modes,
    graph-replayed past the formation step: the same records to rounding (the
    same per-site arithmetic, evaluated at different places; the fused step
    pushes three quarters of them as stragglers)."""
    N, L = 48, 4.8
    g = glasma(N, L, n_sheets=2, steps=60, seed=13)
    p = dict(n=4 * N * N, mass_GeV=1.27, pT_min_GeV=0.0, pT_max_GeV=3.0, azimuth_uniform=1, tau_form_fm=0.3, rep=0,
             seed=14)
    out = []
    for mode in (cp.PUSH_GATHER, cp.PUSH_TABLE, cp.PUSH_TILE):
        ctx = cp.Context(g, p)
        assert ctx.push_mode() == cp.PUSH_TABLE          # the default for more particles than sites
        ctx.set_push_mode(mode)
        assert ctx.push_mode() == mode
        ctx.init_mv()
        ctx.evolve(1e9)
        out.append((ctx.get_state(cp.STATE_PARTICLES), ctx.observables()))
        ctx.close()
    for o in out[1:]:
        assert np.array_equal(out[0][0][:, 14:16], o[0][:, 14:16])
        assert rel_err(o[0], out[0][0]) < 1e-12
        assert rel_err(o[1], out[0][1]) < 1e-12


@pytest.mark.parametrize("launch", ["ctile32x8", "tile32x8", "site64x4", "link32x4w2"])
def test_links_are_kept_as_two_rows(launch):
    """The device keeps the first two rows of each link (include/cpic.h): the
    third rows given to cpic_set_state are never read, so zeroing them leaves
    every result bit for bit the same in every field decomposition, and
    cpic_get_state returns the third row as the conjugate cross product of
    the first two (for a unitary link of unit determinant: its third row)."""
    N, L, n0, steps, n = 32, 6.0, 4, 20, 500
    a = oracle.lattice_spacing(L, N)
    st = inputs.random_state(N, 71, eps_link=0.5)
    P = inputs.random_particles(n, N, 72, p_scale=0.6)
    cut = dict(st, U=st["U"].copy())
    cut["U"][..., 2, :] = 0.0
    out = []
    for state in (st, cut):
        ctx = cp.Context(glasma(N, L, steps=n0 + steps), particle_params(n, 0.3 / a, N, L, 0))
        ctx.set_launch(*LAUNCHES[launch])
        ctx.load_state(state, n=n0, particles=P)
        U0 = ctx.get_state(cp.STATE_U)
        ctx.step(steps)
        ctx.sync()
        out.append([U0] + [ctx.get_state(w) for w in (cp.STATE_U, cp.STATE_E, cp.STATE_PHI, cp.STATE_PI,
                                                      cp.STATE_PARTICLES)] + [ctx.observables()])
        ctx.close()
    for x, y in zip(out[0], out[1]):
        assert np.array_equal(x, y)
    # the third row handed back is the one of the (unitary) input links
    assert np.max(np.abs(out[0][0] - st["U"])) < 1e-14
    U = out[0][1]
    r3 = np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
    assert np.max(np.abs(U[..., 2, :] - r3)) < 1e-15


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_store_policy_does_not_change_results(precision):
    """The compressed-tile field update stores the new links and phi
    non-temporal or with the default cache policy (cpic_set_store_policy):
    the same run under either policy, switched mid-run, ends in identical
    bits (fields, particle records, samples)."""
    print(f"case store policy {precision}", flush=True)
    N, L, n0, steps, n = 48, 9.0, 4, 40, 2000
    a = oracle.lattice_spacing(L, N)
    prec = cp.FP64 if precision == "fp64" else cp.FP32
    st = inputs.random_state(N, 61, eps_link=0.4)
    P = inputs.random_particles(n, N, 62, p_scale=0.6)
    out = []
    for policy in ((1, 1), (0, 0), (0, 1)):
        ctx = cp.Context(glasma(N, L, steps=n0 + steps, precision=prec, reunit_every=8 if prec == cp.FP32 else 0),
                         particle_params(n, 0.3 / a, N, L, 1))
        ctx.set_launch(64, 8, 1, 1, 3)
        ctx.load_state(st, n=n0, particles=P)
        ctx.set_store_policy(policy[0])
        assert ctx.get_launch()["nt_store"] == policy[0]
        ctx.step(steps // 2)
        ctx.set_store_policy(policy[1])
        ctx.step(steps - steps // 2)
        ctx.sync()
        out.append([ctx.get_state(w) for w in (cp.STATE_U, cp.STATE_E, cp.STATE_PHI, cp.STATE_PI,
                                               cp.STATE_PARTICLES)] + [ctx.observables()])
        ctx.close()
    for run in out[1:]:
        for x, y in zip(out[0], run):
            assert np.array_equal(x, y)


class _CkptHeader(ctypes.Structure):
    _fields_ = [("magic", ctypes.c_char * 8), ("version", ctypes.c_int32), ("N", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("n", ctypes.c_int32), ("cur", ctypes.c_int32),
                ("nsamples", ctypes.c_int32), ("np", ctypes.c_int64), ("nslots", ctypes.c_int32),
                ("jets", ctypes.c_int32), ("gp", cp.GlasmaParams), ("pp", cp.ParticleParams)]


def internal_order(path, reals_per_site=68, part_reals=19):
    """Cells and original indices of the records in the library's internal
    order, read from a checkpoint (state, records, cells, pid in that order)."""
    raw = open(path, "rb").read()
    h = _CkptHeader.from_buffer_copy(raw)
    tsz = 8 if h.prec == cp.FP64 else 4
    off = ctypes.sizeof(h) + 8 * h.nsamples + reals_per_site * h.N * h.N * tsz + part_reals * h.np * tsz
    cell = np.frombuffer(raw, np.int32, 2 * h.np, off).reshape(2, h.np)
    pid = np.frombuffer(raw, np.int32, h.np, off + 8 * h.np)
    return h, cell, pid


@pytest.mark.parametrize("n,static,shape,piled", [(3000, False, None, 0), (3000, True, None, 0),
                                                  (40000, False, None, 0), (3000, False, (16, 16), 0),
                                                  (3000, True, None, 900)])
def test_reordering_is_a_stable_sort_by_tile(tmp_path, n, static, shape, piled):
    """Right after the first reordering (from the input order) the records are
    ordered by their tile key (32 x 16 cell tiles for the gather push, the
    fused kernel's tiles for the fused step; row-major inside a tile), records
    of one cell in ascending input index: the permutation of a stable sort.
    40000 records on 48^2 put 17 on a cell on average; `piled` records of the
    input (every third one) sit on one cell, a run longer than the insertion
    sort handles."""
    print(f"case reorder n={n} static={static} shape={shape} piled={piled}", flush=True)
    N, L, n_form = 48, 9.0, 3
    a = oracle.lattice_spacing(L, N)
    st = inputs.random_state(N, 91, eps_link=0.4)
    P = inputs.random_particles(n, N, 92, p_scale=0.6)
    if piled:
        sel = np.arange(0, 3 * piled, 3)
        P[sel, 0], P[sel, 1] = 17.2, 30.4
        P[sel, 14], P[sel, 15] = 17, 30
    ctx = cp.Context(glasma(N, L, steps=20), particle_params(n, math.inf if static else 0.3 / a, N, L, n_form))
    if shape:
        ctx.set_launch(shape[0], shape[1], 1, 1, 4)
    ctx.load_state(st, n=0, particles=P)
    ctx.step(n_form + 1)   # the reordering before the push of step n_form; the cells of that step stored by it
    path = tmp_path / "order.ckpt"
    ctx.save(str(path))
    ctx.close()
    h, cell, pid = internal_order(path)
    assert h.np == n and sorted(pid.tolist()) == list(range(n))
    tx, ty = shape or (32, 16)
    cx, cy = cell[0].astype(np.int64), cell[1].astype(np.int64)
    ntx = (N + tx - 1) // tx
    key = ((cy // ty) * ntx + cx // tx) * (tx * ty) + (cy % ty) * tx + cx % tx
    order = np.lexsort((pid, key))       # by key, then by input index
    assert np.array_equal(order, np.arange(n))
