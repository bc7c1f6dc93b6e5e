"""The drift watchdog (cpic_set_watchdog) through the C ABI: each breach
forced from the host and reported by cpic_sync, and silence on sound runs.

  * a non-unitary link installed with cpic_set_state -> CPIC_E_DRIFT (unitarity);
  * a non-finite field value -> CPIC_E_NAN;
  * Gauss-law and Casimir drift: the leapfrog keeps both to rounding, so a
    threshold below rounding trips them and the default one does not;
  * every = 0 switches the checks off; a reported breach is cleared.
"""
import numpy as np
import pytest

import inputs

cp = pytest.importorskip("paper_2303_05599_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E_DRIFT, E_NAN = -6, -5


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    cp.lib()
    yield


def context(N=32, steps=200, n=500, precision=None, **kw):
    L = 6.0
    g = dict(N=N, L_fm=L, g2mu_GeV=2.0, m_ir_GeV=0.2, uv_GeV=10.0, n_sheets=2, dtau_over_a=0.125,
             tau_max_fm=steps * (L / N) * 0.125, seed=31, precision=precision or cp.FP64, reunit_every=16,
             record_every=8)
    g.update(kw)
    p = dict(n=n, mass_GeV=1.27, pT_min_GeV=0.0, pT_max_GeV=2.0, azimuth_uniform=1, tau_form_fm=0.05, rep=0, seed=32)
    return cp.Context(g, p)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sound_run_is_silent(precision):
    """An MV event evolved 200 steps with the default thresholds: no report."""
    print(f"case watchdog silent {precision}", flush=True)
    ctx = context(precision=cp.FP64 if precision == "fp64" else cp.FP32)
    ctx.init_mv()
    ctx.evolve(1e9)
    ctx.sync()
    ctx.close()


def test_non_unitary_link_is_reported():
    print("case watchdog unitarity", flush=True)
    ctx = context()
    ctx.init_mv()
    ctx.step(10)
    st = ctx.state()
    st["U"][0, 5, 7] *= 1.05          # one link off the group manifold
    ctx.load_state(st, n=10)
    ctx.step(60)                      # past the check after step 63
    with pytest.raises(cp.CpicError) as e:
        ctx.sync()
    assert e.value.status == E_DRIFT and "unitarity" in str(e.value)
    ctx.sync()                        # reported once, then cleared
    ctx.close()


def test_non_finite_field_is_reported():
    """(Without particles: a particle in a non-finite field would first be
    reported as a cell jump.)"""
    print("case watchdog nan", flush=True)
    ctx = context(n=0)
    ctx.set_watchdog(every=8)
    ctx.init_mv()
    ctx.step(3)
    st = ctx.state()
    st["E"][1, 3, 4, 2] = np.nan
    ctx.load_state(st, n=3)
    ctx.step(8)
    with pytest.raises(cp.CpicError) as e:
        ctx.sync()
    assert e.value.status == E_NAN and "non-finite" in str(e.value)
    ctx.close()


@pytest.mark.parametrize("which", ["gauss", "casimir"])
def test_drift_thresholds(which):
    """A random state (its Gauss residual and charge Casimirs far from zero
    and from q2(R)) drifts only by rounding: a threshold of 1e-30 trips the
    check, the default 1e-8 does not."""
    print(f"case watchdog {which}", flush=True)
    N = 32
    st = inputs.random_state(N, 33, eps_link=0.4)
    P = inputs.random_particles(500, N, 34, p_scale=0.6)
    for thr, trips in ((1e-8, False), (1e-30, True)):
        ctx = context(N, steps=80)
        kw = dict(max_gauss_drift=thr) if which == "gauss" else dict(max_casimir_drift=thr)
        ctx.set_watchdog(every=16, **kw)
        ctx.load_state(st, n=4, particles=P)
        ctx.step(40)
        if trips:
            with pytest.raises(cp.CpicError) as e:
                ctx.sync()
            assert e.value.status == E_DRIFT
            assert ("Gauss" if which == "gauss" else "Casimir") in str(e.value)
        else:
            ctx.sync()
        ctx.close()


def test_watchdog_off():
    print("case watchdog off", flush=True)
    ctx = context()
    ctx.set_watchdog(every=0)
    ctx.init_mv()
    st = ctx.state()
    st["U"][1, 2, 3] *= 1.05
    ctx.load_state(st, n=0)
    ctx.step(70)
    ctx.sync()
    ctx.close()
