"""GPU tests of the error behaviour the C ABI documents (include/cpic.h):
every condition is set up from the host, and every kernel still runs to its
normal end.

  * a particle whose stored cell is two cells from its position: the push
    counts the jump and cpic_sync reports CPIC_E_CELL_JUMP;
  * a non-finite field value: cpic_diagnostics reports CPIC_E_NAN;
  * caller buffers of the wrong size: CPIC_E_CAPACITY, nothing written;
  * checkpoint files that cannot be read or written: CPIC_E_IO;
  * calls out of order or with bad arguments: CPIC_E_INVALID, and the
    context stays usable afterwards; the same for the batch API.
"""
import ctypes

import numpy as np
import pytest

import inputs

cp = pytest.importorskip("paper_2303_05599_amd")
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    cp.lib()
    yield


def glasma(N=16, steps=40):
    L = 0.75 * N / 16
    return dict(N=N, L_fm=L, g2mu_GeV=2.0, m_ir_GeV=0.2, uv_GeV=10.0, n_sheets=1, dtau_over_a=0.125,
                tau_max_fm=steps * 0.125 * L / N, seed=1, precision=cp.FP64, reunit_every=0, record_every=8)


def particles(n=200):
    return dict(n=n, mass_GeV=1.0, pT_min_GeV=0.0, pT_max_GeV=1.0, azimuth_uniform=1, tau_form_fm=0.0, rep=0,
                seed=2)


def status(e):
    return e.value.status


def test_cell_jump_is_reported():
    N = 16
    ctx = cp.Context(glasma(N), particles(200))
    P = inputs.random_particles(200, N, 3, p_scale=0.3)
    P[7, 14] = (P[7, 14] + 2) % N          # stored cell two columns from the position
    ctx.load_state(inputs.random_state(N, 4), n=2, particles=P)
    ctx.step(1)
    with pytest.raises(cp.CpicError) as e:
        ctx.sync()
    assert status(e) == -8 and "cell" in str(e.value).lower()
    ctx.close()


def test_non_finite_field_is_reported():
    N = 16
    ctx = cp.Context(glasma(N), None)
    st = inputs.random_state(N, 5)
    st["E"][1, 3, 4, 2] = np.nan
    ctx.load_state(st, n=2)
    with pytest.raises(cp.CpicError) as e:
        ctx.diagnostics()
    assert status(e) == -5
    ctx.close()


def test_caller_buffers_of_the_wrong_size():
    N = 16
    ctx = cp.Context(glasma(N), particles(64))
    ctx.init_mv()
    ctx.step(17)                            # two samples
    L = cp.lib()
    assert ctx.num_samples() == 2
    out = np.full((1, 6), -1.0)
    assert L.cpic_observables_full(ctx.h, out.ctypes.data, 1) == -7
    assert np.all(out == -1.0)              # nothing written
    phi = np.zeros((N, N, 8))
    assert L.cpic_get_state(ctx.h, cp.STATE_PHI, phi.ctypes.data, phi.nbytes - 8) == -7
    assert L.cpic_set_state(ctx.h, cp.STATE_PHI, phi.ctypes.data, phi.nbytes + 8) == -7
    assert L.cpic_get_state(ctx.h, 99, phi.ctypes.data, phi.nbytes) == -1
    # the context is unharmed
    ctx.step(1)
    ctx.sync()
    assert ctx.n == 18
    ctx.close()


def test_checkpoint_io_errors(tmp_path):
    ctx = cp.Context(glasma(), None)
    ctx.init_mv()
    with pytest.raises(cp.CpicError) as e:
        ctx.load(tmp_path / "missing.bin")
    assert status(e) == -9
    with pytest.raises(cp.CpicError) as e:
        ctx.save(tmp_path / "no_such_dir" / "x.bin")
    assert status(e) == -9
    bad = tmp_path / "garbage.bin"
    bad.write_bytes(b"not a checkpoint" * 4)
    with pytest.raises(cp.CpicError) as e:
        ctx.load(bad)
    assert status(e) in (-9, -1)
    ctx.step(2)
    ctx.close()


def test_calls_out_of_order_and_bad_arguments():
    ctx = cp.Context(glasma(16, steps=20), particles(64))
    with pytest.raises(cp.CpicError) as e:
        ctx.step(1)                         # no state yet
    assert status(e) == -1
    ctx.init_mv()
    with pytest.raises(cp.CpicError) as e:
        ctx.step(21)                        # past n_max
    assert status(e) == -1
    for args in ((48, 4, 1, 1, 3), (64, 4, 1, 2, 3), (64, 4, 1, 1, 7), (100, 3, 1, 1, 0)):
        with pytest.raises(cp.CpicError) as e:
            ctx.set_launch(*args)
        assert status(e) == -1, args
    with pytest.raises(cp.CpicError):
        ctx.set_push_lanes(3)
    with pytest.raises(cp.CpicError):
        ctx.set_push_mode(5)
    ctx.set_timing(True)
    with pytest.raises(cp.CpicError) as e:
        ctx.tune(1)                         # not while kernel timing is on
    assert status(e) == -1
    ctx.set_timing(False)
    launch = ctx.get_launch()
    ctx.step(5)                             # still usable, launch unchanged
    ctx.sync()
    assert ctx.n == 5 and ctx.get_launch() == launch
    ctx.close()


def test_batch_errors():
    """The batch API: mixed precisions, a bad event index, a too small
    observables buffer, bad launch shapes; the batch stays usable."""
    g = glasma(16, steps=20)
    with pytest.raises(cp.CpicError) as e:
        cp.Batch([g, dict(g, precision=cp.FP32)], [particles(64), particles(64)])
    assert status(e) == -1
    b = cp.Batch([g, dict(g, N=24, L_fm=g["L_fm"] * 24 / 16)], [particles(64), dict(n=0)])
    b.init_mv()
    b.step(17)
    b.sync()
    L = cp.lib()
    ns = ctypes.c_int32()
    out = np.zeros((1, 6))
    assert L.cpic_batch_observables(b.h, 0, out.ctypes.data, 1, ctypes.byref(ns)) == -7
    assert ns.value == 2
    for ev in (-1, 2):
        assert L.cpic_batch_observables(b.h, ev, out.ctypes.data, 1, ctypes.byref(ns)) == -1
        with pytest.raises(cp.CpicError) as e:
            b.n(ev)
        assert status(e) == -1
    for args in ((48, 4, 1, 4), (64, 4, 1, 3)):
        with pytest.raises(cp.CpicError) as e:
            b.set_launch(*args)
        assert status(e) == -1
    b.run()
    b.sync()
    assert b.n(0) == 20 and b.n(1) == 20
    assert b.observables(0).shape[0] == 3
    b.close()
