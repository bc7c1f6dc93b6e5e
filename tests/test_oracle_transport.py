"""Pins of the oracle's transport coefficients ([eq:kappalt], [eq:qhati]) and
anisotropies (the heavy-quark ratio <dp_L^2>/<dp_T^2> and [eq:jetanisotropy]):
closed forms on series whose derivative is known exactly."""
import numpy as np

import oracle


def test_quadratic_series_exact_at_midpoints():
    """<dp^2>(tau) = a (tau - tau_f)^2 + c (tau - tau_f), sampled at uneven
    times: the derivative at each interval's midpoint is 2 a (tau_mid - tau_f)
    + c exactly, the first interval opening at the formation time."""
    tau_f = 0.1
    tau = np.array([0.13, 0.2, 0.26, 0.41, 0.5, 0.77])
    a = np.array([2.0, -0.5, 1.5, 0.25])
    c = np.array([0.3, 4.0, -1.0, 0.0])
    d = tau - tau_f
    b = a[None, :] * d[:, None] ** 2 + c[None, :] * d[:, None]
    out = oracle.transport_coefficients(tau_f, tau, b)
    mids = 0.5 * (np.concatenate([[tau_f], tau[:-1]]) + tau)
    assert np.allclose(out[:, 0], mids, rtol=0, atol=1e-15)
    want = 2 * a[None, :] * (mids - tau_f)[:, None] + c[None, :]
    assert np.allclose(out[:, 1:5], want, rtol=1e-12, atol=1e-12)
    assert np.array_equal(out[:, 5], tau)


def test_linear_series_constant_coefficient():
    tau_f = 0.0
    tau = np.linspace(0.05, 1.0, 20)
    k = np.array([1.7, 0.2, 3.0, 0.9])
    out = oracle.transport_coefficients(tau_f, tau, tau[:, None] * k[None, :])
    assert np.allclose(out[:, 1:5], k[None, :], rtol=1e-13)


def test_anisotropies_are_the_paper_ratios():
    """Column 6 is <dp_L^2>/<dp_T^2>, column 7 <dp_z^2>/<dp_y^2> with the
    longitudinal component <dp_z^2> = <dp_L^2> and y the direction across the
    initial one."""
    b = np.array([[2.0, 3.0, 5.0, 7.0], [4.0, 1.0, 8.0, 0.5]])
    out = oracle.transport_coefficients(0.0, [0.1, 0.2], b)
    assert np.allclose(out[:, 6], [1.5, 0.25])
    assert np.allclose(out[:, 7], [3.0 / 7.0, 2.0])
