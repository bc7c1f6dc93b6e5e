"""The oracle's Philox4x64-10 against numpy's independent implementation
(numpy.random.Philox, same published algorithm), and the Box-Muller normals."""
import numpy as np

import oracle


def test_philox_matches_numpy():
    for key in ([0, 0], [1, 3], [0xDEADBEEF12345678, 0x0123456789ABCDEF]):
        for ctr in ([0, 0, 0, 0], [5, 7, 0, 0], [2 ** 64 - 2, 1, 2, 3]):
            bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
            # numpy increments the counter before producing its first block
            ref = bg.random_raw(4)
            c1 = list(ctr)
            c1[0] = (c1[0] + 1) % 2 ** 64
            if c1[0] == 0:
                c1[1] += 1
            got = oracle.philox(c1, key)
            assert np.array_equal(got, ref)


def test_mv_charge_statistics():
    """Gaussian colour charges: mean 0, variance sigma^2, no colour correlation
    (the regularised correlator [eq:MVchargecorrnum] with a Kronecker delta)."""
    N, sigma = 128, 0.37
    rho = oracle.mv_charges(N, 11, 0, 3, sigma).reshape(-1, 8)
    n = rho.shape[0]
    assert np.all(np.abs(rho.mean(0)) < 5 * sigma / np.sqrt(n))
    var = rho.var(0)
    assert np.all(np.abs(var / sigma ** 2 - 1) < 5 * np.sqrt(2.0 / n))
    cov = np.cov(rho.T) / sigma ** 2
    off = cov - np.diag(np.diag(cov))
    assert np.max(np.abs(off)) < 5 / np.sqrt(n)
    # different sheets and nuclei are independent streams
    rho2 = oracle.mv_charges(N, 11, 0, 4, sigma).reshape(-1, 8)
    rho3 = oracle.mv_charges(N, 11, 1, 3, sigma).reshape(-1, 8)
    for other in (rho2, rho3):
        c = np.mean(rho * other) / sigma ** 2
        assert abs(c) < 5 / np.sqrt(rho.size)
