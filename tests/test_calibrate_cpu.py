"""CPU checks of the host-only calibration plan (eqs. 35-41) against the
oracle's formulas, on sums that exercise every branch."""
import numpy as np
import pytest

from paper_2301_05780_amd import pdd
from oracle.calibrate import plan, STATS_WIDTH


def test_plan_matches_the_oracle():
    rng = np.random.default_rng(0)
    n, N = 200, 500
    phi = rng.normal(1.0, 0.3, size=(n, N))
    xi = -0.8 * (phi - 1.0) + rng.normal(0.0, 0.05, size=(n, N))
    diff = rng.normal(rng.normal(0, 0.003, size=(n, 1)), 0.01, size=(n, N))
    st = np.stack([diff.sum(1), phi.sum(1), (phi * phi).sum(1), xi.sum(1), (xi * xi).sum(1), (phi * xi).sum(1),
                   np.full(n, 7.0 * N), np.full(n, 9.0 * N)], axis=1)
    st[0, 0] = 0.0                     # no bias: h = h0
    st[1, 3:6] = 0.0                   # no control variate: rho^2 = 0
    st[2, 1:3] = (N, N)                # zero variance: one job
    got = pdd.calibration_plan(st, N, 1e-3, 0.01, 64)
    ref = plan(st, N, 1e-3, 0.01, 64)
    assert np.allclose(got["h"], ref["h"], rtol=1e-14, atol=0)
    assert np.array_equal(got["n_paths"], ref["n_paths"])
    for key in ("bias", "var", "rho2"):
        assert np.allclose(got[key], ref[key], rtol=1e-12, atol=1e-15), key
    assert got["h"][0] == 1e-3 and got["rho2"][1] == 0.0 and got["n_paths"][2] == 64
    # calibration at h0' = 4 h0: eq. 40's numerator takes h0', the cap stays h0
    eps = 1e-3
    got1 = pdd.calibration_plan(st, N, 1e-3, eps, 64)
    got4 = pdd.calibration_plan(st, N, 1e-3, eps, 64, h0_cal=4e-3)
    ref4 = plan(st, N, 1e-3, eps, 64, h0_cal=4e-3)
    assert np.allclose(got4["h"], ref4["h"], rtol=1e-14, atol=0) and np.all(got4["h"] <= 1e-3)
    mdiff = np.abs(st[:, 0] / N)
    big = mdiff > 2.0 * 4e-3 * eps / 3.0 / 1e-3             # knots where eq. 40's second term binds
    assert big.sum() > 10 and np.allclose(got4["h"][big], 2.0 * 4e-3 * eps / (3.0 * mdiff[big]), rtol=1e-14)
    assert np.allclose(got4["h"][big], 4.0 * got1["h"][big], rtol=1e-14)


def test_plan_rejects_bad_arguments():
    st = np.zeros((3, STATS_WIDTH))
    for args in ((st, 0, 1e-3, 0.01, 10), (st, 10, 0.0, 0.01, 10), (st, 10, 1e-3, -1.0, 10), (st, 10, 1e-3, 0.01, 0)):
        with pytest.raises(pdd.PddError):
            pdd.calibration_plan(*args)
    with pytest.raises(pdd.PddError):                       # h0' below the production cap h0
        pdd.calibration_plan(st, 10, 1e-3, 0.01, 10, h0_cal=5e-4)
