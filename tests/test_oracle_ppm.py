"""Pins of the oracle's 1-D PPM face value (the inner operator of fv_tp_2d,
Sec. IX-C, Lin-Rood transport): closed forms on constant and linear data,
the exact upwind shift at Courant number +-1, and the monotone bound of the
1-D flux-form update."""
import numpy as np
import pytest


def test_constant_data_exact(orc):
    for c in (-1.0, -0.6, -0.01, 0.0, 0.3, 0.99, 1.0):
        assert orc.ppm_face(np.full(6, 3.25), c) == 3.25


@pytest.mark.parametrize("c", [0.05, 0.37, 0.5, 0.81, 1.0, -0.05, -0.37, -0.5, -0.81, -1.0])
def test_linear_data_closed_form(orc, c):
    # cells m-3..m+2 hold alpha + beta*s (cell s centred at s); face m at m - 1/2.
    # The swept interval's mean of the exact linear profile is alpha + beta(m - 1/2 - c/2).
    rng = np.random.default_rng(11)
    for _ in range(20):
        alpha, beta = rng.normal(size=2) * 5
        m = 3
        q = alpha + beta * np.arange(6)
        want = alpha + beta * (m - 0.5 - 0.5 * c)
        got = orc.ppm_face(q, c)
        assert abs(got - want) <= 1e-14 * (abs(alpha) + 6 * abs(beta))


def test_courant_one_is_upwind_cell(orc):
    rng = np.random.default_rng(5)
    for _ in range(200):
        q = rng.random(6)
        assert orc.ppm_face(q, 1.0) == q[2]      # cell m-1
        assert orc.ppm_face(q, -1.0) == q[3]     # cell m


def test_local_extremum_flat(orc):
    # a local maximum in the upwind cell has zero slope: the face value is the cell mean
    q = np.array([0.0, 1.0, 5.0, 1.0, 0.0, 0.0])
    assert orc.ppm_face(q, 0.4) == 5.0


def _update_1d(orc, q, c):
    """Periodic 1-D flux-form update q_m += c (F_m - F_{m+1}) with uniform c."""
    n = len(q)
    F = np.array([orc.ppm_face(np.array([q[(m + s - 3) % n] for s in range(6)]), c)
                  for m in range(n)])
    return q + c * (F - np.roll(F, -1))


def test_monotone_1d_update_no_new_extrema(orc):
    rng = np.random.default_rng(7)
    viol = 0
    for trial in range(300):
        n = 12
        q = rng.random(n) if trial % 2 else np.where(rng.random(n) > 0.6, 1.0, 0.0)
        c = rng.uniform(-1, 1)
        qn = _update_1d(orc, q, c)
        for m in range(n):
            nb = [q[(m + d) % n] for d in (-2, -1, 0, 1, 2)]
            if qn[m] > max(nb) + 1e-14 or qn[m] < min(nb) - 1e-14:
                viol += 1
        assert qn.min() >= q.min() - 1e-14 and qn.max() <= q.max() + 1e-14
        assert abs(qn.sum() - q.sum()) <= 1e-13
    assert viol == 0


def test_shift_one_cell_per_step(orc):
    rng = np.random.default_rng(3)
    q = rng.random(16)
    qn = _update_1d(orc, q, 1.0)
    np.testing.assert_allclose(qn, np.roll(q, 1), rtol=0, atol=2e-16)
    qn = _update_1d(orc, q, -1.0)
    np.testing.assert_allclose(qn, np.roll(q, -1), rtol=0, atol=2e-16)
