"""Pins of the oracle's fv_tp_2d (Sec. IX-C: two-dimensional, mass-conserving
horizontal flux-form transport after Lin & Rood) on the doubly periodic
grid: exact one- and two-direction shifts at Courant number 1 (the splitting
reduces to the composition of two 1-D shifts), mass conservation, no new
extrema for uniform flow, constant preservation."""
import numpy as np
import pytest

H = 3


def _step(orc, g, q, cx, cy):
    n, N = g.n, g.N
    A = g.metric("area")[0, H, H]
    Q = g.field(1)
    Q[0, 0, H:H + n, H:H + n] = q
    orc.halo_fill(g, Q)
    crx = np.full((N, N), float(cx))
    cry = np.full((N, N), float(cy))
    xfx = crx * A
    yfx = cry * A
    FX, FY = orc.fv_tp_2d(g, 0, Q[0, 0], crx, cry, xfx, yfx)
    F = FX[H:H + n, H:H + n + 1]
    G = FY[H:H + n + 1, H:H + n]
    return q + (F[:, :-1] - F[:, 1:] + G[:-1, :] - G[1:, :]) / A


@pytest.fixture(scope="module")
def g(orc):
    return orc.Grid(0, 16, 1, delta=1000.0)


def test_shift_x(orc, g):
    q = np.random.default_rng(1).random((16, 16))
    np.testing.assert_allclose(_step(orc, g, q, 1.0, 0.0), np.roll(q, 1, axis=1), rtol=0, atol=1e-15)
    np.testing.assert_allclose(_step(orc, g, q, -1.0, 0.0), np.roll(q, -1, axis=1), rtol=0, atol=1e-15)


def test_shift_y(orc, g):
    q = np.random.default_rng(2).random((16, 16))
    np.testing.assert_allclose(_step(orc, g, q, 0.0, 1.0), np.roll(q, 1, axis=0), rtol=0, atol=1e-15)
    np.testing.assert_allclose(_step(orc, g, q, 0.0, -1.0), np.roll(q, -1, axis=0), rtol=0, atol=1e-15)


def test_shift_diagonal_and_repeated(orc, g):
    q = np.random.default_rng(3).random((16, 16))
    np.testing.assert_allclose(_step(orc, g, q, 1.0, 1.0), np.roll(q, (1, 1), axis=(0, 1)),
                               rtol=0, atol=1e-15)
    np.testing.assert_allclose(_step(orc, g, q, -1.0, 1.0), np.roll(q, (1, -1), axis=(0, 1)),
                               rtol=0, atol=1e-15)
    r = q.copy()
    for _ in range(5):
        r = _step(orc, g, r, 1.0, 0.0)
    np.testing.assert_allclose(r, np.roll(q, 5, axis=1), rtol=0, atol=1e-14)


def test_uniform_flow_monotone_and_conservative(orc, g):
    rng = np.random.default_rng(4)
    q0 = np.where(rng.random((16, 16)) > 0.7, 1.0, 0.0) + 0.2 * rng.random((16, 16))
    q = q0.copy()
    for _ in range(30):
        q = _step(orc, g, q, 0.37, -0.81)
        assert q.min() >= q0.min() - 1e-14
        assert q.max() <= q0.max() + 1e-14
    assert abs(q.sum() - q0.sum()) <= 1e-13 * q0.sum()


def test_constant_preserved(orc, g):
    q = np.full((16, 16), 0.7)
    for cx, cy in ((0.3, 0.9), (-0.6, 0.2), (1.0, -1.0)):
        np.testing.assert_allclose(_step(orc, g, q, cx, cy), 0.7, rtol=1e-15, atol=0)


def test_split_average_of_orderings(orc, g):
    # For uniform flow the result is 1/2 (X o Y + Y o X) of the 1-D operators.
    q = np.random.default_rng(6).random((16, 16))
    cx, cy = 0.45, 0.7
    xy = _step(orc, g, _step(orc, g, q, 0.0, cy), cx, 0.0)
    yx = _step(orc, g, _step(orc, g, q, cx, 0.0), 0.0, cy)
    np.testing.assert_allclose(_step(orc, g, q, cx, cy), 0.5 * (xy + yx), rtol=0, atol=1e-14)
