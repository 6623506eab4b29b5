"""Pins of the oracle's 1-D PPM face value (the inner operator of fv_tp_2d,
Sec. IX-C, Lin-Rood transport): closed forms on constant and linear data,
the exact upwind shift at Courant number +-1, the monotone bound of the
1-D flux-form update, and for the unlimited order (hord 6) the exact swept
mean of quadratics, agreement with the monotone order on linear data and the
new extrema it is allowed to make."""
import numpy as np
import pytest

H = 3


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


# ---- the unlimited order (hord 6) ----------------------------------------

def _quad_cells(a, b, c2, s):
    """Mean of a + b x + c2 x^2 over the cell [s - 1/2, s + 1/2]."""
    P = lambda x: a * x + b * x * x / 2 + c2 * x ** 3 / 3
    return P(s + 0.5) - P(s - 0.5)


def _quad_swept(a, b, c2, x0, x1):
    P = lambda x: a * x + b * x * x / 2 + c2 * x ** 3 / 3
    return (P(x1) - P(x0)) / (x1 - x0)


@pytest.mark.parametrize("c", [0.05, 0.37, 0.5, 0.81, 1.0, -0.05, -0.37, -0.5, -0.81, -1.0])
def test_unlimited_quadratic_exact(orc, c):
    """Fourth-order edges are exact for cell means of a quadratic, and the
    parabola through two exact edges with the exact mean is the quadratic
    itself: the face value is the exact mean over the swept interval
    [m - 1/2 - c, m - 1/2] (c > 0) or [m - 1/2, m - 1/2 - c] (c < 0)."""
    rng = np.random.default_rng(21)
    for _ in range(20):
        a, b, c2 = rng.normal(size=3) * (4, 2, 1)
        q = np.array([_quad_cells(a, b, c2, s) for s in range(6)])
        f = 2.5
        want = _quad_swept(a, b, c2, f - c, f) if c > 0 else _quad_swept(a, b, c2, f, f - c)
        got = orc.ppm_face(q, c, hord=6)
        assert abs(got - want) <= 2e-14 * (abs(a) + 6 * abs(b) + 36 * abs(c2)), (got, want)


def test_unlimited_equals_monotone_on_linear(orc):
    rng = np.random.default_rng(22)
    for _ in range(50):
        alpha, beta = rng.normal(size=2) * 5
        q = alpha + beta * np.arange(6)
        c = rng.uniform(-1, 1)
        assert abs(orc.ppm_face(q, c, hord=6) - orc.ppm_face(q, c)) <= 1e-14 * (abs(alpha) + 6 * abs(beta))


def test_unlimited_courant_one_is_upwind_cell(orc):
    rng = np.random.default_rng(23)
    for _ in range(100):
        q = rng.random(6)
        assert orc.ppm_face(q, 1.0, hord=6) == q[2]
        assert orc.ppm_face(q, -1.0, hord=6) == q[3]


def test_unlimited_extremum_not_flattened(orc):
    """Without the limiter a local maximum keeps its curvature, where the
    monotone order returns the cell mean itself.  Closed form: both edges of
    cell 2 from the fourth-order interpolation 7/12 (q0 + q1) - 1/12 (q- + q+)
    are 41/12; the parabola with those edges and mean 5 is e + 6 (5 - e) x (1 - x),
    and its mean over the swept part x in [0.6, 1] follows from the integral
    of x - x^2."""
    q = np.array([0.0, 1.0, 5.0, 1.0, 0.0, 0.0])
    assert orc.ppm_face(q, 0.4) == 5.0
    e = 7 / 12 * (1.0 + 5.0) - 1 / 12 * (0.0 + 1.0)
    assert abs(e - 41 / 12) < 1e-15
    want = e + 6 * (5.0 - e) * (1 / 6 - (0.6 ** 2 / 2 - 0.6 ** 3 / 3)) / 0.4
    assert abs(orc.ppm_face(q, 0.4, hord=6) - want) <= 1e-14


def _update_1d_order(orc, q, c, hord):
    n = len(q)
    F = np.array([orc.ppm_face(np.array([q[(m + s - 3) % n] for s in range(6)]), c, hord=hord)
                  for m in range(n)])
    return q + c * (F - np.roll(F, -1))


def test_unlimited_update_conserves_and_overshoots(orc):
    """The flux-form update conserves the sum for any face values; on a step
    the unlimited order creates new extrema (its defining difference from the
    monotone order, which keeps the data in [0, 1])."""
    q = np.array([0.0] * 6 + [1.0] * 6)
    for c in (0.3, 0.6, -0.45):
        qu = _update_1d_order(orc, q, c, 6)
        qm = _update_1d_order(orc, q, c, 8)
        assert abs(qu.sum() - q.sum()) <= 1e-13
        assert qu.min() < -1e-3 or qu.max() > 1 + 1e-3
        assert qm.min() >= -1e-15 and qm.max() <= 1 + 1e-15


@pytest.mark.parametrize("axis", ["x", "y"])
def test_unlimited_transport_quadratic_faces(orc, axis):
    """fv_tp_2d on a grid built with hord 6, flow along one axis only: at every
    face whose six-cell stencil lies inside the quadratic (away from the
    periodic seam), the flux over the Courant-weighted area is the exact
    swept mean of the quadratic."""
    n = 24
    g = orc.Grid(0, n, 1, delta=1000.0, hord=6)
    N = g.N
    A = g.metric("area")[0, H, H]
    a, b, c2 = 0.3, 0.07, -0.011
    prof = np.array([_quad_cells(a, b, c2, s) for s in range(n)])
    Q = g.field(1)
    Q[0, 0, H:H + n, H:H + n] = prof[None, :] if axis == "x" else prof[:, None]
    orc.halo_fill(g, Q)
    for c in (0.42, -0.77):
        zero = np.zeros((N, N))
        cr = np.full((N, N), c)
        if axis == "x":
            FX, _ = orc.fv_tp_2d(g, 0, Q[0, 0], cr, zero, cr * A, zero)
            face = FX[H + n // 2, H:H + n + 1] / (c * A)
        else:
            _, FY = orc.fv_tp_2d(g, 0, Q[0, 0], zero, cr, zero, cr * A)
            face = FY[H:H + n + 1, H + n // 2] / (c * A)
        for m in range(3, n - 2):
            f = m - 0.5
            want = _quad_swept(a, b, c2, f - c, f) if c > 0 else _quad_swept(a, b, c2, f, f - c)
            assert abs(face[m] - want) <= 1e-13, (axis, c, m, face[m], want)
        g8 = orc.Grid(0, n, 1, delta=1000.0)
        if axis == "x":
            F8, _ = orc.fv_tp_2d(g8, 0, Q[0, 0], cr, zero, cr * A, zero)
            f8 = F8[H + n // 2, H:H + n + 1] / (c * A)
        else:
            _, F8 = orc.fv_tp_2d(g8, 0, Q[0, 0], zero, cr, zero, cr * A)
            f8 = F8[H:H + n + 1, H + n // 2] / (c * A)
        # the monotone order flattens the quadratic's extremum at s = -b / (2 c2) ~ 3.2
        assert np.abs(f8[3:n - 2] - face[3:n - 2]).max() > 1e-6


def test_unlimited_order_reaches_kinetic_energy(orc):
    """The hord switch also reaches the kinetic-energy faces of the momentum
    update: with every transport of the substep on one order the C-grid half
    step (which has no PPM) is the same for both orders and the D-grid winds
    are not."""
    import fv3_inputs as fi
    n, nz = 16, 2
    init = fi.periodic_state(n=n, nz=nz, seed=4)
    out = {}
    for hord in (6, 8):
        g = orc.Grid(0, n, nz, delta=1000.0, hord=hord)
        for stage in (2, 6):
            s = orc.new_state(g, init)
            assert orc.acoustic_substeps(g, s, 2.0, 1, stop_stage=stage) == 0
            out[hord, stage] = {k: s[k].copy() for k in ("uc", "vc", "u", "v", "pt", "w")}
    for k in ("uc", "vc"):
        np.testing.assert_array_equal(out[6, 2][k], out[8, 2][k])
    for k in ("u", "v", "pt"):
        assert np.abs(out[6, 6][k] - out[8, 6][k]).max() > 0, k


@pytest.mark.parametrize("axis", ["x", "y"])
def test_unlimited_order_in_kinetic_energy_alone(orc, axis):
    """D-grid winds that are the differences of a corner potential varying
    along one axis only: zero circulation around every cell, so the vorticity
    flux of the momentum update vanishes for both orders, and only the wind
    along that axis is non-zero, so the kinetic energy holds that wind's face
    value alone.  The updated winds then differ between the orders only
    through that face value: a difference far above rounding shows that it
    follows the order."""
    import fv3_inputs as fi
    n, nz, dx = 16, 1, 1000.0
    init = fi.periodic_state(n=n, nz=nz, seed=4)
    x = np.arange(n) * 2 * np.pi / n
    p1 = 2.5e4 * np.sin(x) + 1.0e4 * np.cos(2 * x)
    psi = np.tile(p1, (n, 1)) if axis == "x" else np.tile(p1[:, None], (1, n))
    u = (np.roll(psi, -1, axis=1) - psi) / dx          # edge (i, j)-(i+1, j)
    v = (np.roll(psi, -1, axis=0) - psi) / dx          # edge (i, j)-(i, j+1)
    init["u"][0, 0, H:H + n, H:H + n] = u
    init["u"][0, 0, H + n, H:H + n] = u[0]
    init["v"][0, 0, H:H + n, H:H + n] = v
    init["v"][0, 0, H:H + n, H + n] = v[:, 0]
    out = {}
    for hord in (6, 8):
        g = orc.Grid(0, n, nz, delta=dx, hord=hord)
        s = orc.new_state(g, init)
        assert orc.acoustic_substeps(g, s, 2.0, 1, stop_stage=6) == 0
        out[hord] = s
    k = "u" if axis == "x" else "v"
    ref = np.abs(init[k]).max()
    assert np.abs(out[6][k] - out[8][k]).max() > 1e-6 * ref
