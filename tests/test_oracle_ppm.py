"""Pins of the oracle's 1-D PPM face value (the inner operator of fv_tp_2d,
Sec. IX-C, Lin-Rood transport): closed forms on constant and linear data,
the exact upwind shift at Courant number +-1, the monotone bound of the
1-D flux-form update, and for the unlimited order (hord 6) the exact swept
mean of quadratics, agreement with the monotone order on linear data and the
new extrema it is allowed to make; the 2dx-filtered order (hord 5) and the
positive-definite tracer order (hord 7) against first-order upwind on
two-cell oscillations, the unlimited order on smooth data, and non-negative
1-D and 2-D updates."""
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


# ---- the 2dx-filtered order (hord 5) ------------------------------------

@pytest.mark.parametrize("c", [0.3, 0.8, 1.0, -0.3, -0.8, -1.0])
def test_2dx_oscillation_is_upwind(orc, c):
    """On data alternating between two values every cell is a local extremum,
    so the face takes the upwind cell mean and the 1-D update is first-order
    upwind: q_m - c (q_m - q_{m-1}) for c > 0, q_m - |c| (q_m - q_{m+1})
    for c < 0."""
    q = np.where(np.arange(12) % 2 == 0, 0.2, 1.7)
    got = _update_1d_order(orc, q, c, 5)
    want = q - c * (q - np.roll(q, 1)) if c > 0 else q + c * (q - np.roll(q, -1))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)
    assert np.abs(_update_1d_order(orc, q, c, 6) - want).max() > 1e-2 or abs(c) == 1.0


def test_2dx_one_neighbour_suffices(orc):
    # upwind cell 2 and cell 3 are extrema, cell 1 is not: filtered
    q = np.array([0.0, 0.0, 1.0, -1.0, 0.0, 0.0])
    assert orc.ppm_face(q, 0.4, hord=5) == 1.0
    assert orc.ppm_face(q, -0.4, hord=5) == -1.0
    # an isolated spike: its neighbours are not strict extrema, no filter
    q = np.array([0.0, 0.0, 1.0, 0.0, 0.0, 0.0])
    assert orc.ppm_face(q, 0.4, hord=5) == orc.ppm_face(q, 0.4, hord=6)
    assert orc.ppm_face(q, 0.4, hord=5) != 1.0


def test_2dx_smooth_equals_unlimited(orc):
    """Twelve cells per wavelength: extrema are single cells, never adjacent,
    so every face equals the unlimited one (the same arithmetic, bit for bit),
    and quadratics keep their exact swept means."""
    q = np.sin(np.arange(24) * 2 * np.pi / 12) + 0.3 * np.cos(np.arange(24) * 2 * np.pi / 8)
    for c in (0.45, -0.7):
        for m in range(24):
            w = np.array([q[(m + s - 3) % 24] for s in range(6)])
            assert orc.ppm_face(w, c, hord=5) == orc.ppm_face(w, c, hord=6)
    a, b, c2 = 0.4, -0.3, 0.05
    qq = np.array([_quad_cells(a, b, c2, s) for s in range(6)])
    assert abs(orc.ppm_face(qq, 0.3, hord=5) - _quad_swept(a, b, c2, 2.2, 2.5)) <= 1e-14


def test_2dx_conserves(orc):
    rng = np.random.default_rng(31)
    for _ in range(20):
        q = rng.random(14)
        c = rng.uniform(-1, 1)
        assert abs(_update_1d_order(orc, q, c, 5).sum() - q.sum()) <= 1e-13


@pytest.mark.parametrize("axis", ["x", "y"])
def test_2dx_transport_faces(orc, axis):
    """fv_tp_2d on a grid built with hord 5: a field alternating along the
    flow axis has every face equal to its upwind cell (both sweeps filter)."""
    n = 16
    g = orc.Grid(0, n, 1, delta=1000.0, hord=5)
    N = g.N
    A = g.metric("area")[0, H, H]
    prof = np.where(np.arange(n) % 2 == 0, 0.25, 1.5)
    Q = g.field(1)
    Q[0, 0, H:H + n, H:H + n] = prof[None, :] if axis == "x" else prof[:, None]
    orc.halo_fill(g, Q)
    zero = np.zeros((N, N))
    for c in (0.6, -0.35):
        cr = np.full((N, N), c)
        if axis == "x":
            FX, _ = orc.fv_tp_2d(g, 0, Q[0, 0], cr, zero, cr * A, zero)
            face = FX[H + 5, H:H + n + 1] / (c * A)
        else:
            _, FY = orc.fv_tp_2d(g, 0, Q[0, 0], zero, cr, zero, cr * A)
            face = FY[H:H + n + 1, H + 5] / (c * A)
        up = np.array([prof[(m - 1) % n] if c > 0 else prof[m % n] for m in range(n + 1)])
        np.testing.assert_allclose(face, up, rtol=1e-14, atol=0)


def _winds_along_x(fi, n, u1):
    """D-grid u varying along x only, v = 0: zero circulation around every cell."""
    init = fi.periodic_state(n=n, nz=1, seed=4)
    init["u"][0, 0, H:H + n + 1, H:H + n] = u1[None, :]
    init["v"][0, 0, H:H + n, H:H + n + 1] = 0.0
    return init


def test_2dx_order_in_kinetic_energy(orc):
    """Irrotational D-grid winds along x (no vorticity flux): a wind
    alternating every cell about a mean changes the momentum update between
    hord 5 and 6 (through the kinetic-energy faces alone); a smooth one leaves
    it bit for bit equal."""
    import fv3_inputs as fi
    n = 16
    x = np.arange(n)
    for u1, differ in ((10.0 + 2.0 * (-1.0) ** x, True),
                       (10.0 + 3.0 * np.sin(x * 2 * np.pi / n) + np.cos(x * 4 * np.pi / n), False)):
        init = _winds_along_x(fi, n, u1)
        out = {}
        for hord in (5, 6):
            g = orc.Grid(0, n, 1, delta=1000.0, hord=hord)
            s = orc.new_state(g, init)
            assert orc.acoustic_substeps(g, s, 2.0, 1, stop_stage=6) == 0
            out[hord] = s["u"]
        d = np.abs(out[5] - out[6]).max()
        assert (d > 1e-6 * np.abs(u1).max()) if differ else (d == 0.0), (differ, d)


# ---- the positive-definite tracer order (hord 7) ------------------------

def _pd_data(rng, n):
    q = np.where(rng.random(n) > 0.6, rng.random(n) * 5.0, 0.0)
    q[rng.integers(n)] = 0.0
    return q


def test_pd_update_non_negative(orc):
    """For non-negative data every scaled parabola is non-negative with the
    cell's mean, so each swept part carries at most the cell's content and the
    1-D update stays non-negative for |c| <= 1; the unlimited order on the same
    data goes negative."""
    rng = np.random.default_rng(41)
    neg6 = 0
    for _ in range(300):
        q = _pd_data(rng, 12)
        c = rng.uniform(-1, 1)
        q7 = _update_1d_order(orc, q, c, 7)
        assert q7.min() >= -1e-15, (q, c, q7.min())
        assert abs(q7.sum() - q.sum()) <= 1e-13
        neg6 += _update_1d_order(orc, q, c, 6).min() < -1e-3
    assert neg6 > 50


def test_pd_scaling_closed_form(orc):
    """A small cell next to a large one: the unlimited parabola dips below
    zero.  Its minimum from a dense sampling of that parabola (edges by
    7/12, -1/12 interpolation), theta = q / (q - min), and the swept mean of
    the scaled parabola integrated exactly."""
    q = np.array([0.0, 5.0, 0.1, 0.0, 0.0, 0.0])
    e = lambda k: 7 / 12 * (q[k - 1] + q[k]) - 1 / 12 * (q[k - 2] + q[k + 1])
    aL, aR, m = e(2), e(3), q[2]
    a6 = 6 * m - 3 * (aL + aR)
    P = lambda x: aL + x * (aR - aL + a6 * (1 - x))
    xs = np.linspace(0, 1, 200001)
    mn = P(xs).min()
    assert mn < 0
    th = m / (m - mn)
    c = 0.35
    # mean of m + th (P - m) over x in [1 - c, 1]
    Pint = lambda x: aL * x + (aR - aL + a6) * x * x / 2 - a6 * x ** 3 / 3
    want = m + th * ((Pint(1.0) - Pint(1 - c)) / c - m)
    assert abs(orc.ppm_face(q, c, hord=7) - want) <= 1e-9
    assert orc.ppm_face(q, c, hord=6) < 0


def test_pd_positive_parabola_unchanged(orc):
    rng = np.random.default_rng(43)
    for _ in range(100):
        q = 1.0 + rng.random(6)
        c = rng.uniform(-1, 1)
        assert orc.ppm_face(q, c, hord=7) == orc.ppm_face(q, c, hord=6)


def _uniform_tracer(orc, n, hord_tr, cx, cy):
    g = orc.Grid(0, n, 1, hord_tr=hord_tr)
    dp0 = g.field(1)
    dp0[:] = 1000.0
    A = 1000.0 * 1000.0
    CX, CY = g.field(1), g.field(1)
    CX[:] = cx
    CY[:] = cy
    return g, dp0, CX * dp0 * A, CY * dp0 * A, CX, CY


def test_pd_tracer_transport_non_negative(orc):
    """Tracer transport with hord_tr 7 under uniform flow (the 2-D result is
    the mean of the two orderings of 1-D updates, each non-negative) keeps a
    sparse non-negative field non-negative over 20 steps and conserves its
    sum; with hord_tr 6 the same run goes negative."""
    n = 16
    rng = np.random.default_rng(44)
    q0 = np.where(rng.random((n, n)) > 0.7, rng.random((n, n)) * 3.0, 0.0)
    mins = {}
    for hord_tr in (7, 6):
        g, dp0, mfx, mfy, cx, cy = _uniform_tracer(orc, n, hord_tr, 0.55, -0.3)
        q = g.field(1)
        q[0, 0, H:H + n, H:H + n] = q0
        lo = np.inf
        for _ in range(20):
            orc.tracer_transport(g, [q], dp0, mfx, mfy, cx, cy)
            lo = min(lo, q[0, 0, H:H + n, H:H + n].min())
        mins[hord_tr] = lo
        assert abs(q[0, 0, H:H + n, H:H + n].sum() - q0.sum()) <= 1e-12 * q0.sum()
    assert mins[7] >= -1e-15, mins
    assert mins[6] < -1e-3, mins


def test_pd_only_in_tracer_transport(orc):
    """hord_tr changes the tracer transport only: the substep is bit-equal
    under hord_tr 7 and 0, and hord 7 is rejected for the substep."""
    import fv3_inputs as fi
    init = fi.periodic_state(n=16, nz=2, seed=4)
    out = []
    for hord_tr in (0, 7):
        g = orc.Grid(0, 16, 2, hord_tr=hord_tr)
        s = orc.new_state(g, init)
        assert orc.acoustic_substeps(g, s, 2.0, 2) == 0
        out.append(s["u"].copy())
    np.testing.assert_array_equal(out[0], out[1])
    with pytest.raises(ValueError):
        orc.Grid(0, 16, 2, hord=7)
