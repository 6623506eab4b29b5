"""Pins of the oracle's Smagorinsky-scaled divergence damping (the damping
family of d_sw; the paper's Smagorinsky kernel, Sec. VII-C, computes
dt sqrt(DT^2 + DS^2) from the tension DT and the shear DS): the magnitude
vanishes for uniform flow and solid-body rotation and equals the closed
forms for a linear shear and a pure strain (finite-volume differences are
exact for linear winds on the uniform periodic grid); the coefficient is
capped at 0.2 and never below d2_bg (checked by whole-substep equalities)."""
import numpy as np
import pytest

import fv3_inputs as fi
import oracle as orc

H = 3


def _winds(g, fu, fv):
    """D-grid u on y-faces (x = (i + 1/2) d, y = j d) and v on x-faces
    (x = i d, y = (j + 1/2) d) of a periodic grid of spacing d, halos included."""
    N, d = g.N, 1000.0
    I, J = np.meshgrid(np.arange(N) - H, np.arange(N) - H)
    u = fu((I + 0.5) * d, J * d)
    v = fv(I * d, (J + 0.5) * d)
    return u.astype(np.float64), v.astype(np.float64)


def _inner(g, a):
    # corners whose dual cell and four cells use only non-wrapped halo points
    return a[H + 2:H + g.n - 1, H + 2:H + g.n - 1]


@pytest.mark.parametrize("case", ["uniform", "rotation"])
def test_no_deformation(orc, case):
    g = orc.Grid(0, 16, 1)
    if case == "uniform":
        u, v = _winds(g, lambda x, y: 7.0 + 0 * x, lambda x, y: -3.0 + 0 * x)
    else:
        om = 1e-4
        u, v = _winds(g, lambda x, y: -om * y, lambda x, y: om * x)
    s = orc.smag_corner(g, 0, u, v, 15.0)
    assert np.abs(_inner(g, s)).max() <= 1e-15


def test_linear_shear_closed_form(orc):
    alpha, dt = 2e-4, 15.0
    g = orc.Grid(0, 16, 1)
    u, v = _winds(g, lambda x, y: alpha * y, lambda x, y: 0 * x)
    s = _inner(g, orc.smag_corner(g, 0, u, v, dt))
    assert np.abs(s - dt * alpha).max() <= 1e-12 * dt * alpha


def test_pure_strain_closed_form(orc):
    alpha, dt = 3e-4, 10.0
    g = orc.Grid(0, 16, 1)
    u, v = _winds(g, lambda x, y: alpha * x, lambda x, y: -alpha * y)
    s = _inner(g, orc.smag_corner(g, 0, u, v, dt))
    assert np.abs(s - 2 * dt * alpha).max() <= 1e-12 * dt * alpha


def test_shear_and_strain_combine_in_quadrature(orc):
    a, b, dt = 2e-4, 1e-4, 5.0
    g = orc.Grid(0, 16, 1)
    u, v = _winds(g, lambda x, y: a * y + b * x, lambda x, y: -b * y)
    s = _inner(g, orc.smag_corner(g, 0, u, v, dt))
    assert np.abs(s - dt * np.hypot(a, 2 * b)).max() <= 1e-12 * dt * a


def _sheared_state(n=24, nz=4):
    init = fi.periodic_state(n=n, nz=nz, seed=3)
    N = n + 2 * H + 1
    J = np.arange(N)[:, None] - H
    init["u"] = init["u"] + 20.0 * np.sin(2 * np.pi * J / n)[None, None, :, :] * np.ones((1, nz, 1, N))
    return init


def _run(d2_bg, dddmp, init, n=24, nz=4):
    g = orc.Grid(0, n, nz, d2_bg=d2_bg, dddmp=dddmp)
    s = orc.new_state(g, init)
    assert orc.acoustic_substeps(g, s, 4.0, 2) == 0
    return s


def test_cap_and_floor_of_the_coefficient(orc):
    init = _sheared_state()
    # a huge Smagorinsky coefficient saturates at 0.2 everywhere: the same run
    # as a constant 0.2
    a = _run(0.0, 1e6, init)
    b = _run(0.2, 0.0, init)
    for k in ("u", "v", "delp", "pt"):
        assert np.array_equal(a[k], b[k]), k
    # a vanishing one never lowers the coefficient below d2_bg
    c = _run(0.1, 1e-30, init)
    d = _run(0.1, 0.0, init)
    for k in ("u", "v", "delp", "pt"):
        assert np.array_equal(c[k], d[k]), k


def test_smagorinsky_raises_damping_where_sheared(orc):
    """With d2_bg = 0 the only damping is the Smagorinsky part: the run
    differs from the undamped one, and by more where the shear is strong."""
    init = _sheared_state()
    a = _run(0.0, 0.0, init)
    b = _run(0.0, 0.15, init)
    diff = np.abs(a["v"] - b["v"])[0, 0, H:H + 24, H:H + 24]
    assert diff.max() > 0.0
    assert np.isfinite(b["u"]).all()


def test_shear_averaged_to_the_corner(orc):
    """u = a y^2: the finite-volume shear of a cell is exact (2 a y at its
    centre) and the mean of the cells above and below a corner is 2 a y at
    the corner; one cell alone would be half a cell off."""
    a, dt, d = 1e-8, 10.0, 1000.0
    g = orc.Grid(0, 16, 1)
    u, v = _winds(g, lambda x, y: a * y * y, lambda x, y: 0 * x)
    s = orc.smag_corner(g, 0, u, v, dt)
    J = (np.arange(g.N) - H)[:, None] * np.ones((1, g.N))
    want = dt * 2 * a * np.abs(J * d)
    assert np.abs(_inner(g, s) - _inner(g, want)).max() <= 1e-12 * dt * 2 * a * 16 * d
