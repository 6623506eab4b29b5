"""Pins of the oracle's whole acoustic substep loop (the innermost loop of
Sec. II) on the doubly periodic grid and the cubed sphere.

Pins: delp mass and pt*delp conserved to 1e-14 (flux form on a periodic
domain); a hydrostatic rest state and a uniform flow are steady states; the
transposed initial state evolves into the transposed result (catches any
index or sign slip that breaks the x/y mirror structure); a compressed column
pushes air outward in both directions (signs of both pressure gradients); the
cube run stays finite with small global mass drift."""
import numpy as np
import pytest

import fv3_inputs as fi

H = 3


def _int(a, n, st="C", lev=None):
    ni = n + 1 if st in ("X", "B") else n
    nj = n + 1 if st in ("Y", "B") else n
    return a[..., H:H + nj, H:H + ni]


def test_cfg1_mass_conservation(orc):
    g = orc.Grid(0, 48, 8)
    s = orc.new_state(g, fi.periodic_state())
    m0 = orc.mass_sums(g, s["delp"], s["pt"])
    assert orc.acoustic_substeps(g, s, 2.0, 10) == 0
    m1 = orc.mass_sums(g, s["delp"], s["pt"])
    assert np.all(np.abs(m1 - m0) <= 1e-14 * np.abs(m0))
    # delp changed: the test is not vacuous
    assert np.abs(_int(s["delp"], 48) - _int(fi.periodic_state()["delp"], 48)).max() > 1e-3


def test_offcentred_substeps_conserve_mass_and_differ(orc):
    """Ten substeps with an off-centred vertical solve (beta = 0.6): delp and
    pt delp mass conserved to rounding, the run finite, and w different from
    the backward-Euler run (the weight reaches the solve)."""
    init = fi.periodic_state()
    ga, gb = orc.Grid(0, 48, 8), orc.Grid(0, 48, 8, beta=0.6)
    sa, sb = orc.new_state(ga, init), orc.new_state(gb, init)
    m0 = orc.mass_sums(gb, sb["delp"], sb["pt"])
    assert orc.acoustic_substeps(ga, sa, 2.0, 10) == 0
    assert orc.acoustic_substeps(gb, sb, 2.0, 10) == 0
    m1 = orc.mass_sums(gb, sb["delp"], sb["pt"])
    assert np.all(np.abs(m1 - m0) <= 1e-14 * np.abs(m0))
    wa, wb = _int(sa["w"], 48), _int(sb["w"], 48)
    assert np.isfinite(wb).all()
    assert np.abs(wa - wb).max() > 1e-3 * np.abs(wa).max()


def _rest(n=16, nz=6, f0=0.0):
    init = fi.periodic_state(n=n, nz=nz, wind=0.0)
    init["u"][:] = 0.0
    init["v"][:] = 0.0
    return init


@pytest.mark.parametrize("f0", [0.0, 1e-4])
def test_rest_state_is_steady(orc, f0):
    n, nz = 16, 6
    g = orc.Grid(0, n, nz, f0=f0)
    init = _rest(n, nz)
    s = orc.new_state(g, init)
    assert orc.acoustic_substeps(g, s, 20.0, 10) == 0
    for k in ("delp", "pt", "delz"):
        np.testing.assert_allclose(_int(s[k], n), _int(init[k], n), rtol=1e-13, atol=0)
    assert np.abs(_int(s["w"], n)).max() <= 1e-12
    assert np.abs(_int(s["u"], n, "Y")).max() <= 1e-12
    assert np.abs(_int(s["v"], n, "X")).max() <= 1e-12


def test_uniform_flow_is_steady(orc):
    n, nz = 16, 6
    g = orc.Grid(0, n, nz)
    init = _rest(n, nz)
    init["u"][0, :, H:H + n + 1, H:H + n] = 10.0
    init["v"][0, :, H:H + n, H:H + n + 1] = 10.0
    s = orc.new_state(g, init)
    assert orc.acoustic_substeps(g, s, 20.0, 10) == 0
    for k, st in (("u", "Y"), ("v", "X"), ("delp", "C"), ("pt", "C"), ("delz", "C")):
        np.testing.assert_allclose(_int(s[k], n, st), _int(init[k], n, st), rtol=1e-13, atol=1e-12)
    assert np.abs(_int(s["w"], n)).max() <= 1e-12
    # accumulated Courant number of 10 substeps of 2 s at 10 m/s over 1 km
    np.testing.assert_allclose(_int(s["cx"], n, "X"), 10 * 2.0 * 10.0 / 1000.0, rtol=1e-13)


def _transpose_state(init):
    out = dict(init)
    out["u"] = np.ascontiguousarray(init["v"].swapaxes(-1, -2))
    out["v"] = np.ascontiguousarray(init["u"].swapaxes(-1, -2))
    for k in ("w", "delp", "pt", "delz"):
        out[k] = np.ascontiguousarray(init[k].swapaxes(-1, -2))
    return out


def test_transpose_symmetry(orc):
    n, nz = 20, 5
    g = orc.Grid(0, n, nz)
    init = fi.periodic_state(n=n, nz=nz, seed=12, temp_noise=1.0)
    a = orc.new_state(g, init)
    b = orc.new_state(g, _transpose_state(init))
    assert orc.acoustic_substeps(g, a, 4.0, 4) == 0
    assert orc.acoustic_substeps(g, b, 4.0, 4) == 0
    pairs = (("u", "v", "Y", "X"), ("v", "u", "X", "Y"), ("w", "w", "C", "C"),
             ("delp", "delp", "C", "C"), ("pt", "pt", "C", "C"), ("delz", "delz", "C", "C"),
             ("mfx", "mfy", "X", "Y"), ("cx", "cy", "X", "Y"))
    for ka, kb, sa, sb in pairs:
        A = _int(a[ka], n, sa)
        Bt = _int(b[kb], n, sb).swapaxes(-1, -2)
        scale = np.abs(A).max()
        assert np.abs(A - Bt).max() <= 1e-12 * scale, ka


def test_compressed_column_pushes_outward(orc):
    n, nz = 16, 6
    g = orc.Grid(0, n, nz)
    init = _rest(n, nz)
    c = n // 2
    init["delz"][0, :, H + c, H + c] *= 0.995      # squeeze one column: high pressure
    s = orc.new_state(g, init)
    assert orc.acoustic_substeps(g, s, 1.0, 1) == 0
    k = nz - 1
    u = s["u"][0, k]          # D-grid u on the y-face from corner (i, j) to (i+1, j)
    # C-grid winds on the faces of the squeezed cell
    west, east = s["uc"][0, k, H + c, H + c], s["uc"][0, k, H + c, H + c + 1]
    assert west < 0 < east
    south, north = s["vc"][0, k, H + c, H + c], s["vc"][0, k, H + c + 1, H + c]
    assert south < 0 < north
    # D-grid u on the edges east and west of the cell's top corners
    assert u[H + c + 1, H + c + 1] > 0 and u[H + c + 1, H + c - 1] < 0


def test_cube_runs_finite(orc):
    n, nz = 12, 4
    g = orc.Grid(1, n, nz)
    s = orc.new_state(g, fi.cube_state(n=n, nz=nz))
    m0 = orc.mass_sums(g, s["delp"], s["pt"])
    assert orc.acoustic_substeps(g, s, 10 * 300.0, 10) == 0
    m1 = orc.mass_sums(g, s["delp"], s["pt"])
    assert np.all(np.abs(m1 / m0 - 1) < 1e-5)
    for k in ("u", "v", "w", "delp", "pt", "delz"):
        assert np.all(np.isfinite(s[k][:, :, H:H + n, H:H + n]))


def _pure_wind_state(n, nz, u_cells, v_cells):
    """Isothermal periodic columns at rest except the given D-grid winds
    u (y-faces, [nz][n][n] for rows 0..n-1) and v (x-faces, columns 0..n-1);
    the duplicate periodic faces n copy faces 0."""
    st = fi.periodic_state(n=n, nz=nz, seed=3, wind=0.0)
    st["u"][:] = 0.0
    st["v"][:] = 0.0
    st["u"][0, :, H:H + n, H:H + n] = u_cells
    st["u"][0, :, H + n, H:H + n] = u_cells[:, 0, :]
    st["v"][0, :, H:H + n, H:H + n] = v_cells
    st["v"][0, :, H:H + n, H + n] = v_cells[:, :, 0]
    return st


def _one_substep(orc, st, n, nz, d2_bg, dt=0.2):
    g = orc.Grid(0, n, nz, d2_bg=d2_bg)
    s = orc.new_state(g, st)
    assert orc.acoustic_substeps(g, s, dt, 1) == 0
    return s


def test_divergence_damping_closed_form(orc):
    """A purely divergent mode u = a cos(2 pi (i + 1/2) / n), v = 0: the damping
    changes u by nu times the discrete second difference of u over dx^2,
    i.e. by -(4 nu / dx^2) sin^2(pi / n) u (del-2 diffusion of the
    divergence; nu = d2_bg times the smallest dual-cell area = d2_bg dx^2)."""
    n, nz, d2 = 16, 2, 0.1
    i = np.arange(n)
    ucol = np.cos(2 * np.pi * (i + 0.5) / n)
    u = np.broadcast_to(ucol, (nz, n, n)).copy()
    st = _pure_wind_state(n, nz, u, np.zeros((nz, n, n)))
    a = _one_substep(orc, st, n, nz, 0.0)
    b = _one_substep(orc, st, n, nz, d2)
    du = (b["u"] - a["u"])[0, :, H:H + n, H:H + n]
    want = -(4 * d2) * np.sin(np.pi / n) ** 2 * u
    np.testing.assert_allclose(du, want, rtol=0, atol=1e-12)
    np.testing.assert_allclose((b["v"] - a["v"])[0, :, H:H + n, H:H + n], 0.0, atol=1e-13)


def test_divergence_damping_leaves_rotational_flow(orc):
    """D-grid winds from a streamfunction at cell centres have zero discrete
    divergence at every corner: the damping changes nothing beyond rounding."""
    n, nz = 16, 2
    rng = np.random.default_rng(9)
    psi = rng.standard_normal((nz, n, n)) * 1000.0          # psi [m^2/s] at cells
    dx = 1000.0
    u = -(psi - np.roll(psi, 1, axis=1)) / dx               # y-face (i, j): cells (i, j-1), (i, j)
    v = (psi - np.roll(psi, 1, axis=2)) / dx                # x-face (i, j): cells (i-1, j), (i, j)
    st = _pure_wind_state(n, nz, u, v)
    a = _one_substep(orc, st, n, nz, 0.0)
    b = _one_substep(orc, st, n, nz, 0.2)
    scale = np.abs(a["u"]).max()
    assert np.abs(b["u"] - a["u"]).max() <= 1e-12 * scale
    assert np.abs(b["v"] - a["v"]).max() <= 1e-12 * scale
