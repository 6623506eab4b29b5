"""Pins of the oracle's higher-order divergence damping (nord 1: del-4,
nord 2: del-6, coefficient nu = (d4_bg da_min)^(nord+1)): the corner
divergence with nord corner Laplacians applied enters the kinetic energy with
sign (-1)^(nord+1), so the divergence obeys dD/dt = (-1)^nord nu Lap^(nord+1) D.

Pins: the closed-form decay of a divergent Fourier mode for nord 1 and 2
(the 1-D corner Laplacian's eigenvalue -(4/dx^2) sin^2(pi/n) raised to
nord + 1); a streamfunction flow is untouched; on the cube the corner
Laplacian of a constant is 0 at every corner (cube vertices included), and
for corner fields that are divergences of winds (so the two tiles of a shared
edge agree) the Laplacian sums to 0 over the sphere and is self-adjoint
(weights: dual areas, each shared corner counted once)."""
import numpy as np
import pytest

import fv3_inputs as fi

H = 3


def _pure_wind_state(n, nz, u_cells, v_cells):
    st = fi.periodic_state(n=n, nz=nz, seed=3, wind=0.0)
    st["u"][:] = 0.0
    st["v"][:] = 0.0
    st["u"][0, :, H:H + n, H:H + n] = u_cells
    st["u"][0, :, H + n, H:H + n] = u_cells[:, 0, :]
    st["v"][0, :, H:H + n, H:H + n] = v_cells
    st["v"][0, :, H:H + n, H + n] = v_cells[:, :, 0]
    return st


def _one(orc, st, n, nz, nord, d4, dt=0.2):
    g = orc.Grid(0, n, nz, nord=nord, d4_bg=d4)
    s = orc.new_state(g, st)
    assert orc.acoustic_substeps(g, s, dt, 1) == 0
    return s


@pytest.mark.parametrize("nord,d4", [(1, 0.15), (2, 0.12)])
def test_higher_order_damping_closed_form(orc, nord, d4):
    """u = a cos(2 pi (i + 1/2) / n), v = 0: the damping changes u by
    -(4 d4 sin^2(pi/n))^(nord+1) u (da_min = dx^2 on the periodic grid)."""
    n, nz = 16, 2
    i = np.arange(n)
    ucol = np.cos(2 * np.pi * (i + 0.5) / n)
    u = np.broadcast_to(ucol, (nz, n, n)).copy()
    st = _pure_wind_state(n, nz, u, np.zeros((nz, n, n)))
    a = _one(orc, st, n, nz, 0, 0.0)
    b = _one(orc, st, n, nz, nord, d4)
    du = (b["u"] - a["u"])[0, :, H:H + n, H:H + n]
    want = -((4 * d4) * np.sin(np.pi / n) ** 2) ** (nord + 1) * u
    np.testing.assert_allclose(du, want, rtol=0, atol=1e-13)
    np.testing.assert_allclose((b["v"] - a["v"])[0, :, H:H + n, H:H + n], 0.0, atol=1e-13)
    # the shortest resolved mode is damped hardest: (2 dx) wave, sin^2 = 1
    ucol = np.cos(np.pi * (i + 0.5))
    st = _pure_wind_state(n, nz, np.broadcast_to(ucol, (nz, n, n)).copy(), np.zeros((nz, n, n)))
    du = (_one(orc, st, n, nz, nord, d4)["u"] - _one(orc, st, n, nz, 0, 0.0)["u"])[0, :, H:H + n, H:H + n]
    np.testing.assert_allclose(du, -(4 * d4) ** (nord + 1) * np.broadcast_to(ucol, (nz, n, n)), rtol=0,
                               atol=1e-12)


@pytest.mark.parametrize("nord", [1, 2])
def test_higher_order_damping_leaves_rotational_flow(orc, nord):
    n, nz = 16, 2
    rng = np.random.default_rng(19)
    psi = rng.standard_normal((nz, n, n)) * 1000.0
    dx = 1000.0
    u = -(psi - np.roll(psi, 1, axis=1)) / dx
    v = (psi - np.roll(psi, 1, axis=2)) / dx
    st = _pure_wind_state(n, nz, u, v)
    a = _one(orc, st, n, nz, 0, 0.0)
    b = _one(orc, st, n, nz, nord, 0.2)
    scale = np.abs(a["u"]).max()
    assert np.abs(b["u"] - a["u"]).max() <= 1e-12 * scale
    assert np.abs(b["v"] - a["v"]).max() <= 1e-12 * scale


def _cube_divergence(orc, n, nz, seed):
    """Corner divergence of smooth winds: the jet plus 60 seeded bumps (some
    near every cube vertex) without noise, so that the wind on a face shared by two tiles (stored by both) is
    the same in each, and so is the divergence of a shared corner."""
    g = orc.Grid(1, n, nz, delta=1.0e5)
    init = fi.cube_state(n=n, nz=nz, seed=seed, noise=0.0, bumps=60)
    U, V = init["u"].copy(), init["v"].copy()
    orc.halo_fill_pair(g, U, "Y", V, "X")
    return g, orc.corner_div(g, U, V)


def _phys_weights(n):
    w = np.ones((n + 1, n + 1))
    w[0, :] = w[n, :] = w[:, 0] = w[:, n] = 0.5
    for a in (0, n):
        for b in (0, n):
            w[a, b] = 1.0 / 3.0
    return w


def test_corner_laplacian_of_constant_is_zero(orc):
    n, nz = 10, 1
    g = orc.Grid(1, n, nz, delta=1.0e5)
    D = g.field(nz)
    D[:, :, H:H + n + 1, H:H + n + 1] = 3.7
    L, _ = orc.corner_lap(g, D)
    assert np.abs(L[:, :, H:H + n + 1, H:H + n + 1]).max() <= 1e-20


def test_corner_laplacian_conserves_and_is_self_adjoint(orc):
    n, nz = 10, 1
    g, D = _cube_divergence(orc, n, nz, 4)
    _, E = _cube_divergence(orc, n, nz, 5)
    ac = g.metric("area_c")[:, H:H + n + 1, H:H + n + 1]
    wts = _phys_weights(n)[None] * ac
    LD, D = orc.corner_lap(g, D)
    LE, E = orc.corner_lap(g, E)
    sl = (slice(None), 0, slice(H, H + n + 1), slice(H, H + n + 1))
    assert np.abs(D[sl] - E[sl]).max() > 0.1 * np.abs(D[sl]).max()
    # the cube vertices take part (their divergence is not zero)
    vert = [abs(D[t, 0, H + a, H + b]) for t in range(6) for a in (0, n) for b in (0, n)]
    assert np.median(vert) > 1e-3 * np.abs(D[sl]).max()
    scale = np.abs(LD[sl]).max()
    total = float((wts * LD[sl]).sum())
    assert abs(total) <= 1e-11 * scale * wts.sum(), total
    a = float((wts * E[sl] * LD[sl]).sum())
    b = float((wts * LE[sl] * D[sl]).sum())
    assert abs(a - b) <= 1e-10 * max(abs(a), abs(b)), (a, b)
    assert abs(a) > 0


# ---- del-2 vorticity damping (vtdm) -------------------------------------

def _one_v(orc, st, n, nz, vtdm, dt=0.2):
    g = orc.Grid(0, n, nz, vtdm=vtdm)
    s = orc.new_state(g, st)
    assert orc.acoustic_substeps(g, s, dt, 1) == 0
    return s


@pytest.mark.parametrize("m", [1, 4, 8])
@pytest.mark.parametrize("axis", ["x", "y"])
def test_vorticity_damping_closed_form(orc, m, axis):
    """A purely rotational mode, v = cos(2 pi m i / n) on x-faces (or
    u = cos(2 pi m j / n) on y-faces), the other wind 0: its vorticity is a
    Fourier mode of the 1-D cell Laplacian, and the damping changes that wind
    by -4 vtdm sin^2(pi m / n) times itself (del-2 diffusion of the vorticity;
    nu_v = vtdm dx^2), the other wind not at all."""
    n, nz, vt = 16, 2, 0.1
    i = np.arange(n)
    col = np.cos(2 * np.pi * m * i / n)
    z = np.zeros((nz, n, n))
    if axis == "x":
        w = np.broadcast_to(col, (nz, n, n)).copy()
        st = _pure_wind_state(n, nz, z, w)
        k, o = "v", "u"
    else:
        w = np.broadcast_to(col[:, None], (nz, n, n)).copy()
        st = _pure_wind_state(n, nz, w, z)
        k, o = "u", "v"
    a = _one_v(orc, st, n, nz, 0.0)
    b = _one_v(orc, st, n, nz, vt)
    d = (b[k] - a[k])[0, :, H:H + n, H:H + n]
    want = -(4 * vt) * np.sin(np.pi * m / n) ** 2 * w
    np.testing.assert_allclose(d, want, rtol=0, atol=1e-13)
    np.testing.assert_allclose((b[o] - a[o])[0, :, H:H + n, H:H + n], 0.0, atol=1e-13)


def test_vorticity_damping_on_the_cube(orc):
    """On the cube (uneven metrics) the change of the D-grid winds in the
    momentum update is the diffusive vorticity flux alone: for v on x-face
    (i, j), -nu_v (w(i-1, j) - w(i, j)) / dxc, for u on y-face (i, j),
    nu_v (w(i, j-1) - w(i, j)) / dyc, w the relative vorticity (circulation
    of the halo-filled winds over the cell area)."""
    n, nz, vt = 10, 2, 0.15
    st = fi.cube_state(n=n, nz=nz, seed=8)
    g0 = orc.Grid(1, n, nz, delta=1.0e5)
    g1 = orc.Grid(1, n, nz, delta=1.0e5, vtdm=vt)
    out = []
    for g in (g0, g1):
        s = orc.new_state(g, st)
        assert orc.acoustic_substeps(g, s, 300.0, 1, stop_stage=6) == 0
        out.append(s)
    U, V = st["u"].copy(), st["v"].copy()
    orc.halo_fill_pair(g0, U, "Y", V, "X")
    dx, dy, dxc, dyc = (g0.metric(k) for k in ("dx", "dy", "dxc", "dyc"))
    area = g0.metric("area")
    nuv = vt * g0.metric("area_c")[:, H:H + n + 1, H:H + n + 1].min()
    c = slice(H - 1, H + n)
    w = np.zeros_like(U)
    e = slice(H, H + n + 1)
    with np.errstate(divide="ignore", invalid="ignore"):   # the cube-corner halo cells have no area
        w[:, :, c, c] = (U[:, :, c, c] * dx[:, None, c, c] - U[:, :, e, c] * dx[:, None, e, c] -
                         V[:, :, c, c] * dy[:, None, c, c] + V[:, :, c, e] * dy[:, None, c, e]) / area[:, None, c, c]
    I = slice(H, H + n)
    dv = (out[1]["v"] - out[0]["v"])[:, :, I, I]
    want_v = -nuv * (w[:, :, I, H - 1:H + n - 1] - w[:, :, I, I]) / dxc[:, None, I, I]
    du = (out[1]["u"] - out[0]["u"])[:, :, I, I]
    want_u = nuv * (w[:, :, H - 1:H + n - 1, I] - w[:, :, I, I]) / dyc[:, None, I, I]
    scale = max(np.abs(want_v).max(), np.abs(want_u).max())
    assert scale > 1e-6
    assert np.abs(dv - want_v).max() <= 1e-8 * scale
    assert np.abs(du - want_u).max() <= 1e-8 * scale


def test_vorticity_damping_leaves_divergent_flow(orc):
    """D-grid winds that are differences of a corner potential have zero
    relative vorticity in every cell: the damping changes nothing."""
    n, nz = 16, 2
    rng = np.random.default_rng(29)
    chi = rng.standard_normal((nz, n, n)) * 1000.0          # potential at corners
    dx = 1000.0
    u = (np.roll(chi, -1, axis=2) - chi) / dx               # y-face (i, j): corners (i, j), (i+1, j)
    v = (np.roll(chi, -1, axis=1) - chi) / dx               # x-face (i, j): corners (i, j), (i, j+1)
    st = _pure_wind_state(n, nz, u, v)
    a = _one_v(orc, st, n, nz, 0.0)
    b = _one_v(orc, st, n, nz, 0.2)
    scale = np.abs(a["u"]).max()
    assert np.abs(b["u"] - a["u"]).max() <= 1e-12 * scale
    assert np.abs(b["v"] - a["v"]).max() <= 1e-12 * scale


def test_vorticity_damping_ignores_coriolis(orc):
    """On the cube f varies (its Laplacian is not zero): D-grid winds at rest
    have zero relative vorticity, so the momentum update with the damping
    equals the one without bit for bit (stage 6), which would not hold if the
    absolute vorticity were diffused."""
    n, nz = 10, 3
    st = fi.cube_state(n=n, nz=nz, noise=0.0)
    st["u"][:] = 0.0
    st["v"][:] = 0.0
    out = []
    for vt in (0.0, 0.2):
        g = orc.Grid(1, n, nz, delta=1.0e5, vtdm=vt)
        s = orc.new_state(g, st)
        assert orc.acoustic_substeps(g, s, 300.0, 1, stop_stage=6) == 0
        out.append((s["u"].copy(), s["v"].copy()))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
