"""Pins of the oracle's C-grid wind update in c_sw (the half-step of the C-D
grid method, Sec. II; the D-grid winds are interpolated to the C grid, then
advanced over dt/2 by the vorticity flux and the kinetic-energy gradient).

Each pin compares with the continuous equations of motion in vector-invariant
form, du/dt = +zeta_abs v - dK/dx, dv/dt = -zeta_abs u - dK/dy, evaluated
analytically for a flow whose fields are closed-form on the doubly periodic
grid, within a bound set by the discretisation error of that flow (the
interpolations are fourth order, the vorticity a second-order circulation,
the kinetic energy upwinded):

* f-plane uniform flow: the change over the half step is exactly the
  Coriolis term (+f v dt/2 in uc, -f u dt/2 in vc);
* a shear flow u(y) crossed by a uniform v (and the transposed case): the
  change of uc is the relative-vorticity flux with the vorticity taken at
  the corner upwind of the crossing wind; the downwind corner is off by a
  whole grid step of the vorticity gradient;
* a one-dimensional flow u(x), v = 0: the change of uc is minus the
  gradient of the kinetic energy;
* circulation (P8): the corner vorticity of c_sw and the cell vorticity of
  d_sw integrate over a periodic tile to the integral of f exactly.
"""
import math

import numpy as np
import pytest

import fv3_inputs as fi

H = 3
N = 48
DX = 1000.0
BDT = 10.0          # dt2 = 5 s: large increments next to the interpolation error
DT2 = 0.5 * BDT
K = 2.0 * math.pi / (N * DX)


def _run(orc, u_fn, v_fn, f0=0.0, nz=1):
    """One half step of c_sw (stop after it) from D-grid winds u(x, y),
    v(x, y) given at their own positions; returns the C-grid winds on the
    interior faces and the debug fields."""
    init = fi.periodic_state(n=N, nz=nz, wind=0.0, nq=0)
    i = np.arange(N + 1)
    # D-grid u on y-faces (i, j - 1/2): x = (i + 1/2) dx, y = j dx
    xu, yu = np.meshgrid((i + 0.5) * DX, i * DX)
    # D-grid v on x-faces (i - 1/2, j): x = i dx, y = (j + 1/2) dx
    xv, yv = np.meshgrid(i * DX, (i + 0.5) * DX)
    for k in range(nz):
        init["u"][0, k, H:H + N + 1, H:H + N + 1] = u_fn(xu, yu)
        init["v"][0, k, H:H + N + 1, H:H + N + 1] = v_fn(xv, yv)
    g = orc.Grid(0, N, nz, delta=DX, f0=f0)
    s = orc.new_state(g, init)
    st, dbg = orc.acoustic_substeps(g, s, BDT, 1, stop_stage=2, debug=True)
    assert st == 0
    uc = s["uc"][0, :, H:H + N, H:H + N + 1]        # x-faces i = 0..n, rows 0..n-1
    vc = s["vc"][0, :, H:H + N + 1, H:H + N]        # y-faces j = 0..n, cols 0..n-1
    return g, uc, vc, dbg


def _cpos():
    """Positions of the C-grid faces: uc at (i dx, (j + 1/2) dx), vc at
    ((i + 1/2) dx, j dx)."""
    i = np.arange(N + 1)
    j = np.arange(N)
    xuc, yuc = np.meshgrid(i * DX, (j + 0.5) * DX)
    xvc, yvc = np.meshgrid((j + 0.5) * DX, i * DX)
    return xuc, yuc, xvc, yvc


@pytest.mark.parametrize("U,V", [(10.0, 5.0), (-7.0, 12.0), (3.0, -9.0)])
def test_fplane_uniform_flow_coriolis(orc, U, V):
    """Uniform winds on an f-plane: no relative vorticity, no kinetic-energy
    gradient, so the half-step change is the Coriolis acceleration alone,
    +f0 V dt/2 in uc and -f0 U dt/2 in vc (interpolations are exact on a
    constant)."""
    f0 = 1.0e-4
    _, uc, vc, _ = _run(orc, lambda x, y: U + 0 * x, lambda x, y: V + 0 * x, f0=f0)
    du, dv = uc - U, vc - V
    np.testing.assert_allclose(du, f0 * V * DT2, rtol=1e-10, atol=0)
    np.testing.assert_allclose(dv, -f0 * U * DT2, rtol=1e-10, atol=0)


@pytest.mark.parametrize("V", [8.0, -8.0])
def test_shear_flow_upwind_vorticity_flux_in_uc(orc, V):
    """u = U0 + A sin(k y), v = V: relative vorticity zeta = -A k cos(k y).
    The change of uc at a face is V zeta dt/2 with zeta at the corner on the
    upwind side of V (lower corner for V > 0, upper for V < 0); the kinetic
    energy does not vary along x.  Bound: interpolation and circulation
    error of this flow, far below the one-grid-step shift of the corner."""
    U0, A = 4.0, 6.0
    _, uc, _, _ = _run(orc, lambda x, y: U0 + A * np.sin(K * y), lambda x, y: V + 0 * x)
    _, yuc, _, _ = _cpos()
    y_up = yuc - 0.5 * DX if V > 0 else yuc + 0.5 * DX
    zeta = -A * K * np.cos(K * y_up)
    expect = U0 + A * np.sin(K * yuc) + DT2 * V * zeta
    incr = np.abs(DT2 * V * zeta).max()
    err = np.abs(uc[0] - expect).max()
    # the downwind corner would be off by dt2 |V| A k^2 dx ~ 13 % of the increment
    assert err < 0.02 * incr, (err, incr)


@pytest.mark.parametrize("U", [8.0, -8.0])
def test_shear_flow_upwind_vorticity_flux_in_vc(orc, U):
    """Transposed case: v = V0 + B sin(k x), u = U: zeta = B k cos(k x); the
    change of vc is -U zeta dt/2 with zeta on the upwind corner of U."""
    V0, B = 4.0, 6.0
    _, _, vc, _ = _run(orc, lambda x, y: U + 0 * x, lambda x, y: V0 + B * np.sin(K * x))
    _, _, xvc, _ = _cpos()
    x_up = xvc - 0.5 * DX if U > 0 else xvc + 0.5 * DX
    zeta = B * K * np.cos(K * x_up)
    expect = V0 + B * np.sin(K * xvc) - DT2 * U * zeta
    incr = np.abs(DT2 * U * zeta).max()
    err = np.abs(vc[0] - expect).max()
    assert err < 0.02 * incr, (err, incr)


def test_one_dimensional_flow_kinetic_energy_gradient(orc):
    """u = U0 + A sin(k x), v = 0: no vorticity, so uc changes by
    -dt/2 d(u^2/2)/dx = -dt/2 u u'.  Bound: the upwinded kinetic energy is
    first-order accurate (a quarter-cell shift), about k dx / 4 of the term."""
    U0, A = 12.0, 5.0
    _, uc, vc, _ = _run(orc, lambda x, y: U0 + A * np.sin(K * x), lambda x, y: 0 * x)
    xuc, _, _, _ = _cpos()
    u = U0 + A * np.sin(K * xuc)
    expect = u - DT2 * u * A * K * np.cos(K * xuc)
    incr = np.abs(DT2 * u * A * K * np.cos(K * xuc)).max()
    err = np.abs(uc[0] - expect).max()
    assert err < 0.1 * incr, (err, incr)
    # v stays zero: nothing drives it
    assert np.abs(vc).max() == 0.0


def test_one_dimensional_flow_kinetic_energy_gradient_in_vc(orc):
    """v = V0 + B sin(k y), u = 0: vc changes by -dt/2 v v'."""
    V0, B = 12.0, 5.0
    _, uc, vc, _ = _run(orc, lambda x, y: 0 * x, lambda x, y: V0 + B * np.sin(K * y))
    _, _, _, yvc = _cpos()
    v = V0 + B * np.sin(K * yvc)
    expect = v - DT2 * v * B * K * np.cos(K * yvc)
    incr = np.abs(DT2 * v * B * K * np.cos(K * yvc)).max()
    err = np.abs(vc[0] - expect).max()
    assert err < 0.1 * incr, (err, incr)
    assert np.abs(uc).max() == 0.0


def test_vorticity_integrates_to_coriolis_on_periodic_tile(orc):
    """P8: on a doubly periodic tile the circulation terms telescope, so the
    area integral of the absolute vorticity equals the integral of f, for
    c_sw's corner vorticity (C-grid circulation) and for d_sw's cell
    vorticity (D-grid circulation), on a noisy flow."""
    f0 = 1.0e-4
    init = fi.periodic_state(n=N, nz=3, seed=7)
    g = orc.Grid(0, N, 3, delta=DX, f0=f0)
    s = orc.new_state(g, init)
    st, dbg = orc.acoustic_substeps(g, s, 2.0, 1, stop_stage=6, debug=True)
    assert st == 0
    area_c = g.metric("area_c")[0, H:H + N, H:H + N]    # corners 0..n-1 (n repeats 0)
    area = g.metric("area")[0, H:H + N, H:H + N]
    for k in range(3):
        vc_ = dbg["vortc"][0, k, H:H + N, H:H + N]
        vd_ = dbg["vortd"][0, k, H:H + N, H:H + N]
        # the flow has vorticity: the check is not vacuous
        assert np.abs(vc_ - f0).max() > 10 * f0
        assert np.abs(vd_ - f0).max() > 10 * f0
        ref_c = f0 * area_c.sum()
        ref_d = f0 * area.sum()
        assert abs((vc_ * area_c).sum() - ref_c) <= 1e-11 * ref_c
        assert abs((vd_ * area).sum() - ref_d) <= 1e-11 * ref_d


@pytest.mark.parametrize("comp", ["u", "v"])
def test_linear_flow_upwinded_kinetic_energy_closed_form(orc, comp):
    """A flow linear in x (sawtooth over the period), u = U0 + a (x - L/2) > 0,
    v = 0: away from the jump every four-point interpolation is exact (it is
    exact for cubics), so the centre kinetic energy upwinded with u > 0 is
    K_i = u(x_i) u(x_i - dx/2) / 2, a quadratic in x whose centred difference
    is exact: the change of uc at x is -dt/2 (a u(x) - a^2 dx / 4).  Taking
    the downwind face instead flips the a^2 dx / 4 term (1.7 % of the
    change).  The transposed flow pins vc the same way."""
    U0, a = 30.0, 1.0e-3
    L = N * DX

    def saw(s):
        return U0 + a * (np.mod(s, L) - 0.5 * L)

    xuc, yuc, xvc, yvc = _cpos()
    if comp == "u":
        _, uc, _, _ = _run(orc, lambda x, y: saw(x), lambda x, y: 0 * x)
        pos, got = xuc, uc[0]
    else:
        _, _, vc, _ = _run(orc, lambda x, y: 0 * x, lambda x, y: saw(y))
        pos, got = yvc, vc[0]
    far = (pos >= 5 * DX) & (pos <= L - 5 * DX)
    w = saw(pos)
    expect = w - DT2 * (a * w - a * a * DX / 4.0)
    incr = DT2 * a * np.abs(w[far]).max()
    err = np.abs(got - expect)[far].max()
    assert err < 1e-9 * incr + 1e-12 * U0, (err, incr)


def test_potential_flows_have_no_vorticity_on_the_cube(orc):
    """The circulation weights on the cube's uneven metrics.  C-grid winds
    that are differences of any cell-centred potential over the
    centre-to-centre lengths (uc = (phi_E - phi_W) / dxc, vc = (phi_N -
    phi_S) / dyc) have zero circulation around every dual cell, so c_sw's
    corner vorticity is exactly f at every corner off the cube vertices;
    D-grid winds that are differences of any corner potential over the edge
    lengths (u = (phi_E - phi_W) / dx, v = (phi_N - phi_S) / dy) leave d_sw's
    cell vorticity exactly f in every cell.  An index or weight slip in
    either circulation breaks the telescoping sum."""
    import fv3_inputs as fi

    n, nz = 12, 1
    g = orc.Grid(1, n, nz)
    T, N = 6, n + 2 * H + 1
    rng = np.random.default_rng(23)
    dxc, dyc, dx, dy = g.metric("dxc"), g.metric("dyc"), g.metric("dx"), g.metric("dy")
    fB, fC = g.metric("fB"), g.metric("fC")
    # C-grid: cell potential on cells -1..n
    phi = rng.normal(size=(T, N, N)) * 1e6
    uc = np.zeros((T, N, N))
    vc = np.zeros((T, N, N))
    for j in range(-1, n + 1):
        for i in range(0, n + 1):
            uc[:, j + H, i + H] = (phi[:, j + H, i + H] - phi[:, j + H, i - 1 + H]) / dxc[:, j + H, i + H]
    for j in range(0, n + 1):
        for i in range(-1, n + 1):
            vc[:, j + H, i + H] = (phi[:, j + H, i + H] - phi[:, j - 1 + H, i + H]) / dyc[:, j + H, i + H]
    vort = orc.corner_vorticity(g, uc, vc)
    scale = np.abs(uc).max() * dxc[:, H:H + n, H:H + n].max() / g.metric("area_c")[:, H:H + n, H:H + n].min()
    for t in range(T):
        for j in range(0, n + 1):
            for i in range(0, n + 1):
                if (i in (0, n)) and (j in (0, n)):
                    continue
                assert abs(vort[t, j + H, i + H] - fB[t, j + H, i + H]) <= 1e-12 * scale, (t, i, j)
    # D-grid: corner potential on corners 0..n, winds on the tile's faces;
    # the substep's halo fill supplies the rest, d_sw's vorticity is read back
    init = fi.cube_state(n=n, nz=nz)
    psi = rng.normal(size=(T, N, N)) * 1e6
    u = np.zeros_like(init["u"])
    v = np.zeros_like(init["v"])
    for j in range(0, n + 1):
        for i in range(0, n):
            u[:, 0, j + H, i + H] = (psi[:, j + H, i + 1 + H] - psi[:, j + H, i + H]) / dx[:, j + H, i + H]
    for j in range(0, n):
        for i in range(0, n + 1):
            v[:, 0, j + H, i + H] = (psi[:, j + 1 + H, i + H] - psi[:, j + H, i + H]) / dy[:, j + H, i + H]
    init["u"], init["v"] = u, v
    s = orc.new_state(g, init)
    st, dbg = orc.acoustic_substeps(g, s, 1.0, 1, stop_stage=6, debug=True)
    om = dbg["vortd"][:, 0, H:H + n, H:H + n]
    scale = np.abs(u).max() * dx.max() / g.metric("area")[:, H:H + n, H:H + n].min()
    assert np.abs(om - fC[:, H:H + n, H:H + n]).max() <= 1e-12 * scale
    # the same winds with the metric weights taken one face off are not
    # irrotational: the pin sees the weights
    uc2 = uc.copy()
    uc2[:, H:H + n, H + 1:H + n] *= dxc[:, H:H + n, H + 1:H + n] / dxc[:, H:H + n, H:H + n - 1]
    vort2 = orc.corner_vorticity(g, uc2, vc)
    assert np.abs(vort2 - fB)[:, H + 1:H + n, H + 1:H + n].max() > 1e-6 * scale
