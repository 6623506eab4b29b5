"""Oracle pins of the one-sided interpolations at cube tile edges (option
edge_interp): c_sw's D -> A and A -> C point interpolations and nh_p_grad's
cell-to-corner values.

On a sweep with tile edges at the interfaces 0 and n, every stencil that
would reach across an edge uses the three nearest points on its own side
(the quadratic through them), and an interface on the edge itself takes the
mean of the two linear extrapolations from the two nearest points of each
side.  Pinned by: exactness for linear data everywhere and for quadratic data
at the one-sided positions (the straddling stencils are not exact there when
the two sides carry different data), blindness to the points across the
edge, mirror symmetry of the two ends, the closed form of the edge value for
data with a kink at the edge, bit-equality with the centred stencils away
from the edges, and on the cube: interior corner values and C-grid winds
unchanged, quadratic corner data reproduced next to the edges, the doubly
periodic grid untouched."""
import numpy as np
import pytest

import fv3_inputs as fi
import oracle as orc

H = 3
N = 12
LO, HI = -4, N + 5          # index range held in the test arrays
KINDS = ("face_pt", "cell_pt", "face_mean")


def _arr(f):
    """Values f(k) for k = LO .. HI - 1 (x[k - LO])."""
    return np.array([f(k) for k in range(LO, HI)], dtype=np.float64)


def _data(kind, poly):
    """Inputs of `kind` for the polynomial poly(x) and the exact output at
    index m: point values at interfaces (cell_pt inputs) or cell centres
    (face_pt inputs), cell means (face_mean)."""
    p = np.polynomial.Polynomial(poly)
    P = p.integ()
    if kind == "cell_pt":
        return _arr(lambda k: p(k)), lambda m: p(m + 0.5)
    if kind == "face_pt":
        return _arr(lambda k: p(k + 0.5)), lambda m: p(m)
    return _arr(lambda k: P(k + 1) - P(k)), lambda m: p(m)


def _ms(kind):
    # output positions each kind is used at (c_sw: cells -2 .. n+1 and faces
    # -1 .. n+1; corners 0 .. n)
    return range(-2, N + 2) if kind == "cell_pt" else (range(-1, N + 2) if kind == "face_pt" else range(0, N + 1))


def _one_sided(kind):
    return (-1, 0, N - 1, N) if kind == "cell_pt" else (-1, 1, N - 1, N + 1)


def _val(kind, x, m, edge):
    return orc.interp(kind, x, LO, m, N, edge)


@pytest.mark.parametrize("kind", KINDS)
def test_linear_exact_everywhere(kind):
    x, exact = _data(kind, [0.7, -1.3])
    for edge in (False, True):
        for m in _ms(kind):
            assert abs(_val(kind, x, m, edge) - exact(m)) <= 1e-13, (kind, edge, m)


@pytest.mark.parametrize("kind", KINDS)
def test_quadratic_exact_at_one_sided_positions(kind):
    x, exact = _data(kind, [0.3, -0.9, 0.45])
    for m in _one_sided(kind):
        if kind == "face_mean" and m not in range(0, N + 1):
            continue
        assert abs(_val(kind, x, m, True) - exact(m)) <= 1e-12, (kind, m)
    # the centred stencils are exact for cubics, so away from the edges both
    # settings agree bit for bit
    x3, exact3 = _data(kind, [0.3, -0.9, 0.45, 0.2])
    for m in _ms(kind):
        if m in (-1, 0, 1, N - 1, N, N + 1):
            continue
        assert _val(kind, x3, m, True) == _val(kind, x3, m, False)
        assert abs(_val(kind, x3, m, False) - exact3(m)) <= 1e-11


@pytest.mark.parametrize("kind", KINDS)
def test_blind_across_the_edge(kind):
    """A one-sided value does not see the points across its edge; the
    straddling stencil does."""
    rng = np.random.default_rng(3)
    x = rng.normal(size=HI - LO)
    for m in _one_sided(kind):
        if kind == "face_mean" and m not in range(0, N + 1):
            continue
        # the edge the stencil sits next to, and the side it lies on
        if kind == "cell_pt":
            e = 0 if m in (-1, 0) else N
            inside_after = m == e          # cell e lies after the edge
        else:
            e = 0 if m in (-1, 1) else N
            inside_after = m > e
        y = x.copy()
        for k in range(LO, HI):
            # cell-centred inputs: cell k lies after edge e when k >= e;
            # interface inputs (cell_pt): interface k after the edge when k > e
            after = k >= e if kind != "cell_pt" else k > e
            before = k < e if kind != "cell_pt" else k < e
            if (inside_after and before) or (not inside_after and after):
                y[k - LO] += 10.0
        assert _val(kind, y, m, True) == _val(kind, x, m, True), (kind, m)
        assert _val(kind, y, m, False) != _val(kind, x, m, False), (kind, m)


@pytest.mark.parametrize("kind", KINDS)
def test_mirror_symmetry(kind):
    """Reversing the sweep maps each end onto the other."""
    rng = np.random.default_rng(5)
    x = rng.normal(size=HI - LO)
    # reversed data: interface k -> n - k, cell k -> n - 1 - k
    if kind == "cell_pt":
        xr = _arr(lambda k: x[(N - k) - LO] if LO <= N - k < HI else 0.0)
        mirror = lambda m: N - 1 - m
    else:
        xr = _arr(lambda k: x[(N - 1 - k) - LO] if LO <= N - 1 - k < HI else 0.0)
        mirror = lambda m: N - m
    for m in _ms(kind):
        mm = mirror(m)
        if mm not in _ms(kind):
            continue
        if kind == "cell_pt" and not (-1 <= mm <= N):
            continue
        a = _val(kind, x, m, True)
        b = _val(kind, xr, mm, True)
        assert abs(a - b) <= 1e-14 * (1 + abs(a)), (kind, m, a, b)


@pytest.mark.parametrize("kind", ["face_pt", "face_mean"])
def test_edge_value_is_mean_of_one_sided_extrapolations(kind):
    """Data linear on each side of the edge at interface 0 with different
    slopes (a kink): each side's linear extrapolation is exact for its own
    piece, so the edge value is the mean of the two pieces' values there."""
    aL, sL, aR, sR = 2.0, 0.5, -1.0, 3.0

    def piece(k):
        # value of the cell k (its centre, or its mean: the same for linear data)
        xc = k + 0.5
        return aR + sR * xc if k >= 0 else aL + sL * xc

    x = _arr(piece)
    want = 0.5 * (aL + aR)
    assert abs(_val(kind, x, 0, True) - want) <= 1e-13
    # the straddling stencil gives another value
    assert abs(_val(kind, x, 0, False) - want) > 1e-3


def _cube_corner_case(edge_interp, q):
    g = orc.Grid(1, N, 2, edge_interp=edge_interp)
    f = np.ascontiguousarray(q, dtype=np.float64).copy()
    orc.halo_fill(g, f)
    return orc.corner_values(g, f)


def test_corner_values_on_the_cube():
    """nh_p_grad's corner values: cell means of data quadratic in each tile's
    lattice coordinates are reproduced at the corners one cell inside the
    edges (one-sided x pass, centred y pass) whatever the neighbours hold;
    corners two or more cells inside the edges are bit-equal with and
    without the option; the vertices keep the three-cell mean."""
    T, NN = 6, N + 2 * H + 1
    q = np.zeros((T, NN, NN))
    # cell means of p(x, y) = 1 + 0.2 x - 0.05 x^2 + 0.1 y + 0.03 y^2 on every tile
    px = np.polynomial.Polynomial([0.0, 0.2, -0.05]).integ()
    py = np.polynomial.Polynomial([0.0, 0.1, 0.03]).integ()
    for j in range(-H, N + H + 1):
        for i in range(-H, N + H + 1):
            q[:, j + H, i + H] = 1.0 + (px(i + 1) - px(i)) + (py(j + 1) - py(j))
    on = _cube_corner_case(True, q)
    off = _cube_corner_case(False, q)
    exact = lambda i, j: 1.0 + 0.2 * i - 0.05 * i * i + 0.1 * j + 0.03 * j * j
    for t in range(T):
        for j in range(2, N - 1):
            for i in (1, N - 1):
                assert abs(on[t, j + H, i + H] - exact(i, j)) <= 1e-12, (t, i, j)
            for i in (1, N - 1):
                assert abs(off[t, j + H, i + H] - exact(i, j)) > 1e-6   # sees the rotated neighbour
        for j in range(2, N - 1):
            for i in range(2, N - 1):
                assert on[t, j + H, i + H] == off[t, j + H, i + H]
        for (i, j) in ((0, 0), (N, 0), (0, N), (N, N)):
            assert on[t, j + H, i + H] == off[t, j + H, i + H]


def test_corner_values_blind_to_the_neighbour_tile():
    """Changing the cells of the neighbour tiles (every halo cell) leaves the
    corner values one cell inside an edge unchanged on rows where both passes
    stay on the tile."""
    T, NN = 6, N + 2 * H + 1
    rng = np.random.default_rng(11)
    g = orc.Grid(1, N, 2, edge_interp=True)
    q = rng.normal(size=(T, NN, NN))
    a = q.copy()
    orc.halo_fill(g, a)
    b = a.copy()
    b[:, :, :H] += 5.0          # west halo columns
    b[:, :, N + H:] += 5.0      # east halo columns
    ca, cb = orc.corner_values(g, a), orc.corner_values(g, b)
    for j in range(2, N - 1):
        for i in (1, N - 1):
            assert ca[:, j + H, i + H].tolist() == cb[:, j + H, i + H].tolist()


def test_csw_winds_interior_unchanged_and_edges_changed():
    """After c_sw on the cube the C-grid winds are bit-equal with and without
    the option from four faces inside the tile edges, and differ next to
    them; on the doubly periodic grid the option changes nothing."""
    n, nz = 24, 3
    init = fi.cube_state(n=n, nz=nz)
    res = {}
    for ei in (False, True):
        g = orc.Grid(1, n, nz, edge_interp=ei)
        s = orc.new_state(g, init)
        assert orc.acoustic_substeps(g, s, 200.0, 1, stop_stage=2) == 0
        res[ei] = s
    for k in ("uc", "vc"):
        a, b = res[False][k], res[True][k]
        inner = np.s_[..., H + 4:H + n - 3, H + 4:H + n - 3]
        assert np.array_equal(a[inner], b[inner]), k
        assert np.abs(a - b).max() > 1e-6, k
    # every substep stage runs with the option, and the run stays finite
    g = orc.Grid(1, n, nz, edge_interp=True)
    s = orc.new_state(g, init)
    assert orc.acoustic_substeps(g, s, 2000.0, 10) == 0
    # doubly periodic: no tile edges
    pinit = fi.periodic_state(n=24, nz=3)
    out = []
    for ei in (False, True):
        g = orc.Grid(0, 24, 3, edge_interp=ei)
        s = orc.new_state(g, pinit)
        assert orc.acoustic_substeps(g, s, 1.0, 3) == 0
        out.append(s)
    for k in ("u", "v", "w", "delp", "pt", "delz"):
        assert np.array_equal(out[0][k], out[1][k]), k


def test_corner_values_one_sided_y_pass():
    """Corners one cell inside a y-edge (j = 1, n - 1) away from the x-edges
    take the one-sided y pass over rows on the tile: quadratic cell means are
    reproduced there (the centred pass would read a row of the rotated
    neighbour tile)."""
    T, NN = 6, N + 2 * H + 1
    q = np.zeros((T, NN, NN))
    px = np.polynomial.Polynomial([0.0, 0.2, -0.05]).integ()
    py = np.polynomial.Polynomial([0.0, 0.1, 0.03]).integ()
    for j in range(-H, N + H + 1):
        for i in range(-H, N + H + 1):
            q[:, j + H, i + H] = 1.0 + (px(i + 1) - px(i)) + (py(j + 1) - py(j))
    on = _cube_corner_case(True, q)
    exact = lambda i, j: 1.0 + 0.2 * i - 0.05 * i * i + 0.1 * j + 0.03 * j * j
    for t in range(T):
        for j in (1, N - 1):
            for i in range(1, N):
                assert abs(on[t, j + H, i + H] - exact(i, j)) <= 1e-12, (t, i, j)


def test_corner_values_rows_outside_keep_the_centred_x_pass():
    """At the corners on a y-edge (j = 0, n) one cell from an x-edge, the
    edge mean of the y pass combines the x-pass values of two rows inside
    the tile (one-sided in x) and two rows of the neighbour tile, which keep
    the centred x pass through the corner view: the composition of the
    one-dimensional interpolations written out."""
    T, NN = 6, N + 2 * H + 1
    rng = np.random.default_rng(17)
    g = orc.Grid(1, N, 2, edge_interp=True)
    q = rng.normal(size=(T, NN, NN))
    orc.halo_fill(g, q)
    got = orc.corner_values(g, q)
    for t in range(T):
        qx = orc.corner_view(g, q[t], "C", "x")
        for (i, j) in ((1, 0), (N - 1, 0), (1, N), (N - 1, N)):
            rows = [orc.interp("face_mean", qx[r + H, :], -H, i, N, 0 <= r < N) for r in range(j - 2, j + 2)]
            want = orc.interp("face_mean", rows, j - 2, j, N, True)
            assert abs(got[t, j + H, i + H] - want) <= 1e-14 * (1 + abs(want)), (t, i, j)


def test_csw_one_sided_face_winds():
    """c_sw's A -> C winds one face inside an edge: D-grid winds that depend
    only on the position along the wind (u = f(x) at the y-faces, v = f(y)
    at the x-faces, f quadratic) give cell-centre winds f exactly on the tile
    (one-sided D -> A next to the y-edges) and face winds f exactly at the
    faces 1 and n - 1 (one-sided A -> C), read back from the half-step area
    fluxes ax = dt/2 (u_c - v cos) / sin dy (and ay); without the option those faces
    read the rotated neighbour tile."""
    n, nz = 16, 2
    f = lambda x: 3.0 + 0.4 * x - 0.02 * x * x
    init = fi.cube_state(n=n, nz=nz)
    for key, shape in (("u", "Y"), ("v", "X")):
        a = np.zeros_like(init[key])
        for jj in range(a.shape[2]):
            for ii in range(a.shape[3]):
                i, j = ii - H, jj - H
                a[:, :, jj, ii] = f(i + 0.5) if key == "u" else f(j + 0.5)
        init[key] = a
    dt = 100.0
    res = {}
    for ei in (False, True):
        g = orc.Grid(1, n, nz, edge_interp=ei)
        s = orc.new_state(g, init)
        st, dbg = orc.acoustic_substeps(g, s, dt, 1, stop_stage=2, debug=True)
        assert st == 0
        dt2 = 0.5 * dt
        sin_u, cos_u, dy = g.metric("sin_u"), g.metric("cos_u"), g.metric("dy")
        sin_v, cos_v, dx = g.metric("sin_v"), g.metric("cos_v"), g.metric("dx")
        with np.errstate(invalid="ignore", divide="ignore"):
            ucp = dbg["ax"] * sin_u[:, None] / (dt2 * dy[:, None]) + init["v"] * cos_u[:, None]
            vcp = dbg["ay"] * sin_v[:, None] / (dt2 * dx[:, None]) + init["u"] * cos_v[:, None]
        res[ei] = (ucp, vcp)
    for ei, (ucp, vcp) in res.items():
        for m in (1, n - 1):
            e_u = np.abs(ucp[..., H:H + n, H + m] - f(m)).max()
            e_v = np.abs(vcp[..., H + m, H:H + n] - f(m)).max()
            if ei:
                assert e_u <= 1e-12 and e_v <= 1e-12, (m, e_u, e_v)
            else:
                assert e_u > 1e-6 and e_v > 1e-6, (m, e_u, e_v)


def test_csw_halo_columns_keep_the_centred_d_to_a():
    """Sweeps outside the tile keep the centred stencil: the outer face -1 of
    row 0 takes the one-sided A -> C value from the cells -1, -2, -3 of the
    neighbour tile, whose cell-centre winds come from the centred D -> A
    along their column (through the y-sweep view), as written out here from
    the one-dimensional interpolations."""
    n, nz = 16, 2
    init = fi.cube_state(n=n, nz=nz)
    dt = 100.0
    g = orc.Grid(1, n, nz, edge_interp=True)
    s = orc.new_state(g, init)
    st, dbg = orc.acoustic_substeps(g, s, dt, 1, stop_stage=2, debug=True)
    assert st == 0
    dt2 = 0.5 * dt
    sin_u, cos_u, dy = g.metric("sin_u"), g.metric("cos_u"), g.metric("dy")
    for t in range(6):
        for k in range(nz):
            uY, _ = orc.corner_view_pair(g, s["u"][t, k], "Y", s["v"][t, k], "X", "y")
            ua = {i: orc.interp("cell_pt", uY[:, i + H], -H, 0, n, False) for i in (-1, -2, -3)}
            want = 0.375 * ua[-1] + 0.75 * ua[-2] - 0.125 * ua[-3]
            f = (t, k, H, H - 1)
            got = dbg["ax"][f] * sin_u[t, H, H - 1] / (dt2 * dy[t, H, H - 1]) + s["v"][f] * cos_u[t, H, H - 1]
            assert abs(got - want) <= 1e-12 * (1 + abs(want)), (t, k, got, want)
