"""Pins of the oracle's one-sided PPM edge values at cube tile edges (option
edge_ppm; the panel-edge treatment of Putman & Lin 2007, on which the paper
is silent): exactness for data linear in physical distance at the edge on an
uneven grid, one-sidedness of the inner and outer edge values, the mirror
symmetry between the two ends of a sweep, exactness for linear data at every
order, the Colella-Woodward constraint of order 8 in the edge cells
(flattening at an extremum, no overshoot of the swept means), faces away from
the edges left as they were, and the x/y symmetry of a cube tile under its
diagonal reflection.  Of the one-sided weights, linear exactness leaves one
free parameter; its value (the published 5/14, 11/14, -2/14) has no
independent pin."""
import numpy as np
import pytest

H = 3
ORDERS = (5, 6, 7, 8)


def _linear_window(rng, pe):
    """Cell widths (uneven) and the cell means of a linear function of the
    distance, with the edge position x_e of window interface pe."""
    w = rng.uniform(0.6, 1.6, 6)
    edges = np.concatenate([[0.0], np.cumsum(w)])
    centres = 0.5 * (edges[:-1] + edges[1:])
    a, b = rng.normal(), rng.normal()
    return w, a + b * centres, a + b * edges[pe]


@pytest.mark.parametrize("hord", [6, 8])
def test_edge_value_exact_for_linear_data_on_uneven_grid(orc, hord):
    rng = np.random.default_rng(5)
    for _ in range(20):
        w, q, exact = _linear_window(rng, 3)
        for west in (True, False):
            for c in (1e-13, -1e-13):
                f = orc.ppm_face_edge(q, w, c, hord, 3, west)
                assert abs(f - exact) < 1e-10 * (1 + abs(exact))
        # the stencil that straddles the edge is not exact there
        assert abs(orc.ppm_face(q, 1e-13, 6) - exact) > 1e-6


def test_inner_and_outer_values_are_one_sided(orc):
    rng = np.random.default_rng(6)
    for _ in range(20):
        q, w = rng.normal(size=6), rng.uniform(0.5, 1.5, 6)
        c = rng.uniform(0.05, 0.95)
        # west edge two faces below the upwind cell: face 2, upwind cell e+1
        f = orc.ppm_face_edge(q, w, c, 6, 1, True)
        q2 = q.copy()
        q2[0] += rng.normal()
        assert orc.ppm_face_edge(q2, w, c, 6, 1, True) == pytest.approx(f, abs=1e-14)
        assert orc.ppm_face(q2, c, 6) != pytest.approx(orc.ppm_face(q, c, 6), abs=1e-6)
        # the east mirror: face n-2, upwind cell e-2, blind to cell e
        f = orc.ppm_face_edge(q, w, -c, 6, 5, False)
        q2 = q.copy()
        q2[5] += rng.normal()
        assert orc.ppm_face_edge(q2, w, -c, 6, 5, False) == pytest.approx(f, abs=1e-14)
        # the outer value from the halo side alone: with the upwind cell e-1
        # and the edge value fixed by the cells beside the edge, cells beyond
        # them on the tile side do not enter
        f = orc.ppm_face_edge(q, w, c, 6, 3, True)
        q2 = q.copy()
        q2[5] += rng.normal()
        assert orc.ppm_face_edge(q2, w, c, 6, 3, True) == pytest.approx(f, abs=1e-14)


@pytest.mark.parametrize("hord", ORDERS)
def test_mirror_symmetry_of_the_two_ends(orc, hord):
    rng = np.random.default_rng(7)
    for _ in range(30):
        q = rng.normal(size=6) + (3.0 if hord == 7 else 0.0)
        w = rng.uniform(0.5, 1.5, 6)
        c = rng.uniform(-0.95, 0.95)
        for pe in range(1, 6):
            for west in (True, False):
                a = orc.ppm_face_edge(q, w, c, hord, pe, west)
                b = orc.ppm_face_edge(q[::-1], w[::-1], -c, hord, 6 - pe, not west)
                assert a == pytest.approx(b, rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("hord", ORDERS)
def test_linear_data_gives_the_exact_swept_mean(orc, hord):
    # unit cells, q = cell index: every edge value of every order is exact,
    # the parabola is the line, and the face value is the mean over the
    # swept interval next to the face at 2.5: 2.5 - c/2 for either sign
    q = np.arange(6, dtype=float) + 1.0
    w = np.ones(6)
    for pe in range(1, 6):
        for west in (True, False):
            for c in (-0.9, -0.4, -0.05, 0.05, 0.4, 0.9):
                f = orc.ppm_face_edge(q, w, c, hord, pe, west)
                assert f == pytest.approx(3.5 - c / 2, abs=1e-14)


def test_order8_flattens_an_extremum_in_an_edge_cell(orc):
    rng = np.random.default_rng(8)
    for _ in range(20):
        q = rng.uniform(0.0, 1.0, 6)
        q[2] = 2.0 + rng.uniform()        # a maximum in the upwind cell
        w = rng.uniform(0.5, 1.5, 6)
        for pe, west in ((2, True), (3, True), (3, False), (4, False)):
            for c in (0.1, 0.5, 0.9):
                assert orc.ppm_face_edge(q, w, c, 8, pe, west) == q[2]


def test_order8_swept_means_do_not_overshoot_in_edge_cells(orc):
    # increasing data: the parabola of an edge cell must be monotone, so the
    # mean over the swept part [1 - c, 1] of the cell falls as c grows, and
    # stays within the cell's edge values
    rng = np.random.default_rng(9)
    cs = np.linspace(0.02, 0.98, 25)
    for _ in range(200):
        q = np.cumsum(rng.exponential(size=6) ** 3)
        w = rng.uniform(0.5, 1.5, 6)
        for pe, west in ((1, True), (2, True), (3, True), (3, False), (4, False), (5, False)):
            s_edge = 2 in ((pe - 1, pe, pe + 1) if west else (pe - 2, pe - 1, pe))
            if not s_edge:
                continue
            f = np.array([orc.ppm_face_edge(q, w, c, 8, pe, west) for c in cs])
            assert np.all(np.diff(f) <= 1e-12 * (1 + abs(f).max()))


def _cube_fluxes(orc, edge_ppm, hord=8, seed=3, n=12):
    g = orc.Grid(1, n, 1, hord=hord, edge_ppm=edge_ppm)
    rng = np.random.default_rng(seed)
    N = g.N
    Q = g.field(1)
    Q[:, 0, H:H + n, H:H + n] = 1.0 + rng.random((6, n, n))
    orc.halo_fill(g, Q)
    A = g.metric("area")[0]
    crx = rng.uniform(-0.4, 0.4, (N, N))
    cry = rng.uniform(-0.4, 0.4, (N, N))
    return g, orc.fv_tp_2d(g, 0, Q[0, 0], crx, cry, crx * A, cry * A)


@pytest.mark.parametrize("hord", [6, 8])
def test_only_faces_near_tile_edges_change(orc, hord):
    n = 12
    _, (fx0, fy0) = _cube_fluxes(orc, False, hord)
    _, (fx1, fy1) = _cube_fluxes(orc, True, hord)
    # x-faces 3..n-3 in rows 3..n-4 see no edge window (the row's inner
    # y-update reaches y-face j+1 <= n-3), and the transpose for y-faces
    sl = (slice(H + 3, H + n - 3), slice(H + 3, H + n - 2))
    np.testing.assert_array_equal(fx1[sl], fx0[sl])
    np.testing.assert_array_equal(fy1[sl[::-1]], fy0[sl[::-1]])
    # in the same band of rows (columns), the faces with an edge cell upwind
    # change (there the difference can come only from the sweep's own edge
    # values); faces 2 and n-2 have one upwind only for one flow direction
    band = slice(H + 3, H + n - 3)
    for i in (0, 1, 2, n - 2, n - 1, n):
        assert (np.abs(fx1[band, H + i] - fx0[band, H + i]) > 1e-8).any()
        assert (np.abs(fy1[H + i, band] - fy0[H + i, band]) > 1e-8).any()


def test_periodic_grid_has_no_tile_edges(orc):
    rng = np.random.default_rng(4)
    out = []
    for on in (False, True):
        g = orc.Grid(0, 12, 1, edge_ppm=on)
        Q = g.field(1)
        Q[0, 0, H:H + 12, H:H + 12] = rng.random((12, 12)) if not out else q
        q = Q[0, 0, H:H + 12, H:H + 12].copy()
        orc.halo_fill(g, Q)
        A = g.metric("area")[0]
        c = np.full((g.N, g.N), 0.3)
        out.append(orc.fv_tp_2d(g, 0, Q[0, 0], c, -c, c * A, -c * A))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_diagonal_reflection_of_a_tile(orc):
    # a cube tile is symmetric under i <-> j with dxa <-> dya: transposing the
    # field and swapping the x and y Courant numbers swaps the flux arrays,
    # which ties the y-sweep's edge treatment (dya) to the x-sweep's (dxa)
    n = 12
    g = orc.Grid(1, n, 1, hord=8, edge_ppm=True)
    dxa, dya = g.metric("dxa")[0], g.metric("dya")[0]
    np.testing.assert_allclose(dxa, dya.T, rtol=1e-12)
    rng = np.random.default_rng(11)
    N = g.N
    q = 1.0 + rng.random((N, N))
    q = 0.5 * (q + q.T) + 0.1 * rng.random((N, N))
    A = g.metric("area")[0]
    crx = rng.uniform(-0.4, 0.4, (N, N))
    cry = rng.uniform(-0.4, 0.4, (N, N))
    fx, fy = orc.fv_tp_2d(g, 0, q, crx, cry, crx * A, cry * A)
    gx, gy = orc.fv_tp_2d(g, 0, q.T.copy(), cry.T.copy(), crx.T.copy(), (cry * A).T.copy(), (crx * A).T.copy())
    sl = (slice(H, H + n), slice(H, H + n + 1))
    np.testing.assert_allclose(gy.T[sl], fx[sl], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(gx.T[sl[::-1]], fy[sl[::-1]], rtol=1e-12, atol=1e-14)


def test_one_dsw_changes_winds_only_near_tile_edges(orc):
    # the kinetic-energy upwinding and every fv_tp_2d of d_sw take the edge
    # values only next to a tile edge: after one d_sw the winds
    # of the tile interior are bit-equal with and without the option, and the
    # winds next to the edges differ (through the edge-corner kinetic energy)
    import fv3_inputs as fi

    n, nz = 24, 2
    init = fi.cube_state(n=n, nz=nz, nq=0)
    out = []
    for on in (False, True):
        g = orc.Grid(1, n, nz, delta=1.0e5, edge_ppm=on)
        s = orc.new_state(g, init)
        assert orc.acoustic_substeps(g, s, 300.0, 1, stop_stage=6) == 0
        out.append(s)
    lo, hi = H + 5, H + n - 4    # measured: bit-equal from four cells in
    for k in ("u", "v"):
        a, b = out[0][k], out[1][k]
        np.testing.assert_array_equal(a[:, :, lo:hi, lo:hi], b[:, :, lo:hi, lo:hi])
        assert np.abs(a[:, :, H:H + n, H:H + 2] - b[:, :, H:H + n, H:H + 2]).max() > 1e-8
