"""Pins of the oracle's cubed-sphere grid (Sec. II: gnomonic cubed sphere)
and its halos, corner views and tile-edge rule.

Grid: total area 4 pi a^2; each tile a sixth; dual (corner) areas also tile
the sphere; a cube edge is the arc arccos(1/3); in-tile mirror and transpose
symmetries of the equiangular grid.  Halos: every halo cell is a geometric
neighbour of the cell next to it (distance about one spacing, outward
direction), vector halos of a solid-body rotation reproduce the local
covariant components, the corner view of the paper's corner fragment
(Sec. VII-C) holds, and the tile-edge faces carry cos = 0 / sin = 1 so the
general normal-flux formula reduces to the printed edge rule (Sec. V-B)."""
import math
import os

import numpy as np
import pytest

H = 3
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def cube(orc):
    return orc.Grid(1, 16, 1)


def _int(a, n, ni=None, nj=None):
    ni = n if ni is None else ni
    nj = n if nj is None else nj
    return a[:, H:H + nj, H:H + ni]


def test_total_and_tile_area(orc, cube):
    n, a = cube.n, orc.RADIUS
    A = _int(cube.metric("area"), n)
    S = 4 * math.pi * a * a
    assert abs(A.sum() / S - 1) <= 1e-12
    for t in range(6):
        assert abs(A[t].sum() / (S / 6) - 1) <= 1e-12


def test_dual_area_tiles_sphere(orc, cube):
    n, a = cube.n, orc.RADIUS
    Ac = _int(cube.metric("area_c"), n, n + 1, n + 1)
    w = np.ones((n + 1, n + 1))
    w[0, :] = w[-1, :] = w[:, 0] = w[:, -1] = 0.5
    for jj in (0, n):
        for ii in (0, n):
            w[jj, ii] = 1.0 / 3.0
    assert abs((Ac * w[None]).sum() / (4 * math.pi * a * a) - 1) <= 1e-12


def test_cube_edge_length(orc, cube):
    n, a = cube.n, orc.RADIUS
    dx = cube.metric("dx")       # on y-faces: rows j = 0..n, i = 0..n-1
    edge = dx[:, H, H:H + n].sum(axis=1)
    np.testing.assert_allclose(edge, a * math.acos(1.0 / 3.0), rtol=1e-13)


def test_in_tile_symmetries(cube):
    n = cube.n
    for name in ("area", "dxa", "sin_a"):
        A = _int(cube.metric(name), n)[0]
        np.testing.assert_allclose(A, A[:, ::-1], rtol=1e-13)
        np.testing.assert_allclose(A, A[::-1, :], rtol=1e-13)
    A = _int(cube.metric("area"), n)[0]
    np.testing.assert_allclose(A, A.T, rtol=1e-13)
    dxa = _int(cube.metric("dxa"), n)[0]
    dya = _int(cube.metric("dya"), n)[0]
    np.testing.assert_allclose(dxa, dya.T, rtol=1e-13)
    # cos at cells is antisymmetric under one mirror (the frame is skewed the other way)
    ca = _int(cube.metric("cos_a"), n)[0]
    np.testing.assert_allclose(ca, -ca[:, ::-1], atol=1e-14)
    # all tiles are congruent
    allA = _int(cube.metric("area"), n)
    for t in range(1, 6):
        np.testing.assert_allclose(allA[t], allA[0], rtol=1e-13)


def test_connectivity_is_an_involution(cube):
    nbr, rot = cube.connectivity()
    for t in range(6):
        assert len(set(nbr[t])) == 4 and t not in nbr[t]
        for e in range(4):
            tb = nbr[t, e]
            back = list(nbr[tb]).index(t)
            R = rot[t, e]
            Rb = rot[tb, back]
            np.testing.assert_array_equal(Rb @ R, np.eye(2, dtype=int))
            assert round(np.linalg.det(R)) == 1


def test_edge_faces_reduce_to_printed_rule(orc, cube):
    n = cube.n
    with open(os.path.join(GOLD, "edge_flux_sec5b.txt")) as f:
        dt2, vel, velc, want = [float(x) for x in
                                [l for l in f if not l.startswith("#")][0].split()]
    for cname, sname, axis in (("cos_u", "sin_u", "x"), ("cos_v", "sin_v", "y")):
        c, s = cube.metric(cname), cube.metric(sname)
        if axis == "x":
            ce, se = c[:, H:H + n, [H, H + n]], s[:, H:H + n, [H, H + n]]
        else:
            ce, se = c[:, [H, H + n], H:H + n], s[:, [H, H + n], H:H + n]
        assert np.all(ce == 0.0) and np.all(se == 1.0)
        flux = dt2 * (vel - velc * ce) / se
        assert np.all(flux == want)
    # away from tile edges the grid is skewed: cos != 0 in general
    assert np.abs(cube.metric("cos_u")[:, H:H + n, H + 1:H + n]).max() > 1e-3


def test_halo_cells_are_geometric_neighbours(orc, cube):
    n = cube.n
    P = [cube.metric(k).copy() for k in ("cx", "cy", "cz")]
    raw = [p.copy() for p in P]
    for p in P:
        orc.halo_fill(cube, p[:, None], "C")
    pos = np.stack(P, axis=-1)          # [t][jj][ii][3]
    spacing = math.pi / 2 / n
    for t in range(6):
        for jj in range(H, H + n):
            for d in (1, 2, 3):
                # west / east / south / north halo at depth d vs the first interior cell
                for (hi, hj, ii, ij) in ((H - d, jj, H, jj), (H + n - 1 + d, jj, H + n - 1, jj),
                                         (jj, H - d, jj, H), (jj, H + n - 1 + d, jj, H + n - 1)):
                    a = pos[t, hj, hi]
                    b = pos[t, ij, ii]
                    ang = math.acos(max(-1.0, min(1.0, float(a @ b))))
                    assert 0.5 * d * spacing < ang < 1.6 * d * spacing
                    # the halo point is not on this tile's face
                    assert np.allclose(np.linalg.norm(a), 1.0)
    # interior untouched
    for p, r in zip(P, raw):
        np.testing.assert_array_equal(_int(p, n), _int(r, n))


def _solid_body(p):
    # velocity of a rigid rotation about the axis (0.3, -0.5, 0.81), |omega| = 1
    ax = np.array([0.3, -0.5, 0.81])
    ax /= np.linalg.norm(ax)
    return np.cross(ax, p)


def _face_tables(cube):
    """Midpoints and unit edge tangents of every interior D-grid face of every tile."""
    n = cube.n
    B = np.stack([cube.metric(k) for k in ("bx", "by", "bz")], axis=-1)
    mids, tans, keys = [], [], []
    for t in range(6):
        for j in range(n + 1):
            for i in range(n):          # y-faces: edge B(i,j) -> B(i+1,j)
                p0, p1 = B[t, H + j, H + i], B[t, H + j, H + i + 1]
                m = (p0 + p1) / np.linalg.norm(p0 + p1)
                e = (p1 - p0) - ((p1 - p0) @ m) * m
                mids.append(m); tans.append(e / np.linalg.norm(e)); keys.append((t, "Y", i, j))
        for j in range(n):
            for i in range(n + 1):      # x-faces: edge B(i,j) -> B(i,j+1)
                p0, p1 = B[t, H + j, H + i], B[t, H + j + 1, H + i]
                m = (p0 + p1) / np.linalg.norm(p0 + p1)
                e = (p1 - p0) - ((p1 - p0) @ m) * m
                mids.append(m); tans.append(e / np.linalg.norm(e)); keys.append((t, "X", i, j))
    return np.array(mids), np.array(tans), keys


def test_vector_halo_orientation(orc, cube):
    """D-grid covariant components of a rigid rotation V.  After the vector
    fill, every west/south halo value equals V . e of the neighbour-tile edge
    it sits on (located geometrically from the halo cell centres), with the
    sign that aligns that edge with this tile's lattice direction."""
    n, N = cube.n, cube.N
    mids, tans, keys = _face_tables(cube)
    u = np.zeros((6, 1, N, N))
    v = np.zeros((6, 1, N, N))
    for (t, st, i, j), m, e in zip(keys, mids, tans):
        (u if st == "Y" else v)[t, 0, H + j, H + i] = _solid_body(m) @ e
    orc.halo_fill_pair(cube, u, "Y", v, "X")
    C = [cube.metric(k).copy() for k in ("cx", "cy", "cz")]
    for c in C:
        orc.halo_fill(cube, c[:, None], "C")
    C = np.stack(C, axis=-1)

    def check(t, got, c0, c1, along):
        # face between halo cells c0, c1; its true midpoint is the nearest face midpoint
        guess = (c0 + c1) / np.linalg.norm(c0 + c1)
        k = int(np.argmax(mids @ guess))
        e_true = tans[k]
        sign = 1.0 if e_true @ along > 0 else -1.0
        assert abs(e_true @ along) > 0.5 * np.linalg.norm(along)
        assert abs(got - sign * (_solid_body(mids[k]) @ e_true)) <= 1e-12

    checked = 0
    for t in range(6):
        for d in (1, 2, 3):
            i = -d
            for j in range(1, n):       # west-halo y-faces (x components)
                c0, c1 = C[t, H + j - 1, H + i], C[t, H + j, H + i]
                along = (C[t, H + j, H + i + 1] - C[t, H + j, H + i - 1]) if d < 3 else \
                        (C[t, H + j, H + i + 1] - C[t, H + j, H + i])
                check(t, u[t, 0, H + j, H + i], c0, c1, along)
                checked += 1
            j = -d
            for i in range(1, n):       # south-halo x-faces (y components)
                c0, c1 = C[t, H + j, H + i - 1], C[t, H + j, H + i]
                along = (C[t, H + j + 1, H + i] - C[t, H + j - 1, H + i]) if d < 3 else \
                        (C[t, H + j + 1, H + i] - C[t, H + j, H + i])
                check(t, v[t, 0, H + j, H + i], c0, c1, along)
                checked += 1
    assert checked == 6 * 3 * 2 * (n - 1)


def test_printed_corner_fill(orc, cube):
    with open(os.path.join(GOLD, "corner_fill_sec7c.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    rng = np.random.default_rng(8)
    plane = rng.random((cube.N, cube.N))
    for mode, corner, di, dj, si, sj, mult in rows:
        assert corner == "SW"
        view = orc.corner_view(cube, plane, "C", mode)
        assert view[H + int(dj), H + int(di)] == float(mult) * plane[H + int(sj), H + int(si)]


def test_corner_view_rotation_rules(orc, cube):
    """x-sweep: SW (-a,-b) <- (-b, a-1); y-sweep: SW (-a,-b) <- (b-1, -a);
    the other corners by mirroring i -> n-1-i and/or j -> n-1-j."""
    n = cube.n
    rng = np.random.default_rng(9)
    plane = rng.random((cube.N, cube.N))
    vx = orc.corner_view(cube, plane, "C", "x")
    vy = orc.corner_view(cube, plane, "C", "y")
    P = lambda i, j: plane[H + j, H + i]
    for a in (1, 2, 3):
        for b in (1, 2, 3):
            for mi in (False, True):
                for mj in (False, True):
                    fi = (lambda i: n - 1 - i) if mi else (lambda i: i)
                    fj = (lambda j: n - 1 - j) if mj else (lambda j: j)
                    ci, cj = fi(-a), fj(-b)
                    assert vx[H + cj, H + ci] == P(fi(-b), fj(a - 1))
                    assert vy[H + cj, H + ci] == P(fi(b - 1), fj(-a))


def test_periodic_halo_wraps(orc):
    g = orc.Grid(0, 8, 2)
    f = g.field(2)
    rng = np.random.default_rng(3)
    f[0, :, H:H + 8, H:H + 8] = rng.random((2, 8, 8))
    orc.halo_fill(g, f, "C")
    inner = f[0, :, H:H + 8, H:H + 8]
    full = np.tile(inner, (1, 3, 3))[:, 8 - H:16 + H, 8 - H:16 + H]
    np.testing.assert_array_equal(f[0, :, :8 + 2 * H, :8 + 2 * H], full)
