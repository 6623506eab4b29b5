"""Pins of the learned-correction oracle (NumPy FP64): the analytic gradients
equal central finite differences, a linear network's gradient equals the
closed form 2 X^T (X W - T) / N, the first bias-corrected Adam step is
-lr * sign(g), BF16 rounding is round-to-nearest-even, and the coarsening
conserves mass and circulation and preserves constants."""
import math

import numpy as np
import pytest

import fv3_inputs as fi
from oracle import mlp

H = 3


def _params(rng, sizes):
    ps = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        ps += [rng.standard_normal((a, b)) / math.sqrt(a), 0.1 * rng.standard_normal(b)]
    return ps


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    ps = _params(rng, [7, 6, 5, 4])
    X = rng.standard_normal((9, 7))
    T = rng.standard_normal((9, 4))
    _, grads, _ = mlp.loss_grad(ps, X, T, bf=False)
    h = 1e-6
    for p, g in zip(ps, grads):
        flat = p.reshape(-1)
        gf = g.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _, _ = mlp.loss_grad(ps, X, T, bf=False)
            flat[idx] = old - h
            lm, _, _ = mlp.loss_grad(ps, X, T, bf=False)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gf[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_output_layer_gradient_closed_form():
    # with the hidden activations fixed, the last layer is linear least squares
    rng = np.random.default_rng(1)
    ps = _params(rng, [5, 4, 3, 2])
    X = rng.standard_normal((11, 5))
    T = rng.standard_normal((11, 2))
    _, grads, Y = mlp.loss_grad(ps, X, T, bf=False)
    _, cache = mlp.forward(ps, X, bf=False)
    H2 = cache[4]
    want = 2.0 * H2.T @ (Y - T) / Y.size
    np.testing.assert_allclose(grads[4], want, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(grads[5], 2.0 * (Y - T).sum(0) / Y.size, rtol=1e-13, atol=1e-15)


def test_adam_first_step_is_signed_lr():
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -1e-3, 2.0])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    mlp.adam(p, g, m, v, step=1, lr=1e-3, eps=1e-12)
    np.testing.assert_allclose(p[0], [1.0 - 1e-3, -2.0 + 1e-3, 3.0 - 1e-3], rtol=0, atol=1e-12)


def test_bf16_rounding():
    # 1 + 2^-8 is exactly between 1 and the next bfloat16 (1 + 2^-7): ties to even -> 1
    assert mlp.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert mlp.bf16(np.array([1.0 + 3 * 2.0 ** -9]))[0] == 1.0 + 2.0 ** -7
    x = np.random.default_rng(2).standard_normal(1000)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))   # half an ulp of 8 significant bits
    np.testing.assert_array_equal(mlp.bf16(r), r)


@pytest.fixture(scope="module")
def grids(orc):
    return orc.Grid(1, 16, 3), orc.Grid(1, 4, 3)


def test_coarse_areas_tile_fine(grids):
    gf, gc = grids
    Af = gf.metric("area")[:, H:H + 16, H:H + 16]
    Ac = gc.metric("area")[:, H:H + 4, H:H + 4]
    s = Af.reshape(6, 4, 4, 4, 4).sum(axis=(2, 4))
    np.testing.assert_allclose(s, Ac, rtol=1e-12)


def test_coarsening_conserves(grids):
    gf, gc = grids
    init = fi.cube_state(n=16, nz=3)
    c = mlp.coarsen(init, gf, gc, 4)
    Af = gf.metric("area")[:, H:H + 16, H:H + 16]
    Ac = gc.metric("area")[:, H:H + 4, H:H + 4]
    mf = (init["delp"][:, :, H:H + 16, H:H + 16] * Af[:, None]).sum()
    mc = (c["delp"][:, :, H:H + 4, H:H + 4] * Ac[:, None]).sum()
    assert abs(mc / mf - 1) <= 1e-13
    tf = (init["pt"][:, :, H:H + 16, H:H + 16] * init["delp"][:, :, H:H + 16, H:H + 16] * Af[:, None]).sum()
    tc = (c["pt"][:, :, H:H + 4, H:H + 4] * c["delp"][:, :, H:H + 4, H:H + 4] * Ac[:, None]).sum()
    assert abs(tc / tf - 1) <= 1e-13
    # circulation along the south edge of every coarse row of y-faces
    dxf = gf.metric("dx")[:, H:H + 17, H:H + 16]
    dxc = gc.metric("dx")[:, H:H + 5, H:H + 4]
    circ_f = (init["u"][:, :, H:H + 17:4, H:H + 16] * dxf[:, None, ::4, :]).sum(-1)
    circ_c = (c["u"][:, :, H:H + 5, H:H + 4] * dxc[:, None]).sum(-1)
    np.testing.assert_allclose(circ_c, circ_f, rtol=1e-12)
    # constants stay constant
    k = dict(init)
    k["pt"] = np.full_like(init["pt"], 305.0)
    c2 = mlp.coarsen(k, gf, gc, 4)
    np.testing.assert_allclose(c2["pt"][:, :, H:H + 4, H:H + 4], 305.0, rtol=1e-14)


def test_features_layout(grids):
    gf, gc = grids
    init = fi.cube_state(n=4, nz=3)
    F = mlp.features(init, 4)
    assert F.shape == (6 * 16, 15)
    # column (t=1, j=2, i=3): pt block holds the three levels top to bottom
    col = 1 * 16 + 2 * 4 + 3
    np.testing.assert_array_equal(F[col, 6:9], init["pt"][1, :, H + 2, H + 3])
    np.testing.assert_allclose(F[col, 0:3], 0.5 * (init["u"][1, :, H + 2, H + 3] + init["u"][1, :, H + 3, H + 3]))


def test_correction_periodic_closed_form(orc):
    """On a doubly periodic tile the face increment is the mean of its two
    cells: a cell tendency cos(2 pi j / n) in ua comes back in the face-mean
    wind ua as cos(2 pi j / n) (1 + cos(2 pi / n)) / 2, exactly the discrete
    filter of two successive two-point means; pt changes by seconds x its
    tendency."""
    n, nz = 16, 2
    g = orc.Grid(0, n, nz)
    st = fi.periodic_state(n=n, nz=nz, seed=3)
    sec = 600.0
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    cu = np.cos(2 * np.pi * jj / n)
    cv = np.sin(2 * np.pi * ii / n)
    dY = np.zeros((n * n, 3 * nz))
    for k in range(nz):
        dY[:, k] = (k + 1) * cu.ravel()
        dY[:, nz + k] = (k + 2) * cv.ravel()
        dY[:, 2 * nz + k] = 1e-3 * (k + 1)
    out = mlp.apply_correction(g, st, dY, sec)
    d = mlp.features(out, n) - mlp.features(st, n)
    filt = (1 + np.cos(2 * np.pi / n)) / 2
    for k in range(nz):
        np.testing.assert_allclose(d[:, k], sec * (k + 1) * cu.ravel() * filt, atol=1e-11)
        np.testing.assert_allclose(d[:, nz + k], sec * (k + 2) * cv.ravel() * filt, atol=1e-11)
        np.testing.assert_allclose(d[:, 2 * nz + k], sec * 1e-3 * (k + 1), rtol=1e-12)
    # the periodic copies of the boundary faces stay identical
    np.testing.assert_array_equal(out["u"][:, :, H, H:H + n], out["u"][:, :, H + n, H:H + n])
    np.testing.assert_array_equal(out["v"][:, :, H:H + n, H], out["v"][:, :, H:H + n, H + n])


def test_correction_cube_edges_consistent(orc):
    """A D-grid face on a tile edge is stored by both tiles; after a random
    correction the two copies carry the same increment up to the sign that
    aligns the two tiles' edge directions (found from the vertex positions)."""
    n, nz = 8, 1
    g = orc.Grid(1, n, nz)
    N = n + 2 * H + 1
    zero = {k: np.zeros((6, nz, N, N)) for k in ("u", "v", "pt", "w", "delp", "delz")}
    dY = np.random.default_rng(5).standard_normal((6 * n * n, 3 * nz))
    out = mlp.apply_correction(g, zero, dY, 1.0)
    B = np.stack([g.metric(k) for k in ("bx", "by", "bz")], axis=-1)
    faces = []
    for t in range(6):
        for j in (0, n):
            for i in range(n):
                p0, p1 = B[t, H + j, H + i], B[t, H + j, H + i + 1]
                faces.append((p0 + p1, p1 - p0, out["u"][t, 0, H + j, H + i]))
        for i in (0, n):
            for j in range(n):
                p0, p1 = B[t, H + j, H + i], B[t, H + j + 1, H + i]
                faces.append((p0 + p1, p1 - p0, out["v"][t, 0, H + j, H + i]))
    mids = np.array([f[0] / np.linalg.norm(f[0]) for f in faces])
    matched = 0
    for a, (m, e, val) in enumerate(faces):
        d = mids @ mids[a]
        d[a] = -2
        b = int(np.argmax(d))
        assert d[b] > 1 - 1e-12          # every edge face has a twin on another tile
        sign = 1.0 if e @ faces[b][1] > 0 else -1.0
        assert abs(val - sign * faces[b][2]) <= 1e-14 * max(1.0, abs(val))
        assert val != 0.0
        matched += 1
    assert matched == 6 * 4 * n


def test_out_of_range_flag():
    lo = np.array([-1.0, -2.0])
    hi = np.array([1.0, 2.0])
    assert not mlp.out_of_range(np.array([[6.9, -7.9]]), lo, hi)
    assert mlp.out_of_range(np.array([[7.1, 0.0]]), lo, hi)
    assert mlp.out_of_range(np.array([[0.0, np.nan]]), lo, hi)
