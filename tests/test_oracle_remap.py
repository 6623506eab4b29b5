"""Pins of the oracle's vertical remapping (Lagrangian layers back to the
reference coordinate of the remapping step, Sec. II).  Each test checks a
property the mathematics fixes independently of the code: exactness on
polynomials the reconstruction can represent, conservation of the
mass-weighted column integral, boundedness and the limiter's behaviour at a
discontinuity, identity when nothing moved, and the global invariants of a
whole-state remap."""
import numpy as np
import pytest

import fv3_inputs as fi
import oracle as orc

H = 3


def _grid(nz, seed, lo=0.5, hi=2.0, top=0.0):
    rng = np.random.default_rng(seed)
    d = rng.uniform(lo, hi, nz)
    return np.concatenate([[top], top + np.cumsum(d)])


def _shifted(pe, seed, frac=0.45):
    """Target interfaces: every interior interface moved by up to frac of the
    thinner neighbouring layer (ends fixed, order kept)."""
    rng = np.random.default_rng(seed)
    d = np.diff(pe)
    out = pe.copy()
    for K in range(1, len(pe) - 1):
        out[K] = pe[K] + rng.uniform(-frac, frac) * min(d[K - 1], d[K])
    return out


def _means(F, pe):
    """Exact layer means of the function with antiderivative F."""
    return (F(pe[1:]) - F(pe[:-1])) / np.diff(pe)


def test_identity_when_interfaces_equal():
    pe = _grid(16, 1)
    q = np.random.default_rng(2).normal(size=16)
    out = orc.remap_column(pe, pe, q)
    assert np.abs(out - q).max() <= 1e-14 * np.abs(q).max()


def test_constant_preserved():
    pe = _grid(20, 3)
    q = np.full(20, 3.7)
    out = orc.remap_column(pe, _shifted(pe, 4), q)
    assert np.abs(out - 3.7).max() <= 1e-14


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_column_integral_conserved(seed):
    pe1 = _grid(30, seed)
    pe2 = _shifted(pe1, seed + 100)
    q = np.random.default_rng(seed + 200).normal(size=30) * 5.0 + 2.0
    out = orc.remap_column(pe1, pe2, q)
    m1 = np.sum(q * np.diff(pe1))
    m2 = np.sum(out * np.diff(pe2))
    assert abs(m2 - m1) <= 1e-13 * np.sum(np.abs(q) * np.diff(pe1))


def test_linear_profile_exact_away_from_boundary_layers():
    """Edges are exact for a linear profile (fourth- and second-order
    interpolation alike) and the limiter stays off for monotone data; the top
    and bottom layers are constant, so target layers that reach into them are
    excluded."""
    nz = 24
    pe1 = _grid(nz, 8)
    pe2 = _shifted(pe1, 9)
    a, b = 1.5, -0.7
    F = lambda p: a * p + b * p * p / 2.0
    out = orc.remap_column(pe1, pe2, _means(F, pe1))
    exact = _means(F, pe2)
    inner = [m for m in range(nz) if pe2[m] >= pe1[1] and pe2[m + 1] <= pe1[nz - 1]]
    assert len(inner) >= nz - 4
    err = np.abs(out - exact)[inner].max()
    assert err <= 1e-12 * np.abs(exact).max(), err


def test_quadratic_profile_exact_in_fourth_order_interior():
    """The parabola of a layer whose two edges come from the fourth-order
    interpolation equals a quadratic profile exactly (the interpolation is
    exact up to cubics); checked where the target layer overlaps only such
    layers (2..nz-3) with a monotone, gently curved profile."""
    nz = 24
    pe1 = _grid(nz, 10, lo=0.8, hi=1.25)
    pe2 = _shifted(pe1, 11)
    F = lambda p: 2.0 * p + 0.02 * p ** 3 / 3.0        # q = 2 + 0.02 p^2, monotone for p > 0
    out = orc.remap_column(pe1, pe2, _means(F, pe1))
    exact = _means(F, pe2)
    inner = [m for m in range(nz) if pe2[m] >= pe1[2] and pe2[m + 1] <= pe1[nz - 2]]
    assert len(inner) >= nz - 8
    err = np.abs(out - exact)[inner].max()
    assert err <= 1e-12 * np.abs(exact).max(), err
    # a dropped curvature term would leave an error of order the curvature
    d = np.diff(pe1)
    aL, aR, a6 = orc.ppm_profile(d, _means(F, pe1))
    f = lambda p: 2.0 + 0.02 * p * p
    for k in range(2, nz - 2):
        assert abs(aL[k] - f(pe1[k])) <= 1e-12 * f(pe1[k])
        assert abs(aR[k] - f(pe1[k + 1])) <= 1e-12 * f(pe1[k + 1])
        assert abs(a6[k] - (-0.02 * d[k] ** 2)) <= 1e-10     # q(x) curvature: -a6 = f'' d^2 / 2


def test_cubic_edges_exact():
    """Interface values of the fourth-order interpolation reproduce a cubic
    profile (monotone, limiter inactive) on non-uniform layers."""
    nz = 16
    pe = _grid(nz, 12, lo=0.9, hi=1.1, top=1.0)
    c = (1.0, 0.4, 0.05, 0.002)
    F = lambda p: c[0] * p + c[1] * p ** 2 / 2 + c[2] * p ** 3 / 3 + c[3] * p ** 4 / 4
    f = lambda p: c[0] + c[1] * p + c[2] * p ** 2 + c[3] * p ** 3
    aL, aR, _ = orc.ppm_profile(np.diff(pe), _means(F, pe))
    # an edge from two layers on either side: aR of layer k for k in 1..nz-3
    # unless the parabola limiter moved it; for this gentle cubic it does not
    for k in range(2, nz - 2):
        assert abs(aL[k] - f(pe[k])) <= 1e-12 * f(pe[k]), k
    for k in range(1, nz - 3):
        assert abs(aR[k] - f(pe[k + 1])) <= 1e-12 * f(pe[k + 1]), k


@pytest.mark.parametrize("seed", [13, 14])
def test_bounded_by_source_extremes(seed):
    rng = np.random.default_rng(seed)
    pe1 = _grid(40, seed)
    pe2 = _shifted(pe1, seed + 1, frac=0.49)
    q = rng.normal(size=40)
    out = orc.remap_column(pe1, pe2, q)
    assert out.max() <= q.max() + 1e-14 and out.min() >= q.min() - 1e-14


def test_step_shifted_half_a_layer_gives_half():
    """At a jump between two plateaus the limiter flattens both adjacent
    layers, so the reconstruction is the step itself: a target layer
    straddling it by half gets exactly the mean of the plateaus, and all
    others keep their plateau value.  Without the limiter the layers next to
    the jump would carry parabolas and the straddling mean would differ."""
    nz, K = 12, 6
    pe1 = np.arange(nz + 1, dtype=np.float64) * 10.0
    q = np.where(np.arange(nz) < K, 0.0, 1.0)
    pe2 = pe1.copy()
    pe2[1:-1] += 5.0
    out = orc.remap_column(pe1, pe2, q)
    want = np.where(np.arange(nz) < K - 1, 0.0, 1.0)
    want[K - 1] = 0.5
    assert np.array_equal(out, want), out


def test_single_and_two_layer_columns():
    out = orc.remap_column(np.array([0.0, 3.0]), np.array([0.0, 3.0]), np.array([2.5]))
    assert out[0] == 2.5
    out = orc.remap_column(np.array([0.0, 1.0, 3.0]), np.array([0.0, 2.0, 3.0]), np.array([1.0, 4.0]))
    # constant layers: [0,2] holds 1 x 1 + 4 x 1, [2,3] holds 4 x 1
    assert np.allclose(out, [2.5, 4.0], rtol=0, atol=1e-15)


def _state(kind, n, nz, seed):
    init = fi.periodic_state(n=n, nz=nz, seed=seed) if kind == 0 else fi.cube_state(n=n, nz=nz, seed=seed)
    og = orc.Grid(kind, n, nz, delta=1000.0 if kind == 0 else 1.0e5)
    s = orc.new_state(og, init)
    s["delp"] = fi.deform_layers(s["delp"], seed=seed + 1)
    qs = [np.ascontiguousarray(q, dtype=np.float64).copy() for q in init["q"]][:2]
    return og, s, qs


@pytest.mark.parametrize("kind,n,nz", [(0, 8, 10), (1, 6, 9)])
def test_state_remap_invariants(kind, n, nz):
    og, s, qs = _state(kind, n, nz, 21)
    ak, bk = fi.hybrid_coefficients(nz, og.ptop)
    cs = np.s_[..., H:H + n, H:H + n]
    before = orc.mass_sums(og, s["delp"], s["pt"], qs)
    depth = s["delz"][cs].sum(axis=1)
    wmom = (s["w"] * s["delp"])[cs].sum(axis=1)
    ps = og.ptop + s["delp"][cs].sum(axis=1)
    assert orc.remap(og, s, ak, bk, qs) == 0
    after = orc.mass_sums(og, s["delp"], s["pt"], qs)
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before)), (before, after)
    # every column now sits on the reference interfaces
    pe = og.ptop + np.concatenate([np.zeros_like(ps[:, None]), np.cumsum(s["delp"][cs], axis=1)], axis=1)
    ref = ak[None, :, None, None] + bk[None, :, None, None] * ps[:, None]
    assert np.abs(pe - ref).max() <= 1e-9
    assert np.abs(s["delz"][cs].sum(axis=1) - depth).max() <= 1e-12 * np.abs(depth).max()
    assert np.abs((s["w"] * s["delp"])[cs].sum(axis=1) - wmom).max() <= 1e-12 * (np.abs(wmom).max() + 1e-30) + 1e-12


def test_state_remap_identity_on_reference_layers():
    """A state whose layers already are the reference ones (evenly spaced
    sigma, the coordinate the inputs are built on) comes back unchanged,
    winds included (their face interfaces are the mean of two sigma columns,
    which is again the sigma column of the mean surface pressure)."""
    n, nz = 8, 10
    init = fi.cube_state(n=n, nz=nz, seed=31)
    og = orc.Grid(1, n, nz, delta=1.0e5)
    s = orc.new_state(og, init)
    ref = {k: s[k].copy() for k in ("u", "v", "w", "delp", "pt", "delz")}
    ak, bk = fi.sigma_coefficients(nz, og.ptop)
    assert orc.remap(og, s, ak, bk) == 0
    views = {"u": (n + 1, n), "v": (n, n + 1), "w": (n, n), "delp": (n, n), "pt": (n, n), "delz": (n, n)}
    for k, (nj, ni) in views.items():
        a = s[k][..., H:H + nj, H:H + ni]
        b = ref[k][..., H:H + nj, H:H + ni]
        scale = np.abs(b).max() + 1e-30
        assert np.abs(a - b).max() <= 1e-12 * scale + 1e-14, k


def test_face_momentum_conserved():
    """u at a y-face is remapped on the mean interfaces of its two cells:
    the face column's sum of u times the mean thickness is unchanged."""
    og, s, _ = _state(1, 6, 8, 41)
    orc.halo_fill(og, s["delp"])
    ak, bk = fi.hybrid_coefficients(8, og.ptop)
    t, i, j = 2, 3, 0      # j = 0: the second cell is in the halo (neighbour tile)
    da = s["delp"][t, :, j + H, i + H].copy()
    db = s["delp"][t, :, j - 1 + H, i + H].copy()
    u0 = s["u"][t, :, j + H, i + H].copy()
    m0 = np.sum(u0 * 0.5 * (da + db))
    psf = og.ptop + 0.5 * (da.sum() + db.sum())
    assert orc.remap(og, s, ak, bk) == 0
    m1 = np.sum(s["u"][t, :, j + H, i + H] * np.diff(ak + bk * psf))
    assert abs(m1 - m0) <= 1e-12 * np.sum(np.abs(u0) * 0.5 * (da + db))


@pytest.mark.parametrize("seed", [51, 52, 53])
def test_edges_between_adjacent_means(seed):
    """Monotonised slopes keep every interface value between the means of
    the two layers it separates (random, non-smooth data)."""
    rng = np.random.default_rng(seed)
    nz = 40
    d = rng.uniform(0.3, 3.0, nz)
    a = rng.normal(size=nz) * np.where(rng.random(nz) < 0.3, 10.0, 1.0)
    e = orc.ppm_edges(d, a)
    for K in range(1, nz):
        lo, hi = min(a[K - 1], a[K]), max(a[K - 1], a[K])
        assert lo - 1e-13 <= e[K] <= hi + 1e-13, (K, a[K - 1], e[K], a[K])


@pytest.mark.parametrize("seed", [61, 62])
def test_monotone_data_give_monotone_parabolas_and_result(seed):
    """For monotone layer means the limited parabola of every layer has no
    turning point inside the layer (|a6| <= |aR - aL|), and the remapped
    means stay monotone."""
    rng = np.random.default_rng(seed)
    nz = 40
    pe1 = _grid(nz, seed)
    a = np.cumsum(rng.exponential(size=nz) ** 3)      # increasing, with sharp jumps
    aL, aR, a6 = orc.ppm_profile(np.diff(pe1), a)
    # a moved edge puts the turning point exactly on it (|a6| = |aR - aL|),
    # so allow rounding at the size of the field
    tol = 1e-13 * np.abs(a).max()
    assert np.all(np.abs(a6) <= np.abs(aR - aL) + tol)
    assert np.all(aR >= aL - tol)
    out = orc.remap_column(pe1, _shifted(pe1, seed + 7, frac=0.49), a)
    assert np.all(np.diff(out) >= -1e-12 * np.abs(a).max())


def test_dynamics_loop_conserves_and_lands_on_reference():
    """The oracle's remapping loop (k_split passes of substeps, tracer
    transport and remap) on the doubly periodic grid: the global sums of
    mass, pt mass and tracer masses are those of the start (each of the three
    steps conserves them there), every column ends on the reference
    interfaces, and with k_split = 1 the loop is the three calls in order,
    bit for bit."""
    n, nz = 16, 6
    init = fi.periodic_state(n=n, nz=nz, seed=5, nq=2)
    ak, bk = fi.hybrid_coefficients(nz, 100.0)
    og = orc.Grid(0, n, nz)
    s = orc.new_state(og, init)
    qs = [np.ascontiguousarray(q, dtype=np.float64).copy() for q in init["q"]]
    before = orc.mass_sums(og, s["delp"], s["pt"], qs)
    assert orc.dynamics(og, s, qs, ak, bk, 3 * 4 * 0.3, 3, 4) == 0
    after = orc.mass_sums(og, s["delp"], s["pt"], qs)
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before)), (before, after)
    cs = np.s_[..., H:H + n, H:H + n]
    ps = og.ptop + s["delp"][cs].sum(axis=1)
    pe = og.ptop + np.concatenate([np.zeros_like(ps[:, None]), np.cumsum(s["delp"][cs], axis=1)], axis=1)
    ref = ak[None, :, None, None] + bk[None, :, None, None] * ps[:, None]
    assert np.abs(pe - ref).max() <= 1e-9
    # k_split = 1: the loop is substeps, tracer transport, remap
    a = orc.new_state(og, init)
    b = orc.new_state(og, init)
    qa = [np.ascontiguousarray(q, dtype=np.float64).copy() for q in init["q"]]
    qb = [q.copy() for q in qa]
    assert orc.dynamics(og, a, qa, ak, bk, 4 * 0.3, 1, 4) == 0
    assert orc.acoustic_substeps(og, b, 4 * 0.3, 4) == 0
    orc.tracer_transport(og, qb, b["dp0"], b["mfx"], b["mfy"], b["cx"], b["cy"])
    assert orc.remap(og, b, ak, bk, qb) == 0
    for k in ("u", "v", "w", "delp", "pt", "delz"):
        assert np.array_equal(a[k], b[k]), k
    for x, y in zip(qa, qb):
        assert np.array_equal(x, y)
