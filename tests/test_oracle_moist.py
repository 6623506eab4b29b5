"""Pins of the oracle's moist column solves: with specific humidity q the
equation of state of both column solves takes the virtual potential
temperature theta (1 + (Rv/Rd - 1) q), q fixed over the call (tracers move in
the remapping step, Sec. II).  Pins: q = 0 is the dry path bit for bit; a
uniform q gives exactly the dry run started from pt (1 + eps q) (the pt that
comes out scaled by the same factor, every other field equal: transport and
the solves are homogeneous in pt), on the doubly periodic grid and on the
cube, whose C-grid solve reaches into the halo; a humid layer in a column at
rest pushes its neighbours away."""
import numpy as np
import pytest

import fv3_inputs as fi

H = 3
RD, RV = 287.05, 461.5
EPS = RV / RD - 1.0


def _run(orc, kind, n, nz, init, dt, ns, qv=None):
    g = orc.Grid(kind, n, nz, delta=1000.0 if kind == 0 else 1.0e5)
    d = dict(init)
    d["qv"] = qv
    s = orc.new_state(g, d)
    assert orc.acoustic_substeps(g, s, dt, ns) == 0
    return s


def _inner(a, n):
    return a[..., H:H + n, H:H + n]


@pytest.mark.parametrize("kind,n,nz,dt", [(0, 16, 6, 2.0), (1, 12, 6, 2000.0)])
def test_zero_humidity_is_dry(orc, kind, n, nz, dt):
    init = fi.periodic_state(n=n, nz=nz) if kind == 0 else fi.cube_state(n=n, nz=nz)
    dry = _run(orc, kind, n, nz, init, dt, 5)
    wet = _run(orc, kind, n, nz, init, dt, 5, qv=np.zeros_like(init["pt"]))
    for k in ("u", "v", "w", "delp", "pt", "delz", "pfull", "phi"):
        np.testing.assert_array_equal(dry[k], wet[k])


@pytest.mark.parametrize("kind,n,nz,dt", [(0, 16, 6, 2.0), (1, 12, 6, 2000.0)])
def test_uniform_humidity_scales_pt(orc, kind, n, nz, dt):
    init = fi.periodic_state(n=n, nz=nz) if kind == 0 else fi.cube_state(n=n, nz=nz)
    q = 0.012
    lam = 1.0 + EPS * q
    qv = np.zeros_like(init["pt"])
    qv[..., H:H + n, H:H + n] = q      # interior only: the halo is the call's to fill
    wet = _run(orc, kind, n, nz, init, dt, 10, qv=qv)
    scaled = dict(init)
    scaled["pt"] = init["pt"] * lam
    dry = _run(orc, kind, n, nz, scaled, dt, 10)
    for k in ("u", "v", "w", "delp", "delz", "pfull", "phi"):
        a, b = _inner(wet[k], n), _inner(dry[k], n)
        assert np.abs(a - b).max() <= 1e-11 * max(np.abs(b).max(), 1e-30), k
    a, b = _inner(wet["pt"], n) * lam, _inner(dry["pt"], n)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    # and the humidity matters: the dry run from the unscaled pt is different
    plain = _run(orc, kind, n, nz, init, dt, 10)
    assert np.abs(_inner(plain["w"], n) - _inner(wet["w"], n)).max() > 1e-6


def test_humid_layer_expands(orc):
    """A column at rest: moistening layer 3 raises its virtual temperature
    and hence its pressure, so the layer thickens, the layer above (k = 2)
    gains upward velocity and the one below (k = 4) downward velocity
    (w positive upward, k counted from the top)."""
    n, nz = 8, 6
    init = fi.periodic_state(n=n, nz=nz, wind=0.0)
    for k in ("u", "v"):
        init[k][:] = 0.0
    qv = np.zeros_like(init["pt"])
    qv[0, 3] = 0.02
    dry = _run(orc, 0, n, nz, init, 1.0, 1)
    wet = _run(orc, 0, n, nz, init, 1.0, 1, qv=qv)
    c = (0, slice(None), H + 2, H + 2)
    dz_dry, dz_wet = -dry["delz"][c], -wet["delz"][c]
    assert dz_wet[3] > dz_dry[3]
    assert wet["w"][0, 2, H + 2, H + 2] > dry["w"][0, 2, H + 2, H + 2]
    assert wet["w"][0, 4, H + 2, H + 2] < dry["w"][0, 4, H + 2, H + 2]


def test_humidity_per_tile_in_the_solve(orc):
    """Humidity that differs between tiles and levels: the D-grid solve's w
    equals the column solve with theta (1 + eps q) of each sampled column's
    own tile and levels, applied to the state it receives."""
    n, nz, dt = 10, 6, 300.0
    init = fi.cube_state(n=n, nz=nz, seed=5)
    rng = np.random.default_rng(60)
    qv = np.zeros_like(init["pt"])
    qv[..., H:H + n, H:H + n] = rng.uniform(0.0, 0.02, size=(6, nz, 1, 1))
    g = orc.Grid(1, n, nz, delta=1.0e5)
    d = dict(init, qv=qv)
    s7 = orc.new_state(g, d)
    assert orc.acoustic_substeps(g, s7, dt, 1, stop_stage=7) == 0
    s8 = orc.new_state(g, d)
    assert orc.acoustic_substeps(g, s8, dt, 1, stop_stage=8) == 0
    for _ in range(12):
        t, j, i = int(rng.integers(6)), int(rng.integers(n)) + H, int(rng.integers(n)) + H
        col = lambda k: s7[k][t, :, j, i]
        th = col("pt") * (1.0 + EPS * qv[t, :, j, i])
        r = orc.sim1(dt, g.ptop, 0.0, col("delp"), th, col("delz"), col("w"))
        assert np.abs(r["w"] - s8["w"][t, :, j, i]).max() <= 1e-13 * max(np.abs(r["w"]).max(), 1e-30)


def test_humidity_of_one_tile_in_the_c_grid_solve(orc):
    """Humidity on tile 3 only: after the C-grid solve (stage 3) its interface
    pressure on tile 3 differs from the dry run, and away from tile 3's halo
    ring the other tiles' columns are bit-equal to the dry run."""
    n, nz, dt = 10, 6, 300.0
    init = fi.cube_state(n=n, nz=nz, seed=6)
    qv = np.zeros_like(init["pt"])
    qv[3, :, H:H + n, H:H + n] = 0.015
    g = orc.Grid(1, n, nz, delta=1.0e5)
    dry = orc.new_state(g, init)
    st, d0 = orc.acoustic_substeps(g, dry, dt, 1, stop_stage=3, debug=True)
    wet = orc.new_state(g, dict(init, qv=qv))
    st1, d1 = orc.acoustic_substeps(g, wet, dt, 1, stop_stage=3, debug=True)
    assert st == 0 and st1 == 0
    inner = (slice(None), slice(H + 1, H + n - 1), slice(H + 1, H + n - 1))
    below_top = (slice(1, None),) + inner[1:]      # the top interface is ptop in both
    assert np.abs(d1["pkc"][3][below_top] - d0["pkc"][3][below_top]).min() > 0.0
    for t in (0, 1, 2, 4, 5):
        np.testing.assert_array_equal(d1["pkc"][t][inner], d0["pkc"][t][inner])
