"""GPU parity of the vertical remapping (fv3_remap) against the oracle.

Inputs: the seeded initial states with every column's layers redistributed
(fv3_inputs.deform_layers, standing in for the Lagrangian deformation of a
remapping step), seeded N(0, 1) vertical velocity and two U[0, 1] tracers,
remapped to the hybrid reference coordinate of fv3_inputs.

Error measure: max |gpu - oracle| / max |oracle| per field over interior
points.  FP64 bar 1e-12: each value is a sum of a few overlap integrals of
parabolas whose coefficients take some tens of operations, and the layer
coordinates x = (p - p_top) / dp lose about two digits (p ~ 1e5 Pa against
dp ~ 1e3 Pa), so rounding differences of the two implementations stay near
1e-14.  Mixed precision: both sides start from the same FP32-rounded bulk
fields (rounded on the host for the oracle), the remap computes in FP64 and
rounds its bulk outputs to FP32 once: bar 2.5e-7 (two FP32 half-ulps of the
field's largest value), delz (FP64 storage) 1e-12."""
import numpy as np
import pytest

import fv3_inputs as fi

pytestmark = pytest.mark.gpu
H = 3
VIEWS = {"u": "Y", "v": "X", "w": "C", "delp": "C", "pt": "C", "delz": "C"}


def _int(a, n, st):
    ni = n + 1 if st in ("X", "B") else n
    nj = n + 1 if st in ("Y", "B") else n
    return a[..., H:H + nj, H:H + ni]


def _relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def fv3():
    import torch

    import paper_2205_04148_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def _inputs(kind, n, nz, seed, nq=2):
    init = fi.periodic_state(n=n, nz=nz, seed=seed, nq=nq) if kind == 0 else \
        fi.cube_state(n=n, nz=nz, seed=seed, nq=nq)
    init["delp"] = fi.deform_layers(init["delp"], seed=seed + 1)
    rng = np.random.default_rng(seed + 2)
    w = np.zeros_like(init["delp"])
    w[..., H:H + n, H:H + n] = rng.normal(size=w[..., H:H + n, H:H + n].shape)
    init["w"] = w
    return init


def _fp32(init, precision):
    """The oracle's copy of the inputs: bulk fields rounded as the device stores them."""
    out = dict(init)
    if precision == "mixed":
        for k in ("u", "v", "w", "delp", "pt"):
            out[k] = init[k].astype(np.float32).astype(np.float64)
        out["q"] = [q.astype(np.float32).astype(np.float64) for q in init["q"]]
    return out


def _run_pair(fv3, orc, kind, n, nz, precision, seed=3, coef="hybrid"):
    import torch

    init = _inputs(kind, n, nz, seed)
    dx = 1000.0 if kind == 0 else 1.0e5
    g = fv3.Grid(kind, n, nz, dx=dx, precision=precision)
    s = fv3.State.allocate(g)
    s.load(init)
    qd = [g.upload(q, nz) for q in init["q"]]
    ak, bk = fi.hybrid_coefficients(nz, g.ptop) if coef == "hybrid" else fi.sigma_coefficients(nz, g.ptop)
    print(f"remap kind={kind} n={n} nz={nz} {precision}", flush=True)
    fv3.remap(s, g, ak, bk, qd)
    assert fv3.check_status(g) == 0
    torch.cuda.synchronize()
    oi = _fp32(init, precision)
    og = orc.Grid(kind, n, nz, delta=dx)
    os_ = orc.new_state(og, oi)
    qh = [q.copy() for q in oi["q"]]
    assert orc.remap(og, os_, ak, bk, qh) == 0
    errs = {k: _relerr(_int(s.get(k), n, st), _int(os_[k], n, st)) for k, st in VIEWS.items()}
    for m, (a, b) in enumerate(zip(qd, qh)):
        errs[f"q{m}"] = _relerr(_int(g.download(a, nz), n, "C"), _int(b, n, "C"))
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    return errs, g, s, qd


def _bars(precision):
    if precision == "fp64":
        return lambda k: 1e-12
    return lambda k: 1e-12 if k == "delz" else 2.5e-7


@pytest.mark.parametrize("kind,n,nz", [(0, 70, 12), (1, 12, 9)])
def test_remap_parity_fp64(fv3, orc, kind, n, nz):
    """Periodic n = 70 spans two 64-wide blocks with a ragged tail; the cube
    exercises tile-edge faces, whose second cell comes from the neighbour
    tile through the halo."""
    errs, *_ = _run_pair(fv3, orc, kind, n, nz, "fp64")
    bar = _bars("fp64")
    for k, e in errs.items():
        assert e <= bar(k), (k, e)


def test_remap_parity_mixed_cube(fv3, orc):
    errs, *_ = _run_pair(fv3, orc, 1, 24, 10, "mixed")
    bar = _bars("mixed")
    for k, e in errs.items():
        assert e <= bar(k), (k, e)


@pytest.mark.parametrize("nz", [1, 2, 3, 4])
def test_remap_few_layers(fv3, orc, nz):
    """Columns too short for any fourth-order interface (nz < 4) or with a
    single one (nz = 4): the boundary rules alone."""
    errs, *_ = _run_pair(fv3, orc, 0, 20, nz, "fp64", seed=5)
    for k, e in errs.items():
        assert e <= 1e-12, (k, e)


def test_remap_identity_on_reference_layers(fv3):
    """Undeformed sigma layers remapped to the same sigma coordinate come back
    unchanged (up to rounding), winds included."""
    import torch

    n, nz = 16, 8
    init = fi.cube_state(n=n, nz=nz, seed=7)
    g = fv3.Grid(1, n, nz, dx=1.0e5)
    s = fv3.State.allocate(g)
    s.load(init)
    before = {k: s.get(k) for k in VIEWS}
    ak, bk = fi.sigma_coefficients(nz, g.ptop)
    fv3.remap(s, g, ak, bk)
    assert fv3.check_status(g) == 0
    torch.cuda.synchronize()
    for k, st in VIEWS.items():
        a, b = _int(s.get(k), n, st), _int(before[k], n, st)
        assert np.abs(a - b).max() <= 1e-12 * (np.abs(b).max() + 1e-30) + 1e-14, k


def test_remap_conserves_mass_sums(fv3, orc):
    """Global mass, pt mass and tracer masses (compensated FP64 sums on the
    device) are unchanged by the remap."""
    kind, n, nz = 1, 12, 9
    init = _inputs(kind, n, nz, 11)
    g = fv3.Grid(kind, n, nz, dx=1.0e5)
    s = fv3.State.allocate(g)
    s.load(init)
    qd = [g.upload(q, nz) for q in init["q"]]
    m0 = fv3.mass_sums(g, s.f["delp"], s.f["pt"], qd)
    ak, bk = fi.hybrid_coefficients(nz, g.ptop)
    fv3.remap(s, g, ak, bk, qd)
    m1 = fv3.mass_sums(g, s.f["delp"], s.f["pt"], qd)
    assert np.all(np.abs(m1 - m0) <= 1e-13 * np.abs(m0)), (m0, m1)


def test_remap_errors(fv3):
    n, nz = 8, 4
    g = fv3.Grid(0, n, nz)
    s = fv3.State.allocate(g)
    s.load(fi.periodic_state(n=n, nz=nz))
    ak, bk = fi.sigma_coefficients(nz, g.ptop)
    bad = ak.copy()
    bad[0] = g.ptop + 1.0
    with pytest.raises(fv3.FV3Error) as e:
        fv3.remap(s, g, bad, bk)
    assert e.value.status == -1
    bad = bk.copy()
    bad[-1] = 0.99
    with pytest.raises(fv3.FV3Error):
        fv3.remap(s, g, ak, bad)
    bad = ak.copy()
    bad[2] = np.nan
    with pytest.raises(fv3.FV3Error):
        fv3.remap(s, g, bad, bk)
    g2 = fv3.Grid(0, 8, 129)
    s2 = fv3.State.allocate(g2)
    a2, b2 = fi.sigma_coefficients(129, g2.ptop)
    with pytest.raises(fv3.FV3Error) as e:
        fv3.remap(s2, g2, a2, b2)
    assert e.value.status == -2
    # reference interfaces that fold back: every access stays in bounds, the
    # kernel latches the condition
    ak2, bk2 = ak.copy(), bk.copy()
    ak2[2], bk2[2] = ak[1], bk[1] - 0.2
    fv3.remap(s, g, ak2, bk2)
    assert fv3.check_status(g) == -9
    assert fv3.check_status(g) == 0


def test_remap_full_size_sampled(fv3, orc):
    """C192 x 79, mixed precision, the launch configuration the benchmark
    times: 48 sampled cell columns (all fields) and 24 faces of each wind
    against the oracle's column remap, computed one by one."""
    import torch

    n, nz = 192, 79
    init = _inputs(1, n, nz, 2, nq=2)
    g = fv3.Grid(1, n, nz, dx=1.0e5, precision="mixed")
    s = fv3.State.allocate(g)
    s.load(init)
    qd = [g.upload(q, nz) for q in init["q"]]
    oi = _fp32(init, "mixed")
    ak, bk = fi.hybrid_coefficients(nz, g.ptop)
    print("remap C192x79 mixed", flush=True)
    fv3.remap(s, g, ak, bk, qd)
    assert fv3.check_status(g) == 0
    torch.cuda.synchronize()
    out = {k: s.get(k) for k in ("u", "v", "w", "pt", "delz", "delp")}
    qo = [g.download(q, nz) for q in qd]
    rng = np.random.default_rng(17)
    ptop = g.ptop
    dp = oi["delp"]

    def pe_of(t, j, i):
        return ptop + np.concatenate([[0.0], np.cumsum(dp[t, :, j + H, i + H])])

    worst = {}
    for _ in range(48):
        t, j, i = int(rng.integers(6)), int(rng.integers(n)), int(rng.integers(n))
        pe1 = pe_of(t, j, i)
        pe2 = ak + bk * pe1[-1]
        cols = {"pt": oi["pt"], "w": oi["w"], "q0": oi["q"][0], "q1": oi["q"][1]}
        for k, f in cols.items():
            want = orc.remap_column(pe1, pe2, f[t, :, j + H, i + H])
            got = out[k][t, :, j + H, i + H] if k[0] != "q" else qo[int(k[1])][t, :, j + H, i + H]
            worst[k] = max(worst.get(k, 0.0), float(np.abs(got - want).max() / np.abs(want).max()))
        ratio = oi["delz"][t, :, j + H, i + H] / dp[t, :, j + H, i + H]
        want = orc.remap_column(pe1, pe2, ratio) * np.diff(pe2)
        got = out["delz"][t, :, j + H, i + H]
        worst["delz"] = max(worst.get("delz", 0.0), float(np.abs(got - want).max() / np.abs(want).max()))
        got = out["delp"][t, :, j + H, i + H]
        worst["delp"] = max(worst.get("delp", 0.0), float(np.abs(got - np.diff(pe2)).max() / np.diff(pe2).max()))
    for k, (dj, di, ni, nj) in {"u": (-1, 0, n, n + 1), "v": (0, -1, n + 1, n)}.items():
        for _ in range(24):
            t, j, i = int(rng.integers(6)), int(rng.integers(nj)), int(rng.integers(ni))
            if (j + dj < 0) or (i + di < 0):
                continue   # the second cell is a halo cell of another tile: covered at small sizes
            pa, pb = pe_of(t, j, i), pe_of(t, j + dj, i + di)
            pe1 = 0.5 * (pa + pb)
            pe2 = ak + bk * pe1[-1]
            want = orc.remap_column(pe1, pe2, oi[k][t, :, j + H, i + H])
            got = out[k][t, :, j + H, i + H]
            worst[k] = max(worst.get(k, 0.0), float(np.abs(got - want).max() / np.abs(want).max()))
    print({k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    for k, e in worst.items():
        assert e <= (1e-12 if k == "delz" else 2.5e-7), (k, e)


# ------------------------------------------------------------ remapping loop
@pytest.mark.parametrize("kind,n,nz,bdt,k_split,n_split", [(0, 48, 8, 0.2, 3, 4), (1, 24, 10, 200.0, 2, 5)])
def test_dynamics_loop_matches_oracle(fv3, orc, kind, n, nz, bdt, k_split, n_split):
    """fv3_dynamics (k_split x (n_split substeps, tracer transport, remap))
    against the oracle running the same loop, FP64: bar 1e-11 per field
    (the substep bar; the remap adds ~1e-14) and tracer masses conserved by
    the device to 1e-13 on the periodic grid."""
    import torch

    init = fi.periodic_state(n=n, nz=nz, nq=2) if kind == 0 else fi.cube_state(n=n, nz=nz, nq=2)
    ak, bk = fi.hybrid_coefficients(nz, 100.0)
    dt = bdt * n_split * k_split
    g = fv3.Grid(kind, n, nz)
    s = fv3.State.allocate(g)
    s.load(init)
    qd = [g.upload(q, nz) for q in init["q"]]
    m0 = fv3.mass_sums(g, s.f["delp"], s.f["pt"], qd)
    fv3.dynamics(s, g, qd, ak, bk, dt, k_split, n_split)
    torch.cuda.synchronize()
    assert fv3.check_status(g) == 0
    m1 = fv3.mass_sums(g, s.f["delp"], s.f["pt"], qd)
    og = orc.Grid(kind, n, nz)
    os_ = orc.new_state(og, init)
    qh = [q.copy() for q in init["q"]]
    assert orc.dynamics(og, os_, qh, ak, bk, dt, k_split, n_split) == 0
    errs = {k: _relerr(_int(s.get(k), n, st), _int(os_[k], n, st)) for k, st in VIEWS.items()}
    for m, (a, b) in enumerate(zip(qd, qh)):
        errs[f"q{m}"] = _relerr(_int(g.download(a, nz), n, "C"), _int(b, n, "C"))
    print(f"dynamics kind{kind} C{n}x{nz} k_split {k_split} n_split {n_split}",
          {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= 1e-11, (k, e)
    if kind == 0:
        rel = np.abs(m1 - m0) / np.abs(m0)
        assert np.all(rel <= 1e-13), rel
    # the state ends on the reference interfaces: delp = the reference thickness
    ps = 100.0 + _int(os_["delp"], n, "C").sum(axis=1)
    dref = (np.diff(ak)[None, :, None, None] + np.diff(bk)[None, :, None, None] * ps[:, None])
    assert np.abs(_int(s.get("delp"), n, "C") - dref).max() <= 1e-9 * np.abs(dref).max()


def test_dynamics_errors(fv3):
    g = fv3.Grid(0, 16, 2)
    s = fv3.State.allocate(g)
    s.load(fi.periodic_state(n=16, nz=2, nq=0))
    ak, bk = fi.hybrid_coefficients(2, 100.0)
    with pytest.raises(fv3.FV3Error) as e:
        fv3.dynamics(s, g, [], ak, bk, 1.0, 0, 2)
    assert e.value.status == -1
    bad = ak.copy()
    bad[0] = 50.0
    with pytest.raises(fv3.FV3Error) as e:
        fv3.dynamics(s, g, [], bad, bk, 1.0, 1, 2)
    assert e.value.status == -1
