"""Batched ensemble: uneven members run by one launch per kernel must equal
their standalone runs bit for bit (the same device code computes every
point), with and without a captured HIP graph and after block shapes are
retuned; one member is also held against the oracle."""
import numpy as np
import pytest

import fv3_inputs as fi

pytestmark = pytest.mark.gpu
H = 3
FIELDS = ("u", "v", "w", "delp", "pt", "delz", "uc", "vc", "mfx", "mfy", "cx", "cy", "dp0", "pfull",
          "phi")
# (kind, n, nz) of uneven members
MEMBERS = [(0, 24, 5), (0, 40, 8), (0, 16, 3), (0, 64, 6)]


@pytest.fixture(scope="module")
def fv3():
    import torch

    import paper_2205_04148_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def _init(kind, n, nz, seed):
    return fi.periodic_state(n=n, nz=nz, seed=seed) if kind == 0 else fi.cube_state(n=n, nz=nz, seed=seed)


def _make(fv3, precision, members=MEMBERS, dx=1000.0):
    grids, states, inits = [], [], []
    for q, (kind, n, nz) in enumerate(members):
        g = fv3.Grid(kind, n, nz, dx=dx, precision=precision)
        s = fv3.State.allocate(g)
        init = _init(kind, n, nz, 20 + q)
        s.load(init)
        grids.append(g)
        states.append(s)
        inits.append(init)
    return grids, states, inits


def _snap(s):
    return {k: s.get(k) for k in FIELDS}


def _equal(a, b, label):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k], equal_nan=True), (label, k, float(np.nanmax(np.abs(a[k] - b[k]))))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_equals_standalone(fv3, precision):
    import torch

    dt, ns = 0.8, 2
    grids, states, inits = _make(fv3, precision)
    fv3.acoustic_substeps_batched(states, grids, dt, ns)
    got = [_snap(s) for s in states]
    for q, (g, init) in enumerate(zip(grids, inits)):
        s = fv3.State.allocate(g)
        s.load(init)
        fv3.acoustic_substeps(s, g, dt, ns)
        torch.cuda.synchronize()
        _equal(got[q], _snap(s), f"member {q}")
        assert fv3.check_status(g) == 0


def test_cube_member_and_oracle(fv3, orc):
    """A cube member among periodic ones (100 km spacing, so that one substep
    length suits all): every member equals its standalone run, and each kind
    of member matches the oracle (1e-11; w 1e-10, the column-solve bar of the
    stage parity tests)."""
    import torch

    members = [(0, 24, 4), (1, 12, 4), (0, 32, 4)]
    dt, ns, dx = 400.0, 2, 1.0e5
    grids, states, inits = _make(fv3, "fp64", members, dx=dx)
    fv3.acoustic_substeps_batched(states, grids, dt, ns)
    torch.cuda.synchronize()
    for q, (g, init) in enumerate(zip(grids, inits)):
        s = fv3.State.allocate(g)
        s.load(init)
        fv3.acoustic_substeps(s, g, dt, ns)
        torch.cuda.synchronize()
        _equal(_snap(states[q]), _snap(s), f"member {q}")
        assert fv3.check_status(g) == 0
    for q in (0, 1):
        kind, n, nz = members[q]
        og = orc.Grid(kind, n, nz, delta=dx)
        os_ = orc.new_state(og, inits[q])
        assert orc.acoustic_substeps(og, os_, dt, ns) == 0
        for k, (nj, ni) in {"u": (n + 1, n), "v": (n, n + 1), "w": (n, n), "delp": (n, n), "pt": (n, n),
                            "delz": (n, n)}.items():
            a = states[q].get(k)[..., H:H + nj, H:H + ni]
            b = os_[k][..., H:H + nj, H:H + ni]
            e = float(np.abs(a - b).max() / np.abs(b).max())
            print(f"member {q} {k}: {e:.2e}", flush=True)
            assert e <= (3e-11 if k == "w" else 1e-11), (q, k, e)


def test_graph_replays_match_eager(fv3):
    """Three replays of the captured call, with eager library work and
    synchronisations between them, each equal to the eager ensemble."""
    import torch

    members = [(0, 24, 5), (0, 16, 3), (0, 40, 4)]
    ga, sa, _ = _make(fv3, "fp64", members)
    gb, sb, _ = _make(fv3, "fp64", members)
    ea = fv3.Ensemble(sa, ga, 0.8, 2, graph=False)
    eb = fv3.Ensemble(sb, gb, 0.8, 2, graph=True)
    for rep in range(3):
        ea.run()
        eb.run()
        torch.cuda.synchronize()
        fv3.halo_fill(ga[0], [sa[0].f["pt"]], ga[0].nz)     # eager work between replays
        fv3.halo_fill(gb[0], [sb[0].f["pt"]], gb[0].nz)
        torch.cuda.synchronize()
        for q in range(len(members)):
            _equal(_snap(sa[q]), _snap(sb[q]), f"replay {rep} member {q}")


def test_tuning_keeps_results_and_reuses(fv3):
    import torch

    members = [(0, 24, 5), (0, 40, 8), (0, 16, 3)]
    # tune on scratch copies
    gs, ss, _ = _make(fv3, "fp64", members)
    e = fv3.Ensemble(ss, gs, 0.8, 2)
    rep = e.tune(reps=2)
    print("tune report:", rep, flush=True)
    assert rep["tunable_sites"] > 0 and rep["searched"] + rep["reused"] == rep["tunable_sites"]
    assert rep["reused"] > 0 and rep["search_ms"] > 0
    shapes = e.shapes()
    assert all(bx * by in (256,) for _, bx, by in shapes)
    # a new ensemble finds every plane kernel in the cache
    gt, st, _ = _make(fv3, "fp64", members)
    e2 = fv3.Ensemble(st, gt, 0.8, 2)
    rep2 = e2.tune(reps=1)
    assert rep2["searched"] == 0 and rep2["reused"] == rep2["tunable_sites"]
    # tuned shapes: still bit-identical to the standalone runs
    gr, sr, inits = _make(fv3, "fp64", members)
    e3 = fv3.Ensemble(sr, gr, 0.8, 2, graph=True)
    e3.run()
    torch.cuda.synchronize()
    for q, (g, init) in enumerate(zip(gr, inits)):
        s = fv3.State.allocate(g)
        s.load(init)
        fv3.acoustic_substeps(s, g, 0.8, 2)
        torch.cuda.synchronize()
        _equal(_snap(sr[q]), _snap(s), f"tuned member {q}")


def test_ensemble_errors(fv3):
    g1 = fv3.Grid(0, 16, 3, precision="fp64")
    g2 = fv3.Grid(0, 16, 3, precision="mixed")
    s1, s2 = fv3.State.allocate(g1), fv3.State.allocate(g2)
    with pytest.raises(fv3.FV3Error) as e:
        fv3.acoustic_substeps_batched([s1, s2], [g1, g2], 1.0, 2)
    assert e.value.status == -3
    with pytest.raises(fv3.FV3Error):
        fv3.acoustic_substeps_batched([s1], [g1], -1.0, 2)
    # a member whose options choose other kernels (tile-edge PPM on a cube,
    # a different PPM order) is refused with its own status
    for opts in ({"edge_ppm": True}, {"hord": 6}):
        g3 = fv3.Grid(1, 12, 3, precision="fp64", **opts)
        g4 = fv3.Grid(1, 12, 3, precision="fp64")
        s3, s4 = fv3.State.allocate(g3), fv3.State.allocate(g4)
        with pytest.raises(fv3.FV3Error) as e:
            fv3.acoustic_substeps_batched([s4, s3], [g4, g3], 1.0, 2)
        assert e.value.status == -8, opts
