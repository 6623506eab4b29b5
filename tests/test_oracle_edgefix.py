"""Pins of the oracle's edge-flux fix-up on the cube (each face on a tile
edge is stored by both tiles; after each flux-form transport both fluxes are
replaced by their mean and the cells next to the edge take the difference):
the global sums of delp, pt delp and the tracer masses are then exact over
10 substeps and a tracer transport (without the fix they drift by ~1e-8);
the accumulated mass fluxes of the two copies of every shared face agree;
a constant tracer stays constant; only cells next to tile edges change; the
doubly periodic grid is untouched; the partner map is an involution."""
import numpy as np
import pytest

import fv3_inputs as fi

H = 3


def _run(orc, ef, n=16, nz=6, dt=2000.0, ns=10, stop=0, nq=2):
    init = fi.cube_state(n=n, nz=nz, nq=nq)
    g = orc.Grid(1, n, nz, delta=1.0e5, edge_fix=ef)
    s = orc.new_state(g, init)
    assert orc.acoustic_substeps(g, s, dt, ns, stop_stage=stop) == 0
    return g, init, s


def test_partner_map_is_an_involution(orc):
    n = 8
    g = orc.Grid(1, n, 1, delta=1.0e5)
    area = g.metric("dx")
    for t in range(6):
        for st, faces in (("X", [(0, j) for j in range(n)] + [(n, j) for j in range(n)]),
                          ("Y", [(i, 0) for i in range(n)] + [(i, n) for i in range(n)])):
            for i, j in faces:
                tp, stp, ip, jp, sg = orc.edge_partner(g, t, st, i, j)
                assert tp != t and sg in (-1, 1)
                assert (ip in (0, n)) if stp == "X" else (jp in (0, n))
                back = orc.edge_partner(g, tp, stp, ip, jp)
                assert back == (t, st, i, j, sg)


def test_exact_conservation_on_the_cube(orc):
    sums = {}
    for ef in (False, True):
        g, init, s = _run(orc, ef)
        m0 = orc.mass_sums(g, s["dp0"], init["pt"], init["q"])
        mp = orc.mass_sums(g, s["delp"], s["pt"])
        qs = [q.copy() for q in init["q"]]
        orc.tracer_transport(g, qs, s["dp0"], s["mfx"], s["mfy"], s["cx"], s["cy"])
        mq = orc.mass_sums(g, s["delp"], s["pt"], qs)
        sums[ef] = (np.abs(mp[0] / m0[0] - 1), np.abs(mq[2:] / m0[2:] - 1).max())
    # the initial pt delp sum: pt at entry times dp0
    assert sums[True][0] <= 1e-14 and sums[True][1] <= 1e-14, sums
    assert sums[False][0] > 1e-10 and sums[False][1] > 1e-10, sums


def test_pt_mass_exact(orc):
    g, init, s = _run(orc, True)
    a0 = orc.mass_sums(g, s["dp0"], init["pt"])[1]
    a1 = orc.mass_sums(g, s["delp"], s["pt"])[1]
    assert abs(a1 / a0 - 1) <= 1e-14


def test_shared_face_mass_fluxes_agree(orc):
    n = 12
    g, init, s = _run(orc, True, n=n, ns=3)
    worst = 0.0
    for t in range(6):
        for k in range(g.nz):
            for i, j in [(0, j) for j in range(n)] + [(n, j) for j in range(n)]:
                tp, stp, ip, jp, sg = orc.edge_partner(g, t, "X", i, j)
                a = s["mfx"][t, k, H + j, H + i]
                b = (s["mfx"] if stp == "X" else s["mfy"])[tp, k, H + jp, H + ip] * sg
                worst = max(worst, abs(a - b) / abs(s["mfx"]).max())
    assert worst <= 1e-15, worst


def test_constant_tracer_stays_constant(orc):
    g, init, s = _run(orc, True, ns=4)
    q = g.field(g.nz)
    q[:] = 0.37
    orc.tracer_transport(g, [q], s["dp0"], s["mfx"], s["mfy"], s["cx"], s["cy"])
    np.testing.assert_allclose(q[:, :, H:H + 16, H:H + 16], 0.37, rtol=1e-13, atol=0)


def test_only_edge_cells_change(orc):
    n = 12
    _, _, a = _run(orc, False, n=n, ns=1, stop=6)
    _, _, b = _run(orc, True, n=n, ns=1, stop=6)
    inner = (slice(None), slice(None), slice(H + 1, H + n - 1), slice(H + 1, H + n - 1))
    for k in ("delp", "pt", "w"):
        np.testing.assert_array_equal(a[k][inner], b[k][inner])
    for k in ("delp", "pt"):     # w starts at 0 and carries no flux in the first d_sw
        assert np.abs(a[k][..., H:H + n, H:H + n] - b[k][..., H:H + n, H:H + n]).max() > 0, k


def test_periodic_grid_untouched(orc):
    init = fi.periodic_state(n=16, nz=4, nq=1)
    out = []
    for ef in (False, True):
        g = orc.Grid(0, 16, 4, edge_fix=ef)
        s = orc.new_state(g, init)
        assert orc.acoustic_substeps(g, s, 2.0, 5) == 0
        qs = [init["q"][0].copy()]
        orc.tracer_transport(g, qs, s["dp0"], s["mfx"], s["mfy"], s["cx"], s["cy"])
        out.append((s["delp"].copy(), s["pt"].copy(), qs[0]))
    for x, y in zip(*out):
        np.testing.assert_array_equal(x, y)
