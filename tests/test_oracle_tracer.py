"""Pins of the oracle's tracer transport (tracer advection of the remapping
step, Sec. II) with the fluxes accumulated over the acoustic substeps:
tracer mass conserved to 1e-14, a constant tracer stays constant, Courant
number 1 shifts the field by exactly one cell, the sub-cycle count keeps a
Courant number of exactly 1 in one sub-cycle and splits 1.5 into two."""
import numpy as np
import pytest

import fv3_inputs as fi

H = 3


@pytest.fixture(scope="module")
def run(orc):
    g = orc.Grid(0, 48, 8)
    init = fi.periodic_state(nq=2)
    s = orc.new_state(g, init)
    assert orc.acoustic_substeps(g, s, 2.0, 10) == 0
    return g, init, s


def test_tracer_mass_conserved(orc, run):
    g, init, s = run
    qs = [q.copy() for q in init["q"]]
    m0 = orc.mass_sums(g, s["dp0"], s["pt"], qs)[2:]
    used = orc.tracer_transport(g, qs, s["dp0"], s["mfx"], s["mfy"], s["cx"], s["cy"])
    assert used >= 1
    m1 = orc.mass_sums(g, s["delp"], s["pt"], qs)[2:]
    assert np.all(np.abs(m1 - m0) <= 1e-14 * np.abs(m0))
    assert np.abs(qs[0] - init["q"][0])[0, :, H:H + 48, H:H + 48].max() > 1e-4


def test_constant_tracer_preserved(orc, run):
    g, init, s = run
    q = g.field(g.nz)
    q[:] = 0.7
    orc.tracer_transport(g, [q], s["dp0"], s["mfx"], s["mfy"], s["cx"], s["cy"])
    np.testing.assert_allclose(q[0, :, H:H + 48, H:H + 48], 0.7, rtol=1e-14, atol=0)


def _uniform(orc, n, nz, cx, cy):
    g = orc.Grid(0, n, nz)
    dp0 = g.field(nz)
    dp0[:] = 1000.0
    A = 1000.0 * 1000.0
    CX, CY = g.field(nz), g.field(nz)
    CX[:] = cx
    CY[:] = cy
    return g, dp0, CX * dp0 * A, CY * dp0 * A, CX, CY


def test_courant_one_shift(orc):
    n, nz = 12, 2
    g, dp0, mfx, mfy, cx, cy = _uniform(orc, n, nz, 1.0, 0.0)
    q = g.field(nz)
    rng = np.random.default_rng(5)
    q0 = rng.random((nz, n, n))
    q[0, :, H:H + n, H:H + n] = q0
    used = orc.tracer_transport(g, [q], dp0, mfx, mfy, cx, cy)
    assert used == 1
    np.testing.assert_allclose(q[0, :, H:H + n, H:H + n], np.roll(q0, 1, axis=2), rtol=0, atol=1e-15)
    g, dp0, mfx, mfy, cx, cy = _uniform(orc, n, nz, 1.0, -1.0)
    q[0, :, H:H + n, H:H + n] = q0
    orc.tracer_transport(g, [q], dp0, mfx, mfy, cx, cy)
    np.testing.assert_allclose(q[0, :, H:H + n, H:H + n], np.roll(q0, (-1, 1), axis=(1, 2)),
                               rtol=0, atol=1e-15)


def test_subcycle_count(orc):
    n, nz = 12, 1
    g, dp0, mfx, mfy, cx, cy = _uniform(orc, n, nz, 1.5, 0.2)
    q = g.field(nz)
    q[0, :, H:H + n, H:H + n] = np.random.default_rng(1).random((nz, n, n))
    assert orc.tracer_transport(g, [q], dp0, mfx, mfy, cx, cy) == 2
    assert orc.tracer_transport(g, [q], dp0, mfx, mfy, cx, cy, nsplt=3) == 3
