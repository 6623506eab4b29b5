"""Pins of the synthetic initial states (the analytic baroclinic-instability
jet of the paper's test case, Sec. X, and the isothermal periodic column):
closed-form values, hydrostatic and gradient-wind balance of the jet, and a
zero discrete nonhydrostatic perturbation of the generated columns."""
import math

import numpy as np
import pytest

import fv3_inputs as fi

H = 3


def test_jet_closed_form_values():
    jet = fi.BaroclinicJet()
    assert abs(jet.temperature(0.0, 0.0) - 310.0) <= 1e-12
    assert abs(jet.temperature(math.pi / 2, 0.0) - 240.0) <= 1e-12
    for lat in (-1.2, -0.3, 0.0, 0.7, 1.4):
        assert abs(jet.pressure(lat, 0.0) - 1.0e5) <= 1e-9
    assert abs(jet.zonal_wind(0.0, 5000.0)) <= 1e-9
    assert abs(jet.zonal_wind(math.pi / 2, 5000.0)) <= 1e-6
    u45 = jet.zonal_wind(math.radians(45.0), 10000.0)
    assert 20.0 < u45 < 40.0


def test_jet_hydrostatic_balance():
    jet = fi.BaroclinicJet()
    for lat in (0.1, 0.6, 1.1):
        for z in (500.0, 5000.0, 15000.0):
            h = 0.5
            dpdz = (jet.pressure(lat, z + h) - jet.pressure(lat, z - h)) / (2 * h)
            rhs = -fi.GRAV * jet.pressure(lat, z) / (fi.RDGAS * jet.temperature(lat, z))
            assert abs(dpdz - rhs) <= 1e-7 * abs(rhs)


def test_jet_gradient_wind_balance():
    jet = fi.BaroclinicJet()
    a, om = fi.RADIUS, fi.OMEGA
    for lat in (0.3, 0.8, 1.2):
        for z in (1000.0, 8000.0):
            h = 1e-5
            dpdl = (jet.pressure(lat + h, z) - jet.pressure(lat - h, z)) / (2 * h)
            u = jet.zonal_wind(lat, z)
            rho = jet.pressure(lat, z) / (fi.RDGAS * jet.temperature(lat, z))
            lhs = u * u * math.tan(lat) / a + 2 * om * math.sin(lat) * u
            rhs = -dpdl / (rho * a)
            assert abs(lhs - rhs) <= 1e-6 * (abs(rhs) + 1e-6)


def _discrete_pprime(delp, pt, delz, ptop):
    nz = delp.shape[0]
    pi = ptop + np.concatenate([np.zeros((1,) + delp.shape[1:]), np.cumsum(delp, axis=0)])
    pibar = delp / (np.log(pi[1:]) - np.log(pi[:-1]))
    m = delp / fi.GRAV
    gam = 1.0 / (1.0 - fi.KAPPA)
    p = fi.P0 * (fi.RDGAS * pt * m / (-delz * fi.P0)) ** gam
    return (p - pibar) / pibar


def test_periodic_columns_hydrostatic():
    s = fi.periodic_state(n=8, nz=8)
    n = 8
    rel = _discrete_pprime(s["delp"][0, :, H:H + n, H:H + n], s["pt"][0, :, H:H + n, H:H + n],
                           s["delz"][0, :, H:H + n, H:H + n], 100.0)
    assert np.max(np.abs(rel)) <= 1e-13
    # the duplicate periodic faces equal face 0
    np.testing.assert_array_equal(s["u"][0, :, H + n, H:H + n], s["u"][0, :, H, H:H + n])
    np.testing.assert_array_equal(s["v"][0, :, H:H + n, H + n], s["v"][0, :, H:H + n, H])


def test_cube_columns_hydrostatic_and_jet_shape():
    n, nz = 8, 10
    s = fi.cube_state(n=n, nz=nz, noise=0.0)
    rel = _discrete_pprime(s["delp"][:, :, H:H + n, H:H + n].transpose(1, 0, 2, 3),
                           s["pt"][:, :, H:H + n, H:H + n].transpose(1, 0, 2, 3),
                           s["delz"][:, :, H:H + n, H:H + n].transpose(1, 0, 2, 3), 100.0)
    assert np.max(np.abs(rel)) <= 1e-12
    # surface at z = 0: the column heights sum to the top height, all layers thin
    assert np.all(s["delz"][:, :, H:H + n, H:H + n] < 0)
    # the winds are bounded by the jet maximum
    assert np.abs(s["u"]).max() < 60.0
