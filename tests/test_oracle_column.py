"""Pins of the oracle's semi-implicit vertical solve (riem_solver_c /
riem_solver3, Sec. IX-B: nonhydrostatic w and pressure perturbation through a
tridiagonal solver) and of the finite-volume pressure-gradient force.

Pins: the Thomas elimination equals a dense LU solve of the same system; the
closed-form single-layer solution; a column at hydrostatic rest stays at rest;
the top-down scan of the new perturbation equals the implicitly linearised
interface pressure (so the returned w solves the discrete momentum equation);
the thickness inversion reproduces the new pressure through the equation of
state; all pivots positive; the pressure gradient is zero for identical
columns, equals -dt*dp/(rho*L) for a uniform offset, and is antisymmetric.
The cubic interface perturbation (pp_order 4): exact interface values of
cubic profiles on uneven layers, the 7/12, -1/12 weights on even ones, the
mass-linear rule where one side has a single layer, and its use in both
column solves of the substep."""
import math

import numpy as np
import pytest

G, RD, CP, P0 = 9.80665, 287.05, 1004.6, 1.0e5
KAPPA = RD / CP
GAM = 1.0 / (1.0 - KAPPA)


def _column(nz, rng, perturb=0.02):
    pi = np.linspace(100.0, 1.0e5, nz + 1)
    dpi = np.diff(pi)
    T = 250.0 + 50.0 * rng.random(nz)
    lnr = np.log(pi[1:] / pi[:-1])
    pibar = dpi / lnr
    theta = T * (P0 / pibar) ** KAPPA
    delz = -(RD * T / G) * lnr * (1.0 + perturb * rng.standard_normal(nz))
    w = rng.standard_normal(nz)
    return pi, dpi, theta, delz, w


def _assemble(dt, pi, dpi, theta, delz, w, pps=None):
    """Dense matrix of the implicit system, assembled from the discrete
    equations (interface pressure linearised in the new w); pps replaces the
    mass-linear interface perturbation when given."""
    nz = len(dpi)
    m = dpi / G
    h = -delz
    pibar = dpi / (np.log(pi[1:]) - np.log(pi[:-1]))
    p = P0 * (RD * theta * m / (h * P0)) ** GAM
    pp = p - pibar
    PPs = np.zeros(nz + 1)
    for K in range(1, nz):
        PPs[K] = (dpi[K] * pp[K - 1] + dpi[K - 1] * pp[K]) / (dpi[K - 1] + dpi[K])
    PPs[nz] = pp[nz - 1]
    if pps is not None:
        PPs = np.asarray(pps, dtype=float)
    d = np.zeros(nz + 1)
    d[1:nz] = 0.5 * (h[:-1] + h[1:])
    d[nz] = 0.5 * h[-1]
    A = np.zeros(nz + 1)
    A[1:] = GAM * (pi[1:] + PPs[1:]) * dt * dt / d[1:]
    M = np.zeros((nz, nz))
    rhs = m * w + dt * (PPs[1:] - PPs[:-1])
    for k in range(nz):
        M[k, k] = m[k] + A[k] + A[k + 1]
        if k > 0:
            M[k, k - 1] = -A[k]
        if k < nz - 1:
            M[k, k + 1] = -A[k + 1]
    return M, rhs, PPs, A, m, pibar


@pytest.mark.parametrize("nz", [1, 2, 3, 5, 8, 20])
def test_thomas_matches_dense_lu(orc, nz):
    rng = np.random.default_rng(100 + nz)
    for _ in range(5):
        pi, dpi, theta, delz, w = _column(nz, rng)
        dt = 7.5
        r = orc.sim1(dt, 100.0, 0.0, dpi, theta, delz, w)
        M, rhs, *_ = _assemble(dt, pi, dpi, theta, delz, w)
        wd = np.linalg.solve(M, rhs)
        assert np.max(np.abs(r["w"] - wd)) <= 1e-13 * max(1.0, np.max(np.abs(wd)))
        assert r["min_pivot"] > 0


def test_single_layer_closed_form(orc):
    rng = np.random.default_rng(9)
    pi, dpi, theta, delz, w = _column(1, rng, perturb=0.05)
    dt = 3.0
    r = orc.sim1(dt, 100.0, 0.0, dpi, theta, delz, w)
    m = dpi[0] / G
    h = -delz[0]
    pibar = dpi[0] / math.log(pi[1] / pi[0])
    pp0 = P0 * (RD * theta[0] * m / (h * P0)) ** GAM - pibar
    A1 = GAM * (pi[1] + pp0) * dt * dt / (0.5 * h)
    want = (m * w[0] + dt * pp0) / (m + A1)
    assert abs(r["w"][0] - want) <= 1e-14 * max(1.0, abs(want))


def test_rest_column_stays_at_rest(orc):
    nz = 12
    pi = np.linspace(100.0, 1.0e5, nz + 1)
    dpi = np.diff(pi)
    lnr = np.log(pi[1:] / pi[:-1])
    T = np.linspace(220.0, 300.0, nz)
    theta = T * (P0 / (dpi / lnr)) ** KAPPA
    delz = -(RD * T / G) * lnr
    r = orc.sim1(15.0, 100.0, 0.0, dpi, theta, delz, np.zeros(nz))
    assert np.max(np.abs(r["w"])) <= 1e-12
    np.testing.assert_allclose(r["delz"], delz, rtol=1e-14)
    # hydrostatic interfaces and heights
    np.testing.assert_allclose(r["pfull"], pi, rtol=1e-13)
    z = np.concatenate([np.cumsum(-delz[::-1])[::-1], [0.0]])
    np.testing.assert_allclose(r["phi"], G * z, rtol=1e-13, atol=1e-9)


def test_scanned_perturbation_is_linearised_interface_pressure(orc):
    rng = np.random.default_rng(21)
    for nz in (2, 5, 9):
        pi, dpi, theta, delz, w = _column(nz, rng)
        dt = 10.0
        r = orc.sim1(dt, 100.0, 0.0, dpi, theta, delz, w)
        M, rhs, PPs, A, m, pibar = _assemble(dt, pi, dpi, theta, delz, w)
        wn = r["w"]
        wext = np.concatenate([wn, [0.0]])                # surface w = 0
        Plin = PPs.copy()
        for K in range(1, nz + 1):
            Plin[K] = PPs[K] - (A[K] / dt) * (wext[K - 1] - wext[K])
        scanned = r["pfull"] - pi
        assert np.max(np.abs(scanned - Plin)) <= 1e-12 * np.max(np.abs(pi))


def test_thickness_inverts_equation_of_state(orc):
    rng = np.random.default_rng(31)
    nz = 6
    pi, dpi, theta, delz, w = _column(nz, rng)
    dt = 5.0
    r = orc.sim1(dt, 100.0, 0.0, dpi, theta, delz, w)
    pnew = 0.5 * (r["pfull"][:-1] + r["pfull"][1:]) - 0.5 * (pi[:-1] + pi[1:]) + dpi / np.log(pi[1:] / pi[:-1])
    m = dpi / G
    p_eos = P0 * (RD * theta * m / (-r["delz"] * P0)) ** GAM
    np.testing.assert_allclose(p_eos, pnew, rtol=1e-13)


def test_compressed_layer_pushes_outward(orc):
    # a squeezed middle layer has excess pressure: the layer above accelerates up,
    # the one below down
    nz = 5
    pi = np.linspace(100.0, 1.0e5, nz + 1)
    dpi = np.diff(pi)
    lnr = np.log(pi[1:] / pi[:-1])
    T = np.full(nz, 280.0)
    theta = T * (P0 / (dpi / lnr)) ** KAPPA
    delz = -(RD * T / G) * lnr
    delz[2] *= 0.99
    r = orc.sim1(2.0, 100.0, 0.0, dpi, theta, delz, np.zeros(nz))
    assert r["w"][1] > 0 and r["w"][3] < 0


def test_pgf_closed_forms(orc):
    dt, L = 20.0, 5.0e4
    # identical columns: exactly zero
    assert orc.pgf(dt, L, 900.0, 900.0, 5e4, 4e4, 5e4, 4e4, 3e4, 3.09e4, 3e4, 3.09e4) == 0.0
    # uniform offset of the east column's pressure: -dt * dp / (rho L)
    phi0, phi1, dpi, dp = 5.0e4, 4.9e4, 900.0, 37.0
    got = orc.pgf(dt, L, dpi, dpi, phi0, phi1, phi0, phi1, 3.0e4, 3.0e4 + dpi, 3.0e4 + dp, 3.0e4 + dpi + dp)
    rho = dpi / (phi0 - phi1)          # delta-pi / (g dz), with phi = g z
    want = -dt * dp / (rho * L)
    assert abs(got - want) <= 1e-13 * abs(want)
    assert got < 0                      # force toward the low pressure (west)
    # antisymmetric under exchange of the two columns
    args = (870.0, 910.0, 5.1e4, 4.0e4, 5.0e4, 4.1e4, 3.0e4, 3.09e4, 3.01e4, 3.1e4)
    a = orc.pgf(dt, L, *args)
    b = orc.pgf(dt, L, args[1], args[0], args[4], args[5], args[2], args[3], args[8], args[9], args[6], args[7])
    assert abs(a + b) <= 1e-15 * abs(a)


def test_long_step_limit_is_hydrostatic(orc):
    # backward Euler with a very long step relaxes the column to zero
    # nonhydrostatic perturbation (P'_{k+1} - P'_k = m dw/dt -> 0, P'_top = 0)
    rng = np.random.default_rng(41)
    pi, dpi, theta, delz, w = _column(7, rng, perturb=0.03)
    r = orc.sim1(1.0e7, 100.0, 0.0, dpi, theta, delz, np.zeros(7))
    pert = r["pfull"] - pi
    assert np.max(np.abs(pert)) <= 1e-6 * pi[-1]
    # w decays like (displacement needed to rebalance) / dt
    assert np.max(np.abs(r["w"])) * 1.0e7 <= 0.1 * np.max(np.abs(delz))


def _coupled_solution(dt, beta, dpi, w, pstar, coup):
    """Solve the off-centred defining equations directly, unknowns w^{n+1}
    (nz) and P^{n+1} at interfaces 1..nz (the top stays 0, the surface is
    rigid):  P_K + beta C_K (w_{K-1} - w_K) = P*_K - (1-beta) C_K (w^n_{K-1} - w^n_K)
    and  m_k (w_k - w^n_k)/dt = P^b_{k+1} - P^b_k,  P^b = beta P + (1-beta) P*."""
    nz = len(dpi)
    m = dpi / G
    N = 2 * nz
    M = np.zeros((N, N))
    b = np.zeros(N)
    wn = np.concatenate([w, [0.0]])
    for K in range(1, nz + 1):        # rows 0..nz-1: interface relation for P_K (column nz + K - 1)
        r = K - 1
        M[r, nz + K - 1] = 1.0
        M[r, K - 1] += beta * coup[K]
        if K < nz:
            M[r, K] += -beta * coup[K]
        b[r] = pstar[K] - (1.0 - beta) * coup[K] * (wn[K - 1] - wn[K])
    for k in range(nz):               # rows nz..2nz-1: momentum of layer k
        r = nz + k
        M[r, k] = m[k] / dt
        M[r, nz + k] -= beta          # P_{k+1}
        if k > 0:
            M[r, nz + k - 1] += beta  # P_k
        b[r] = m[k] * w[k] / dt + (1.0 - beta) * (pstar[k + 1] - pstar[k])
    x = np.linalg.solve(M, b)
    return x[:nz], np.concatenate([[0.0], x[nz:]])


@pytest.mark.parametrize("beta", [1.0, 0.9, 0.7, 0.5])
def test_offcentred_solve_equals_coupled_system(orc, beta):
    """The tridiagonal reduction (coupling scaled by beta^2, explicit part on
    the right-hand side, P^{n+1} recovered from the scanned P^b) equals the
    direct solution of the defining equations for w^{n+1} and P^{n+1}."""
    rng = np.random.default_rng(40)
    nz, dt = 12, 20.0
    pi, dpi, theta, delz, w = _column(nz, rng)
    r = orc.sim1(dt, pi[0], 0.0, dpi, theta, delz, w, beta=beta)
    w_ref, P_ref = _coupled_solution(dt, beta, dpi, w, r["pstar"], r["coupling"])
    assert np.abs(r["w"] - w_ref).max() <= 1e-10 * np.abs(w_ref).max()
    P_new = r["pfull"] - pi
    assert np.abs(P_new - P_ref).max() <= 1e-9 * np.abs(r["pfull"]).max()


@pytest.mark.parametrize("beta", [0.5, 0.75])
def test_offcentred_rest_column_stays_at_rest(orc, beta):
    rng = np.random.default_rng(41)
    nz = 10
    pi, dpi, theta, delz, _ = _column(nz, rng, perturb=0.0)
    r = orc.sim1(30.0, pi[0], 0.0, dpi, theta, delz, np.zeros(nz), beta=beta)
    ref = orc.sim1(30.0, pi[0], 0.0, dpi, theta, delz, np.zeros(nz), beta=1.0)
    # the discrete state is not exactly p' = 0 here; at rest with w = 0 the
    # off-centred and backward-Euler solves differ only through the scaling
    # of the same pressure imbalance, so both keep the thicknesses close
    assert np.abs(r["delz"] - delz).max() <= 1e-2 * np.abs(delz).max()
    assert np.isfinite(r["w"]).all() and np.isfinite(ref["w"]).all()


def test_offcentring_weight_changes_the_response(orc):
    """A squeezed layer: with beta < 1 part of the pressure response is
    explicit, so the new w differs from backward Euler (and the sign of the
    response is the same)."""
    rng = np.random.default_rng(42)
    nz = 10
    pi, dpi, theta, delz, _ = _column(nz, rng, perturb=0.0)
    dz = delz.copy()
    dz[5] *= 0.98
    a = orc.sim1(10.0, pi[0], 0.0, dpi, theta, dz, np.zeros(nz), beta=1.0)
    b = orc.sim1(10.0, pi[0], 0.0, dpi, theta, dz, np.zeros(nz), beta=0.6)
    assert np.sign(a["w"][4]) == np.sign(b["w"][4]) and np.sign(a["w"][6]) == np.sign(b["w"][6])
    assert np.abs(a["w"] - b["w"]).max() > 1e-6 * np.abs(a["w"]).max()


# ---- cubic interface perturbation (pp_order 4) --------------------------

def _cubic_means(coef, x):
    """Layer means of sum coef[q] s^q, s = x / 1e4, over the layers between
    the interfaces x, and the profile at the interfaces."""
    F = lambda xx: sum(c * 1e4 * (xx / 1e4) ** (q + 1) / (q + 1) for q, c in enumerate(coef))
    f = lambda xx: sum(c * (xx / 1e4) ** q for q, c in enumerate(coef))
    return (F(x[1:]) - F(x[:-1])) / np.diff(x), f(x)


def test_pp_interfaces_cubic_exact(orc):
    rng = np.random.default_rng(50)
    for _ in range(10):
        nz = 12
        dpi = rng.uniform(300.0, 3000.0, nz)
        x = np.concatenate([[0.0], np.cumsum(dpi)])
        coef = rng.normal(size=4) * (50.0, 30.0, 10.0, 5.0)
        pp, fx = _cubic_means(coef, x)
        got = orc.pp_interfaces(dpi, pp, order=4)
        scale = np.abs(pp).max()
        for K in range(2, nz - 1):
            assert abs(got[K] - fx[K]) <= 1e-11 * scale, (K, got[K], fx[K])
        for K in (1, nz - 1):
            want = (dpi[K] * pp[K - 1] + dpi[K - 1] * pp[K]) / (dpi[K - 1] + dpi[K])
            assert abs(got[K] - want) <= 1e-14 * scale
        assert got[0] == 0.0 and got[nz] == pp[nz - 1]
        two = orc.pp_interfaces(dpi, pp, order=2)
        mid = (dpi[1:] * pp[:-1] + dpi[:-1] * pp[1:]) / (dpi[:-1] + dpi[1:])
        np.testing.assert_allclose(two[1:nz], mid, rtol=1e-15, atol=1e-15 * scale)
        # the mass-linear rule is not exact for curved profiles
        assert np.abs(two[2:nz - 1] - fx[2:nz - 1]).max() > 1e-6 * scale


def test_pp_interfaces_even_layers(orc):
    rng = np.random.default_rng(51)
    pp = rng.normal(size=9)
    got = orc.pp_interfaces(np.full(9, 700.0), pp, order=4)
    for K in range(2, 8):
        want = 7 / 12 * (pp[K - 1] + pp[K]) - 1 / 12 * (pp[K - 2] + pp[K + 1])
        assert abs(got[K] - want) <= 1e-14 * np.abs(pp).max()


def test_cubic_interfaces_in_the_solve(orc):
    """With pp_order 4 the solve's P* is the cubic interface value of the
    equation-of-state perturbation, and the returned w solves the implicit
    system assembled with those interface values (dense solve)."""
    rng = np.random.default_rng(52)
    nz, dt = 14, 15.0
    pi, dpi, theta, delz, w = _column(nz, rng)
    pibar = dpi / (np.log(pi[1:]) - np.log(pi[:-1]))
    pp = P0 * (RD * theta * (dpi / G) / (-delz * P0)) ** GAM - pibar
    pps = orc.pp_interfaces(dpi, pp, order=4)
    r = orc.sim1(dt, pi[0], 0.0, dpi, theta, delz, w, pp_order=4)
    assert np.abs(r["pstar"] - pps).max() <= 1e-12 * np.abs(pps).max()
    M, rhs, *_ = _assemble(dt, pi, dpi, theta, delz, w, pps=pps)
    wd = np.linalg.solve(M, rhs)
    assert np.abs(r["w"] - wd).max() <= 1e-10 * np.abs(wd).max()
    r2 = orc.sim1(dt, pi[0], 0.0, dpi, theta, delz, w)
    assert np.abs(r["w"] - r2["w"]).max() > 1e-8 * np.abs(wd).max()


def test_cubic_interfaces_reach_both_solves(orc):
    """Substep threading: the C-grid solve is the first place the order acts
    (its interface pressure differs between the orders while the stages
    before it are bit-equal), and the D-grid solve's w equals the column
    solve with pp_order 4 applied to the state it receives."""
    import fv3_inputs as fi
    n, nz, dt = 12, 10, 300.0
    init = fi.cube_state(n=n, nz=nz, seed=3)
    dbg = {}
    for order in (2, 4):
        g = orc.Grid(1, n, nz, delta=1.0e5, pp_order=order)
        s = orc.new_state(g, init)
        st, d = orc.acoustic_substeps(g, s, dt, 1, stop_stage=3, debug=True)
        assert st == 0
        dbg[order] = d
    np.testing.assert_array_equal(dbg[2]["ptc"], dbg[4]["ptc"])
    assert np.abs(dbg[2]["pkc"] - dbg[4]["pkc"]).max() > 1e-8 * np.abs(dbg[2]["pkc"]).max()
    g = orc.Grid(1, n, nz, delta=1.0e5, pp_order=4)
    s7 = orc.new_state(g, init)
    assert orc.acoustic_substeps(g, s7, dt, 1, stop_stage=7) == 0
    s8 = orc.new_state(g, init)
    assert orc.acoustic_substeps(g, s8, dt, 1, stop_stage=8) == 0
    H = 3
    rng = np.random.default_rng(53)
    for _ in range(12):
        t, j, i = int(rng.integers(6)), int(rng.integers(n)) + H, int(rng.integers(n)) + H
        col = lambda k: s7[k][t, :, j, i]
        r = orc.sim1(dt, g.ptop, 0.0, col("delp"), col("pt"), col("delz"),
                     col("w"), pp_order=4)
        assert np.abs(r["w"] - s8["w"][t, :, j, i]).max() <= 1e-13 * max(np.abs(r["w"]).max(), 1e-30)
