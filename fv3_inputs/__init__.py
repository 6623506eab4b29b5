"""Seeded synthetic initial states for the FV3 acoustic-substep path.

These generators are shared by the oracle tests, the GPU parity tests, the
benchmark and the smoke check.  They hold no step of the substep method: they
only build initial conditions (hydrostatically balanced columns, an analytic
baroclinic jet, seeded noise) in a plain host layout

    field[t][k][j + H][i + H],   H = 3,   N = n + 2H + 1 points per side,

with halos left at zero.  Staggering: D-grid ``u`` on y-faces (point
(i+1/2, j), i in [0,n-1], j in [0,n]), ``v`` on x-faces (point (i, j+1/2),
i in [0,n], j in [0,n-1]), cell fields on i,j in [0,n-1].

Workloads (the paper's own test is the analytic baroclinic-instability case
of Sec. X, a uniform zonal jet with a perturbation; no dataset is involved):

* ``periodic_state`` -- doubly periodic isothermal 300 K column, evenly
  spaced sigma layers, winds 10 m/s plus N(0,1) noise, tracers U[0,1].
* ``cube_state`` -- cubed sphere, closed-form baroclinic jet (balanced zonal
  jet with temperature and surface pressure from the closed form), discretely
  hydrostatic columns, N(0,1) m/s noise on the covariant D-grid winds, four
  tracers U[0,1].
* ``ensemble_sizes`` -- the uneven member sizes of the batched ensemble.
* ``sigma_coefficients`` / ``hybrid_coefficients`` -- reference vertical
  coordinates pe_K = ak_K + bk_K ps for the remapping step, and
  ``deform_layers`` -- seeded redistribution of the layer thicknesses of
  every column (fixed column mass), standing in for Lagrangian deformation.
"""
from __future__ import annotations

import math

import numpy as np

H = 3

# Constants of the dry system (the library and the oracle hold their own copies).
GRAV = 9.80665
RDGAS = 287.05
CP_AIR = 1004.6
KAPPA = RDGAS / CP_AIR
P0 = 1.0e5
OMEGA = 7.2921e-5
RADIUS = 6.3712e6

# Cube face frames (centre c, first lattice axis e1, second e2), e1 x e2 = c.
# This table is a convention that the oracle, the library and this module
# each hold in their own code.
CUBE_FRAMES = (
    ((1, 0, 0), (0, 1, 0), (0, 0, 1)),
    ((0, 1, 0), (-1, 0, 0), (0, 0, 1)),
    ((0, 0, 1), (-1, 0, 0), (0, -1, 0)),
    ((-1, 0, 0), (0, -1, 0), (0, 0, 1)),
    ((0, -1, 0), (1, 0, 0), (0, 0, 1)),
    ((0, 0, -1), (0, 1, 0), (1, 0, 0)),
)


def sigma_interfaces(nz: int, ptop: float = 100.0, ps: float = 1.0e5) -> np.ndarray:
    """Hydrostatic interface pressures pi_K = ptop + (ps - ptop) K / nz."""
    K = np.arange(nz + 1, dtype=np.float64)
    return ptop + (ps - ptop) * K / nz


def _empty(T, nlev, n):
    N = n + 2 * H + 1
    return np.zeros((T, nlev, N, N), dtype=np.float64)


def periodic_state(n: int = 48, nz: int = 8, seed: int = 1, temp: float = 300.0,
                   wind: float = 10.0, ptop: float = 100.0, ps: float = 1.0e5,
                   nq: int = 1, temp_noise: float = 0.0) -> dict:
    """Doubly periodic isothermal state.

    Draw order with ``numpy.random.default_rng(seed)``: u noise (nz,n,n) on
    y-faces 0..n-1, v noise on x-faces 0..n-1, then the tracers (nq,nz,n,n),
    then (only if temp_noise > 0) a temperature perturbation (nz,n,n).  The
    duplicate periodic face n is set equal to face 0.
    """
    rng = np.random.default_rng(seed)
    N = n + 2 * H + 1
    s = {}
    u = _empty(1, nz, n)
    v = _empty(1, nz, n)
    un = wind + rng.standard_normal((nz, n, n))
    vn = wind + rng.standard_normal((nz, n, n))
    u[0, :, H:H + n, H:H + n] = un
    u[0, :, H + n, H:H + n] = un[:, 0, :]
    v[0, :, H:H + n, H:H + n] = vn
    v[0, :, H:H + n, H + n] = vn[:, :, 0]
    qs = rng.random((nq, nz, n, n))
    tnoise = rng.standard_normal((nz, n, n)) * temp_noise if temp_noise > 0 else None
    pi = sigma_interfaces(nz, ptop, ps)
    delp = _empty(1, nz, n)
    pt = _empty(1, nz, n)
    delz = _empty(1, nz, n)
    for k in range(nz):
        dpi = pi[k + 1] - pi[k]
        lnr = math.log(pi[k + 1] / pi[k])
        pibar = dpi / lnr
        T = np.full((n, n), temp) if tnoise is None else temp + tnoise[k]
        delp[0, k, H:H + n, H:H + n] = dpi
        pt[0, k, H:H + n, H:H + n] = T * (P0 / pibar) ** KAPPA
        delz[0, k, H:H + n, H:H + n] = -(RDGAS * T / GRAV) * lnr
    s.update(u=u, v=v, w=_empty(1, nz, n), delp=delp, pt=pt, delz=delz,
             phis=np.zeros((1, N, N)))
    qq = []
    for m in range(nq):
        q = _empty(1, nz, n)
        q[0, :, H:H + n, H:H + n] = qs[m]
        qq.append(q)
    s["q"] = qq
    s["meta"] = dict(kind=0, n=n, nz=nz, T=1, ptop=ptop)
    return s


# ---------------------------------------------------------------- cube state
def _gnomonic_corners(n: int) -> np.ndarray:
    """Unit-sphere corner points [t][J][I][xyz] for I,J in [0,n]."""
    idx = np.arange(n + 1)
    ta = np.tan((2 * idx - n) * math.pi / (4.0 * n))
    ta[0], ta[-1] = -1.0, 1.0
    out = np.zeros((6, n + 1, n + 1, 3))
    for t, (c, e1, e2) in enumerate(CUBE_FRAMES):
        c, e1, e2 = (np.asarray(x, dtype=np.float64) for x in (c, e1, e2))
        X = c[None, None, :] + ta[None, :, None] * e1[None, None, :] + ta[:, None, None] * e2[None, None, :]
        out[t] = X / np.linalg.norm(X, axis=-1, keepdims=True)
    return out


def _unit(x):
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


class BaroclinicJet:
    """Closed-form balanced baroclinic jet (deep-atmosphere form with shallow
    geometry) used by the paper's test case; constants as published for the
    test: T_E = 310 K, T_P = 240 K, lapse 0.005 K/m, K = 3, b = 2."""

    def __init__(self, te=310.0, tp=240.0, lapse=0.005, kexp=3, b=2.0):
        self.te, self.tp, self.lapse, self.K, self.b = te, tp, lapse, kexp, b
        self.t0 = 0.5 * (te + tp)
        self.A = 1.0 / lapse
        self.B = (self.t0 - tp) / (self.t0 * tp)
        self.C = 0.5 * (kexp + 2.0) * (te - tp) / (te * tp)
        self.Hs = RDGAS * self.t0 / GRAV

    def _tau(self, z):
        zeta = z / (self.b * self.Hs)
        e = np.exp(-zeta * zeta)
        ez = np.exp(self.lapse * z / self.t0)
        tau1 = ez / self.t0 + self.B * (1.0 - 2.0 * zeta * zeta) * e
        tau2 = self.C * (1.0 - 2.0 * zeta * zeta) * e
        itau1 = self.A * (ez - 1.0) + self.B * z * e
        itau2 = self.C * z * e
        return tau1, tau2, itau1, itau2

    def _FG(self, lat):
        c = np.cos(lat)
        K = self.K
        F = c ** K - K / (K + 2.0) * c ** (K + 2)
        G = K * (c ** (K - 1) - c ** (K + 1))
        return F, G

    def temperature(self, lat, z):
        tau1, tau2, _, _ = self._tau(z)
        F, _ = self._FG(lat)
        return 1.0 / (tau1 - tau2 * F)

    def pressure(self, lat, z):
        _, _, i1, i2 = self._tau(z)
        F, _ = self._FG(lat)
        return P0 * np.exp(-(GRAV / RDGAS) * i1 + (GRAV / RDGAS) * i2 * F)

    def zonal_wind(self, lat, z):
        _, _, _, i2 = self._tau(z)
        _, G = self._FG(lat)
        T = self.temperature(lat, z)
        U = (GRAV / RADIUS) * i2 * G * T
        rc = RADIUS * np.cos(lat)
        return -OMEGA * rc + np.sqrt(OMEGA * OMEGA * rc * rc + rc * U)

    def height_at_pressure(self, lat, p, tol=1e-9, maxit=60):
        """Solve p(lat, z) = p for z by Newton on ln p (dlnp/dz = -g/(Rd T))."""
        lat = np.asarray(lat, dtype=np.float64)
        p = np.broadcast_to(np.asarray(p, dtype=np.float64), lat.shape)
        z = -(RDGAS * self.t0 / GRAV) * np.log(p / P0)
        for _ in range(maxit):
            f = np.log(self.pressure(lat, z)) - np.log(p)
            dz = f / (-GRAV / (RDGAS * self.temperature(lat, z)))
            z = z - dz
            if np.max(np.abs(dz)) < tol:
                break
        return z


def cube_geometry(n: int) -> dict:
    """Cell-centre latitudes and the D-grid edge tangents/latitudes."""
    B = _gnomonic_corners(n)                              # [t][J][I][3]
    C = _unit(B[:, :-1, :-1] + B[:, 1:, :-1] + B[:, 1:, 1:] + B[:, :-1, 1:])   # [t][j][i]
    # y-faces (i, j): edge from B(i,j) to B(i+1,j)  -> arrays [t][j=0..n][i=0..n-1]
    my = _unit(B[:, :, :-1] + B[:, :, 1:])
    dy_ = B[:, :, 1:] - B[:, :, :-1]
    ey = _unit(dy_ - np.sum(dy_ * my, axis=-1, keepdims=True) * my)
    # x-faces (i, j): edge from B(i,j) to B(i,j+1) -> [t][j=0..n-1][i=0..n]
    mx = _unit(B[:, :-1, :] + B[:, 1:, :])
    dx_ = B[:, 1:, :] - B[:, :-1, :]
    ex = _unit(dx_ - np.sum(dx_ * mx, axis=-1, keepdims=True) * mx)
    return dict(C=C, my=my, ty=ey, mx=mx, tx=ex)


def _east(p):
    e = np.stack([-p[..., 1], p[..., 0], np.zeros_like(p[..., 0])], axis=-1)
    return _unit(e)


def _jet_base(n: int, nz: int, ptop: float) -> dict:
    """The deterministic (seed-independent) part of the cubed-sphere jet state,
    cached per (n, nz, ptop): layer pressures, thicknesses, potential
    temperature and the face winds of the balanced jet."""
    key = (n, nz, float(ptop))
    if key in _BASE_CACHE:
        return _BASE_CACHE[key]
    jet = BaroclinicJet()
    geo = cube_geometry(n)
    pi = sigma_interfaces(nz, ptop, P0)
    dpi = np.diff(pi)
    lnr = np.log(pi[1:] / pi[:-1])
    pibar = dpi / lnr
    delp = _empty(6, nz, n)
    pt = _empty(6, nz, n)
    delz = _empty(6, nz, n)

    latc = np.arcsin(np.clip(geo["C"][..., 2], -1, 1))      # [t][j][i]
    zI = np.stack([jet.height_at_pressure(latc, pi[K]) for K in range(nz + 1)], axis=1)
    zI[:, nz] = 0.0
    for k in range(nz):
        dz = zI[:, k + 1] - zI[:, k]
        Tbar = -GRAV * dz / (RDGAS * lnr[k])
        delz[:, k, H:H + n, H:H + n] = dz
        delp[:, k, H:H + n, H:H + n] = dpi[k]
        pt[:, k, H:H + n, H:H + n] = Tbar * (P0 / pibar[k]) ** KAPPA

    def face_wind(mid, tan):
        lat = np.arcsin(np.clip(mid[..., 2], -1, 1))
        e = _east(mid)
        proj = np.sum(e * tan, axis=-1)
        out = np.zeros((6, nz) + lat.shape[1:])
        for k in range(nz):
            z = jet.height_at_pressure(lat, pibar[k])
            out[:, k] = jet.zonal_wind(lat, z) * proj
        return out

    base = dict(delp=delp, pt=pt, delz=delz, uw=face_wind(geo["my"], geo["ty"]),
                vw=face_wind(geo["mx"], geo["tx"]), geo=geo)
    if len(_BASE_CACHE) >= 4:
        _BASE_CACHE.clear()
    _BASE_CACHE[key] = base
    return base


_BASE_CACHE: dict = {}


def cube_state(n: int = 96, nz: int = 79, seed: int = 2, ptop: float = 100.0, nq: int = 4,
               noise: float = 1.0, bumps: int = 0) -> dict:
    """Cubed-sphere baroclinic jet.

    Columns: for each cell centre, interface heights z_K with p(lat, z_K) =
    pi_K (sigma-uniform pi, flat surface at p0); delz_k = z_{K+1} - z_K, layer
    temperature from the hydrostatic relation over the layer, theta from the
    log-mean layer pressure, so the discrete nonhydrostatic perturbation is 0.
    Winds: covariant D-grid components V.e of the zonal jet at each edge, at
    the edge's latitude and the height of the layer's log-mean pressure, plus
    N(0, noise) drawn with ``default_rng(seed)`` (u then v, then tracers).
    ``bumps`` > 0 adds, after those draws, that many seeded Gaussian wind
    perturbations (centre uniform on the sphere, radius 600 km, amplitude
    U(2, 8) m/s, direction U(0, 2 pi), all levels), the large-scale
    variability of the learned-correction samples.
    """
    base = _jet_base(n, nz, ptop)
    geo = base["geo"]
    rng = np.random.default_rng(seed)
    u = _empty(6, nz, n)
    v = _empty(6, nz, n)
    uw = base["uw"] + noise * rng.standard_normal(base["uw"].shape)
    vw = base["vw"] + noise * rng.standard_normal(base["vw"].shape)
    qs = rng.random((nq, 6, nz, n, n))
    for _ in range(bumps):
        c = rng.standard_normal(3)
        c /= np.linalg.norm(c)
        amp = rng.uniform(2.0, 8.0)
        ang = rng.uniform(0.0, 2 * np.pi)
        east = _east(c[None])[0]
        north = np.cross(c, east)
        d = math.cos(ang) * east + math.sin(ang) * north       # bump wind direction at its centre
        for w, mid, tan in ((uw, geo["my"], geo["ty"]), (vw, geo["mx"], geo["tx"])):
            dist = np.arccos(np.clip(np.sum(mid * c, axis=-1), -1, 1)) * RADIUS
            vec = d - np.sum(mid * d, axis=-1, keepdims=True) * mid   # transported to the face
            w += (amp * np.exp(-(dist / 6.0e5) ** 2) * np.sum(vec * tan, axis=-1))[:, None]
    u[:, :, H:H + n + 1, H:H + n] = uw
    v[:, :, H:H + n, H:H + n + 1] = vw
    qq = []
    for m in range(nq):
        q = _empty(6, nz, n)
        q[:, :, H:H + n, H:H + n] = qs[m]
        qq.append(q)
    return dict(u=u, v=v, w=_empty(6, nz, n), delp=base["delp"].copy(), pt=base["pt"].copy(),
                delz=base["delz"].copy(), phis=np.zeros((6, n + 2 * H + 1, n + 2 * H + 1)), q=qq,
                meta=dict(kind=1, n=n, nz=nz, T=6, ptop=ptop))


def sigma_coefficients(nz: int, ptop: float = 100.0):
    """Evenly spaced sigma layers: ak_K = ptop (1 - K/nz), bk_K = K/nz, so that
    ak + bk ps reproduces ``sigma_interfaces(nz, ptop, ps)``."""
    eta = np.arange(nz + 1, dtype=np.float64) / nz
    ak = ptop * (1.0 - eta)
    bk = eta.copy()
    ak[-1], bk[-1] = 0.0, 1.0
    return ak, bk


def hybrid_coefficients(nz: int, ptop: float = 100.0, ps0: float = 1.0e5, eta_c: float = 0.3):
    """Hybrid pressure-sigma interfaces: pure pressure above eta_c, bk rising
    quadratically to 1 below; at ps = ps0 the interfaces are evenly spaced.
    Interfaces increase downwards for every ps above about ps0 - (ps0 - ptop)
    (1 - eta_c) / 2."""
    eta = np.arange(nz + 1, dtype=np.float64) / nz
    bk = np.clip((eta - eta_c) / (1.0 - eta_c), 0.0, None) ** 2
    ak = ptop + (ps0 - ptop) * eta - bk * ps0
    ak[0], bk[0] = ptop, 0.0
    ak[-1], bk[-1] = 0.0, 1.0
    return ak, bk


def deform_layers(delp: np.ndarray, seed: int = 9, amp: float = 0.25) -> np.ndarray:
    """Redistribute each column's layer thicknesses by seeded factors in
    [1 - amp, 1 + amp] (smooth in k, random per column), keeping the column
    sum.  Works on any [T][K][N][N] array; returns a new array."""
    rng = np.random.default_rng(seed)
    T, K, N, _ = delp.shape
    k = np.arange(K, dtype=np.float64)[None, :, None, None]
    ph = rng.uniform(0.0, 2.0 * math.pi, size=(T, 1, N, N))
    wav = rng.uniform(1.0, 3.0, size=(T, 1, N, N))
    f = 1.0 + amp * np.sin(wav * 2.0 * math.pi * k / K + ph)
    out = delp * f
    tot0 = delp.sum(axis=1, keepdims=True)
    tot1 = out.sum(axis=1, keepdims=True)
    return out * np.where(tot1 != 0.0, tot0 / np.where(tot1 != 0.0, tot1, 1.0), 1.0)


def ensemble_sizes(members: int = 32, seed: int = 4):
    """Uneven (n, nz) of the batched ensemble: n in 64..256 step 16, nz in [32, 79]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(members):
        n = 16 * int(rng.integers(4, 17))
        nz = int(rng.integers(32, 80))
        out.append((n, nz))
    return out


def interior(a: np.ndarray, stagger: str, n: int) -> np.ndarray:
    """Interior view of a [T][K][N][N] (or [T][N][N]) array for a staggering."""
    ni = n + 1 if stagger in ("X", "B") else n
    nj = n + 1 if stagger in ("Y", "B") else n
    return a[..., H:H + nj, H:H + ni]
