"""FV3 acoustic-substep ORACLE: test infrastructure only.

A plain FP64 CPU implementation (C, built with ``-O2 -ffp-contract=off``)
of the acoustic substep loop, the tracer transport and the global mass sums,
wrapped with ctypes over numpy arrays in the oracle's own unpadded layout
``f[t][k][j+3][i+3]``.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the HIP library
never does, and the two share no code.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRCS = ["grid.c", "halo.c", "ppm.c", "column.c", "dyn.c", "remap.c", "api.c"]

ST = {"C": 0, "X": 1, "Y": 2, "B": 3}
MODE = {"x": 0, "y": 1}
PAIR = {"signed": 0, "abs": 1, "cos": 2}
METRICS = ["dx", "dy", "dxc", "dyc", "dxa", "dya", "area", "area_c", "fC", "fB", "sin_u",
           "cos_u", "sin_v", "cos_v", "sin_a", "cos_a", "cx", "cy", "cz", "bx", "by", "bz"]
H = 3
OMEGA = 7.2921e-5
RADIUS = 6.3712e6


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-o", _LIB] + [os.path.join(_HERE, s) for s in _SRCS] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_grid_new.restype = C.c_void_p
        L.orc_grid_new.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                   C.c_double, C.c_double, C.c_char_p, C.c_int]
        L.orc_grid_free.argtypes = [C.c_void_p]
        L.orc_set_damping.argtypes = [C.c_void_p, C.c_double]
        L.orc_set_beta.argtypes = [C.c_void_p, C.c_double]
        L.orc_set_smag.argtypes = [C.c_void_p, C.c_double]
        L.orc_smag_corner.argtypes = [C.c_void_p, C.c_int, dp, dp, C.c_double, dp]
        L.orc_sim1b.restype = C.c_double
        L.orc_sim1b.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double] + [dp] * 10
        L.orc_pp_interfaces.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        L.orc_set_pp_order.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_damp4.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.orc_set_vtdm.argtypes = [C.c_void_p, C.c_double]
        L.orc_set_edge_fix.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_edge_ppm.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_edge_interp.argtypes = [C.c_void_p, C.c_int]
        L.orc_interp.argtypes = [C.c_int, C.POINTER(C.c_double), C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_interp.restype = C.c_double
        L.orc_corner_values.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_corner_vort.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
        L.orc_ppm_face_edge.restype = C.c_double
        L.orc_ppm_face_edge.argtypes = [dp, dp, C.c_double, C.c_int, C.c_int, C.c_int]
        L.orc_edge_partner.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int)]
        L.orc_corner_div.argtypes = [C.c_void_p, C.c_int, dp, dp, dp]
        L.orc_corner_lap.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.orc_grid_metric.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_grid_conn.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_halo_fill.argtypes = [C.c_void_p, dp, C.c_int, C.c_int, C.c_int]
        L.orc_halo_fill_pair.argtypes = [C.c_void_p, dp, C.c_int, dp, C.c_int, C.c_int, C.c_int]
        L.orc_corner_view.argtypes = [C.c_void_p, dp, C.c_int, C.c_int, dp]
        L.orc_corner_view_pair.argtypes = [C.c_void_p, dp, C.c_int, dp, C.c_int, C.c_int, dp, dp]
        L.orc_ppm_face.restype = C.c_double
        L.orc_ppm_face.argtypes = [dp, C.c_double]
        L.orc_ppm_face_order.restype = C.c_double
        L.orc_ppm_face_order.argtypes = [dp, C.c_double, C.c_int]
        L.orc_set_hord.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_fv_tp_2d.argtypes = [C.c_void_p, C.c_int] + [dp] * 9
        L.orc_sim1.restype = C.c_double
        L.orc_sim1.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double] + [dp] * 8
        L.orc_pgf.restype = C.c_double
        L.orc_pgf.argtypes = [C.c_double] * 12
        L.orc_acoustic_substeps.argtypes = [C.c_void_p] + [dp] * 17 + [C.c_double, C.c_int,
                                                                      C.c_int, C.POINTER(dp)]
        L.orc_tracer_transport.argtypes = [C.c_void_p, C.POINTER(dp), C.c_int] + [dp] * 5 + [
            C.c_int, C.POINTER(C.c_int)]
        L.orc_mass_sums.argtypes = [C.c_void_p, dp, dp, C.POINTER(dp), C.c_int, dp]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_ppm_profile.argtypes = [C.c_int] + [dp] * 5
        L.orc_ppm_edges.argtypes = [C.c_int] + [dp] * 3
        L.orc_remap_column.argtypes = [C.c_int] + [dp] * 4
        L.orc_remap.argtypes = [C.c_void_p] + [dp] * 6 + [C.POINTER(dp), C.c_int, dp, dp]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "oracle wants C-contiguous float64"
    return a.ctypes.data_as(C.POINTER(C.c_double))


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


class Grid:
    """Oracle grid: kind 0 = doubly periodic (one tile), 1 = cubed sphere (6 tiles)."""

    def __init__(self, kind: int, n: int, nz: int, delta: float = 1000.0, f0: float = 0.0,
                 radius: float = RADIUS, omega: float = OMEGA, ptop: float = 100.0,
                 d2_bg: float = 0.0, beta: float = 1.0, dddmp: float = 0.0, hord: int = 8,
                 hord_tr: int = 0, pp_order: int = 2, nord: int = 0, d4_bg: float = 0.0,
                 vtdm: float = 0.0, edge_fix: bool = False,
                 edge_ppm: bool = False, edge_interp: bool = False):
        if hord not in (5, 6, 8) or hord_tr not in (0, 5, 6, 7, 8):
            raise ValueError("PPM orders: hord 5, 6 or 8; hord_tr 0, 5, 6, 7 or 8")
        if pp_order not in (2, 4):
            raise ValueError("pp_order must be 2 or 4")
        if nord not in (0, 1, 2):
            raise ValueError("nord must be 0, 1 or 2")
        err = C.create_string_buffer(256)
        h = lib().orc_grid_new(kind, n, nz, delta, f0, radius, omega, ptop, err, 256)
        if not h:
            raise RuntimeError("oracle grid: " + err.value.decode())
        self._h = h
        self.d2_bg = d2_bg
        lib().orc_set_damping(h, float(d2_bg))
        self.beta = beta
        lib().orc_set_beta(h, float(beta))
        self.dddmp = dddmp
        lib().orc_set_smag(h, float(dddmp))
        self.hord, self.hord_tr = hord, hord_tr
        lib().orc_set_hord(h, int(hord), int(hord_tr))
        self.pp_order = pp_order
        lib().orc_set_pp_order(h, int(pp_order))
        self.nord, self.d4_bg = nord, d4_bg
        lib().orc_set_damp4(h, int(nord), float(d4_bg))
        self.vtdm = vtdm
        lib().orc_set_vtdm(h, float(vtdm))
        self.edge_fix = edge_fix
        lib().orc_set_edge_fix(h, int(bool(edge_fix)))
        self.edge_ppm = edge_ppm
        lib().orc_set_edge_ppm(h, int(bool(edge_ppm)))
        self.edge_interp = edge_interp
        lib().orc_set_edge_interp(h, int(bool(edge_interp)))
        self.kind, self.n, self.nz = kind, n, nz
        self.T = 6 if kind == 1 else 1
        self.N = n + 2 * H + 1
        self.ptop = ptop

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_grid_free(h)
            self._h = None

    def metric(self, name: str) -> np.ndarray:
        out = np.zeros((self.T, self.N, self.N))
        if lib().orc_grid_metric(self._h, METRICS.index(name), _p(out)) != 0:
            raise KeyError(name)
        return out

    def connectivity(self):
        nbr = np.zeros(24, dtype=np.int32)
        rot = np.zeros(96, dtype=np.int32)
        lib().orc_grid_conn(self._h, nbr.ctypes.data_as(C.POINTER(C.c_int)),
                            rot.ctypes.data_as(C.POINTER(C.c_int)))
        return nbr.reshape(6, 4), rot.reshape(6, 4, 2, 2)

    def field(self, nlev: int) -> np.ndarray:
        return np.zeros((self.T, nlev, self.N, self.N))


def halo_fill(g: Grid, f: np.ndarray, stagger: str = "C", coslike: bool = False) -> None:
    lib().orc_halo_fill(g._h, _p(f), f.shape[1] if f.ndim == 4 else 1, ST[stagger], int(coslike))


def halo_fill_pair(g: Grid, fx, stx, fy, sty, kind="signed") -> None:
    nlev = fx.shape[1] if fx.ndim == 4 else 1
    lib().orc_halo_fill_pair(g._h, _p(fx), ST[stx], _p(fy), ST[sty], nlev, PAIR[kind])


def corner_view(g: Grid, plane: np.ndarray, stagger: str, mode: str) -> np.ndarray:
    plane = np.ascontiguousarray(plane)
    out = np.zeros_like(plane)
    lib().orc_corner_view(g._h, _p(plane), ST[stagger], MODE[mode], _p(out))
    return out


def corner_view_pair(g: Grid, px, stx, py, sty, mode):
    px = np.ascontiguousarray(px)
    py = np.ascontiguousarray(py)
    ox, oy = np.zeros_like(px), np.zeros_like(py)
    lib().orc_corner_view_pair(g._h, _p(px), ST[stx], _p(py), ST[sty], MODE[mode], _p(ox), _p(oy))
    return ox, oy


def ppm_face(q6, c: float, hord: int = 8) -> float:
    q = np.ascontiguousarray(q6, dtype=np.float64)
    assert q.shape == (6,)
    if hord == 8:
        return lib().orc_ppm_face(_p(q), float(c))
    return lib().orc_ppm_face_order(_p(q), float(c), int(hord))


def ppm_face_edge(q6, w6, c: float, hord: int, pe: int, west: bool) -> float:
    """Face value between window cells 2 and 3 when window interface pe
    (1..5, between cells pe-1 and pe) is a cube tile edge; w6 are the cell
    widths along the sweep, west says the tile lies at cells >= pe."""
    q = np.ascontiguousarray(q6, dtype=np.float64)
    w = np.ascontiguousarray(w6, dtype=np.float64)
    assert q.shape == (6,) and w.shape == (6,) and 1 <= pe <= 5
    return lib().orc_ppm_face_edge(_p(q), _p(w), float(c), int(hord), int(pe), int(bool(west)))


def fv_tp_2d(g: Grid, t: int, q, crx, cry, xfx, yfx, mx=None, my=None):
    args = [np.ascontiguousarray(a, dtype=np.float64) if a is not None else None
            for a in (q, crx, cry, xfx, yfx, mx, my)]
    FX = np.zeros((g.N, g.N))
    FY = np.zeros((g.N, g.N))
    lib().orc_fv_tp_2d(g._h, t, *[_p(a) for a in args], _p(FX), _p(FY))
    return FX, FY


def sim1(dt, ptop, zs, dpi, theta, delz, w, beta: float = 1.0, pp_order: int = 2):
    """One column solve; also returns the interface perturbation P* ("pstar")
    and the unscaled coupling dt x linearised pressure response ("coupling")."""
    nz = len(dpi)
    ins = [np.ascontiguousarray(a, dtype=np.float64) for a in (dpi, theta, delz, w)]
    wo, dzo = np.zeros(nz), np.zeros(nz)
    pf, ph = np.zeros(nz + 1), np.zeros(nz + 1)
    ps, cp = np.zeros(nz + 1), np.zeros(nz + 1)
    minpiv = lib().orc_sim1b(nz, dt, float(beta), int(pp_order), ptop, zs, *[_p(a) for a in ins], _p(wo), _p(dzo),
                             _p(pf), _p(ph), _p(ps), _p(cp))
    return dict(w=wo, delz=dzo, pfull=pf, phi=ph, min_pivot=minpiv, pstar=ps, coupling=cp)


def pp_interfaces(dpi, pp, order: int = 2) -> np.ndarray:
    """Interface values (nz + 1) of the layer perturbation pp used by the column solve."""
    d = np.ascontiguousarray(dpi, dtype=np.float64)
    q = np.ascontiguousarray(pp, dtype=np.float64)
    out = np.zeros(len(d) + 1)
    lib().orc_pp_interfaces(len(d), int(order), _p(d), _p(q), _p(out))
    return out


def pgf(dt, L, dpiW, dpiE, phW0, phW1, phE0, phE1, pW0, pW1, pE0, pE1) -> float:
    return lib().orc_pgf(dt, L, dpiW, dpiE, phW0, phW1, phE0, phE1, pW0, pW1, pE0, pE1)


STATE_FIELDS = ["u", "v", "w", "delp", "pt", "delz", "uc", "vc", "mfx", "mfy", "cx", "cy",
                "dp0", "pfull", "phi"]
DEBUG_FIELDS = ["delpc", "ptc", "wc", "ax", "ay", "crx", "cry", "xfx", "yfx", "pkc", "gz", "vortc",
                "vortd"]


def new_state(g: Grid, init: dict) -> dict:
    """Copy an input state (from fv3_inputs) into a full oracle state."""
    s = {}
    for k in ("u", "v", "w", "delp", "pt", "delz"):
        s[k] = np.ascontiguousarray(init[k], dtype=np.float64).copy()
    for k in ("uc", "vc", "mfx", "mfy", "cx", "cy", "dp0"):
        s[k] = g.field(g.nz)
    s["pfull"] = g.field(g.nz + 1)
    s["phi"] = g.field(g.nz + 1)
    s["phis"] = np.ascontiguousarray(init.get("phis", np.zeros((g.T, g.N, g.N))), dtype=np.float64)
    # specific humidity (moist column solves) or None (dry)
    s["qv"] = np.ascontiguousarray(init["qv"], dtype=np.float64).copy() if init.get("qv") is not None else None
    return s


def acoustic_substeps(g: Grid, s: dict, dt: float, n_split: int, stop_stage: int = 0,
                      debug: bool = False):
    """Run n_split substeps in place.  Returns the status (0 ok, -6 Courant > 1,
    -7 non-finite) and, with debug=True, the intermediate fields of the last
    substep."""
    dbg = None
    dbg_arr = None
    if debug:
        dbg = {k: g.field(g.nz + (1 if k in ("pkc", "gz") else 0)) for k in DEBUG_FIELDS}
        dbg_arr = (C.POINTER(C.c_double) * len(DEBUG_FIELDS))(*[_p(dbg[k]) for k in DEBUG_FIELDS])
    st = lib().orc_acoustic_substeps(g._h, *[_p(s[k]) for k in STATE_FIELDS], _p(s["phis"]),
                                     _p(s.get("qv")), float(dt), int(n_split), int(stop_stage), dbg_arr)
    return (st, dbg) if debug else st


def tracer_transport(g: Grid, qs, dp0, mfx, mfy, cx, cy, nsplt: int = 0) -> int:
    arr = (C.POINTER(C.c_double) * len(qs))(*[_p(q) for q in qs])
    used = C.c_int(0)
    lib().orc_tracer_transport(g._h, arr, len(qs), _p(dp0), _p(mfx), _p(mfy), _p(cx), _p(cy),
                               int(nsplt), C.byref(used))
    return used.value


def smag_corner(g: "Grid", t: int, u_plane, v_plane, dt: float) -> np.ndarray:
    """Smagorinsky magnitude dt sqrt(DT^2 + DS^2) at the corners of one level
    (u, v planes [N][N] with halos filled)."""
    u = np.ascontiguousarray(u_plane, dtype=np.float64)
    v = np.ascontiguousarray(v_plane, dtype=np.float64)
    out = np.zeros((g.N, g.N))
    lib().orc_smag_corner(g._h, int(t), _p(u), _p(v), float(dt), _p(out))
    return out


def ppm_edges(d, a):
    """Interface values of a column before the parabola limiter: e[K] for
    K = 1..nz-1 (e[0] and e[nz] are unused and returned as 0)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    e = np.zeros(len(a) + 1)
    lib().orc_ppm_edges(len(a), _p(d), _p(a), _p(e))
    return e


def ppm_profile(d, a):
    """Limited parabola of every layer of a column (thicknesses d, means a):
    top value aL, bottom value aR, curvature a6."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    aL, aR, a6 = np.zeros_like(a), np.zeros_like(a), np.zeros_like(a)
    lib().orc_ppm_profile(len(a), _p(d), _p(a), _p(aL), _p(aR), _p(a6))
    return aL, aR, a6


INTERP_KINDS = {"face_pt": 0, "cell_pt": 1, "face_mean": 2}


def interp(kind: str, x, m0: int, m: int, n: int, edge: bool) -> float:
    """One interpolation of c_sw (kind "cell_pt": D -> A, "face_pt": A -> C)
    or of nh_p_grad's corner values ("face_mean") at index m along a sweep
    whose tile edges are the interfaces 0 and n; x[k - m0] is the value at
    index k.  edge: the one-sided stencils of the option edge_interp."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().orc_interp(INTERP_KINDS[kind], _p(x), len(x), int(m0), int(m), int(n), int(bool(edge)))


def corner_values(g: Grid, q) -> np.ndarray:
    """nh_p_grad's corner values of one level, q [T][N][N] with filled halos
    (the cell-to-corner interpolation of the D-grid pressure gradient)."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.zeros_like(q)
    lib().orc_corner_values(g._h, _p(q), _p(out))
    return out


def corner_vorticity(g: Grid, uc, vc) -> np.ndarray:
    """c_sw's absolute vorticity at the corners of one level of every tile
    from C-grid winds uc (x-faces) and vc (y-faces), [T][N][N] each."""
    uc = np.ascontiguousarray(uc, dtype=np.float64)
    vc = np.ascontiguousarray(vc, dtype=np.float64)
    out = np.zeros_like(uc)
    lib().orc_corner_vort(g._h, _p(uc), _p(vc), _p(out))
    return out


def remap_column(pe1, pe2, q1) -> np.ndarray:
    """Remap the layer means q1 on interfaces pe1 to interfaces pe2."""
    pe1 = np.ascontiguousarray(pe1, dtype=np.float64)
    pe2 = np.ascontiguousarray(pe2, dtype=np.float64)
    q1 = np.ascontiguousarray(q1, dtype=np.float64)
    assert pe1.shape == pe2.shape == (len(q1) + 1,)
    q2 = np.zeros_like(q1)
    lib().orc_remap_column(len(q1), _p(pe1), _p(pe2), _p(q1), _p(q2))
    return q2


def remap(g: Grid, s: dict, ak, bk, qs=()) -> int:
    """Remap a state in place to the reference interfaces ak + bk * ps
    (u, v, w, delp, pt, delz and the tracer fields qs)."""
    ak = np.ascontiguousarray(ak, dtype=np.float64)
    bk = np.ascontiguousarray(bk, dtype=np.float64)
    assert ak.shape == bk.shape == (g.nz + 1,)
    arr = (C.POINTER(C.c_double) * max(1, len(qs)))(*[_p(q) for q in qs])
    return lib().orc_remap(g._h, *[_p(s[k]) for k in ("u", "v", "w", "delp", "pt", "delz")], arr,
                           len(qs), _p(ak), _p(bk))


def dynamics(g: Grid, s: dict, qs, ak, bk, dt: float, k_split: int, n_split: int, nsplt: int = 0) -> int:
    """One pass of the remapping loop (the middle of FV3's three nested
    loops, Sec. II): k_split times, n_split acoustic substeps over dt /
    k_split, the tracer transport of qs with the fluxes they accumulated,
    and the vertical remap of the state and qs to ak + bk * ps.  Returns the
    first non-zero status, else 0."""
    for _ in range(k_split):
        st = acoustic_substeps(g, s, dt / k_split, n_split)
        if st != 0:
            return st
        if len(qs):
            tracer_transport(g, qs, s["dp0"], s["mfx"], s["mfy"], s["cx"], s["cy"], nsplt)
        st = remap(g, s, ak, bk, qs)
        if st != 0:
            return st
    return 0


def mass_sums(g: Grid, delp, pt, qs=()) -> np.ndarray:
    out = np.zeros(2 + len(qs))
    arr = (C.POINTER(C.c_double) * max(1, len(qs)))(*[_p(q) for q in qs])
    lib().orc_mass_sums(g._h, _p(delp), _p(pt), arr, len(qs), _p(out))
    return out


def corner_div(g: "Grid", U, V) -> np.ndarray:
    """Corner divergence of D-grid fields U (y-faces), V (x-faces) of shape (T, L, N, N)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    out = np.zeros_like(U)
    lib().orc_corner_div(g._h, U.shape[1], _p(U), _p(V), _p(out))
    return out


def corner_lap(g: "Grid", D) -> np.ndarray:
    """Corner Laplacian of a corner field (T, L, N, N); fills D's corner halo in place."""
    D = np.ascontiguousarray(D, dtype=np.float64)
    out = np.zeros_like(D)
    lib().orc_corner_lap(g._h, D.shape[1], _p(D), _p(out))
    return out, D


def edge_partner(g: "Grid", t: int, stagger: str, i: int, j: int):
    """The other tile's copy of a face on a tile edge of the cube: (tile,
    stagger, i, j, sign of its flux along ours)."""
    out = (C.c_int * 4)()
    sg = lib().orc_edge_partner(g._h, t, 1 if stagger == "X" else 2, i, j, out)
    return out[0], "X" if out[1] == 1 else "Y", out[2], out[3], sg
