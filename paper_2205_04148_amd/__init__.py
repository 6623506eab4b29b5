"""Python binding of the MI355X FV3 acoustic-substep library (libfv3.so).

Argument marshalling only: every step of the acoustic substep loop and the
tracer transport runs in the HIP kernels of libfv3.so.  PyTorch provides the
device memory (tensors in the library's padded layout) and the stream.  If
the shared library is missing the import of the entry points raises; there is
no CPU fallback.

    g = Grid(kind=1, n=96, nz=79)            # cubed sphere C96 x 79 levels
    s = State.allocate(g)
    s.load(init)                             # host arrays f[t][k][j+3][i+3]
    acoustic_substeps(s, g, dt=1800.0, n_split=60)
    tracer_transport([q...], s, g)
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libfv3.so")
H = 3
RADIUS = 6.3712e6
OMEGA = 7.2921e-5

STATUS = {0: "ok", -1: "EINVAL", -2: "ESHAPE", -3: "EDTYPE", -4: "EDEVICE", -5: "ENOMEM",
          -6: "ECFL", -7: "ENONFINITE", -8: "EUNSUPPORTED", -9: "EREMAP", -99: "EINTERNAL"}
METRICS = ["dx", "dy", "dxc", "dyc", "dxa", "dya", "area", "area_c", "fC", "fB", "sin_u",
           "cos_u", "sin_v", "cos_v", "sin_a", "cos_a"]
EXPORTS = ["fv3_init_grid", "fv3_free_grid", "fv3_grid_layout", "fv3_workspace_bytes",
           "fv3_grid_metric", "fv3_acoustic_substeps", "fv3_acoustic_substeps_debug",
           "fv3_tracer_transport", "fv3_remap", "fv3_dynamics", "fv3_mass_sums", "fv3_mass_sums_noalloc", "fv3_halo_fill", "fv3_check_status",
           "fv3_status_string", "fv3_last_error", "fv3_host_grid_metric", "fv3_timing_start", "fv3_device_copy",
           "fv3_timing_stop", "fv3_acoustic_substeps_batched", "fv3_ensemble_create",
           "fv3_ensemble_run", "fv3_ensemble_free", "fv3_ensemble_tune", "fv3_ensemble_shapes",
           "fv3_coarsen", "fv3_column_features", "fv3_apply_correction",
           "fv3_mlp_create", "fv3_mlp_free", "fv3_mlp_param_count", "fv3_mlp_set_params",
           "fv3_mlp_get_params", "fv3_mlp_forward", "fv3_mlp_gradients", "fv3_mlp_train_step"]


class FV3Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class GridParams(C.Structure):
    _fields_ = [("kind", C.c_int), ("n", C.c_int), ("nz", C.c_int), ("dx", C.c_double),
                ("f0", C.c_double), ("radius", C.c_double), ("omega", C.c_double),
                ("ptop", C.c_double), ("precision", C.c_int), ("hord", C.c_int),
                ("d2_bg", C.c_double), ("beta", C.c_double), ("dddmp", C.c_double), ("hord_tr", C.c_int),
                ("pp_order", C.c_int), ("nord", C.c_int), ("d4_bg", C.c_double),
                ("vtdm", C.c_double), ("edge_fix", C.c_int), ("edge_ppm", C.c_int), ("edge_interp", C.c_int),
                ("device", C.c_int)]


class Layout(C.Structure):
    _fields_ = [("tiles", C.c_int), ("n", C.c_int), ("nz", C.c_int), ("halo", C.c_int),
                ("pitch", C.c_long), ("rows", C.c_long), ("level_elems", C.c_long),
                ("offset0", C.c_long), ("bulk_elem_bytes", C.c_int)]


class TuneReport(C.Structure):
    _fields_ = [("sites", C.c_int), ("tunable_sites", C.c_int), ("searched", C.c_int),
                ("reused", C.c_int), ("search_ms", C.c_double), ("substep_ms_before", C.c_double),
                ("substep_ms_after", C.c_double)]


class FeatureNorm(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("mean", "inv_std", "lo", "hi")]


class StateStruct(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("u", "v", "w", "delp", "pt", "delz", "uc", "vc", "mfx",
                                          "mfy", "cx", "cy", "dp0", "pfull", "phi", "phis",
                                          "workspace")] + [("workspace_bytes", C.c_size_t),
                                                           ("qv", C.c_void_p)]


_lib = None


def lib():
    """Load libfv3.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            raise ImportError(f"{_LIBPATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(_LIBPATH)
        vp = C.c_void_p
        L.fv3_init_grid.argtypes = [C.POINTER(GridParams), C.POINTER(vp)]
        L.fv3_free_grid.argtypes = [vp]
        L.fv3_grid_layout.argtypes = [vp, C.POINTER(Layout)]
        L.fv3_workspace_bytes.argtypes = [vp]
        L.fv3_workspace_bytes.restype = C.c_size_t
        L.fv3_grid_metric.argtypes = [vp, C.c_int, C.POINTER(C.c_double)]
        L.fv3_host_grid_metric.argtypes = [C.POINTER(GridParams), C.c_int, C.POINTER(C.c_double),
                                           C.c_long]
        L.fv3_acoustic_substeps.argtypes = [C.POINTER(StateStruct), vp, C.c_double, C.c_int, vp]
        L.fv3_acoustic_substeps_debug.argtypes = [C.POINTER(StateStruct), vp, C.c_double, C.c_int,
                                                  C.c_int, vp]
        L.fv3_tracer_transport.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(StateStruct), vp,
                                           C.c_int, vp]
        L.fv3_remap.argtypes = [C.POINTER(StateStruct), vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.POINTER(vp), C.c_int, vp]
        L.fv3_mass_sums.argtypes = [vp, vp, vp, C.POINTER(vp), C.c_int, C.POINTER(C.c_double), vp]
        L.fv3_dynamics.argtypes = [C.POINTER(StateStruct), vp, C.POINTER(vp), C.c_int, C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.c_double, C.c_int, C.c_int, C.c_int, vp]
        L.fv3_mass_sums_noalloc.argtypes = [vp, vp, vp, C.POINTER(vp), C.c_int, vp, vp]
        L.fv3_halo_fill.argtypes = [vp, C.POINTER(vp), C.c_int, C.c_int, C.c_int, vp]
        L.fv3_check_status.argtypes = [vp, vp]
        L.fv3_timing_start.argtypes = [C.c_char_p]
        L.fv3_device_copy.argtypes = [vp, vp, C.c_size_t, vp]
        L.fv3_timing_stop.argtypes = [C.c_char_p, C.c_int, C.POINTER(C.c_double),
                                      C.POINTER(C.c_long), C.c_int]
        L.fv3_acoustic_substeps_batched.argtypes = [C.POINTER(C.POINTER(StateStruct)), C.POINTER(vp),
                                                    C.c_int, C.c_double, C.c_int, vp]
        L.fv3_ensemble_create.argtypes = [C.POINTER(C.POINTER(StateStruct)), C.POINTER(vp), C.c_int,
                                          C.c_double, C.c_int, C.c_int, C.POINTER(vp)]
        L.fv3_ensemble_run.argtypes = [vp, vp]
        L.fv3_ensemble_free.argtypes = [vp]
        L.fv3_ensemble_tune.argtypes = [vp, C.c_int, C.POINTER(TuneReport), vp]
        L.fv3_ensemble_shapes.argtypes = [vp, C.c_char_p, C.c_int, C.POINTER(C.c_int),
                                          C.POINTER(C.c_int), C.c_int]
        L.fv3_coarsen.argtypes = [C.POINTER(StateStruct), vp, C.POINTER(StateStruct), vp, vp]
        L.fv3_column_features.argtypes = [C.POINTER(StateStruct), vp, C.POINTER(FeatureNorm), vp,
                                          vp, vp]
        L.fv3_apply_correction.argtypes = [C.POINTER(StateStruct), vp, vp, vp, vp, C.c_double, vp,
                                           vp]
        fp = C.POINTER(C.c_float)
        L.fv3_mlp_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, fp, C.POINTER(vp)]
        L.fv3_mlp_free.argtypes = [vp]
        L.fv3_mlp_param_count.argtypes = [vp]
        L.fv3_mlp_param_count.restype = C.c_long
        L.fv3_mlp_set_params.argtypes = [vp, fp]
        L.fv3_mlp_get_params.argtypes = [vp, fp]
        L.fv3_mlp_forward.argtypes = [vp, vp, C.c_int, vp, vp]
        L.fv3_mlp_gradients.argtypes = [vp, vp, vp, C.c_int, fp, vp]
        L.fv3_mlp_train_step.argtypes = [vp, vp, vp, C.c_int, C.c_float, C.POINTER(C.c_double), vp]
        L.fv3_status_string.argtypes = [C.c_int]
        L.fv3_status_string.restype = C.c_char_p
        L.fv3_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        raise FV3Error(st, lib().fv3_last_error().decode())


def _params(kind, n, nz, dx, f0, radius, omega, ptop, precision, device, d2_bg=0.0, beta=1.0, dddmp=0.0,
            hord=8, hord_tr=0, pp_order=2, nord=0, d4_bg=0.0, vtdm=0.0, edge_fix=False,
            edge_ppm=False, edge_interp=False):
    return GridParams(kind=kind, n=n, nz=nz, dx=dx, f0=f0, radius=radius, omega=omega, ptop=ptop,
                      precision=0 if precision == "fp64" else 1, hord=hord, d2_bg=d2_bg, beta=beta,
                      dddmp=dddmp, hord_tr=hord_tr, pp_order=pp_order, nord=nord, d4_bg=d4_bg,
                      vtdm=vtdm, edge_fix=int(bool(edge_fix)), edge_ppm=int(bool(edge_ppm)),
                      edge_interp=int(bool(edge_interp)), device=device)


def host_metric(kind, n, nz, name, dx=1000.0, f0=0.0, radius=RADIUS, omega=OMEGA, ptop=100.0,
                precision="fp64"):
    """Metric term computed by the library's host grid builder (no device
    needed), returned as [T][N][N] with N = n + 2*3 + 1."""
    p = _params(kind, n, nz, dx, f0, radius, omega, ptop, precision, 0)
    T = 6 if kind == 1 else 1
    N = n + 2 * H + 1
    out = np.zeros(T * N * N)
    _check(lib().fv3_host_grid_metric(C.byref(p), METRICS.index(name),
                                      out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
    return out.reshape(T, N, N)


def _torch():
    import torch
    return torch


class Grid:
    """A library-owned grid on one HIP device (kind 0 doubly periodic, 1 cube)."""

    def __init__(self, kind: int, n: int, nz: int, dx: float = 1000.0, f0: float = 0.0,
                 radius: float = RADIUS, omega: float = OMEGA, ptop: float = 100.0,
                 precision: str = "fp64", device: int = 0, d2_bg: float = 0.0, beta: float = 1.0,
                 dddmp: float = 0.0, hord: int = 8, hord_tr: int = 0, pp_order: int = 2, nord: int = 0,
                 d4_bg: float = 0.0, vtdm: float = 0.0, edge_fix: bool = False,
                 edge_ppm: bool = False, edge_interp: bool = False):
        torch = _torch()
        torch.cuda.set_device(device)
        p = _params(kind, n, nz, dx, f0, radius, omega, ptop, precision, device, d2_bg, beta, dddmp, hord,
                    hord_tr, pp_order, nord, d4_bg, vtdm, edge_fix, edge_ppm, edge_interp)
        h = C.c_void_p()
        _check(lib().fv3_init_grid(C.byref(p), C.byref(h)))
        self._h = h
        lay = Layout()
        _check(lib().fv3_grid_layout(h, C.byref(lay)))
        self.layout = lay
        self.kind, self.n, self.nz, self.T = kind, n, nz, lay.tiles
        self.ptop = ptop
        self.hord, self.hord_tr, self.pp_order = hord, hord_tr, pp_order
        self.precision = precision
        self.device = device
        self.N = n + 2 * H + 1
        self.pitch, self.rows, self.lev, self.off0 = lay.pitch, lay.rows, lay.level_elems, lay.offset0
        self.pre = self.off0 - H * self.pitch - H
        self.bulk_dtype = torch.float64 if precision == "fp64" else torch.float32
        self.ws_bytes = lib().fv3_workspace_bytes(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.fv3_free_grid(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def alloc_elems(self, levels: int) -> int:
        return self.pre + self.T * levels * self.lev + self.pitch

    def new_field(self, levels: int, fp64: bool = False):
        torch = _torch()
        dt = torch.float64 if fp64 else self.bulk_dtype
        return torch.zeros(self.alloc_elems(levels), dtype=dt, device=f"cuda:{self.device}")

    def view(self, buf, levels: int):
        """[T][L][N][N] view of a padded device buffer (i + 3, j + 3 indexing)."""
        n = self.T * levels * self.lev
        return buf[self.pre:self.pre + n].view(self.T, levels, self.rows, self.pitch)[..., :self.N]

    def upload(self, host: np.ndarray, levels: int, fp64: bool = False):
        torch = _torch()
        buf = self.new_field(levels, fp64)
        a = np.asarray(host).reshape(self.T, levels, self.N, self.N)
        self.view(buf, levels).copy_(torch.from_numpy(np.ascontiguousarray(a)).to(buf.dtype))
        return buf

    def download(self, buf, levels: int) -> np.ndarray:
        return self.view(buf, levels).double().cpu().numpy()

    def metric(self, name: str) -> np.ndarray:
        out = np.zeros(self.alloc_elems(1))
        _check(lib().fv3_grid_metric(self._h, METRICS.index(name),
                                     out.ctypes.data_as(C.POINTER(C.c_double))))
        return out[self.pre:self.pre + self.T * self.lev].reshape(
            self.T, self.rows, self.pitch)[:, :, :self.N].copy()


LAYER_BULK = ("u", "v", "w", "delp", "pt", "uc", "vc", "cx", "cy")
LAYER_F64 = ("delz", "mfx", "mfy", "dp0")
IFACE_F64 = ("pfull", "phi")


class State:
    """Device arrays of one model state (torch tensors in the padded layout)."""

    def __init__(self, grid: Grid, fields: dict):
        self.grid = grid
        self.f = fields

    @classmethod
    def allocate(cls, grid: Grid) -> "State":
        torch = _torch()
        f = {}
        for k in LAYER_BULK:
            f[k] = grid.new_field(grid.nz)
        for k in LAYER_F64:
            f[k] = grid.new_field(grid.nz, fp64=True)
        for k in IFACE_F64:
            f[k] = grid.new_field(grid.nz + 1, fp64=True)
        f["phis"] = grid.new_field(1, fp64=True)
        f["workspace"] = torch.empty(grid.ws_bytes, dtype=torch.uint8, device=f"cuda:{grid.device}")
        return cls(grid, f)

    def load(self, init: dict) -> None:
        g = self.grid
        for k in ("u", "v", "w", "delp", "pt"):
            g.view(self.f[k], g.nz).copy_(_torch().from_numpy(
                np.ascontiguousarray(init[k])).to(self.f[k].dtype))
        g.view(self.f["delz"], g.nz).copy_(_torch().from_numpy(np.ascontiguousarray(init["delz"])))
        if "phis" in init:
            g.view(self.f["phis"], 1).copy_(_torch().from_numpy(
                np.ascontiguousarray(init["phis"]).reshape(g.T, 1, g.N, g.N)))
        self.set_humidity(init.get("qv"))

    def set_humidity(self, qv) -> None:
        """Specific humidity for the moist column solves (numpy array in the
        state's field shape, bulk precision on the device), or None: dry."""
        g = self.grid
        if qv is None:
            self.f.pop("qv", None)
            return
        if "qv" not in self.f:
            self.f["qv"] = g.new_field(g.nz)
        g.view(self.f["qv"], g.nz).copy_(_torch().from_numpy(np.ascontiguousarray(qv)).to(self.f["qv"].dtype))

    def get(self, name: str) -> np.ndarray:
        L = self.grid.nz + 1 if name in IFACE_F64 else self.grid.nz
        return self.grid.download(self.f[name], L)

    def struct(self) -> StateStruct:
        s = StateStruct()
        for k in ("u", "v", "w", "delp", "pt", "delz", "uc", "vc", "mfx", "mfy", "cx", "cy",
                  "dp0", "pfull", "phi", "phis", "workspace"):
            setattr(s, k, self.f[k].data_ptr())
        s.workspace_bytes = self.f["workspace"].numel()
        s.qv = self.f["qv"].data_ptr() if "qv" in self.f else None
        return s


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def acoustic_substeps(state: State, grid: Grid, dt: float, n_split: int, stream=None,
                      stop_stage: int = 0) -> None:
    st = state.struct()
    if stop_stage:
        _check(lib().fv3_acoustic_substeps_debug(C.byref(st), grid.handle, float(dt), int(n_split),
                                                 int(stop_stage), _stream(stream)))
    else:
        _check(lib().fv3_acoustic_substeps(C.byref(st), grid.handle, float(dt), int(n_split),
                                           _stream(stream)))


def tracer_transport(qs, state: State, grid: Grid, nsplt: int = 0, stream=None) -> None:
    st = state.struct()
    arr = (C.c_void_p * len(qs))(*[q.data_ptr() for q in qs])
    _check(lib().fv3_tracer_transport(arr, len(qs), C.byref(st), grid.handle, int(nsplt),
                                      _stream(stream)))


def remap(state: State, grid: Grid, ak, bk, qs=(), stream=None) -> None:
    """Remap the state's layers (and the tracer fields qs) in place to the
    reference interfaces ak + bk * ps; ak, bk hold nz + 1 values."""
    ak = np.ascontiguousarray(ak, dtype=np.float64)
    bk = np.ascontiguousarray(bk, dtype=np.float64)
    if ak.shape != (grid.nz + 1,) or bk.shape != (grid.nz + 1,):
        raise ValueError("ak and bk need nz + 1 values")
    st = state.struct()
    arr = (C.c_void_p * max(1, len(qs)))(*[q.data_ptr() for q in qs])
    _check(lib().fv3_remap(C.byref(st), grid.handle, ak.ctypes.data_as(C.POINTER(C.c_double)),
                           bk.ctypes.data_as(C.POINTER(C.c_double)), arr, len(qs), _stream(stream)))


def dynamics(state: State, grid: Grid, qs, ak, bk, dt: float, k_split: int, n_split: int, nsplt: int = 0,
             stream=None) -> None:
    """fv3_dynamics: k_split x (n_split acoustic substeps, tracer transport of
    qs, vertical remap to ak + bk * ps) over the span dt."""
    ak = np.ascontiguousarray(ak, dtype=np.float64)
    bk = np.ascontiguousarray(bk, dtype=np.float64)
    if ak.shape != (grid.nz + 1,) or bk.shape != (grid.nz + 1,):
        raise ValueError("ak and bk need nz + 1 values")
    st = state.struct()
    arr = (C.c_void_p * max(1, len(qs)))(*[q.data_ptr() for q in qs])
    _check(lib().fv3_dynamics(C.byref(st), grid.handle, arr, len(qs), ak.ctypes.data_as(C.POINTER(C.c_double)),
                              bk.ctypes.data_as(C.POINTER(C.c_double)), float(dt), int(k_split), int(n_split),
                              int(nsplt), _stream(stream)))


def mass_sums(grid: Grid, delp, pt, qs=(), stream=None) -> np.ndarray:
    out = np.zeros(2 + len(qs))
    arr = (C.c_void_p * max(1, len(qs)))(*[q.data_ptr() for q in qs])
    _check(lib().fv3_mass_sums(grid.handle, C.c_void_p(delp.data_ptr()), C.c_void_p(pt.data_ptr()),
                               arr, len(qs), out.ctypes.data_as(C.POINTER(C.c_double)),
                               _stream(stream)))
    return out


def device_copy(src, dst, stream=None) -> None:
    """fv3_device_copy of the bytes of device tensor src into dst (same size)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("src and dst must hold the same number of bytes")
    _check(lib().fv3_device_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nb, _stream(stream)))


def mass_sums_noalloc(grid: Grid, delp, pt, qs, out, stream=None) -> None:
    """fv3_mass_sums_noalloc: the sums into `out`, a device float64 tensor of
    2 + len(qs) elements; nothing is allocated and nothing synchronised."""
    if out.dtype != _torch().float64 or not out.is_cuda or out.numel() < 2 + len(qs) or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 device tensor of 2 + nq elements")
    arr = (C.c_void_p * max(1, len(qs)))(*[q.data_ptr() for q in qs])
    _check(lib().fv3_mass_sums_noalloc(grid.handle, C.c_void_p(delp.data_ptr()), C.c_void_p(pt.data_ptr()),
                                       arr, len(qs), C.c_void_p(out.data_ptr()), _stream(stream)))


def halo_fill(grid: Grid, fields, levels: int, fp64: bool = False, stream=None) -> None:
    arr = (C.c_void_p * len(fields))(*[f.data_ptr() for f in fields])
    _check(lib().fv3_halo_fill(grid.handle, arr, len(fields), int(levels), int(fp64),
                               _stream(stream)))


def check_status(grid: Grid, stream=None) -> int:
    return lib().fv3_check_status(grid.handle, _stream(stream))


def timing_start(filter_: str | None = "") -> None:
    """Record HIP events around library kernel launches whose name contains filter_."""
    lib().fv3_timing_start(None if filter_ is None else filter_.encode())


def timing_stop() -> dict:
    """Stop recording; {kernel name: (total ms, launches)} (synchronises the device)."""
    cap = 256
    names = C.create_string_buffer(cap * 64)
    tot = (C.c_double * cap)()
    cnt = (C.c_long * cap)()
    nk = lib().fv3_timing_stop(names, cap * 64, tot, cnt, cap)
    if nk < 0:
        raise FV3Error(nk, "timing_stop failed")
    keys = names.raw.split(b"\0")
    return {keys[q].decode(): (tot[q], cnt[q]) for q in range(nk)}


# ---------------------------------------------------------------- batched ensemble
def _member_arrays(states, grids):
    if len(states) != len(grids) or not states:
        raise ValueError("need one grid per state and at least one member")
    structs = [s.struct() for s in states]
    sp = (C.POINTER(StateStruct) * len(structs))(*[C.pointer(x) for x in structs])
    gp = (C.c_void_p * len(grids))(*[g.handle for g in grids])
    return structs, sp, gp


def acoustic_substeps_batched(states, grids, dt: float, n_split: int, stream=None) -> None:
    """n_split substeps on every (state, grid) member with one launch per kernel
    for all members (synchronises the stream)."""
    keep, sp, gp = _member_arrays(states, grids)
    _check(lib().fv3_acoustic_substeps_batched(sp, gp, len(keep), float(dt), int(n_split),
                                               _stream(stream)))


class Ensemble:
    """Recorded batched substep call over many members (optionally a HIP graph)."""

    def __init__(self, states, grids, dt: float, n_split: int, graph: bool = False):
        self.states, self.grids = list(states), list(grids)
        keep, sp, gp = _member_arrays(self.states, self.grids)
        h = C.c_void_p()
        _check(lib().fv3_ensemble_create(sp, gp, len(keep), float(dt), int(n_split),
                                         1 if graph else 0, C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.fv3_ensemble_free(h)
            self._h = None

    def run(self, stream=None) -> None:
        _check(lib().fv3_ensemble_run(self._h, _stream(stream)))

    def tune(self, reps: int = 3, stream=None) -> dict:
        """Time candidate block shapes (leaves the member states undefined)."""
        r = TuneReport()
        _check(lib().fv3_ensemble_tune(self._h, int(reps), C.byref(r), _stream(stream)))
        return {k: getattr(r, k) for k, _ in TuneReport._fields_}

    def shapes(self):
        cap = 512
        names = C.create_string_buffer(cap * 48)
        bx = (C.c_int * cap)()
        by = (C.c_int * cap)()
        k = lib().fv3_ensemble_shapes(self._h, names, cap * 48, bx, by, cap)
        if k < 0:
            raise FV3Error(k, lib().fv3_last_error().decode())
        ks = names.raw.split(b"\0")
        return [(ks[q].decode(), bx[q], by[q]) for q in range(k)]


# ---------------------------------------------------------------- learned correction
def coarsen(fine: State, gf: Grid, coarse: State, gc: Grid, stream=None) -> None:
    """Conservative coarsening of u, v, w, delp, pt, delz from gf onto gc."""
    a, b = fine.struct(), coarse.struct()
    _check(lib().fv3_coarsen(C.byref(a), gf.handle, C.byref(b), gc.handle, _stream(stream)))


def column_features(state: State, grid: Grid, mean, inv_std, X, flag=None, lo=None, hi=None,
                    stream=None) -> None:
    """Normalised column features into the device float tensor X [T*n*n, 5*nz]."""
    nm = FeatureNorm(mean=mean.data_ptr(), inv_std=inv_std.data_ptr(),
                     lo=lo.data_ptr() if lo is not None else None,
                     hi=hi.data_ptr() if hi is not None else None)
    st = state.struct()
    _check(lib().fv3_column_features(C.byref(st), grid.handle, C.byref(nm), C.c_void_p(X.data_ptr()),
                                     C.c_void_p(flag.data_ptr()) if flag is not None else None,
                                     _stream(stream)))


def apply_correction(state: State, grid: Grid, Y, ymean, ystd, seconds: float, flag,
                     stream=None) -> None:
    """Add seconds x de-normalised tendencies Y [T*n*n, 3*nz] unless *flag is set."""
    st = state.struct()
    _check(lib().fv3_apply_correction(C.byref(st), grid.handle, C.c_void_p(Y.data_ptr()),
                                      C.c_void_p(ymean.data_ptr()), C.c_void_p(ystd.data_ptr()),
                                      float(seconds), C.c_void_p(flag.data_ptr()), _stream(stream)))


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class MLP:
    """Three-layer tanh perceptron trained with BF16 matrix-core kernels.

    params: list [W1 (in, h1), b1, W2, b2, W3, b3] of host arrays."""

    def __init__(self, params, maxrows: int):
        W1, _, W2, _, W3, _ = params
        self.sizes = (W1.shape[0], W1.shape[1], W2.shape[1], W3.shape[1])
        flat = self._pack(params)
        h = C.c_void_p()
        _check(lib().fv3_mlp_create(*[int(x) for x in self.sizes], int(maxrows), _fptr(flat),
                                    C.byref(h)))
        self._h = h

    @staticmethod
    def _pack(params) -> np.ndarray:
        return np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.float32).ravel()
                                                    for p in params]))

    def _unpack(self, flat: np.ndarray):
        i, h1, h2, o = self.sizes
        out, pos = [], 0
        for a, b in ((i, h1), (h1, h2), (h2, o)):
            out.append(flat[pos:pos + a * b].reshape(a, b).copy())
            pos += a * b
            out.append(flat[pos:pos + b].copy())
            pos += b
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.fv3_mlp_free(h)
            self._h = None

    def set_params(self, params) -> None:
        _check(lib().fv3_mlp_set_params(self._h, _fptr(self._pack(params))))

    def get_params(self):
        flat = np.zeros(lib().fv3_mlp_param_count(self._h), dtype=np.float32)
        _check(lib().fv3_mlp_get_params(self._h, _fptr(flat)))
        return self._unpack(flat)

    def forward(self, X, Y, stream=None) -> None:
        _check(lib().fv3_mlp_forward(self._h, C.c_void_p(X.data_ptr()), int(X.shape[0]),
                                     C.c_void_p(Y.data_ptr()), _stream(stream)))

    def gradients(self, X, T, stream=None):
        flat = np.zeros(lib().fv3_mlp_param_count(self._h), dtype=np.float32)
        _check(lib().fv3_mlp_gradients(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                       int(X.shape[0]), _fptr(flat), _stream(stream)))
        return self._unpack(flat)

    def train_step(self, X, T, lr: float = 1e-3, want_loss: bool = False, stream=None):
        loss = C.c_double(0.0)
        _check(lib().fv3_mlp_train_step(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                        int(X.shape[0]), float(lr),
                                        C.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None
