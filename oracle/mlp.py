"""ORACLE (test infrastructure only): the learned per-column correction.

NumPy FP64 reference for the extension that corrects a coarse-grid run of the
method with a per-column neural network trained on coarsened fine-grid runs of
the method itself (the paper motivates coupling machine learning with the
dynamical core, Sec. III; it gives no recipe, so the recipe below is a
reading):

* coarsening by an integer factor r: cell mass delp and thickness delz are
  area means over the r x r fine cells; pt, w and tracers mass-weighted
  means; D-grid winds edge-length-weighted means of the r fine edges on each
  coarse edge (circulation-conserving);
* column features: cell-centred winds (mean of the two D-grid faces), pt, w,
  delp on every level;
* network: x -> tanh(x W1 + b1) -> tanh(. W2 + b2) -> . W3 + b3, mean squared
  error on normalised targets, gradients by the chain rule, Adam.

The GPU kernels feed BF16 operands to the matrix cores and accumulate in FP32;
`bf16=True` applies the same round-to-nearest-even BF16 rounding to the same
operands here, so that the comparison measures only accumulation order.
"""
from __future__ import annotations

import numpy as np

H = 3


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (round to nearest, ties to even) and return as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def forward(params, X, bf: bool = True):
    """Returns (Y, cache).  params = [W1, b1, W2, b2, W3, b3], W as (in, out)."""
    W1, b1, W2, b2, W3, b3 = params
    Xb = _r(X, bf)
    Z1 = Xb @ _r(W1, bf) + b1
    H1 = np.tanh(Z1)
    H1b = _r(H1, bf)
    Z2 = H1b @ _r(W2, bf) + b2
    H2 = np.tanh(Z2)
    H2b = _r(H2, bf)
    Y = H2b @ _r(W3, bf) + b3
    return Y, (Xb, H1, H1b, H2, H2b)


def loss_grad(params, X, T, bf: bool = True):
    """Mean squared error over all outputs and its gradients (chain rule)."""
    W1, b1, W2, b2, W3, b3 = params
    Y, (Xb, H1, H1b, H2, H2b) = forward(params, X, bf)
    N = Y.size
    R = Y - T
    loss = float(np.sum(R * R) / N)
    dY = 2.0 * R / N
    dYb = _r(dY, bf)
    dW3 = H2b.T @ dYb
    db3 = dY.sum(axis=0)
    dH2 = dYb @ _r(W3, bf).T
    dZ2 = dH2 * (1.0 - H2 * H2)
    dZ2b = _r(dZ2, bf)
    dW2 = H1b.T @ dZ2b
    db2 = dZ2.sum(axis=0)
    dH1 = dZ2b @ _r(W2, bf).T
    dZ1 = dH1 * (1.0 - H1 * H1)
    dZ1b = _r(dZ1, bf)
    dW1 = Xb.T @ dZ1b
    db1 = dZ1.sum(axis=0)
    return loss, [dW1, db1, dW2, db2, dW3, db3], Y


def adam(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; `step` counts from 1."""
    for p, g, mm, vv in zip(params, grads, m, v):
        mm *= b1
        mm += (1 - b1) * g
        vv *= b2
        vv += (1 - b2) * g * g
        mh = mm / (1 - b1 ** step)
        vh = vv / (1 - b2 ** step)
        p -= lr * mh / (np.sqrt(vh) + eps)


# ------------------------------------------------------------- coarsening
def coarsen(fine: dict, gf, gc, r: int) -> dict:
    """Coarsen a cubed-sphere state (oracle layout f[t][k][j+3][i+3]) from the
    oracle grid gf (n) to gc (n / r)."""
    n, nc = gf.n, gc.n
    assert n == r * nc
    Af = gf.metric("area")[:, H:H + n, H:H + n]
    Ac = gc.metric("area")[:, H:H + nc, H:H + nc]
    dxf = gf.metric("dx")[:, H:H + n + 1, H:H + n]      # y-faces
    dyf = gf.metric("dy")[:, H:H + n, H:H + n + 1]      # x-faces

    def blocks(a):   # [..., n, n] -> [..., nc, nc] sums of r x r blocks
        s = a.shape[:-2]
        return a.reshape(s + (nc, r, nc, r)).sum(axis=(-3, -1))

    out = {}
    nz = fine["delp"].shape[1]
    N = nc + 2 * H + 1
    z = lambda: np.zeros((6, nz, N, N))
    dp = fine["delp"][:, :, H:H + n, H:H + n]
    mass = dp * Af[:, None]
    msum = blocks(mass)
    d = z()
    d[:, :, H:H + nc, H:H + nc] = msum / Ac[:, None]
    out["delp"] = d
    dz = z()
    dz[:, :, H:H + nc, H:H + nc] = blocks(fine["delz"][:, :, H:H + n, H:H + n] * Af[:, None]) / Ac[:, None]
    out["delz"] = dz
    for k in ("pt", "w"):
        a = z()
        a[:, :, H:H + nc, H:H + nc] = blocks(fine[k][:, :, H:H + n, H:H + n] * mass) / msum
        out[k] = a
    # D-grid winds: coarse y-face (I, J) = fine y-faces (rI .. rI+r-1, rJ)
    u = fine["u"][:, :, H:H + n + 1:r, H:H + n]         # rows j = 0, r, 2r, ... n
    w_ = dxf[:, ::r, :]
    num = (u * w_[:, None]).reshape(6, nz, nc + 1, nc, r).sum(-1)
    den = w_.reshape(6, nc + 1, nc, r).sum(-1)
    uc = z()
    uc[:, :, H:H + nc + 1, H:H + nc] = num / den[:, None]
    out["u"] = uc
    v = fine["v"][:, :, H:H + n, H:H + n + 1:r]
    w_ = dyf[:, :, ::r]
    num = (v * w_[:, None]).reshape(6, nz, nc, r, nc + 1).sum(-2)
    den = w_.reshape(6, nc, r, nc + 1).sum(-2)
    vc = z()
    vc[:, :, H:H + nc, H:H + nc + 1] = num / den[:, None]
    out["v"] = vc
    out["phis"] = np.zeros((6, N, N))
    return out


def features(state: dict, n: int) -> np.ndarray:
    """Column features (T*n*n, 5*nz): ua, va, pt, w, delp per level, with the
    cell-centred winds the means of the two D-grid faces of each cell."""
    u = state["u"][:, :, H:H + n + 1, H:H + n]
    v = state["v"][:, :, H:H + n, H:H + n + 1]
    ua = 0.5 * (u[:, :, :-1, :] + u[:, :, 1:, :])
    va = 0.5 * (v[:, :, :, :-1] + v[:, :, :, 1:])
    cols = []
    for a in (ua, va, state["pt"][:, :, H:H + n, H:H + n], state["w"][:, :, H:H + n, H:H + n],
              state["delp"][:, :, H:H + n, H:H + n]):
        cols.append(a.transpose(0, 2, 3, 1).reshape(-1, a.shape[1]))   # (T*n*n, nz)
    return np.concatenate(cols, axis=1)


def targets(a: dict, b: dict, n: int, seconds: float) -> np.ndarray:
    """Tendency columns (T*n*n, 3*nz) of (ua, va, pt): (a - b) / seconds."""
    fa, fb = features(a, n), features(b, n)
    nz = fa.shape[1] // 5
    return (fa[:, :3 * nz] - fb[:, :3 * nz]) / seconds


def normalise(F: np.ndarray, mean: np.ndarray, std: np.ndarray) -> np.ndarray:
    """Per-feature z-score (x - mean) / std."""
    return (F - mean) / std


def out_of_range(Z: np.ndarray, lo: np.ndarray, hi: np.ndarray, margin: float = 6.0) -> bool:
    """True if any normalised input is not finite or lies more than `margin`
    (in units of the training standard deviation) outside [lo, hi]."""
    ok = np.isfinite(Z) & (Z >= lo - margin) & (Z <= hi + margin)
    return not bool(ok.all())


def apply_correction(g, state: dict, dY: np.ndarray, seconds: float) -> dict:
    """Add `seconds` x the physical tendencies dY (T*n*n, 3*nz: ua, va, pt per
    level) to a copy of `state` (oracle layout).  pt changes at cells; the
    cell wind increments get their halos from the neighbouring tiles (tile
    components, rotated across tile edges) and each D-grid face takes the mean
    of the increments of the two cells that share it."""
    from oracle import halo_fill_pair

    n, T = g.n, g.T
    nz = dY.shape[1] // 3
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in state.items()}
    N = n + 2 * H + 1

    def cells(block):   # (T*n*n, nz) -> [T][nz][n][n]
        return block.reshape(T, n, n, nz).transpose(0, 3, 1, 2)

    dU = np.zeros((T, nz, N, N))
    dV = np.zeros((T, nz, N, N))
    dU[:, :, H:H + n, H:H + n] = seconds * cells(dY[:, :nz])
    dV[:, :, H:H + n, H:H + n] = seconds * cells(dY[:, nz:2 * nz])
    out["pt"][:, :, H:H + n, H:H + n] += seconds * cells(dY[:, 2 * nz:])
    halo_fill_pair(g, dU, "C", dV, "C", kind="signed")
    out["u"][:, :, H:H + n + 1, H:H + n] += 0.5 * (dU[:, :, H - 1:H + n, H:H + n] + dU[:, :, H:H + n + 1, H:H + n])
    out["v"][:, :, H:H + n, H:H + n + 1] += 0.5 * (dV[:, :, H:H + n, H - 1:H + n] + dV[:, :, H:H + n, H:H + n + 1])
    return out
