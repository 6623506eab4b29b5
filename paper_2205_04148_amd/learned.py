"""Learned per-column correction of a coarse cubed-sphere run.

The paper motivates coupling machine-learned components with the dynamical
core (Sec. III) but gives no recipe; this module is the library's recipe,
driven entirely through the C ABI (every numerical step runs in the HIP
kernels: the acoustic substeps, conservative coarsening, column features, the
BF16 matrix-core network and its Adam training, and the application of the
correction).  Host code here only assembles the training matrix and its
normalisation statistics.

* Samples: fine runs (default C192) of the seeded jet with wind bumps, cut
  into windows of `window` seconds.  At the start of each window the fine
  state is coarsened (default C48) and the coarse model runs the window on
  its own; the target is (coarsened fine - coarse) / window for the
  cell-centred winds and pt, the input the 5 x nz column features of the
  coarse state at the end of the window.
* Network: 5 nz -> 256 -> 256 -> 3 nz, tanh, per-feature z-scores on inputs
  and targets, Adam.
* Gain test: held-out seeds; a plain and a corrected coarse run from the
  same coarsened start, the corrected one adding the predicted tendency x
  window after every window unless the device flag reports non-finite
  outputs or inputs more than 6 sigma outside the training range (then the
  window stays plain); RMSE of (ua, va, pt) against the coarsened truth.

    python -m paper_2205_04148_amd.learned --train-seeds 16 --test-seeds 4
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import (MLP, Grid, State, acoustic_substeps, apply_correction, check_status, coarsen,
               column_features, dynamics)

H = 3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Config:
    def __init__(self, fine_n=192, coarse_n=48, nz=79, fine_bdt=15.0, coarse_bdt=60.0,
                 window=10800.0, windows=4, precision="mixed", hidden=256, bumps=4,
                 epochs=20, batch=4096, lr=1e-3, seed0=5000, remap=900.0, test_windows=0):
        self.fine_n, self.coarse_n, self.nz = fine_n, coarse_n, nz
        self.fine_bdt, self.coarse_bdt = fine_bdt, coarse_bdt
        self.window, self.windows = window, windows
        self.precision, self.hidden, self.bumps = precision, hidden, bumps
        self.epochs, self.batch, self.lr, self.seed0 = epochs, batch, lr, seed0
        # seconds between vertical remaps (0: Lagrangian layers for the whole run)
        self.remap = remap
        # windows of the gain test (0: as many as for training)
        self.test_windows = test_windows if test_windows > 0 else windows


def _advance(s: State, g: Grid, seconds: float, bdt: float, remap: float = 0.0, stream=None) -> None:
    """Advance by `seconds` in acoustic substeps of about bdt; with remap > 0
    through the remapping loop (fv3_dynamics: a vertical remap to the hybrid
    reference coordinate every `remap` seconds)."""
    if remap > 0.0:
        import fv3_inputs as fi

        k_split = max(1, int(round(seconds / remap)))
        n_split = max(1, int(round(seconds / k_split / bdt)))
        ak, bk = fi.hybrid_coefficients(g.nz, g.ptop)
        dynamics(s, g, [], ak, bk, seconds, k_split, n_split, stream=stream)
        return
    n_split = max(1, int(round(seconds / bdt)))
    acoustic_substeps(s, g, seconds, n_split, stream=stream)


def _zeros(shape):
    import torch

    return torch.zeros(shape, dtype=torch.float32, device="cuda")


class Features:
    """Raw (un-normalised) column features of a coarse state, on the device."""

    def __init__(self, g: Grid):
        F = 5 * g.nz
        self.rows = g.T * g.n * g.n
        self.X = _zeros((self.rows, F))
        self.zero = _zeros(F)
        self.one = _zeros(F) + 1.0

    def raw(self, s: State, g: Grid) -> np.ndarray:
        column_features(s, g, self.zero, self.one, self.X)
        return self.X.cpu().numpy().astype(np.float64)


def _initial(cfg: Config, seed: int) -> dict:
    import fv3_inputs as fi

    return fi.cube_state(n=cfg.fine_n, nz=cfg.nz, seed=seed, nq=0, bumps=cfg.bumps)


def _initial_states(cfg: Config, seeds, pool=None):
    """The seeds' initial fine states in order; with a process pool they are
    built on the host ahead of the device runs (a few in flight)."""
    if pool is None:
        for seed in seeds:
            yield _initial(cfg, seed)
        return
    import collections

    ahead = collections.deque()
    it = iter(seeds)
    for seed in it:
        ahead.append(pool.submit(_initial, cfg, seed))
        if len(ahead) >= pool._max_workers:
            break
    for seed in it:
        done = ahead.popleft().result()
        ahead.append(pool.submit(_initial, cfg, seed))
        yield done
    while ahead:
        yield ahead.popleft().result()


def make_pool(workers: int):
    """Host process pool for the initial states.  Create it before the
    process touches the GPU: its workers come from a fork server started
    now, so none of them is forked from a process holding a device context."""
    if workers <= 0:
        return None
    import concurrent.futures as cf
    import multiprocessing as mp

    pool = cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("forkserver"))
    pool.submit(int, 0).result()
    return pool


def generate(cfg: Config, seeds, fields=None, pool=None):
    """Training pairs (inputs, targets) as host float64 arrays, one block of
    (6 coarse_n^2) rows per window and seed."""
    gf = Grid(1, cfg.fine_n, cfg.nz, precision=cfg.precision)
    gc = Grid(1, cfg.coarse_n, cfg.nz, precision=cfg.precision)
    sf, sc, st = State.allocate(gf), State.allocate(gc), State.allocate(gc)
    feat = Features(gc)
    nz = cfg.nz
    Xs, Ts = [], []
    bad = 0
    t0 = time.perf_counter()
    for seed, init in zip(seeds, _initial_states(cfg, seeds, pool)):
        sf.load(init)
        del init
        for w in range(cfg.windows):
            coarsen(sf, gf, sc, gc)
            _advance(sf, gf, cfg.window, cfg.fine_bdt, cfg.remap)
            _advance(sc, gc, cfg.window, cfg.coarse_bdt, cfg.remap)
            coarsen(sf, gf, st, gc)
            ok = check_status(gf) == 0 and check_status(gc) == 0
            if not ok:
                bad += 1
                log(f"seed {seed} window {w}: device status not ok, window dropped")
                break
            x = feat.raw(sc, gc)
            y = feat.raw(st, gc)
            Xs.append(x.astype(np.float32))
            Ts.append(((y[:, :3 * nz] - x[:, :3 * nz]) / cfg.window).astype(np.float32))
        log(f"seed {seed}: done at {time.perf_counter() - t0:.1f} s")
    return np.concatenate(Xs), np.concatenate(Ts), bad


def _stats(A: np.ndarray):
    mean = A.mean(0, dtype=np.float64)
    std = A.std(0, dtype=np.float64)
    std = np.where(std > 1e-12 * np.maximum(1.0, np.abs(mean)), std, 1.0)
    return mean, std


def _init_params(sizes, seed):
    rng = np.random.default_rng(seed)
    ps = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        ps += [(rng.standard_normal((a, b)) * math.sqrt(1.0 / a)).astype(np.float32),
               np.zeros(b, np.float32)]
    return ps


class Model:
    """Trained network plus its normalisation (device arrays)."""

    def __init__(self, net, xm, xs, tm, ts, zlo, zhi):
        import torch

        d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
        self.net = net
        self.xm, self.xinv, self.lo, self.hi = d(xm), d(1.0 / xs), d(zlo), d(zhi)
        self.tm, self.ts = d(tm), d(ts)


def train(cfg: Config, X: np.ndarray, T: np.ndarray, log_every: int = 0):
    """Adam on z-scored inputs and targets; returns (Model, report)."""
    import torch

    xm, xs = _stats(X)
    tm, ts = _stats(T)
    Zx = ((X - xm) / xs).astype(np.float32)
    Zt = ((T - tm) / ts).astype(np.float32)
    rng = np.random.default_rng(cfg.seed0)
    perm = rng.permutation(len(Zx))
    Xd = torch.from_numpy(Zx[perm]).cuda()
    Td = torch.from_numpy(Zt[perm]).cuda()
    sizes = (X.shape[1], cfg.hidden, cfg.hidden, T.shape[1])
    # the same network also evaluates every column of the coarse grid at once
    net = MLP(_init_params(sizes, cfg.seed0), maxrows=max(cfg.batch, 6 * cfg.coarse_n ** 2))
    nb = len(Zx) // cfg.batch
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    for ep in range(cfg.epochs):
        order = rng.permutation(nb)
        ep_loss = 0.0
        for q, b in enumerate(order):
            sl = slice(int(b) * cfg.batch, (int(b) + 1) * cfg.batch)
            want = q == nb - 1 or (log_every and q % log_every == 0)
            l = net.train_step(Xd[sl], Td[sl], lr=cfg.lr, want_loss=bool(want))
            steps += 1
            if want:
                ep_loss = l
        losses.append(ep_loss)
        log(f"epoch {ep}: last-batch loss {ep_loss:.4f}")
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    model = Model(net, xm, xs, tm, ts, Zx.min(0), Zx.max(0))
    rep = {"samples": int(len(Zx)), "epochs": cfg.epochs, "batch": cfg.batch, "steps": steps,
           "train_seconds": sec, "samples_per_s": steps * cfg.batch / sec,
           "loss_per_epoch": [float(x) for x in losses]}
    return model, rep


def _rmse(a: np.ndarray, b: np.ndarray, nz: int):
    d = a[:, :3 * nz] - b[:, :3 * nz]
    return [float(np.sqrt(np.mean(d[:, f * nz:(f + 1) * nz] ** 2))) for f in range(3)]


def gain_test(cfg: Config, model: Model, seeds, pool=None):
    """RMSE of (ua, va, pt) against the coarsened truth after each window,
    plain vs corrected coarse runs from the same start."""
    import torch

    import fv3_inputs as fi

    gf = Grid(1, cfg.fine_n, cfg.nz, precision=cfg.precision)
    gc = Grid(1, cfg.coarse_n, cfg.nz, precision=cfg.precision)
    sf, sp, sq, st = (State.allocate(gf), State.allocate(gc), State.allocate(gc),
                      State.allocate(gc))
    feat = Features(gc)
    rows, nz = feat.rows, cfg.nz
    Xn = _zeros((rows, 5 * nz))
    Y = _zeros((rows, 3 * nz))
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    per = {"plain": np.zeros((cfg.test_windows, 3)), "corrected": np.zeros((cfg.test_windows, 3))}
    fallbacks = 0
    infer_s = 0.0
    for seed, init in zip(seeds, _initial_states(cfg, seeds, pool)):
        sf.load(init)
        del init
        coarsen(sf, gf, sp, gc)
        coarsen(sf, gf, sq, gc)
        for w in range(cfg.test_windows):
            _advance(sf, gf, cfg.window, cfg.fine_bdt, cfg.remap)
            _advance(sp, gc, cfg.window, cfg.coarse_bdt, cfg.remap)
            _advance(sq, gc, cfg.window, cfg.coarse_bdt, cfg.remap)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            flag.zero_()
            column_features(sq, gc, model.xm, model.xinv, Xn, flag, model.lo, model.hi)
            model.net.forward(Xn, Y)
            apply_correction(sq, gc, Y, model.tm, model.ts, cfg.window, flag)
            torch.cuda.synchronize()
            infer_s += time.perf_counter() - t0
            if int(flag.item()):
                fallbacks += 1
            coarsen(sf, gf, st, gc)
            truth = feat.raw(st, gc)
            per["plain"][w] += np.array(_rmse(feat.raw(sp, gc), truth, nz)) ** 2
            per["corrected"][w] += np.array(_rmse(feat.raw(sq, gc), truth, nz)) ** 2
        for g in (gf, gc):
            if check_status(g) != 0:
                log(f"seed {seed}: device status not ok")
    out = {}
    for k, a in per.items():
        out[k] = np.sqrt(a / len(seeds)).tolist()
    gain = (1.0 - np.array(out["corrected"]) / np.array(out["plain"])).tolist()
    n_inf = len(seeds) * cfg.test_windows
    return {"hours": [(w + 1) * cfg.window / 3600.0 for w in range(cfg.test_windows)],
            "rmse_plain_ua_va_pt": out["plain"], "rmse_corrected_ua_va_pt": out["corrected"],
            "gain_ua_va_pt": gain, "fallback_windows": fallbacks, "windows": n_inf,
            "inference_columns_per_s": rows * n_inf / infer_s if infer_s > 0 else None}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-seeds", type=int, default=16)
    ap.add_argument("--test-seeds", type=int, default=4)
    ap.add_argument("--fine-n", type=int, default=192)
    ap.add_argument("--coarse-n", type=int, default=48)
    ap.add_argument("--nz", type=int, default=79)
    ap.add_argument("--windows", type=int, default=4)
    ap.add_argument("--window-hours", type=float, default=3.0)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--bumps", type=int, default=4)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--remap", type=float, default=900.0,
                    help="seconds between vertical remaps (0: no remapping)")
    ap.add_argument("--fine-bdt", type=float, default=15.0)
    ap.add_argument("--coarse-bdt", type=float, default=60.0)
    ap.add_argument("--workers", type=int, default=0, help="host processes building initial states ahead")
    ap.add_argument("--test-windows", type=int, default=0, help="windows of the gain test (0: --windows)")
    a = ap.parse_args(argv)
    pool = make_pool(a.workers)   # before any device work
    cfg = Config(fine_n=a.fine_n, coarse_n=a.coarse_n, nz=a.nz, window=3600.0 * a.window_hours,
                 windows=a.windows, precision=a.precision, epochs=a.epochs, batch=a.batch,
                 lr=a.lr, bumps=a.bumps, remap=a.remap, fine_bdt=a.fine_bdt, coarse_bdt=a.coarse_bdt,
                 test_windows=a.test_windows)
    train_seeds = list(range(cfg.seed0, cfg.seed0 + a.train_seeds))
    test_seeds = list(range(cfg.seed0 + 64, cfg.seed0 + 64 + a.test_seeds))
    t0 = time.perf_counter()
    X, T, bad = generate(cfg, train_seeds, pool=pool)
    gen_s = time.perf_counter() - t0
    log(f"training data {X.shape} -> {T.shape} in {gen_s:.1f} s ({bad} windows dropped)")
    model, rep = train(cfg, X, T)
    res = gain_test(cfg, model, test_seeds, pool=pool)
    out = {"config": {"fine": f"C{cfg.fine_n}x{cfg.nz}", "coarse": f"C{cfg.coarse_n}x{cfg.nz}",
                      "window_h": a.window_hours, "windows": cfg.windows, "test_windows": cfg.test_windows, "train_seeds": train_seeds,
                      "test_seeds": test_seeds, "precision": cfg.precision, "bumps": cfg.bumps,
                      "remap_seconds": cfg.remap, "fine_bdt": cfg.fine_bdt, "coarse_bdt": cfg.coarse_bdt},
           "data_seconds": gen_s, "dropped_windows": bad, "training": rep, "gain_test": res}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
