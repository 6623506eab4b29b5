"""GPU parity of the learned-correction path against the NumPy oracle.

Network: the oracle applies the same round-to-nearest-even BF16 rounding to
the operands the matrix-core kernels read (inputs, weights, stored
activations, back-propagated errors), so the residual is FP32 accumulation
order over K <= 400 and single-precision tanh; bar 2e-3 of the largest
magnitude per output / parameter array.  Coarsening, features and the
correction are FP64 element arithmetic: bar 1e-13 relative (features are
stored as FP32: bar 1e-6 absolute on z-scores of size O(1))."""
import math

import numpy as np
import pytest

import fv3_inputs as fi
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
H = 3
SIZES = (395, 256, 256, 237)


@pytest.fixture(scope="module")
def fv3():
    import torch

    import paper_2205_04148_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def _params(seed, sizes=SIZES):
    rng = np.random.default_rng(seed)
    ps = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        ps += [(rng.standard_normal((a, b)) / math.sqrt(a)).astype(np.float32),
               (0.1 * rng.standard_normal(b)).astype(np.float32)]
    return ps


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("rows", [16, 300, 4096])
def test_forward_matches_oracle(fv3, rows):
    import torch

    ps = _params(1)
    X = np.random.default_rng(2).standard_normal((rows, SIZES[0])).astype(np.float32)
    net = fv3.MLP(ps, maxrows=4096)
    Xd = _dev(X)
    Yd = torch.empty((rows, SIZES[3]), dtype=torch.float32, device="cuda")
    net.forward(Xd, Yd)
    torch.cuda.synchronize()
    want, _ = omlp.forward([p.astype(np.float64) for p in ps], X.astype(np.float64), bf=True)
    err = _rel(Yd.cpu().numpy(), want)
    print(f"forward rows={rows}: rel err {err:.2e}", flush=True)
    assert err <= 2e-3


def test_small_layers_exact_products(fv3):
    """With W1 = W2 = 0 every row's second hidden layer is tanh(b2), so each
    output row must equal bf16(tanh(b2)) W3 + b3 with small-integer W3 and b3
    (exact in BF16): checks the output product's operand and bias layout
    against a plain product, independently of the input layers."""
    import torch

    rng = np.random.default_rng(3)
    W1 = np.zeros((20, 16), np.float32)
    b1 = np.zeros(16, np.float32)
    W2 = np.zeros((16, 32), np.float32)
    b2 = rng.integers(-3, 4, 32).astype(np.float32) * 0.25
    W3 = rng.integers(-8, 9, (32, 24)).astype(np.float32)
    b3 = rng.integers(-8, 9, 24).astype(np.float32)
    net = fv3.MLP([W1, b1, W2, b2, W3, b3], maxrows=64)
    X = _dev(rng.standard_normal((40, 20)))
    Y = torch.empty((40, 24), dtype=torch.float32, device="cuda")
    net.forward(X, Y)
    torch.cuda.synchronize()
    h2 = omlp.bf16(np.tanh(b2.astype(np.float64)))
    want = h2 @ W3.astype(np.float64) + b3
    got = Y.cpu().numpy()
    assert np.abs(got - want[None, :]).max() <= 1e-4 * np.abs(want).max()


def test_gradients_match_oracle(fv3):
    ps = _params(4)
    rng = np.random.default_rng(5)
    rows = 300
    X = rng.standard_normal((rows, SIZES[0])).astype(np.float32)
    T = rng.standard_normal((rows, SIZES[3])).astype(np.float32)
    net = fv3.MLP(ps, maxrows=512)
    got = net.gradients(_dev(X), _dev(T))
    _, want, _ = omlp.loss_grad([p.astype(np.float64) for p in ps], X.astype(np.float64),
                                T.astype(np.float64), bf=True)
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    errs = {nm: _rel(g, w) for nm, g, w in zip(names, got, want)}
    print("gradients:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= 2e-3, (k, e)


def test_adam_first_step(fv3):
    """The first bias-corrected Adam step moves every parameter by lr against
    the sign of its gradient (up to eps)."""
    ps = _params(6)
    rng = np.random.default_rng(7)
    rows = 256
    X = rng.standard_normal((rows, SIZES[0])).astype(np.float32)
    T = rng.standard_normal((rows, SIZES[3])).astype(np.float32)
    net = fv3.MLP(ps, maxrows=rows)
    lr = 1e-3
    _, g, _ = omlp.loss_grad([p.astype(np.float64) for p in ps], X.astype(np.float64),
                             T.astype(np.float64), bf=True)
    net.train_step(_dev(X), _dev(T), lr=lr)
    new = net.get_params()
    ref = [p.astype(np.float64) for p in ps]
    omlp.adam(ref, g, [np.zeros_like(a) for a in ref], [np.zeros_like(a) for a in ref], step=1, lr=lr)
    for p, gg, q, want in zip(ps, g, new, ref):
        big = np.abs(gg) > 1e-2 * np.abs(gg).max()
        assert big.any()
        assert np.abs(q[big] - want[big]).max() <= 1e-6
        assert np.abs(q - p).max() <= lr * (1 + 1e-4)


def test_training_reduces_loss(fv3):
    """A teacher network's outputs are learnable: 200 Adam steps on 2048
    columns cut the loss by at least half."""
    teacher = _params(8, (40, 32, 32, 16))
    rng = np.random.default_rng(9)
    X = rng.standard_normal((2048, 40))
    T, _ = omlp.forward([p.astype(np.float64) for p in teacher], X, bf=False)
    net = fv3.MLP(_params(10, (40, 32, 32, 16)), maxrows=2048)
    Xd, Td = _dev(X), _dev(T)
    first = net.train_step(Xd, Td, lr=3e-3, want_loss=True)
    for _ in range(198):
        net.train_step(Xd, Td, lr=3e-3)
    last = net.train_step(Xd, Td, lr=3e-3, want_loss=True)
    print(f"teacher fit: loss {first:.3e} -> {last:.3e}", flush=True)
    assert last < 0.5 * first


def test_mlp_bad_arguments(fv3):
    import torch

    net = fv3.MLP(_params(11, (20, 16, 16, 8)), maxrows=32)
    X = torch.zeros((64, 20), dtype=torch.float32, device="cuda")
    Y = torch.zeros((64, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(fv3.FV3Error):
        net.forward(X, Y)            # more rows than maxrows
    with pytest.raises(fv3.FV3Error):
        fv3.MLP(_params(11, (20, 15, 16, 8)), maxrows=32)   # hidden width not a multiple of 16


# ------------------------------------------------------------------ cube-side kernels
@pytest.fixture(scope="module")
def cube32():
    return fi.cube_state(n=32, nz=3, seed=12, nq=0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_coarsen_matches_oracle(fv3, orc, cube32, precision):
    import torch

    init = cube32
    gf = fv3.Grid(1, 32, 3, precision=precision)
    gc = fv3.Grid(1, 8, 3, precision=precision)
    sf = fv3.State.allocate(gf)
    sf.load(init)
    sc = fv3.State.allocate(gc)
    fv3.coarsen(sf, gf, sc, gc)
    torch.cuda.synchronize()
    if precision == "mixed":   # the oracle coarsens the same FP32-rounded fine state
        init = dict(init)
        for k in ("u", "v", "w", "delp", "pt"):
            init[k] = init[k].astype(np.float32).astype(np.float64)
    want = omlp.coarsen(init, orc.Grid(1, 32, 3), orc.Grid(1, 8, 3), 4)
    tol = 1e-13 if precision == "fp64" else 1e-6
    n = 8
    for k, (nj, ni) in {"u": (n + 1, n), "v": (n, n + 1), "w": (n, n), "delp": (n, n),
                        "pt": (n, n), "delz": (n, n)}.items():
        got = sc.get(k)[..., H:H + nj, H:H + ni]
        ref = want[k][..., H:H + nj, H:H + ni]
        e = float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-30))
        print(f"coarsen {precision} {k}: {e:.2e}", flush=True)
        assert e <= tol, (k, e)


def _norm_arrays(F):
    mean = F.mean(0)
    std = F.std(0) + 1e-6
    return mean, std


def test_features_and_flag(fv3, orc):
    import torch

    init = fi.cube_state(n=8, nz=4, seed=13, nq=0)
    g = fv3.Grid(1, 8, 4)
    s = fv3.State.allocate(g)
    s.load(init)
    F = omlp.features(init, 8)
    mean, std = _norm_arrays(F)
    Z = omlp.normalise(F, mean, std)
    lo, hi = Z.min(0), Z.max(0)
    X = torch.empty(F.shape, dtype=torch.float32, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    fv3.column_features(s, g, _dev(mean), _dev(1.0 / std), X, flag, _dev(lo), _dev(hi))
    torch.cuda.synchronize()
    got = X.cpu().numpy()
    assert np.abs(got - Z).max() <= 1e-6 * max(1.0, np.abs(Z).max())
    assert int(flag.item()) == 0 and not omlp.out_of_range(Z, lo, hi)
    # a training range that ends 7 below the data trips the range check
    lo2, hi2 = lo.copy(), hi.copy()
    hi2[5] = Z[:, 5].max() - 7.0
    fv3.column_features(s, g, _dev(mean), _dev(1.0 / std), X, flag, _dev(lo2), _dev(hi2))
    torch.cuda.synchronize()
    assert int(flag.item()) & 1 and omlp.out_of_range(Z, lo2, hi2)


@pytest.mark.parametrize("kind", [0, 1])
def test_apply_correction_matches_oracle(fv3, orc, kind):
    import torch

    n, nz = (16, 3) if kind == 0 else (8, 3)
    init = fi.periodic_state(n=n, nz=nz, seed=14) if kind == 0 else fi.cube_state(n=n, nz=nz, seed=14, nq=0)
    g = fv3.Grid(kind, n, nz)
    s = fv3.State.allocate(g)
    s.load(init)
    T = g.T
    rng = np.random.default_rng(15)
    Y = rng.standard_normal((T * n * n, 3 * nz)).astype(np.float32)
    ym = (0.1 * rng.standard_normal(3 * nz)).astype(np.float32)
    ys = (0.01 * (1 + rng.random(3 * nz))).astype(np.float32)
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    sec = 900.0
    fv3.apply_correction(s, g, _dev(Y), _dev(ym), _dev(ys), sec, flag)
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
    dY = Y.astype(np.float64) * ys.astype(np.float64) + ym.astype(np.float64)
    want = omlp.apply_correction(orc.Grid(kind, n, nz), init, dY, sec)
    for k, (nj, ni) in {"u": (n + 1, n), "v": (n, n + 1), "pt": (n, n)}.items():
        got = s.get(k)[..., H:H + nj, H:H + ni]
        ref = want[k][..., H:H + nj, H:H + ni]
        e = float(np.abs(got - ref).max() / np.abs(ref).max())
        print(f"correction kind={kind} {k}: {e:.2e}", flush=True)
        assert e <= 1e-13, (k, e)


def test_apply_correction_fallback(fv3):
    """A non-finite network output sets bit 1 of the flag and leaves the
    state exactly as it was (the plain coarse run continues)."""
    import torch

    n, nz = 16, 2
    init = fi.periodic_state(n=n, nz=nz, seed=16)
    g = fv3.Grid(0, n, nz)
    s = fv3.State.allocate(g)
    s.load(init)
    before = {k: s.get(k) for k in ("u", "v", "pt")}
    Y = np.ones((n * n, 3 * nz), np.float32)
    Y[37, 4] = np.nan
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    ones = _dev(np.ones(3 * nz))
    fv3.apply_correction(s, g, _dev(Y), ones, ones, 60.0, flag)
    torch.cuda.synchronize()
    assert int(flag.item()) & 2
    for k, a in before.items():
        np.testing.assert_array_equal(s.get(k), a)
    # a flag already set by the range check also blocks the correction
    Y[37, 4] = 1.0
    flag.fill_(1)
    fv3.apply_correction(s, g, _dev(Y), ones, ones, 60.0, flag)
    torch.cuda.synchronize()
    for k, a in before.items():
        np.testing.assert_array_equal(s.get(k), a)

