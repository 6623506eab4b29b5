"""Learned-correction pipeline at toy size, end to end through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fv3():
    import torch

    import paper_2205_04148_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def test_learned_pipeline_small(fv3):
    """The whole learned-correction recipe at toy size (C32 -> C8, 4 levels,
    two training seeds, one 30-min window): data, training and the gain test
    run through the C ABI and report finite numbers."""
    from paper_2205_04148_amd import learned

    cfg = learned.Config(fine_n=32, coarse_n=8, nz=4, fine_bdt=60.0, coarse_bdt=240.0, window=1800.0,
                         windows=1, precision="fp64", hidden=32, bumps=2, epochs=3, batch=128, lr=1e-3)
    X, T, bad = learned.generate(cfg, [11, 12])
    assert bad == 0 and X.shape == (2 * 6 * 64, 20) and T.shape == (2 * 6 * 64, 12)
    assert np.isfinite(X).all() and np.isfinite(T).all()
    model, rep = learned.train(cfg, X, T)
    assert rep["steps"] == 3 * (len(X) // 128) and all(np.isfinite(rep["loss_per_epoch"]))
    res = learned.gain_test(cfg, model, [13])
    print("toy gain test:", res, flush=True)
    assert res["windows"] == 1
    assert np.isfinite(res["rmse_plain_ua_va_pt"]).all() and np.isfinite(res["rmse_corrected_ua_va_pt"]).all()


def test_learned_gain_c96_c24(fv3):
    """The learned correction at a reduced but real size: C96 x 79 fine runs
    (substeps of 30 s) coarsened to C24 x 79 (substeps of 120 s), both with
    a vertical remap every 15 min (fv3_dynamics), 3-h windows, 8 training
    seeds x 2 windows, 2 held-out seeds.  After the first 3-h window the
    corrected coarse run's RMSE of (ua, va, pt) against the coarsened truth
    is at least 5 % below the plain coarse run's for every field, and no
    window falls back to the plain run."""
    from paper_2205_04148_amd import learned

    cfg = learned.Config(fine_n=96, coarse_n=24, nz=79, fine_bdt=30.0, coarse_bdt=120.0, window=10800.0,
                         windows=2, precision="mixed", hidden=256, bumps=4, epochs=30, batch=1024, lr=1e-3,
                         remap=900.0)
    X, T, bad = learned.generate(cfg, list(range(cfg.seed0, cfg.seed0 + 8)))
    assert bad == 0
    model, rep = learned.train(cfg, X, T)
    res = learned.gain_test(cfg, model, [cfg.seed0 + 64, cfg.seed0 + 65])
    print("C96 -> C24 gain test:", res, flush=True)
    assert res["fallback_windows"] == 0
    gain3h = np.array(res["gain_ua_va_pt"][0])
    assert np.all(gain3h >= 0.05), gain3h
