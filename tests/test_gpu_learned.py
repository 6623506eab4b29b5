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
