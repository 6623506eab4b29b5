"""GPU test of fv3_mass_sums_noalloc, the allocation-free variant of
fv3_mass_sums (block partials in a fixed device array, combined on the
device).  Its sums must equal fv3_mass_sums' bit for bit: both add the same
block partials in the same order with the same compensated steps.  Two calls
in a row, the second on a smaller grid (fewer partials, so stale partials of
the first call lie beyond the ones it reads), then the first grid again."""
import ctypes as C

import numpy as np
import pytest

import fv3_inputs as fi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fv3():
    import torch

    import paper_2205_04148_amd as m

    assert torch.cuda.is_available()
    m.lib()
    return m


def _case(fv3, kind, n, nz, nq, precision, seed):
    if kind == 1:
        init = fi.cube_state(n=n, nz=nz)
        g = fv3.Grid(1, n, nz, precision=precision)
    else:
        init = fi.periodic_state(n=n, nz=nz, seed=seed)
        g = fv3.Grid(0, n, nz, dx=1000.0, precision=precision)
    s = fv3.State.allocate(g)
    s.load(init)
    rng = np.random.default_rng(seed)
    shape = init["delp"].shape
    qs = [g.upload(rng.uniform(0.0, 1.0, size=shape), nz) for _ in range(nq)]
    return g, s, qs


def _check(fv3, g, s, qs, tag):
    import torch

    out = torch.full((2 + len(qs),), float("nan"), dtype=torch.float64, device="cuda")
    fv3.mass_sums_noalloc(g, s.f["delp"], s.f["pt"], qs, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = fv3.mass_sums(g, s.f["delp"], s.f["pt"], qs)
    print(tag, got, ref, flush=True)
    assert np.all(np.isfinite(got)), tag
    # bar: bit-identical (same partials, same order, same additions)
    assert np.array_equal(got, ref), (tag, got - ref)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_mass_sums_match(fv3, precision):
    big = _case(fv3, 1, 24, 6, 3, precision, seed=11)       # C24: 1 x 6 x 6 blocks of 64 x 4
    small = _case(fv3, 0, 20, 4, 1, precision, seed=12)     # 20 x 20: 1 x 5 x 1 blocks
    _check(fv3, *big, f"{precision} C24x6 nq=3")
    _check(fv3, *small, f"{precision} 20x20x4 nq=1 (second call, smaller)")
    _check(fv3, *big, f"{precision} C24x6 nq=3 (again)")


def test_noalloc_mass_sums_errors(fv3):
    import torch

    g, s, qs = _case(fv3, 0, 16, 2, 1, "fp64", seed=13)
    L = fv3.lib()
    arr = (C.c_void_p * 1)(qs[0].data_ptr())
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    d, p = C.c_void_p(s.f["delp"].data_ptr()), C.c_void_p(s.f["pt"].data_ptr())
    assert L.fv3_mass_sums_noalloc(g.handle, d, p, arr, 1, None, None) == -1        # NULL output
    assert L.fv3_mass_sums_noalloc(g.handle, d, p, None, 1, C.c_void_p(out.data_ptr()), None) == -1
    assert L.fv3_mass_sums_noalloc(g.handle, d, p, arr, 65, C.c_void_p(out.data_ptr()), None) == -1
    assert L.fv3_mass_sums_noalloc(None, d, p, arr, 1, C.c_void_p(out.data_ptr()), None) == -1
    with pytest.raises(ValueError):
        fv3.mass_sums_noalloc(g, s.f["delp"], s.f["pt"], qs, torch.zeros(3, dtype=torch.float32, device="cuda"))
