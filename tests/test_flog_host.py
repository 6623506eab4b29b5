"""The column solves' FP64 logarithm (csrc/flog.hpp), compiled for the host
with hipcc and run on the CPU: within one ulp of the host library's log over
about 10^5 arguments spread over the whole positive range, the pressures and
pressure ratios of the equation of state, arguments near 1, the ends of the
reduction interval, powers of two and subnormal numbers; -inf at 0 and NaN
for negative arguments, NaN and +inf."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2205_04148_amd", "csrc")
DRIVER = r"""
#include "flog.hpp"
#include <cstdio>
#include <cstdlib>
int main()
{
    char buf[64];
    while (std::scanf("%63s", buf) == 1) std::printf("%a\n", fv3::flog(std::strtod(buf, nullptr)));
    return 0;
}
"""


@pytest.fixture(scope="module")
def flog(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("flog")
    src, exe = d / "drv.cpp", d / "drv"
    src.write_text(DRIVER)
    subprocess.run([hipcc, "-O2", "-x", "hip", "--offload-arch=gfx950", "-I", CSRC, "-o", str(exe), str(src)],
                   check=True, capture_output=True)

    def run(xs):
        out = subprocess.run([str(exe)], input="\n".join(float(x).hex() for x in xs), capture_output=True,
                             text=True, check=True).stdout.split()
        return np.array([float.fromhex(o) for o in out])

    return run


def test_within_one_ulp(flog):
    rng = np.random.default_rng(7)
    xs = np.concatenate([
        np.exp(rng.uniform(math.log(1e-300), math.log(1e300), 30000)),   # whole range
        np.exp(rng.uniform(math.log(1.0), math.log(1.2e5), 30000)),      # interface pressures (Pa)
        rng.uniform(0.2, 3.0, 20000),                                    # equation-of-state ratios
        1.0 + rng.uniform(-1e-3, 1e-3, 10000), 1.0 + rng.uniform(-1e-12, 1e-12, 5000),
        2.0 ** np.arange(-1022, 1023, 1.0),
        [math.sqrt(0.5), np.nextafter(math.sqrt(0.5), 0.0), np.nextafter(math.sqrt(0.5), 1.0), 1.0,
         np.nextafter(1.0, 0.0), np.nextafter(1.0, 2.0), 2.0, 1e5, 100.0, np.finfo(float).max,
         np.finfo(float).tiny],
    ])
    got, ref = flog(xs), np.log(xs)
    err = np.abs(got - ref) / np.spacing(np.abs(ref))
    err[ref == 0.0] = np.abs(got[ref == 0.0])
    print("max ulp", err.max(), "share off by one ulp", (err > 0.5).mean())
    assert err.max() <= 1.0, xs[err.argmax()]
    assert got[xs == 1.0][0] == 0.0


def test_special_arguments(flog):
    """Subnormal arguments within one ulp; 0 gives -inf; negative arguments,
    NaN and +inf give NaN (straight-line code without the library's log)."""
    sub = np.array([5e-324, 1e-320, 1e-310, 2.2e-308])
    got, ref = flog(sub), np.log(sub)
    assert np.all(np.abs(got - ref) <= np.spacing(np.abs(ref)))
    got = flog([0.0, -0.0, -1.0, -1e-300, float("nan"), float("inf")])
    assert got[0] == -math.inf and got[1] == -math.inf
    assert all(math.isnan(v) for v in got[2:])
