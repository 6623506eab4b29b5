"""CPU tests of the HIP library without a GPU: the shared library loads and
exports every entry point declared in include/fv3.h, and its host-side grid
builder (an implementation independent of the oracle's) produces the same
metric terms as the oracle, interior and halo, on both grid kinds."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
H = 3


@pytest.fixture(scope="module")
def fv3():
    import paper_2205_04148_amd as m

    if not os.path.exists(m._LIBPATH):
        pytest.skip("libfv3.so not built")
    m.lib()
    return m


def test_exports_match_header(fv3):
    hdr = open(os.path.join(ROOT, "include", "fv3.h")).read()
    declared = set(re.findall(r"\b(fv3_[a-z0-9_]+)\s*\(", hdr))
    L = fv3.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(fv3.EXPORTS)


def test_status_strings(fv3):
    L = fv3.lib()
    assert L.fv3_status_string(0) == b"ok"
    assert L.fv3_status_string(-6) == b"Courant number above 1"


METRIC_STAG = {"dx": "Y", "dy": "X", "dxc": "X", "dyc": "Y", "dxa": "C", "dya": "C", "area": "C",
               "area_c": "B", "fC": "C", "fB": "B", "sin_u": "X", "cos_u": "X", "sin_v": "Y",
               "cos_v": "Y", "sin_a": "C", "cos_a": "C"}


def _mask(n, st, interior_only):
    N = n + 2 * H + 1
    sx = 1 if st in ("C", "Y") else 0
    sy = 1 if st in ("C", "X") else 0
    m = np.zeros((N, N), dtype=bool)
    ihi = n + H if st in ("X", "B") else n + H - 1
    jhi = n + H if st in ("Y", "B") else n + H - 1
    for j in range(-H, jhi + 1):
        for i in range(-H, ihi + 1):
            x2, y2 = 2 * i + sx, 2 * j + sy
            inx, iny = 0 <= x2 <= 2 * n, 0 <= y2 <= 2 * n
            if inx and iny:
                m[j + H, i + H] = True
            elif (inx or iny) and not interior_only:
                m[j + H, i + H] = True
    return m


@pytest.mark.parametrize("kind,n", [(1, 12), (1, 16), (0, 10)])
def test_host_metrics_match_oracle(fv3, orc, kind, n):
    g = orc.Grid(kind, n, 2, delta=2500.0, f0=1e-4)
    for name, st in METRIC_STAG.items():
        lib = fv3.host_metric(kind, n, 2, name, dx=2500.0, f0=1e-4)
        ref = g.metric(name)
        # B-point metrics are needed on the interior only; the rest also on edge halos
        m = _mask(n, st, interior_only=(st == "B"))
        a, b = lib[:, m], ref[:, m]
        scale = max(np.abs(b).max(), 1e-300)
        err = np.abs(a - b).max() / scale
        assert err <= 1e-13, (name, err)


def test_pmc_launch_names():
    """Counter rows map to the launch names of the timing hooks: fv_tp_2d by its
    epilogue (not its PPM order), the column solves by pass and site."""
    from paper_2205_04148_amd import pmc

    fvtp = ("_ZN3fv35k_oneITnDaXadL_ZNS_6k_fvtpIfffLi{e}ELi{o}ELi{x}EEEvNS_2BkENS_3GeoENS_6FvArgs"
            "IT_T0_T1_EEEEJS3_NS4_IfffEEEEEvDpT0_")
    for e, want in pmc.FVTP_EPI.items():
        for o in (5, 6, 7, 8):
            for x in (0, 1):
                assert pmc.launch_name(fvtp.format(e=e, o=o, x=x)) == want
    sim1 = ("_ZN3fv35k_oneITnDaXadL_ZNS_6k_sim1IffLi{p}ELi{s}ELb0ELi2ELb0EEEvNS_2BkEiiiiiNS_3GeoE"
            "dddPKT_S6_S6_PKdPKT0_S8_PdSC_SC_PS9_SC_SC_SC_iEEJiiiiiS3_dddPKfSF_SF_S8_SF_S8_SC_SC_SC_"
            "PfSC_SC_SC_iEEEvDpT0_")
    assert pmc.launch_name(sim1.format(p=1, s=0)) == "k_sim1_c.p1"
    assert pmc.launch_name(sim1.format(p=4, s=1)) == "k_sim1_3.p4"
    assert pmc.launch_name("_ZN2at6native18elementwise_kernelIiEEvv") is None
    # plain library kernels, mangled or stored demangled (the learned correction's products)
    assert pmc.launch_name("_ZN3fv311k_gemm_bf16EiiiPKtllS1_llPKfiPflPtl") == "k_gemm_bf16"
    assert pmc.launch_name("fv3::k_gemm_bf16(int, int, int, unsigned short const*, long)") == "k_gemm_bf16"
    assert pmc.launch_name("fv3::k_adam(float*, float const*, float*, float*, long)") == "k_adam"
    assert pmc.launch_name("void at::native::vectorized_elementwise_kernel<4>(int)") is None


def test_pmc_wait_shares(tmp_path):
    """The counter summary derives the wait shares from SQ_WAIT_* over
    SQ_WAVE_CYCLES and the VALU busy share from SQ_ACTIVE_INST_VALU over the
    kernel's duration (GRBM_GUI_ACTIVE summed over the 8 dies)."""
    import json
    import sqlite3

    from paper_2205_04148_amd import pmc

    d = tmp_path / "run"
    d.mkdir()
    con = sqlite3.connect(str(d / "x.db"))
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    sym = "fv3::k_adam(float*, float const*)"
    rows = {"SQ_WAVE_CYCLES": 1000.0, "SQ_WAIT_ANY": 250.0, "SQ_WAIT_INST_ANY": 100.0, "SQ_WAIT_INST_LDS": 10.0,
            "GRBM_GUI_ACTIVE": 8 * 2400.0, "SQ_ACTIVE_INST_VALU": 1024 * 2400.0 / 4 / 2}
    for c, v in rows.items():
        con.execute("insert into counters_collection values (?, ?, ?)", (sym, c, v))
    con.commit()
    con.close()
    out = tmp_path / "o.json"
    pmc.counters_main([str(d), str(out), "test"])
    k = json.loads(out.read_text())["kernels"]["k_adam"]
    assert abs(k["wait_any_share"] - 0.25) < 1e-12 and abs(k["wait_inst_any_share"] - 0.1) < 1e-12
    assert abs(k["wait_inst_lds_share"] - 0.01) < 1e-12
    assert abs(k["valu_busy"] - 0.5) < 1e-12 and abs(k["duration_us_at_2400MHz"] - 1.0) < 1e-12
