"""Benchmark of the FV3 acoustic-substep path on one MI355X.

One step = one pass of the whole hot path over the C192 x 79 cubed-sphere
baroclinic-jet state: fv3_acoustic_substeps with n_split = 100 substeps of
15 s (halo exchanges, c_sw, riem_solver_c, p_grad_c, d_sw with fv_tp_2d,
riem_solver3, nh_p_grad), then fv3_tracer_transport of 4 tracers with the
accumulated fluxes, then the compensated global mass sums.

The headline line is the mixed-precision build (FP32 stencil bulk; FP64
column solves, vertical scans, pressure gradients, mass-flux accumulators and
sums); the FP64 build is measured on the same state beside it ("mixed vs
FP64").  Each build's fields after one call of 100 substeps from the initial
state, with the benchmarked options, are compared with the FP64 oracle's
("error_vs_fp64_oracle": per field max |device - oracle| / max |oracle|).

metric  acoustic-substep cell-updates/s = 6 * 192^2 * 79 * 100 / (seconds per step)
        (the tracer transport and the sums are inside the timed step)
roofline  the kernel with the largest share of the step, timed live with HIP
          events on its stream over the timed region; achieved bandwidth =
          algorithmic bytes per launch / mean launch time, where algorithmic
          bytes = (distinct fields the kernel reads or writes, each counted
          once, at their element sizes) x (cells per launch), the paper's
          bandwidth model of Sec. VII-C.  copy_roof_GBs: the library's own
          streaming copy kernel (fv3_device_copy) over 2 GiB.
cpu_baseline  the oracle (plain C, OpenMP) on a bounded sample of the same
          workload: the first substep of C192 x 79 on one thread, the next
          10 on all usable threads (at most 16); the host's CPU model and
          counts are reported with it.  The oracle then finishes the 100
          substeps (untimed) to serve as the FP64 reference above.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--precision mixed|fp64]
       python bench.py --ensemble     (batched uneven ensemble instead: one JSON line)
       python bench.py --remap        (vertical remapping instead: one JSON line)

--ensemble: 32 doubly periodic members with (n, nz) drawn uniformly from
n in 64..256 (step 16) and nz in 32..79, each an isothermal flow with noise;
one step = one call of 20 substeps of 0.2 s on every member.  Reported:
members run one by one, one batched launch per kernel, the batched call
replayed from a HIP graph, and the same after the block-shape autotuner
(its search cost and reuse count), all in cell-updates/s.

--remap: fv3_remap of the C192 x 79 state with every column's layers
redistributed by up to 25 % (fv3_inputs.deform_layers) and 4 tracers, to the
hybrid reference coordinate; the deformed fields are restored by device copies
before each call, outside the timed region (each call is bracketed by device
synchronisations; its kernels are also timed with HIP events).  Reported in
cells remapped per second (all fields of a cell), with the
roofline of the cell-field kernel: algorithmic bytes = each field read and
written once plus delp read once, per cell.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic traffic of one launch per cell of the launch's planes: for each
# kernel the fields read or written (each element once), split into bulk-type
# fields (8 or 4 bytes) and always-FP64 fields (8 bytes).
BYTES_MODEL = {
    # name: (bulk fields, fp64 fields); a field both read and written counts twice
    "k_csw": (12, 0),          # fused c_sw: u, v, delp, pt, w in | uc, vc, delpc, ptc, wc, ax, ay out
    "k_dzc": (2, 2),
    # column solve in four passes; FP64 scratch columns (elimination coefficients,
    # new w, new thickness) are fields of the passes that write and read them
    "k_sim1_c.p1": (3, 3),     # delpc, ptc, wc | delz_c; c', d' out
    "k_sim1_c.p2": (0, 3),     # c', d' | w new out
    "k_sim1_c.p3": (3, 3),     # delpc, ptc, wc | w new; thickness, pkc out
    "k_sim1_c.p4": (0, 2),     # thickness | gz out
    "k_sim1_3.p1": (3, 3),     # delp, pt, w | delz; c', d' out
    "k_sim1_3.p2": (0, 3),
    "k_sim1_3.p3": (4, 3),     # delp, pt, w in, w out | w new; thickness, pfull out
    "k_sim1_3.p4": (0, 3),     # thickness | phi, delz out
    "k_pgradc": (3, 4), "k_dsw_courant": (8, 0),
    "k_dsw_omke": (6, 0), "k_dsw_update": (13, 0), "k_heights": (0, 2), "k_delz_from_zh": (0, 2),
    "k_nhpgrad": (5, 2),       # delp, u, v in, u, v out | pfull, phi (each interface once)
    # fused fv_tp_2d: the field, 4 Courant / area-flux arrays, weights, outputs, per epilogue
    "k_fvtp_delp": (12, 4),    # delp, crx, cry, xfx, yfx, FX, FY, dn, cx, cy (rw) | mfx, mfy (rw)
    "k_fvtp_massw": (10, 0),   # q, 4 fluxes, mx, my, delp old, delp new, q new
    "k_fvtp_flux": (7, 0),     # q, 4 fluxes, FX, FY
    "k_fvtp_adv": (8, 2),      # 4 Courant / area-flux arrays of the two layers around the interface | zh in, zh out
    "k_fvtp_tracer": (6, 4),   # q, 4 fluxes, q out | mx, my, dp1, dp2
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(name, cells, eb):
    key = name.split("<")[0]
    if key in BYTES_MODEL:
        b, d = BYTES_MODEL[key]
        return (b * eb + d * 8) * cells
    return None


def committed_traffic(precision, n, nz, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    this workload, or None when absent or taken with a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_C{n}x{nz}_{precision}.json")
    if not os.path.exists(path):
        return None
    import paper_2205_04148_amd.pmc as pmc

    with open(path) as f:
        doc = json.load(f)
    if doc.get("kernel_source_sha256") != pmc.source_sha256():
        return None
    k = doc["kernels"].get(kernel)
    if not k or k.get("fetch_bytes") is None or k.get("write_bytes") is None:
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def copy_roof(fv3, torch, nbytes=2 << 30, reps=10):
    """Achievable HBM bandwidth of a plain device-to-device copy with the
    library's streaming copy kernel (fv3_device_copy, 2 GiB, read + write
    counted, HIP events around each launch), the practical roof next to the
    8 TB/s peak."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    fv3.device_copy(a, b)
    torch.cuda.synchronize()
    fv3.timing_start("k_stream_copy")
    for _ in range(reps):
        fv3.device_copy(a, b)
    per = fv3.timing_stop()
    ms, cnt = per["k_stream_copy"]
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms / cnt / 1000.0) / 1e9


def host_cpu():
    """CPU model name and logical CPU counts of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def oracle_reference(init, args, opts):
    """The oracle (plain C, FP64, OpenMP over planes and columns) on the
    benchmarked state and options.  Its first substep runs on one thread and
    the next 10 on all usable threads (at most 16), both timed: those are the
    CPU baseline.  The remaining substeps of the n_split run follow, untimed,
    on all threads, so that the final state is the oracle's after n_split
    substeps (the prognostics do not depend on how the substeps are split
    into calls).  Returns (cpu_baseline dict, final oracle state)."""
    import oracle

    n, nz, ns, bdt = args.n, args.nz, args.n_split, args.bdt
    threads = min(16, len(os.sched_getaffinity(0)))
    og = oracle.Grid(1, n, nz, **opts)
    s = oracle.new_state(og, init)
    cells = 6 * n * n * nz
    oracle.set_threads(1)
    t0 = time.perf_counter()
    st1 = oracle.acoustic_substeps(og, s, bdt, 1)
    t1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    nall = min(10, ns - 1)
    t0 = time.perf_counter()
    st2 = oracle.acoustic_substeps(og, s, bdt * nall, nall) if nall > 0 else 0
    tall = time.perf_counter() - t0
    rest = ns - 1 - nall
    t0 = time.perf_counter()
    st3, done = 0, 0
    while done < rest and st3 == 0:
        m = min(30, rest - done)      # in chunks, with a progress line each
        st3 = oracle.acoustic_substeps(og, s, bdt * m, m)
        done += m
        log(f"oracle: {1 + nall + done} of {ns} substeps, status {st3}")
    trest = time.perf_counter() - t0
    model, ncpu, usable = host_cpu()
    rate_all = cells * nall / tall if nall > 0 else None
    cpu = {"value": rate_all, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"C{n}x{nz} cubed sphere FP64 from the benchmark's state: substep 1 on 1 thread "
                     f"({t1:.1f} s), substeps 2-{1 + nall} on {threads} threads ({tall:.1f} s); "
                     f"status {st1}, {st2}",
           "rate_1_thread": cells / t1, "rate_all_threads": rate_all,
           "threads_all": threads, "nproc": ncpu, "usable_cpus": usable, "cpu_model": model}
    log(f"oracle: 1 substep on 1 thread {t1:.1f} s, {nall} on {threads} threads {tall:.1f} s, "
        f"{rest} more {trest:.1f} s (status {st3})")
    return cpu, s


def run_precision(fv3, torch, init, args, precision):
    n, nz, ns, bdt = args.n, args.nz, args.n_split, args.bdt
    dt = bdt * ns
    g = fv3.Grid(1, n, nz, precision=precision, **grid_opts(args))
    s = fv3.State.allocate(g)
    s.load(init)
    if args.moist:
        # humidity for the moist column solves: 0.02 x the first tracer (U[0, 1])
        s.set_humidity(0.02 * init["q"][0])
    qs = [g.upload(q, nz) for q in init["q"]]
    stream = torch.cuda.current_stream()

    def step():
        fv3.acoustic_substeps(s, g, dt, ns, stream=stream)
        fv3.tracer_transport(qs, s, g, nsplt=0, stream=stream)
        fv3.mass_sums(g, s.f["delp"], s.f["pt"], qs, stream=stream)

    # warm-up; the first warm-up step also times every kernel to find the dominant one
    fv3.timing_start("")
    step()
    per_kernel = fv3.timing_stop()
    for _ in range(max(0, args.warmup - 1)):
        step()
    torch.cuda.synchronize()
    dom = max(per_kernel.items(), key=lambda kv: kv[1][0])[0]
    tot_ms = sum(v[0] for v in per_kernel.values())
    log(f"[{precision}] kernel share of a warm-up step (HIP events):")
    for k, (ms, c) in sorted(per_kernel.items(), key=lambda kv: -kv[1][0]):
        log(f"  {k:28s} {ms:9.2f} ms  {100 * ms / tot_ms:5.1f}%  {c:5d} launches  {1000 * ms / c:8.1f} us/launch")

    fv3.timing_start(dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    live = fv3.timing_stop()
    st = fv3.check_status(g)
    cells = 6 * n * n * nz
    sec = (t1 - t0) / args.steps
    ms_dom, cnt_dom = live.get(dom, (float("nan"), 1))
    avg_s = ms_dom / cnt_dom / 1000.0
    eb = 8 if precision == "fp64" else 4
    bl = kernel_bytes(dom, cells, eb)
    achieved = bl / avg_s / 1e9 if bl else None
    traffic = committed_traffic(precision, n, nz, dom)
    roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": traffic, "bytes_per_launch": bl, "mean_launch_us": avg_s * 1e6,
            "traffic_GBs": traffic / avg_s / 1e9 if traffic else None,
            "launches": cnt_dom, "share_of_step": per_kernel[dom][0] / tot_ms}
    log(f"[{precision}] {1000 * sec:.1f} ms/step, {cells * ns / sec:.3e} cell-updates/s, status {st}")
    del s, qs, g
    torch.cuda.empty_cache()
    return {"value": cells * ns / sec, "ms_per_step": 1000 * sec, "roofline": roof,
            "device_status": int(st), "ms_per_substep": 1000 * sec / ns}


PREC_FIELDS = ("u", "v", "w", "delp", "pt", "delz", "pfull", "phi")


def grid_opts(args):
    """The options of the benchmarked configuration (same names in the
    library binding and the oracle)."""
    return {"beta": args.beta, "d2_bg": args.d2_bg, "dddmp": args.dddmp, "hord": args.hord,
            "hord_tr": args.hord_tr, "pp_order": args.pp_order, "nord": args.nord, "d4_bg": args.d4_bg,
            "vtdm": args.vtdm, "edge_fix": args.edge_fix, "edge_ppm": args.edge_ppm,
            "edge_interp": args.edge_interp}


def gpu_final_fields(fv3, torch, init, args, precision):
    """One call of n_split substeps from the initial state with the
    benchmarked options; the interior of each field of PREC_FIELDS."""
    n, nz, ns, bdt = args.n, args.nz, args.n_split, args.bdt
    g = fv3.Grid(1, n, nz, precision=precision, **grid_opts(args))
    s = fv3.State.allocate(g)
    s.load(init)
    if args.moist:
        s.set_humidity(0.02 * init["q"][0])
    fv3.acoustic_substeps(s, g, bdt * ns, ns)
    torch.cuda.synchronize()
    st = fv3.check_status(g)
    res = {k: interior(s.get(k), n, k) for k in PREC_FIELDS}
    del s, g
    torch.cuda.empty_cache()
    return res, st


def interior(a, n, k, H=3):
    ni = n + 1 if k == "v" else n
    nj = n + 1 if k == "u" else n
    return a[..., H:H + nj, H:H + ni]


def field_errors(res, ref_state, n):
    """max |device - oracle| / max |oracle| over the interior, per field."""
    out = {}
    for k in PREC_FIELDS:
        ref = interior(ref_state[k], n, k)
        out[k] = float(abs(res[k] - ref).max() / max(abs(ref).max(), 1e-300))
    return out


def ensemble_bench(fv3, torch, args):
    import fv3_inputs as fi

    sizes = fi.ensemble_sizes(32, seed=4)
    ns, bdt = 20, 0.2
    dt = ns * bdt
    grids, states, inits = [], [], []
    t0 = time.perf_counter()
    for q, (n, nz) in enumerate(sizes):
        g = fv3.Grid(0, n, nz, precision=args.precision)
        s = fv3.State.allocate(g)
        init = fi.periodic_state(n=n, nz=nz, seed=100 + q, nq=0)
        s.load(init)
        grids.append(g)
        states.append(s)
        inits.append(init)
    cells = sum(n * n * nz for n, nz in sizes)
    log(f"ensemble: {len(sizes)} members, {cells:.3e} cells, set up in {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / reps

    def reload():
        for s, init in zip(states, inits):
            s.load(init)
        torch.cuda.synchronize()

    def one_by_one():
        for s, g in zip(states, grids):
            fv3.acoustic_substeps(s, g, dt, ns, stream=stream)

    res = {}
    res["one_by_one_s"] = timed(one_by_one, args.steps)
    reload()
    e = fv3.Ensemble(states, grids, dt, ns, graph=False)
    res["batched_s"] = timed(lambda: e.run(stream), args.steps)
    reload()
    eg = fv3.Ensemble(states, grids, dt, ns, graph=True)
    res["batched_graph_s"] = timed(lambda: eg.run(stream), args.steps)
    st_ok = all(fv3.check_status(g) == 0 for g in grids)
    # autotune on the same states (left undefined by the search), then reload
    tr = e.tune(reps=3, stream=stream)
    reload()
    et = fv3.Ensemble(states, grids, dt, ns, graph=True)
    res["tuned_graph_s"] = timed(lambda: et.run(stream), args.steps)
    st_ok = st_ok and all(fv3.check_status(g) == 0 for g in grids)
    rate = {k.replace("_s", ""): cells * ns / v for k, v in res.items()}
    for k, v in rate.items():
        log(f"  {k:16s} {v:.3e} cell-updates/s  ({1000 * cells * ns / v / ns:.3f} ms/substep)")
    best = max(rate.values())
    return {
        "metric": "ensemble acoustic-substep cell-updates/s, 32 uneven members, batched vs one by one",
        "value": best, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": 1000 * cells * ns / best, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"32 doubly periodic members n in 64..256, nz in 32..79 "
                               f"({cells} cells), {ns} substeps of {bdt} s per step",
                   "precision": args.precision, "members": [list(x) for x in sizes]},
        "rates": rate, "speedup_batched_graph_vs_one_by_one": rate["batched_graph"] / rate["one_by_one"],
        "autotune": tr, "device_status_ok": st_ok,
    }


def remap_bench(fv3, torch, args):
    import fv3_inputs as fi

    n, nz, nq = args.n, args.nz, 4
    init = fi.cube_state(n=n, nz=nz)
    init["delp"] = fi.deform_layers(init["delp"], seed=3)
    g = fv3.Grid(1, n, nz, precision=args.precision)
    s = fv3.State.allocate(g)
    s.load(init)
    qs = [g.upload(q, nz) for q in init["q"][:nq]]
    keep = {k: s.f[k].clone() for k in ("u", "v", "w", "delp", "pt", "delz")}
    qkeep = [q.clone() for q in qs]
    ak, bk = fi.hybrid_coefficients(nz, g.ptop)
    stream = torch.cuda.current_stream()

    def restore():
        for k, v in keep.items():
            s.f[k].copy_(v)
        for q, v in zip(qs, qkeep):
            q.copy_(v)

    for _ in range(max(1, args.warmup)):
        restore()
        fv3.remap(s, g, ak, bk, qs, stream=stream)
    torch.cuda.synchronize()
    fv3.timing_start("k_remap")
    wall = 0.0
    for _ in range(args.steps):
        restore()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fv3.remap(s, g, ak, bk, qs, stream=stream)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
    per = fv3.timing_stop()
    st = fv3.check_status(g)
    kern_ms = sum(v[0] for v in per.values()) / args.steps
    cells = 6 * n * n * nz
    eb = 8 if args.precision == "fp64" else 4
    for k, (ms, c) in sorted(per.items(), key=lambda kv: -kv[1][0]):
        log(f"  {k:16s} {ms / args.steps:8.3f} ms/call  {c // args.steps:3d} launches/call  "
            f"{1000 * ms / c:8.1f} us/launch")
    ms_c, cnt_c = per["k_remap_cells"]
    avg_s = ms_c / cnt_c / 1000.0
    nf = 3 + nq                                       # pt, w, delz, tracers in one launch
    bl = cells * ((nf - 1) * 2 * eb + 2 * 8 + eb)     # bulk fields r+w, delz r+w, delp r
    achieved = bl / avg_s / 1e9
    return {
        "metric": "vertical remap cells/s at C192x79 (all prognostics + 4 tracers per cell)",
        "value": cells / (wall / args.steps), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000 * wall / args.steps, "kernel_ms_per_call": kern_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": f"C{n}x{nz} cubed-sphere baroclinic jet, layers deformed by up to 25 %, "
                               f"{nq} tracers, hybrid reference coordinate",
                   "precision": args.precision, "cells": cells, "device_status": int(st)},
        "roofline": {"bound": "hbm", "kernel": "k_remap_cells", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": bl, "mean_launch_us": avg_s * 1e6},
        "per_kernel_ms_per_call": {k: v[0] / args.steps for k, v in per.items()},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--n", type=int, default=192)
    ap.add_argument("--nz", type=int, default=79)
    ap.add_argument("--n-split", type=int, default=100)
    ap.add_argument("--bdt", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--ensemble", action="store_true")
    ap.add_argument("--remap", action="store_true")
    ap.add_argument("--beta", type=float, default=1.0, help="off-centring of the vertical solve (0.5 .. 1)")
    ap.add_argument("--hord", type=int, default=8, choices=[5, 6, 8],
                    help="PPM order: 8 monotone, 6 unlimited, 5 2dx-filtered")
    ap.add_argument("--hord-tr", type=int, default=0, choices=[0, 5, 6, 7, 8],
                    help="tracer PPM order (0: as --hord; 7 positive-definite)")
    ap.add_argument("--pp-order", type=int, default=2, choices=[2, 4],
                    help="interface pressure perturbation of the column solves: 2 mass-linear, 4 cubic")
    ap.add_argument("--nord", type=int, default=0, choices=[0, 1, 2],
                    help="higher-order divergence damping: 1 del-4, 2 del-6")
    ap.add_argument("--d4-bg", type=float, default=0.0, help="its coefficient (0 .. 0.25)")
    ap.add_argument("--vtdm", type=float, default=0.0, help="del-2 vorticity damping (0 .. 0.25)")
    ap.add_argument("--edge-fix", action="store_true", help="edge-flux fix-up at the tile edges")
    ap.add_argument("--edge-ppm", action="store_true", help="one-sided PPM edge values at the tile edges")
    ap.add_argument("--edge-interp", action="store_true",
                    help="one-sided c_sw and nh_p_grad interpolations at the tile edges")
    ap.add_argument("--moist", action="store_true",
                    help="moist column solves with humidity 0.02 x the first tracer")
    ap.add_argument("--d2-bg", type=float, default=0.0, help="del-2 divergence damping (0 .. 0.25)")
    ap.add_argument("--dddmp", type=float, default=0.0, help="Smagorinsky divergence damping (0 .. 1)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the acoustic substep path holds all six cube "
              "tiles on a single MI355X (no multi-GPU path in this build)", file=sys.stderr)
        sys.exit(2)

    import torch

    import fv3_inputs as fi
    import paper_2205_04148_amd as fv3

    if args.ensemble:
        print(json.dumps(ensemble_bench(fv3, torch, args)), flush=True)
        return
    if args.remap:
        print(json.dumps(remap_bench(fv3, torch, args)), flush=True)
        return

    n, nz = args.n, args.nz
    t0 = time.perf_counter()
    init = fi.cube_state(n=n, nz=nz)
    log(f"initial state C{n}x{nz}: {time.perf_counter() - t0:.1f} s")

    roof_copy = copy_roof(fv3, torch)
    log(f"device copy roof (library streaming copy): {roof_copy:.0f} GB/s")
    main_res = run_precision(fv3, torch, init, args, args.precision)
    main_res["roofline"]["copy_roof_GBs"] = roof_copy
    main_res["roofline"]["frac_of_copy_roof"] = (main_res["roofline"]["achieved"] or 0) / roof_copy
    other = None
    if not args.no_compare:
        other_prec = "fp64" if args.precision == "mixed" else "mixed"
        r = run_precision(fv3, torch, init, args, other_prec)
        other = {"precision": other_prec, "value": r["value"], "ms_per_step": r["ms_per_step"],
                 "roofline": r["roofline"]}
    cpu = None
    err = None
    if not args.no_cpu:
        # the device's fields after one call of n_split substeps, each
        # precision, then the oracle from the same state with the same options
        precs = [args.precision] + ([] if args.no_compare else [other["precision"]])
        final = {p: gpu_final_fields(fv3, torch, init, args, p) for p in precs}
        log("oracle: CPU baseline and FP64 reference ...")
        oinit = dict(init)
        if args.moist:
            oinit["qv"] = 0.02 * init["q"][0]
        cpu, ref = oracle_reference(oinit, args, grid_opts(args))
        err = {"reference": "FP64 oracle", "substeps": args.n_split,
               "measure": "max |device - oracle| / max |oracle| over the interior"}
        for p, (res, st) in final.items():
            err[p] = field_errors(res, ref, n)
            err[p]["device_status"] = int(st)
            log(f"[{p}] vs FP64 oracle after {args.n_split} substeps: "
                + ", ".join(f"{k} {v:.1e}" for k, v in err[p].items() if k != "device_status"))
        del ref
    cells = 6 * n * n * nz
    out = {
        "metric": "acoustic-substep cell-updates/s at C192x79, mixed vs FP64; % HBM peak",
        "value": main_res["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": main_res["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"C{n}x{nz} cubed-sphere baroclinic jet, {args.n_split} acoustic "
                               f"substeps of {args.bdt:g} s + 4-tracer transport + mass sums per step",
                   "precision": args.precision, "n_split": args.n_split, "cells": cells, "beta": args.beta,
                   "d2_bg": args.d2_bg, "dddmp": args.dddmp, "hord": args.hord,
                   "hord_tr": args.hord_tr, "pp_order": args.pp_order, "moist": args.moist,
                   "nord": args.nord, "d4_bg": args.d4_bg, "vtdm": args.vtdm,
                   "edge_fix": args.edge_fix,
                   "edge_ppm": args.edge_ppm, "edge_interp": args.edge_interp,
                   "ms_per_substep": main_res["ms_per_substep"],
                   "device_status": main_res["device_status"]},
        "roofline": main_res["roofline"],
        "cpu_baseline": cpu,
        "compare": other,
        "error_vs_fp64_oracle": err,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
