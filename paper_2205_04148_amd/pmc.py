"""HBM traffic per kernel launch from two rocprofv3 counter databases.

    python -m paper_2205_04148_amd.pmc FETCH_DIR WRITE_DIR OUT.json WORKLOAD
    python -m paper_2205_04148_amd.pmc counters DIR OUT.json WORKLOAD [DIR2 ...]
    python -m paper_2205_04148_amd.pmc trace DIR OUT.md TITLE COMMAND

FETCH_DIR / WRITE_DIR hold the rocpd databases of one ``rocprofv3 --pmc
FETCH_SIZE`` and one ``--pmc WRITE_SIZE`` run of the same command.  Both
counters are scaled by what they read for the plain copy kernel of the run
(``k_copy``: each thread reads one element of its source type and writes one
of its destination type, so its bytes are known exactly).  The output maps
each launch name used by the library's timing hooks to its mean calibrated
bytes read and written per launch, with the SHA-256 of the kernel source the
counters were taken with (a reader treats the numbers as stale when the
source has changed).
"""
from __future__ import annotations

import collections
import glob
import hashlib
import json
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "kernels.hip")
FVTP_EPI = {0: "k_fvtp_flux", 1: "k_fvtp_delp", 2: "k_fvtp_massw", 3: "k_fvtp_adv", 4: "k_fvtp_tracer"}
TSIZE = {"f": 4, "d": 8}


def source_sha256() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def launch_name(symbol: str):
    """Launch name of a library kernel from its mangled k_one<...> symbol."""
    m = re.search(r"k_oneITnDaXadL_ZNS_(\d+)(k_\w+)", symbol)
    if not m:
        # plain kernels of the library (reductions, copies, the learned
        # correction's products): their own name
        p = re.search(r"_ZN3fv3(\d+)(k_\w+)", symbol) or re.search(r"^_Z(\d+)(k_\w+)", symbol)
        if p:
            return p.group(2)[:int(p.group(1))]
        # names stored demangled ("fv3::k_name(args)")
        p = re.search(r"fv3::(k_\w+)\s*[(<]", symbol)
        return p.group(1) if p else None
    ln = int(m.group(1))
    rest = m.group(2)
    name, targs = rest[:ln], rest[ln:]
    ints = [int(x) for x in re.findall(r"Li(\d+)E", targs.split("EEvNS_")[0])]
    if name == "k_fvtp" and ints:
        # template integers: the epilogue first (then the PPM order and the
        # tile-edge switch)
        return FVTP_EPI.get(ints[0], name)
    if name == "k_sim1" and len(ints) >= 2:
        return f"k_sim1_{'c' if ints[1] == 0 else '3'}.p{ints[0]}"
    if name in ("k_csw", "k_nhpgrad", "k_halo_scalar", "k_halo_pair", "k_fill"):
        return name
    if name == "k_copy":
        t = re.match(r"I([fd])([fd])E", targs)
        return f"k_copy<{t.group(1)}{t.group(2)}>" if t else name
    if name in ("k_heights", "k_delz_from_zh"):
        return name
    return name + "<B>"


def load(dirname: str, counter: str):
    db = glob.glob(os.path.join(dirname, "**", "*.db"), recursive=True)
    if not db:
        raise FileNotFoundError(f"no rocpd database under {dirname}")
    con = sqlite3.connect(db[0])
    out = collections.defaultdict(list)
    for sym, val, grid in con.execute(
            "select kernel_name, value, grid_size from counters_collection where counter_name = ?", (counter,)):
        name = launch_name(sym)
        if name:
            out[name].append((float(val), int(grid)))
    return out


def calibrate(rows, counter: str) -> float:
    """Bytes per counter KiB from the copy kernel of the run."""
    for key in ("k_copy<fd>", "k_copy<dd>", "k_copy<ff>", "k_copy<df>"):
        if key in rows:
            src, dst = key[7], key[8]
            kib, grid = rows[key][0]
            elem = TSIZE[src] if counter == "FETCH_SIZE" else TSIZE[dst]
            return elem * grid / kib
    raise KeyError("no copy kernel in the counter run")


def load_all(dirname: str):
    """Every counter of a rocpd database: {launch name: {counter: [values]}}."""
    db = glob.glob(os.path.join(dirname, "**", "*.db"), recursive=True)
    if not db:
        raise FileNotFoundError(f"no rocpd database under {dirname}")
    con = sqlite3.connect(db[0])
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    for sym, cname, val in con.execute("select kernel_name, counter_name, value from counters_collection"):
        name = launch_name(sym)
        if name:
            out[name][cname].append(float(val))
    return out


SIMDS = 1024          # 256 compute units x 4 SIMDs (MI355X)
XCDS = 8              # GRBM_GUI_ACTIVE comes summed over the 8 accelerator dies
VALU_CYCLES = 4       # a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles


def counters_main(a):
    """counters DIR OUT.json WORKLOAD [DIR2 ...]: per launch name, the mean
    per dispatch of every counter in the databases, plus derived figures:
    valu_busy = SQ_ACTIVE_INST_VALU x 4 / SIMDs / (GRBM_GUI_ACTIVE / XCDs)
    (share of the kernel's cycles in which the average SIMD issues VALU
    work; GRBM_GUI_ACTIVE / XCDs is the kernel's duration in cycles),
    valu_per_wave = SQ_INSTS_VALU / SQ_WAVES, lds_conflict_per_inst =
    SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS (conflict cycles per LDS
    instruction), mfma_busy = SQ_VALU_MFMA_BUSY_CYCLES / SIMDs / duration in
    cycles, mfma_bf16_tflops from SQ_INSTS_VALU_MFMA_MOPS_BF16 (units of 512
    FLOPs) over the duration at 2.4 GHz; wait_any_share, wait_inst_any_share,
    wait_inst_lds_share = SQ_WAIT_ANY, SQ_WAIT_INST_ANY, SQ_WAIT_INST_LDS over
    SQ_WAVE_CYCLES (share of the waves' resident cycles spent waiting for
    outstanding memory or LDS results, for any instruction to issue, for an
    LDS instruction to issue)."""
    dirs, out, workload = [a[0]] + a[3:], a[1], a[2]
    merged = collections.defaultdict(dict)
    for d in dirs:
        for name, cs in load_all(d).items():
            for c, v in cs.items():
                merged[name][c] = v
    kern = {}
    for name, cs in sorted(merged.items()):
        m = {c: sum(v) / len(v) for c, v in cs.items()}
        m["dispatches"] = max(len(v) for v in cs.values())
        g = m.get("GRBM_GUI_ACTIVE")
        if g and "SQ_ACTIVE_INST_VALU" in m:
            m["valu_busy"] = m["SQ_ACTIVE_INST_VALU"] * VALU_CYCLES / SIMDS / (g / XCDS)
            m["duration_us_at_2400MHz"] = g / XCDS / 2400.0
        if m.get("SQ_WAVES") and "SQ_INSTS_VALU" in m:
            m["valu_per_wave"] = m["SQ_INSTS_VALU"] / m["SQ_WAVES"]
        if m.get("SQ_INSTS_LDS") and "SQ_LDS_BANK_CONFLICT" in m:
            m["lds_conflict_per_inst"] = m["SQ_LDS_BANK_CONFLICT"] / m["SQ_INSTS_LDS"]
        if g and "SQ_VALU_MFMA_BUSY_CYCLES" in m:
            # share of the kernel's cycles the average SIMD's matrix core is busy
            m["mfma_busy"] = m["SQ_VALU_MFMA_BUSY_CYCLES"] / SIMDS / (g / XCDS)
        if g and "SQ_INSTS_VALU_MFMA_MOPS_BF16" in m:
            # BF16 matrix FLOPs (the counter counts units of 512) per second
            m["mfma_bf16_tflops"] = m["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512 / (g / XCDS / 2.4e9) / 1e12
        if m.get("SQ_WAVE_CYCLES"):
            for c, k in (("SQ_WAIT_ANY", "wait_any_share"), ("SQ_WAIT_INST_ANY", "wait_inst_any_share"),
                         ("SQ_WAIT_INST_LDS", "wait_inst_lds_share")):
                if c in m:
                    m[k] = m[c] / m["SQ_WAVE_CYCLES"]
        kern[name] = m
    doc = {"workload": workload, "kernel_source_sha256": source_sha256(), "kernels": kern}
    with open(out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"{len(kern)} kernels -> {out}")


def short_name(sym: str) -> str:
    """Readable kernel name with its template arguments from a k_one symbol:
    bulk / Courant / weight types (f, d) and the integer arguments."""
    m = re.search(r"k_oneITnDaXadL_ZNS_(\d+)(k_\w+)", sym)
    if not m:
        return sym[:60]
    ln = int(m.group(1))
    rest = m.group(2)
    name, targs = rest[:ln], rest[ln:]
    head = targs.split("EEvNS_")[0]
    types = "".join(re.findall(r"(?<=I)([fd]+)(?=L|E|$)", head)[:1])
    ints = re.findall(r"Li(\d+)E", head)
    args = ",".join([types] + ints) if types else ",".join(ints)
    return f"{name}<{args}>" if args else name


def trace_main(a):
    """trace DIR OUT.md TITLE COMMAND: the top_kernels view of a rocprofv3
    kernel-trace database as a markdown table."""
    dirname, out, title, command = a[0], a[1], a[2], a[3]
    db = glob.glob(os.path.join(dirname, "**", "*.db"), recursive=True)
    if not db:
        raise FileNotFoundError(f"no rocpd database under {dirname}")
    con = sqlite3.connect(db[0])
    rows = list(con.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    lines = [f"# {title}", "", "Command (GPU box, from the repository root; rocprofv3 run from /tmp with TMPDIR=/tmp):",
             "", "    " + command, "",
             "rocprofv3 top_kernels view (durations in microseconds; template arguments: bulk/Courant/weight "
             "types, then the epilogue of fv_tp_2d (0 flux, 1 delp, 2 mass-weighted, 3 interface heights, "
             "4 tracer) or the pass and site of k_sim1).", "",
             "| kernel | calls | total us | avg us | % |", "|---|---:|---:|---:|---:|"]
    for name, calls, tot, avg, pct in rows:
        if pct < 0.05:
            continue
        lines.append(f"| {short_name(name)} | {calls} | {tot:.1f} | {avg:.1f} | {pct:.2f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"{len(rows)} kernels -> {out}")


def main(argv=None):
    a = argv if argv is not None else sys.argv[1:]
    if a and a[0] == "counters":
        return counters_main(a[1:])
    if a and a[0] == "trace":
        return trace_main(a[1:])
    fdir, wdir, out, workload = a[0], a[1], a[2], a[3]
    f = load(fdir, "FETCH_SIZE")
    w = load(wdir, "WRITE_SIZE")
    ff, wf = calibrate(f, "FETCH_SIZE"), calibrate(w, "WRITE_SIZE")
    kern = {}
    for name in sorted(set(f) | set(w)):
        fv = [v for v, _ in f.get(name, [])]
        wv = [v for v, _ in w.get(name, [])]
        kern[name] = {"dispatches": max(len(fv), len(wv)),
                      "fetch_bytes": (sum(fv) / len(fv) * ff) if fv else None,
                      "write_bytes": (sum(wv) / len(wv) * wf) if wv else None}
    doc = {"workload": workload, "kernel_source_sha256": source_sha256(),
           "fetch_bytes_per_kib": ff, "write_bytes_per_kib": wf, "kernels": kern}
    with open(out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"calibration: FETCH x{ff / 1024:.3f}, WRITE x{wf / 1024:.3f}; {len(kern)} kernels -> {out}")


if __name__ == "__main__":
    main()
