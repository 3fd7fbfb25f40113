"""Summaries of rocprofv3 CSV output for the ``profiles/`` directory.

    python -m paper_2406_18356_amd.prof_summary stats DIR PREFIX OUT.txt --command "..."
    python -m paper_2406_18356_amd.prof_summary traffic DIR FETCH_PREFIX WRITE_PREFIX OUT.json \
        --kernel SUBSTRING --segment I --bytes ALGORITHMIC_BYTES --command "..."
    python -m paper_2406_18356_amd.prof_summary passes DIR PREFIX OUT.txt --command "..." \
        --pass NAME SUBSTRING I [--pass ...]
    python -m paper_2406_18356_amd.prof_summary counters DIR PREFIX OUT.txt --command "..." \
        --pass NAME SUBSTRING I [--pass ...]
    python -m paper_2406_18356_amd.prof_summary mfma DIR PREFIX OUT.txt --command "..." \
        --group NAME SUBSTRING [--group ...]

``stats`` condenses ``<PREFIX>_kernel_stats.csv`` (rocprofv3 --kernel-trace
--stats --output-format csv) into a table.  ``traffic`` reads two --pmc runs
(FETCH_SIZE, WRITE_SIZE, in KiB per dispatch), calibrates each counter against
the largest device-to-device copy in the same run (a copy of B bytes must read
and write B bytes) and records the scaled per-launch HBM traffic of the kernel
whose name contains SUBSTRING, with a hash of the kernel sources so that the
benchmark can tell whether the figure still describes the current code.
``counters`` reads one --pmc run of SQ_* counters and GRBM_GUI_ACTIVE over the
same --profile-pass passes and reports, per named pass, instructions per wave
and the vector-ALU issue share (VALU instructions x 4 cycles over the SIMD
cycles of the kernel; GRBM_GUI_ACTIVE is summed over the 8 XCDs).
``passes`` reads ``<PREFIX>_kernel_trace.csv`` and reports, per named pass, the
mean duration of the dispatches whose kernel name contains SUBSTRING in
segment I.  Segments: in a ``bench.py --profile-pass ...`` run every pass is
preceded by one 64 MiB device copy; segment I holds the dispatches after such
a copy up to the next one, counted from the end when negative (with n
--profile-pass triples, pass i is segment i - n).  The first matching
dispatch of a segment (the untimed warm launch) is dropped.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/fft_engine.hpp", "csrc/kernels.hpp", "csrc/ops.hpp", "csrc/ops_inst.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


_MANGLED_ARG = [(r"DF16b", "bf16"), (r"f", "float"), (r"d", "double"), (r"Lb0E", "false"), (r"Lb1E", "true"),
                (r"Li(\d+)E", r"\1")]


def _demangle_local(name: str) -> str:
    """Names of templates in an anonymous namespace arrive mangled
    (_ZN12_GLOBAL__N_1<len><name>I<args>E...): keep the name and its simple
    template arguments (bf16, float, double, bool and int literals)."""
    m = re.match(r"_ZN12_GLOBAL__N_1(\d+)", name)
    if not m:
        return name
    rest = name[m.end():]
    k = int(m.group(1))
    ident, rest = rest[:k], rest[k:]
    if not rest.startswith("I"):
        return ident
    rest, args = rest[1:], []
    while rest and not rest.startswith("E"):
        for pat, rep in _MANGLED_ARG:
            mm = re.match(pat, rest)
            if mm:
                args.append(mm.expand(rep))
                rest = rest[mm.end():]
                break
        else:
            break
    return f"{ident}<{', '.join(args)}>" if args else ident


def _short(name: str) -> str:
    n = _demangle_local(name)
    n = n.replace("(anonymous namespace)::", "")
    n = re.sub(r"void msr::", "", n)
    n = re.sub(r"msr::(RowArgs|ColArgs)<(float|double)>, ", "", n)
    n = re.sub(r"\(.*", "", n)
    return n


def stats(d, prefix, out, command, top=16):
    rows = list(csv.DictReader(open(os.path.join(d, f"{prefix}_kernel_stats.csv"))))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}", "",
             f"{'kernel':90s} {'calls':>7s} {'avg_us':>9s} {'total_ms':>9s} {'pct':>6s}"]
    for r in rows[:top]:
        lines.append(f"{_short(r['Name'])[:90]:90s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:9.2f} "
                     f"{float(r['TotalDurationNs']) / 1e6:9.2f} {float(r['Percentage']):6.1f}")
    open(out, "w").write("\n".join(lines) + "\n")
    return out


def _segments(rows, name_key):
    """Dispatch lists that follow each marker copy (a device copy of the same
    size as the last copy of the run), in order."""
    copies = [i for i, r in enumerate(rows) if "copyBuffer" in r[name_key]]
    if not copies:
        raise SystemExit("no device copy in the run")
    g_last = int(r_grid(rows[copies[-1]]))
    marks = [i for i in copies if int(r_grid(rows[i])) == g_last]
    segs = []
    for k, i in enumerate(marks):
        end = marks[k + 1] if k + 1 < len(marks) else len(rows)
        segs.append(rows[i + 1:end])
    return segs


def r_grid(r):
    return r.get("Grid_Size_X") or r.get("Grid_Size")


def _pick(seg, sub, name_key):
    ds = [r for r in seg if sub in r[name_key]]
    return ds[1:] if len(ds) > 1 else ds


def passes(d, prefix, out, command, specs):
    rows = list(csv.DictReader(open(os.path.join(d, f"{prefix}_kernel_trace.csv"))))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    segs = _segments(rows, "Kernel_Name")
    lines = [f"# rocprofv3 kernel trace: mean duration of the last dispatches of each pass",
             f"# command: {command}", "",
             f"{'pass':18s} {'dispatches':>10s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s}  kernel"]
    for name, sub, seg in specs:
        ds = _pick(segs[int(seg)], sub, "Kernel_Name")
        if not ds:
            raise SystemExit(f"no dispatch matching {sub!r}")
        us = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in ds]
        lines.append(f"{name:18s} {len(us):10d} {sum(us) / len(us):9.2f} {min(us):9.2f} {max(us):9.2f}  "
                     f"{_short(ds[-1]['Kernel_Name'])[:100]}")
    open(out, "w").write("\n".join(lines) + "\n")
    return out


def _per_dispatch(d, prefix, counter):
    """(name, grid, value) per dispatch, in dispatch order."""
    out = []
    for f in glob.glob(os.path.join(d, f"{prefix}_counter_collection.csv")):
        rows = [r for r in csv.DictReader(open(f)) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0))
        for r in rows:
            out.append({"Kernel_Name": r["Kernel_Name"], "Grid_Size": int(r["Grid_Size"]),
                        "value": float(r["Counter_Value"])})
    return out


def _copy_scale(rows, copy_bytes):
    copies = [r["value"] for r in rows if "copyBuffer" in r["Kernel_Name"]]
    if not copies:
        raise SystemExit("no device copy kernel in the counter run")
    big = max(copies)
    return copy_bytes / 1024.0 / big, big


# MI355X: 256 CUs x 4 SIMDs, 8 XCDs, 2.4 GHz; a wave64 VALU instruction holds a
# 16-lane SIMD for 4 cycles
SIMDS, XCDS, CLOCK_GHZ, VALU_CYCLES = 1024, 8, 2.4, 4


def counters(d, prefix, out, command, specs):
    names = ("GRBM_GUI_ACTIVE", "SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
             "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT")
    per = {n: _per_dispatch(d, prefix, n) for n in names}
    lines = ["# rocprofv3 SQ counters per pass (mean over the pass's timed dispatches)", f"# command: {command}", "",
             f"{'pass':18s} {'us':>7s} {'waves':>7s} {'valu/wave':>9s} {'valu_busy':>9s} {'lds/wave':>8s} "
             f"{'vmem/wave':>9s} {'lds_conflict':>12s}"]
    for name, sub, seg in specs:
        v = {}
        for n in names:
            ds = _pick(_segments(per[n], "Kernel_Name")[int(seg)], sub, "Kernel_Name")
            if not ds:
                raise SystemExit(f"no dispatch matching {sub!r} for {n}")
            v[n] = sum(r["value"] for r in ds) / len(ds)
        cyc = v["GRBM_GUI_ACTIVE"] / XCDS
        waves = max(v["SQ_WAVES"], 1.0)
        busy = v["SQ_INSTS_VALU"] * VALU_CYCLES / (SIMDS * cyc)
        conflict = v["SQ_LDS_BANK_CONFLICT"] / max(v["SQ_ACTIVE_INST_LDS"], 1.0)
        lines.append(f"{name:18s} {cyc / (CLOCK_GHZ * 1e3):7.1f} {waves:7.0f} {v['SQ_INSTS_VALU'] / waves:9.0f} "
                     f"{busy:9.2f} {v['SQ_INSTS_LDS'] / waves:8.0f} "
                     f"{(v['SQ_INSTS_VMEM_RD'] + v['SQ_INSTS_VMEM_WR']) / waves:9.1f} {conflict:12.2f}")
    open(out, "w").write("\n".join(lines) + "\n")
    return out


# one 32x32x16 bf16 MFMA instruction: 32768 flops, 512 of them per MOP
MOP_FLOPS = 512
BF16_PEAK_TFLOPS = 2500.0


def mfma(d, prefix, out, command, specs):
    """Matrix-core use per kernel group (one --pmc run of
    SQ_INSTS_VALU_MFMA_MOPS_BF16, SQ_VALU_MFMA_BUSY_CYCLES,
    SQ_INSTS_VALU_MFMA_BF16 and GRBM_GUI_ACTIVE): MFMA busy cycles over the
    SIMD cycles of the group's dispatches, and its counted bf16 MFMA flops
    per second of GPU-active time against the dense peak."""
    names = ("GRBM_GUI_ACTIVE", "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_INSTS_VALU_MFMA_BF16")
    per = {n: _per_dispatch(d, prefix, n) for n in names}
    lines = ["# rocprofv3 MFMA counters per kernel group (sums over every matching dispatch)", f"# command: {command}",
             "", f"{'group':22s} {'dispatches':>10s} {'mfma_insts':>11s} {'tflop':>9s} {'active_ms':>10s} "
                 f"{'mfma_busy':>9s} {'tflop/s':>8s} {'of_peak':>7s}"]
    for name, sub in specs:
        v = {}
        for n in names:
            ds = _pick(per[n], sub, "Kernel_Name")
            if not ds:
                raise SystemExit(f"no dispatch matching {sub!r} for {n}")
            v[n] = sum(r["value"] for r in ds)
            v["n"] = len(ds)
        cyc = v["GRBM_GUI_ACTIVE"] / XCDS
        busy = v["SQ_VALU_MFMA_BUSY_CYCLES"] / (SIMDS * cyc)
        fl = v["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * MOP_FLOPS
        secs = cyc / (CLOCK_GHZ * 1e9)
        lines.append(f"{name:22s} {v['n']:10d} {v['SQ_INSTS_VALU_MFMA_BF16']:11.4g} {fl / 1e12:9.3f} "
                     f"{secs * 1e3:10.2f} {busy:9.3f} {fl / secs / 1e12:8.1f} {fl / secs / 1e12 / BF16_PEAK_TFLOPS:7.3f}")
    open(out, "w").write("\n".join(lines) + "\n")
    return out


def traffic(d, fprefix, wprefix, out, kernel, alg_bytes, copy_bytes, command, segment):
    fr = _per_dispatch(d, fprefix, "FETCH_SIZE")
    wr = _per_dispatch(d, wprefix, "WRITE_SIZE")
    fs, fbig = _copy_scale(fr, copy_bytes)
    ws, wbig = _copy_scale(wr, copy_bytes)
    fk = [r["value"] for r in _pick(_segments(fr, "Kernel_Name")[segment], kernel, "Kernel_Name")]
    wk = [r["value"] for r in _pick(_segments(wr, "Kernel_Name")[segment], kernel, "Kernel_Name")]
    if not fk or not wk:
        raise SystemExit(f"kernel {kernel!r} not found")
    fetch = sum(fk) / len(fk) * fs * 1024.0
    write = sum(wk) / len(wk) * ws * 1024.0
    rec = {
        "kernel": kernel, "source_sha256": kernel_source_hash(), "command": command,
        "fetch_kib_raw": sum(fk) / len(fk), "write_kib_raw": sum(wk) / len(wk),
        "copy_bytes": copy_bytes, "copy_fetch_kib": fbig, "copy_write_kib": wbig,
        "fetch_scale": fs, "write_scale": ws,
        "dispatches": len(fk), "traffic_bytes": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
        "algorithmic_bytes": alg_bytes,
    }
    json.dump(rec, open(out, "w"), indent=1)
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("prefix")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("dir")
    t.add_argument("fetch_prefix")
    t.add_argument("write_prefix")
    t.add_argument("out")
    t.add_argument("--kernel", required=True)
    t.add_argument("--bytes", type=float, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--segment", type=int, required=True, help="pass index in the --profile-pass run")
    q = sub.add_parser("passes")
    q.add_argument("dir")
    q.add_argument("prefix")
    q.add_argument("out")
    q.add_argument("--command", required=True)
    q.add_argument("--pass", dest="specs", nargs=3, action="append", required=True,
                   metavar=("NAME", "SUBSTRING", "SEGMENT"))
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("prefix")
    c.add_argument("out")
    c.add_argument("--command", required=True)
    c.add_argument("--pass", dest="specs", nargs=3, action="append", required=True,
                   metavar=("NAME", "SUBSTRING", "SEGMENT"))
    m = sub.add_parser("mfma")
    m.add_argument("dir")
    m.add_argument("prefix")
    m.add_argument("out")
    m.add_argument("--command", required=True)
    m.add_argument("--group", dest="specs", nargs=2, action="append", required=True, metavar=("NAME", "SUBSTRING"))
    a = ap.parse_args(argv)
    if a.cmd == "mfma":
        print(mfma(a.dir, a.prefix, a.out, a.command, a.specs))
    elif a.cmd == "counters":
        print(counters(a.dir, a.prefix, a.out, a.command, a.specs))
    elif a.cmd == "stats":
        print(stats(a.dir, a.prefix, a.out, a.command))
    elif a.cmd == "passes":
        print(passes(a.dir, a.prefix, a.out, a.command, a.specs))
    else:
        print(json.dumps(traffic(a.dir, a.fetch_prefix, a.write_prefix, a.out, a.kernel, a.bytes, a.copy_bytes,
                                 a.command, a.segment), indent=1))


if __name__ == "__main__":
    main()
