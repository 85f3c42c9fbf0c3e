"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_2402_08296_amd.profiling stats <kernel_stats.csv> <out.md> --title T --command C
      kernel-trace statistics as a markdown table
  python -m paper_2402_08296_amd.profiling traffic-table <fetch csv> <write csv> <out.md> --kernels K1,K2 ...
      the same scaled bytes per dispatch for several kernels, as one table
  python -m paper_2402_08296_amd.profiling counters <out.md> <counter csv>... --stage K1+K2 --stage-us T ...
      per-dispatch means of SQ counters of a stage's kernels and the VALU/MFMA issue
      floors they imply against the stage time
  python -m paper_2402_08296_amd.profiling traffic <fetch counter_collection.csv> <write counter_collection.csv>
      <out.md> --kernel NAME --copy-bytes B --fetch-command C1 --write-command C2
      HBM bytes per dispatch of a kernel from FETCH_SIZE and WRITE_SIZE (KiB per
      dispatch), each scaled by the ratio of a plain copy kernel's known bytes
      to what the same counter reads for it

The traffic summary records a hash of the kernel sources; bench.py reports
the traffic only while the sources still hash the same.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
# What a kernel is built from: (file, first line marker or None, end marker or None).
# A change in any of these texts invalidates a traffic measurement of the kernel.
_DEVPROB = ("csrc/device.h", "struct DevProb {", "\n};\n")
_CONSTS = ("csrc/device.h", "constexpr int D =", "constexpr size_t LDS_LIMIT")
KERNEL_SOURCES = {
    "dss_mfma_kernel": (("csrc/dss_mfma.hip", None, None), ("csrc/dss_mfma.h", None, None), _DEVPROB, _CONSTS),
    "lu_local_kernel": (("csrc/kernels.hip", "// ---------------------------------------------------------------"
                         "--- reductions", "// ------------------------------------------------------------------ "
                         "DSS forward (VALU)"),
                        ("csrc/kernels.hip", "// ------------------------------------------------------------------ "
                         "exact local solves", "// ------------------------------------------------------------------"
                         " coarse solve"), _DEVPROB, _CONSTS),
}


def _region(rel: str, start: str | None, end: str | None) -> bytes:
    text = open(os.path.join(HERE, rel), encoding="utf-8").read()
    if start is not None:
        i = text.index(start)
        j = text.index(end, i + len(start))
        text = text[i:j]
    return text.encode()


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for part in KERNEL_SOURCES[kernel]:
        h.update(_region(*part))
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """Kernel name without namespaces and argument lists (template arguments kept)."""
    n = re.sub(r"\(anonymous namespace\)::|ddmgnn::", "", name)
    n = re.sub(r"^void ", "", n)
    depth, out = 0, []
    for ch in n:
        if ch == "(" and depth == 0:
            break
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        out.append(ch)
    return "".join(out).strip()


def stats_markdown(csv_path: str, title: str, command: str, notes: str = "") -> str:
    rows = list(csv.DictReader(open(csv_path)))
    lines = [f"# {title}", "", "Command (run from /tmp with TMPDIR=/tmp, repository at <repo>):", "", "```",
             command, "```", "", "| Kernel | Calls | Total ms | Average us | Min us | Max us | % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {short_name(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    if notes:
        lines += ["", notes]
    return "\n".join(lines) + "\n"


def per_dispatch(csv_path: str, counter: str) -> dict:
    """{short kernel name: [counter value per dispatch]} from a counter_collection.csv."""
    out = defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] == counter:
            out[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return out


def traffic_summary(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, fetch_cmd: str,
                    write_cmd: str) -> dict:
    """kernel: one kernel name, or several joined by '+' that run once each per
    step (a stage split over launches): their per-dispatch means are added."""
    fetch = per_dispatch(fetch_csv, "FETCH_SIZE")
    write = per_dispatch(write_csv, "WRITE_SIZE")
    copy_name = next(k for k in fetch if "copyBuffer" in k)
    # the copy dispatches of the calibration buffer are the largest ones
    cf = max(fetch[copy_name])
    cw = max(write[copy_name])
    f_fetch = copy_bytes / (cf * 1024.0)
    f_write = copy_bytes / (cw * 1024.0)
    names = kernel.split("+")
    fk = sum(sum(fetch[k]) / len(fetch[k]) for k in names)
    wk = sum(sum(write[k]) / len(write[k]) for k in names)
    fetch_b = fk * 1024.0 * f_fetch
    write_b = wk * 1024.0 * f_write
    return {
        "kernel": kernel, "dispatches": min(len(fetch[k]) for k in names),
        "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
        "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_scale": f_fetch, "write_scale": f_write,
        "fetch_bytes_per_dispatch": fetch_b, "write_bytes_per_dispatch": write_b,
        "traffic_bytes_per_dispatch": fetch_b + write_b,
        "source_hash": source_hash(names[0].split("<")[0]), "fetch_command": fetch_cmd, "write_command": write_cmd,
    }


def traffic_markdown(res: dict) -> str:
    """Human-readable traffic summary with the figures in a JSON block (read by bench.py)."""
    mb = lambda b: f"{b / 1e6:.1f} MB"
    lines = [f"# HBM traffic per dispatch: {res['kernel']}", "",
             "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two rocprofv3 counter passes, each scaled by",
             "known bytes / counter reading of the largest plain copy (hipMemcpy device-to-device blit) in the",
             "same run. Commands (from /tmp with TMPDIR=/tmp, repository at <repo>):", "", "```",
             res["fetch_command"], res["write_command"], "```", "",
             "| | fetch | write |", "|---|---|---|",
             f"| copy calibration ({mb(res['copy_bytes'])} each way) | {res['copy_fetch_kib']:.0f} KiB | "
             f"{res['copy_write_kib']:.0f} KiB |",
             f"| scale | {res['fetch_scale']:.4f} | {res['write_scale']:.4f} |",
             f"| {res['kernel']} (mean of {res['dispatches']} dispatches) | "
             f"{res['fetch_kib_per_dispatch']:.0f} KiB -> {mb(res['fetch_bytes_per_dispatch'])} | "
             f"{res['write_kib_per_dispatch']:.0f} KiB -> {mb(res['write_bytes_per_dispatch'])} |",
             "", f"Traffic per dispatch: {mb(res['traffic_bytes_per_dispatch'])}. Kernel sources hash "
             f"{res['source_hash']}.", "", "```json", json.dumps(res, indent=1), "```", ""]
    return "\n".join(lines)


def read_traffic(path: str) -> dict | None:
    """The JSON block of a traffic summary, or None when the file is absent."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    return json.loads(m.group(1)) if m else None


def traffic_table_markdown(fetch_csv: str, write_csv: str, kernels: list[str], copy_bytes: int, fetch_cmd: str,
                           write_cmd: str, title: str, notes: str = "") -> str:
    """HBM bytes per dispatch of several kernels (FETCH_SIZE, WRITE_SIZE, each scaled by
    the plain copy's known bytes over the counter's reading for it in the same run)."""
    fetch = per_dispatch(fetch_csv, "FETCH_SIZE")
    write = per_dispatch(write_csv, "WRITE_SIZE")
    copy_name = next(k for k in fetch if "copyBuffer" in k)
    f_fetch = copy_bytes / (max(fetch[copy_name]) * 1024.0)
    f_write = copy_bytes / (max(write[copy_name]) * 1024.0)
    lines = [f"# {title}", "", "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two rocprofv3 counter passes, each "
             "scaled by", "known bytes / counter reading of the largest plain copy (hipMemcpy device-to-device blit) "
             "in the", "same run. Commands (from /tmp with TMPDIR=/tmp, repository at <repo>):", "", "```", fetch_cmd,
             write_cmd, "```", "", f"Scales: fetch {f_fetch:.4f}, write {f_write:.4f} (copy of {copy_bytes} bytes).",
             "", "| Kernel | Dispatches | Fetch MB | Write MB | Total MB |", "|---|---|---|---|---|"]
    for k in kernels:
        fk = sum(fetch[k]) / len(fetch[k]) * 1024.0 * f_fetch
        wk = sum(write[k]) / len(write[k]) * 1024.0 * f_write
        lines.append(f"| {k} | {len(fetch[k])} | {fk / 1e6:.1f} | {wk / 1e6:.1f} | {(fk + wk) / 1e6:.1f} |")
    if notes:
        lines += ["", notes]
    return "\n".join(lines) + "\n"


# Instruction issue model of the hardware (MI355X): 256 compute units of 4 SIMDs at
# 2.4 GHz; a wave64 VALU instruction occupies its SIMD for 4 cycles, a
# v_mfma_f32_32x32x16 (bf16 or f16) for 32 cycles (8 passes).
SIMDS = 256 * 4
CLOCK_HZ = 2.4e9
VALU_CYCLES = 4
MFMA_CYCLES = 32


def counters_markdown(csvs: list[str], stage: list[str], stage_us: float, title: str, commands: list[str],
                      notes: str = "") -> str:
    """Per-dispatch means of every SQ/GRBM counter of the kernels of one stage (several
    kernels joined by '+' that run once each per stage are summed), and the issue floors
    they imply: VALU instructions x 4 cycles and MFMA instructions x 32 cycles spread
    over all SIMDs, against the stage's measured time."""
    vals = defaultdict(lambda: defaultdict(list))
    for path in csvs:
        for r in csv.DictReader(open(path)):
            vals[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for k in stage for c in vals[k]})
    lines = [f"# {title}", "", "Commands (from /tmp with TMPDIR=/tmp, repository at <repo>), one counter pass each:", "",
             "```", *commands, "```", "", "Mean per dispatch (counter units as rocprofv3 reports them):", "",
             "| Counter | " + " | ".join(stage) + " | stage |", "|---" * (len(stage) + 2) + "|"]
    tot = {}
    for c in names:
        row = [sum(vals[k][c]) / len(vals[k][c]) if vals[k][c] else 0.0 for k in stage]
        tot[c] = sum(row)
        lines.append(f"| {c} | " + " | ".join(f"{v:,.0f}" for v in row) + f" | {tot[c]:,.0f} |")
    lines += ["", f"Stage time: {stage_us:.1f} us.", ""]
    if "SQ_INSTS_VALU" in tot:
        fl = tot["SQ_INSTS_VALU"] * VALU_CYCLES / (SIMDS * CLOCK_HZ) * 1e6
        lines.append(f"- VALU issue floor: {tot['SQ_INSTS_VALU']:,.0f} wave instructions x {VALU_CYCLES} cycles over "
                     f"{SIMDS} SIMDs at {CLOCK_HZ / 1e9:.1f} GHz = {fl:.1f} us, i.e. VALU busy "
                     f"{100 * fl / stage_us:.1f}% of the stage.")
    if "SQ_INSTS_MFMA" in tot:
        fm = tot["SQ_INSTS_MFMA"] * MFMA_CYCLES / (SIMDS * CLOCK_HZ) * 1e6
        lines.append(f"- MFMA issue floor: {tot['SQ_INSTS_MFMA']:,.0f} x {MFMA_CYCLES} cycles = {fm:.1f} us, "
                     f"MFMA busy {100 * fm / stage_us:.1f}%.")
    if "SQ_WAVE_CYCLES" in tot and "SQ_WAIT_INST_ANY" in tot:
        lines.append(f"- Waves wait on dependencies (s_waitcnt) {100 * tot['SQ_WAIT_INST_ANY'] / tot['SQ_WAVE_CYCLES']:.1f}% "
                     f"of their cycles; on LDS {100 * tot.get('SQ_WAIT_INST_LDS', 0) / tot['SQ_WAVE_CYCLES']:.1f}%.")
    if "SQ_LDS_BANK_CONFLICT" in tot and "SQ_ACTIVE_INST_LDS" in tot:
        lines.append(f"- LDS bank-conflict cycles per LDS-active cycle: "
                     f"{tot['SQ_LDS_BANK_CONFLICT'] / tot['SQ_ACTIVE_INST_LDS']:.2f}.")
    if notes:
        lines += ["", notes]
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--notes", default="")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("out")
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--fetch-command", required=True)
    t.add_argument("--write-command", required=True)
    tt = sub.add_parser("traffic-table")
    tt.add_argument("fetch_csv")
    tt.add_argument("write_csv")
    tt.add_argument("out")
    tt.add_argument("--kernels", required=True, help="kernel names joined by ','")
    tt.add_argument("--copy-bytes", type=int, required=True)
    tt.add_argument("--fetch-command", required=True)
    tt.add_argument("--write-command", required=True)
    tt.add_argument("--title", required=True)
    tt.add_argument("--notes", default="")
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("csvs", nargs="+")
    c.add_argument("--stage", required=True, help="kernel names of the stage joined by '+'")
    c.add_argument("--stage-us", type=float, required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", action="append", required=True)
    c.add_argument("--notes", default="")
    a = ap.parse_args()
    if a.cmd == "traffic-table":
        with open(a.out, "w") as f:
            f.write(traffic_table_markdown(a.fetch_csv, a.write_csv, a.kernels.split(","), a.copy_bytes,
                                           a.fetch_command, a.write_command, a.title, a.notes))
        return
    if a.cmd == "counters":
        with open(a.out, "w") as f:
            f.write(counters_markdown(a.csvs, a.stage.split("+"), a.stage_us, a.title, a.command, a.notes))
        return
    if a.cmd == "stats":
        with open(a.out, "w") as f:
            f.write(stats_markdown(a.csv, a.title, a.command, a.notes))
    else:
        res = traffic_summary(a.fetch_csv, a.write_csv, a.kernel, a.copy_bytes, a.fetch_command, a.write_command)
        with open(a.out, "w") as f:
            f.write(traffic_markdown(res))
        print(json.dumps(res))


if __name__ == "__main__":
    main()
