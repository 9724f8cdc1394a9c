"""Summarise rocprofv3 runs of the SpMM kernel: HBM traffic per launch from
counter runs, and kernel-time tables from kernel-trace runs.

Traffic (after two rocprofv3 --pmc runs of bench.py with --copy-calibration-mib,
one collecting FETCH_SIZE and one WRITE_SIZE, each with -f csv):

    python -m paper_2009_07226_amd.pmc_summary FETCH.csv WRITE.csv OUT_PREFIX \
        --copy-mib 1024 --command "<the rocprofv3 commands>"

Kernel times (after rocprofv3 --kernel-trace --stats -f csv):

    python -m paper_2009_07226_amd.pmc_summary --trace KERNEL_STATS.csv OUT.md \
        --command "<the rocprofv3 command>" --workload "<workload>"

FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch.  Their scale on a
given device is calibrated with the plain device copy of known size that
bench.py runs (`--copy-calibration-mib`): factor = bytes moved / counter value.
Writes OUT_PREFIX.md (human-readable) and OUT_PREFIX.json (figures and the
SHA-256 of the kernel sources they were measured on; bench.py reports the
traffic only while the sources still match).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/spmm.hip", "csrc/build.hip", "csrc/common.hpp")


def code_only(text: str) -> str:
    """C/C++ source with comments removed and whitespace collapsed (string and
    character literals kept), so that comment edits do not invalidate counters."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == "/" and text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif c == "/" and text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_sources_sha(root: str = HERE) -> str:
    """SHA-256 of the code (not the comments) of the kernel sources."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(root, rel), encoding="utf-8") as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()


def _read(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    by = defaultdict(list)
    for r in rows:
        by[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return by


def summarise(fetch_csv, write_csv, copy_mib):
    f = _read(fetch_csv, "FETCH_SIZE")
    w = _read(write_csv, "WRITE_SIZE")
    nbytes = copy_mib << 20
    copy_f = max(v for k, vs in f.items() if "copyBuffer" in k for v in vs)
    copy_w = max(v for k, vs in w.items() if "copyBuffer" in k for v in vs)
    fscale = nbytes / (copy_f * 1024.0)
    wscale = nbytes / (copy_w * 1024.0)
    out = {"copy_bytes": nbytes, "fetch_scale": fscale, "write_scale": wscale, "kernels": {}}
    for name, vs in f.items():
        if "k_spmm" not in name:
            continue
        ws = w.get(name, [0.0])
        out["kernels"][name] = {
            "launches": len(vs),
            "fetch_bytes_per_launch": sum(vs) / len(vs) * 1024.0 * fscale,
            "write_bytes_per_launch": sum(ws) / len(ws) * 1024.0 * wscale,
            "fetch_kib_raw": vs,
            "write_kib_raw": ws,
        }
    return out


def trace_table(stats_csv, out_md, command, workload, note=""):
    """Markdown table of a rocprofv3 kernel_stats.csv (durations in ns)."""
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# Kernel times: {workload}", "", "Command:", "", "```", command, "```", "",
             "| Kernel | Calls | Total ns | Average ns | % | Min ns | Max ns |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].replace("void ", "").split("(")[0]
        lines.append(f"| {name} | {r['Calls']} | {int(float(r['TotalDurationNs']))} | {float(r['AverageNs']):.0f} | "
                     f"{float(r['Percentage']):.2f} | {int(float(r['MinNs']))} | {int(float(r['MaxNs']))} |")
    if note:
        lines += ["", note]
    lines += ["", f"Kernel sources SHA-256 (code without comments): `{kernel_sources_sha()}`"]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


SQ_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT")


def _last_json(path):
    for line in reversed(open(path).read().splitlines()):
        if line.startswith("{"):
            return json.loads(line)
    raise ValueError(f"no JSON line in {path}")


def sq_table(runs, out_md, command, workload, note=""):
    """Markdown table of SQ counters of the first projection (A) and
    backprojection (A^T) launch of each run.  runs: (label, counter csv,
    bench output holding the JSON line with padded_A / padded_AT); the
    per-group columns divide by the launch's 4-step groups of 64 lanes."""
    lines = [f"# SpMM shader counters (rocprofv3 --pmc, SQ block): {workload}", "", "Command:", "", "```", command,
             "```", "", "Counter values are summed over the device for one launch of A (projection) and one of A^T "
             "(backprojection); the last two columns divide by the launch's 4-step groups (padded entries / 256).",
             "", "| Matrix | Launch | " + " | ".join(SQ_COUNTERS) + " | LDS cycles / LDS instr | conflict cycles / "
             "LDS instr | VALU / group | LDS instr / group |", "|---" * (len(SQ_COUNTERS) + 6) + "|"]
    for label, csv_path, bench_out in runs:
        rows = [r for r in csv.DictReader(open(csv_path)) if "k_spmm" in r["Kernel_Name"]]
        order = []
        vals = defaultdict(dict)
        for r in rows:
            d = int(r["Dispatch_Id"])
            if d not in vals:
                order.append(d)
            vals[d][r["Counter_Name"]] = float(r["Counter_Value"])
        order.sort()
        b = _last_json(bench_out)
        for which, d, padded in (("A", order[0], b["padded_A"]), ("A^T", order[1], b["padded_AT"])):
            v = vals[d]
            groups = padded / 256.0
            lds = v["SQ_INSTS_LDS"]
            lines.append(f"| {label} | {which} | " + " | ".join(f"{v[c]:.4g}" for c in SQ_COUNTERS) +
                         f" | {v['SQ_LDS_IDX_ACTIVE'] / lds:.2f} | {v['SQ_LDS_BANK_CONFLICT'] / lds:.3f} | "
                         f"{v['SQ_INSTS_VALU'] / groups:.1f} | {lds / groups:.1f} |")
    if note:
        lines += ["", note]
    lines += ["", f"Kernel sources SHA-256 (code without comments): `{kernel_sources_sha()}`"]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


STATE_COUNTERS = ("SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU",
                  "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VMEM", "SQ_ACTIVE_INST_SCA", "SQ_WAIT_INST_LDS")


def _first_two_spmm(csv_path):
    """Counter values of the first two k_spmm dispatches of a run (A, then A^T)."""
    vals = defaultdict(dict)
    for r in csv.DictReader(open(csv_path)):
        if "k_spmm" in r["Kernel_Name"]:
            vals[int(r["Dispatch_Id"])][r["Counter_Name"]] = float(r["Counter_Value"])
    order = sorted(vals)
    return vals[order[0]], vals[order[1]]


def states_table(runs, out_md, command, workload, note=""):
    """Markdown table of where the SpMM's wavefronts spend their time: the
    shares of SQ_WAVE_CYCLES spent waiting on a dependency (SQ_WAIT_ANY),
    ready but waiting to issue (SQ_WAIT_INST_ANY) and issuing
    (SQ_ACTIVE_INST_ANY), and the issuing share by instruction kind.  runs:
    (label, csv of one pass, csv of another pass); each pass holds some of
    STATE_COUNTERS for the same launches (first A, then A^T)."""
    lines = [f"# SpMM wavefront states (rocprofv3 --pmc, SQ block): {workload}", "", "Command:", "", "```", command,
             "```", "", "Shares of the wave cycles (SQ_WAVE_CYCLES) of one launch of A (projection) and one of A^T "
             "(backprojection); the three states add up to the whole.", "",
             "| Matrix | Launch | waiting on a dependency | ready, waiting to issue | issuing | of which VALU | LDS | "
             "vector memory | scalar | waiting to issue an LDS instruction |", "|---" * 10 + "|"]
    for label, csv_a, csv_b in runs:
        pa, pb = _first_two_spmm(csv_a), _first_two_spmm(csv_b)
        for which, i in (("A", 0), ("A^T", 1)):
            v = dict(pa[i])
            v.update(pb[i])
            w = v["SQ_WAVE_CYCLES"]
            act = v["SQ_ACTIVE_INST_ANY"]
            lines.append(f"| {label} | {which} | {v['SQ_WAIT_ANY'] / w:.1%} | {v['SQ_WAIT_INST_ANY'] / w:.1%} | "
                         f"{act / w:.1%} | {v['SQ_ACTIVE_INST_VALU'] / act:.1%} | {v['SQ_ACTIVE_INST_LDS'] / act:.1%} | "
                         f"{v['SQ_ACTIVE_INST_VMEM'] / act:.1%} | {v['SQ_ACTIVE_INST_SCA'] / act:.1%} | "
                         f"{v['SQ_WAIT_INST_LDS'] / w:.1%} |")
    if note:
        lines += ["", note]
    lines += ["", f"Kernel sources SHA-256 (code without comments): `{kernel_sources_sha()}`"]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv", nargs="?")
    ap.add_argument("out_prefix", nargs="?")
    ap.add_argument("--trace", action="store_true", help="fetch_csv is a kernel_stats.csv, write_csv the output .md")
    ap.add_argument("--sq", action="append", default=[], metavar="LABEL=CSV,BENCH_OUT",
                    help="SQ counter table instead (repeat per matrix dtype); fetch_csv is then the output .md")
    ap.add_argument("--states", action="append", default=[], metavar="LABEL=CSV,CSV",
                    help="wavefront-state table instead (two counter passes per matrix dtype); fetch_csv is then the "
                         "output .md")
    ap.add_argument("--note", default="")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--command", default="")
    ap.add_argument("--workload", default="")
    a = ap.parse_args()
    if a.states:
        runs = []
        for spec in a.states:
            label, rest = spec.split("=", 1)
            csv_a, csv_b = rest.split(",", 1)
            runs.append((label, csv_a, csv_b))
        states_table(runs, a.fetch_csv, a.command, a.workload, a.note)
        return
    if a.sq:
        runs = []
        for spec in a.sq:
            label, rest = spec.split("=", 1)
            csv_path, bench_out = rest.split(",", 1)
            runs.append((label, csv_path, bench_out))
        sq_table(runs, a.fetch_csv, a.command, a.workload, a.note)
        return
    if a.trace:
        trace_table(a.fetch_csv, a.write_csv, a.command, a.workload, a.note)
        return
    s = summarise(a.fetch_csv, a.write_csv, a.copy_mib)
    s["kernel_sources_sha256"] = kernel_sources_sha()
    s["command"] = a.command
    s["workload"] = a.workload
    with open(a.out_prefix + ".json", "w") as fh:
        json.dump(s, fh, indent=1)
    lines = [f"# SpMM HBM traffic (rocprofv3 FETCH_SIZE / WRITE_SIZE): {a.workload}", "",
             "Command:", "", "```", a.command, "```", "",
             f"Calibration: a plain device copy of {a.copy_mib} MiB reads FETCH_SIZE x {s['fetch_scale']:.4f} "
             f"and writes WRITE_SIZE x {s['write_scale']:.4f} of its true bytes (factors applied below).", "",
             "| Kernel | Launches | Read GB / launch | Written GB / launch | raw FETCH_SIZE KiB | raw WRITE_SIZE KiB |",
             "|---|---|---|---|---|---|"]
    for name, k in s["kernels"].items():
        lines.append(f"| {name.split('(')[0]} | {k['launches']} | {k['fetch_bytes_per_launch'] / 1e9:.3f} | "
                     f"{k['write_bytes_per_launch'] / 1e9:.3f} | {', '.join(f'{v:.6g}' for v in k['fetch_kib_raw'])} | "
                     f"{', '.join(f'{v:.6g}' for v in k['write_kib_raw'])} |")
    lines += ["", f"Kernel sources SHA-256 (code without comments): `{s['kernel_sources_sha256']}`"]
    with open(a.out_prefix + ".md", "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
