"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1003_4322_amd.profsum stats <run_kernel_stats.csv> <out.md> "<command>"
    python -m paper_1003_4322_amd.profsum traffic <fetch.csv> <write.csv> <copy_fetch.csv>
        <copy_write.csv> <bench.json> <out.json> <out.md> "<command>"

``stats`` condenses a --kernel-trace --stats run into a table of the library's
kernels (template arguments shortened).  ``traffic`` turns two --pmc runs
(FETCH_SIZE, then WRITE_SIZE) into HBM bytes per launch of each kernel kind,
scaled by what the same counters read for a plain device copy of known size,
and records the kernel-source hash they belong to.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def short(name: str) -> str:
    name = re.sub(r"ps::Radices<([^>]*)>", r"R<\1>", name)
    name = re.sub(r"\(ps::\w+<\w+>\)", "", name)
    return name.replace("void ps::", "")


def kind_of(name: str) -> str:
    if "k_z_curl" in name:
        return "z_curl"
    if "k_z_epi" in name:
        return "z_epi"
    if "k_x_prod" in name:
        return "x_prod"
    if "k_strided" in name:
        m = re.search(r"k_strided<\w+, \d+, \d+, \d+, (\d)", name)
        return "y_fwd" if m and m.group(1) == "0" else "y_inv"
    if "k_spec" in name:
        return "spectrum"
    if "k_x_r2c" in name:
        return "x_r2c"
    if "k_x_c2r" in name:
        return "x_c2r"
    return "other"


def _code_only(text: str) -> str:
    """Source text without comments and with whitespace runs collapsed, so that
    editing a comment does not count as changing a kernel."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def src_hash() -> str:
    """Hash of the device-side code (kernels, their configurations and
    launchers; comments excluded); host-only code (ps_api.cpp) does not change
    a kernel's traffic."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1003_4322_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            h.update(_code_only(open(os.path.join(d, f), encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def stats(csv_path: str, out_md: str, command: str):
    rows = list(csv.DictReader(open(csv_path)))
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             "| kernel | calls | average (ms) | total (ms) | share |",
             "|---|---:|---:|---:|---:|"]
    for r in rows:
        if "ps::" not in r["Name"]:
            continue
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f}% |")
    lines.append("")
    lines.append("Launches include the autotuner's timing runs of every variant; the variants the "
                 "timed region used are the ones listed in the benchmark line.")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _pmc(path: str, counter: str):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            d[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return d


def traffic(fetch_csv, write_csv, cfetch_csv, cwrite_csv, bench_json, out_json, out_md, command):
    bench = json.loads(open(bench_json).read().strip().splitlines()[-1])
    copy = bench.get("device_copy") or {"bytes_read": 1 << 31, "bytes_written": 1 << 31}
    cf = _pmc(cfetch_csv, "FETCH_SIZE")
    cw = _pmc(cwrite_csv, "WRITE_SIZE")
    copy_name = max(cf, key=lambda k: sum(cf[k]))
    f_scale = (sum(cf[copy_name]) / len(cf[copy_name]) * 1024) / copy["bytes_read"]
    w_scale = (sum(cw[copy_name]) / len(cw[copy_name]) * 1024) / copy["bytes_written"]
    fe, wr = _pmc(fetch_csv, "FETCH_SIZE"), _pmc(write_csv, "WRITE_SIZE")
    variants = bench.get("variants") or {}
    wl = bench["config"].get("workload_key", "mhd512")
    rec = {}
    lines = ["# HBM traffic per launch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)", "",
             f"Command: `{command}`", "",
             f"Copy reference ({copy_name}): FETCH_SIZE reads {f_scale:.3f} x the bytes read, "
             f"WRITE_SIZE {w_scale:.3f} x the bytes written; kernel counters are divided by these.",
             "", "| kernel | launches | read GB | written GB | traffic GB |", "|---|---:|---:|---:|---:|"]
    for name in fe:
        if "ps::" not in name or name not in wr:
            continue
        rd = sum(fe[name]) / len(fe[name]) * 1024 / f_scale
        wt = sum(wr[name]) / len(wr[name]) * 1024 / w_scale
        lines.append(f"| `{short(name)}` | {len(fe[name])} | {rd / 1e9:.3f} | {wt / 1e9:.3f} | "
                     f"{(rd + wt) / 1e9:.3f} |")
        rec.setdefault(kind_of(name), []).append((name, rd + wt, len(fe[name])))
    out = {}
    for kind, lst in rec.items():
        # the variant most launched is the one the timed region used
        name, tb, _ = max(lst, key=lambda t: t[2])
        out[f"{wl}/f32/{kind}"] = {"kernel": short(name), "bytes_per_launch": tb, "src_hash": src_hash()}
    json.dump(out, open(out_json, "w"), indent=1)
    open(out_md, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(*sys.argv[2:5])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:10])
    else:
        raise SystemExit(__doc__)
