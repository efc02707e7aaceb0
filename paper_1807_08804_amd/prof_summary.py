"""Summaries of rocprofv3 CSV output for the profiles/ folder.

Three uses:

``kernels``: per-kernel dispatch statistics of a ``--kernel-trace`` run, plus
the dispatches of one kernel that a bench run times (the last N with at
least a given grid), as a markdown table.

``counters``: the mean per dispatch of every counter of one ``--pmc`` run
(LDS bank conflicts and instructions, for instance) for selected dispatches.

``traffic``: HBM bytes per dispatch from a ``--pmc FETCH_SIZE`` run and a
``--pmc WRITE_SIZE`` run of the same command, each scaled by what the same
counter reads for a device copy of known size (``bench.py --copy-probe``).
The result is merged into a JSON record together with a hash of the kernel
sources, so that ``bench.py`` reports it only while the kernels are
unchanged.

    python -m paper_1807_08804_amd.prof_summary kernels --trace DIR --title T \\
        --command CMD --select k_narrow:262144:6 > profiles/x.md
    python -m paper_1807_08804_amd.prof_summary traffic --fetch DIR --write DIR \\
        --copy-fetch DIR --copy-write DIR --copy-bytes B --key large:persist \\
        --select k_narrow:4096:2 --json profiles/hbm_traffic.json
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
# sources whose change invalidates recorded counters
KERNEL_SOURCES = ["csrc/sgm_narrow.hip", "csrc/sgm_narrow.h", "csrc/sgm_device.h",
                  "csrc/sgm_internal.h"]


def _code_only(text: str) -> str:
    """Source text without comments, trailing blanks and empty lines: the
    hash follows the code, not its documentation."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln)


def kernel_source_hash(read=None) -> str:
    """Hash of the kernel sources' code (read(rel) -> text; default: the
    files beside this module)."""
    if read is None:
        def read(rel):
            with open(os.path.join(HERE, rel), encoding="utf-8") as f:
                return f.read()
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        h.update(_code_only(read(rel)).encode())
    return h.hexdigest()


def _csv(d: str, suffix: str):
    files = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0]


def _grid(r) -> int:
    g = r.get("Grid_Size_X") or r.get("Grid_Size") or "0"
    return int(float(g))


def _select(rows, spec: str):
    """Rows of kernel `name` with grid >= min_grid; the last `last` of them."""
    name, min_grid, last = spec.split(":")
    sel = [r for r in rows if name in r["Kernel_Name"] and _grid(r) >= int(min_grid)]
    return sel[-int(last):] if int(last) > 0 else sel


def cmd_kernels(a):
    rows = _csv(a.trace, "kernel_trace.csv")
    by = collections.defaultdict(list)
    for r in rows:
        by[_short(r["Kernel_Name"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    tot = sum(sum(v) for v in by.values())
    out = [f"# rocprofv3 kernel summary: {a.title}", "", f"Command: `{a.command}`", "",
           f"Kernel dispatches: {len(rows)}; total kernel time {tot / 1e3:.3f} ms", "",
           "| kernel | calls | total ms | avg us | median us | max us | % |",
           "|---|---|---|---|---|---|---|"]
    for n, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| {n} | {len(v)} | {sum(v) / 1e3:.3f} | {statistics.mean(v):.2f} | "
                   f"{statistics.median(v):.2f} | {max(v):.1f} | {100 * sum(v) / tot:.1f} |")
    for spec in a.select or []:
        sel = _select(rows, spec)
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in sel]
        name, min_grid, last = spec.split(":")
        shown = ", ".join(f"{x:.0f}" for x in d[:12]) + (", ..." if len(d) > 12 else "")
        out += ["", f"Timed dispatches of `{name}` (grid >= {min_grid} threads, "
                    f"{'last ' + last if int(last) > 0 else 'all'}): {len(d)}, average "
                    f"{statistics.mean(d):.1f} us, median {statistics.median(d):.1f} us ({shown} us)"]
    print("\n".join(out))


def cmd_traffic(a):
    def per_dispatch(d, spec):
        rows = _select(_csv(d, "counter_collection.csv"), spec)
        return [float(r["Counter_Value"]) for r in rows]

    def copy_factor(d):
        rows = [r for r in _csv(d, "counter_collection.csv") if "copyBuffer" in r["Kernel_Name"]]
        kib = statistics.mean(float(r["Counter_Value"]) for r in rows)
        return (a.copy_bytes / 1024.0) / kib

    ff, wf = copy_factor(a.copy_fetch), copy_factor(a.copy_write)
    fetch = per_dispatch(a.fetch, a.select)
    write = per_dispatch(a.write, a.select)
    if not fetch or len(fetch) != len(write):
        raise SystemExit(f"dispatch counts differ or are empty: {len(fetch)} vs {len(write)}")
    per = [(f * ff + w * wf) * 1024.0 for f, w in zip(fetch, write)]
    rec = {}
    if os.path.exists(a.json):
        with open(a.json) as f:
            rec = json.load(f)
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        rec = {"kernel_source_sha256": kernel_source_hash(), "entries": {}}
    rec["fetch_factor"] = round(ff, 4)
    rec["write_factor"] = round(wf, 4)
    rec["entries"][a.key] = {
        "bytes_per_launch": round(statistics.mean(per), 1),
        "fetch_kib": [round(x, 1) for x in fetch], "write_kib": [round(x, 1) for x in write],
        "select": a.select, "command": a.command}
    with open(a.json, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps(rec["entries"][a.key]))


def cmd_counters(a):
    """Mean per dispatch of every counter of a --pmc run, for the selected
    dispatches of each kernel spec; with SQ_LDS_BANK_CONFLICT and
    SQ_INSTS_LDS both present, also the conflict cycles per LDS
    instruction."""
    rows = _csv(a.pmc, "counter_collection.csv")
    out = [f"# rocprofv3 counters: {a.title}", "", f"Command: `{a.command}`", "",
           "| kernel (selection) | counter | dispatches | mean per dispatch | min | max |",
           "|---|---|---|---|---|---|"]
    ratios = []
    for spec in a.select:
        name, min_grid, last = spec.split(":")
        sel = [r for r in rows if name in r["Kernel_Name"] and _grid(r) >= int(min_grid)]
        by = collections.OrderedDict()
        for r in sel:
            by.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        means = {}
        for c, v in by.items():
            v = v[-int(last):] if int(last) > 0 else v
            means[c] = statistics.mean(v)
            out.append(f"| `{name}` ({spec}) | {c} | {len(v)} | {means[c]:.4g} | {min(v):.4g} | "
                       f"{max(v):.4g} |")
        if "SQ_LDS_BANK_CONFLICT" in means and means.get("SQ_INSTS_LDS"):
            ratios.append(f"`{name}`: {means['SQ_LDS_BANK_CONFLICT'] / means['SQ_INSTS_LDS']:.3f} "
                          "bank-conflict cycles per LDS instruction")
    if ratios:
        out += [""] + ["* " + x for x in ratios]
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("--trace", required=True)
    k.add_argument("--title", required=True)
    k.add_argument("--command", required=True)
    k.add_argument("--select", action="append", help="kernel:min_grid_threads:last_n")
    t = sub.add_parser("traffic")
    for o in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--key", "--select", "--json"):
        t.add_argument(o, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--command", default="")
    c = sub.add_parser("counters")
    c.add_argument("--pmc", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--select", action="append", required=True,
                   help="kernel:min_grid_threads:last_n")
    a = ap.parse_args()
    {"kernels": cmd_kernels, "traffic": cmd_traffic, "counters": cmd_counters}[a.cmd](a)


if __name__ == "__main__":
    main()
