"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2301_05844_amd.profiling trace DIR --title T --cmd C > out.md
        kernel table (calls, average and total time) from a
        ``rocprofv3 --kernel-trace --stats --output-format csv`` run.

    python -m paper_2301_05844_amd.profiling counters DIR [DIR ...] --kernels k_visit4p ... \
        --title T --cmd C [--cmd C ...] > out.md
        per-kernel averages of the counters of ``--pmc`` runs, with the MFMA
        busy fraction and the LDS bank-conflict share where the counters allow.

    python -m paper_2301_05844_amd.profiling traffic --kernel k_visit \
        --kernel-class fit_visit --launches N --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \
        --copy-bytes B --out FILE.json
        HBM bytes per launch of the kernel: FETCH_SIZE and WRITE_SIZE (KiB per
        dispatch) of its last N dispatches, each scaled by what the same
        counter reads for a plain copy of B bytes read and B bytes written.

``source_sha()`` hashes the kernel sources (kernels, launchers and the shapes
they share with the host), so a traffic figure is dropped once the kernels
have changed since the counters were taken.
"""

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ("csrc/bbp_kernels.hip", "csrc/bbp_internal.h")


def source_sha():
    h = hashlib.sha256()
    for rel in SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name):
    """Kernel name without namespaces and argument lists."""
    name = name.replace("(anonymous namespace)::", "").replace("bbp::", "")
    name = re.sub(r"^void ", "", name)
    depth, out = 0, []
    for ch in name:  # drop the parameter list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def _one(pattern):
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise FileNotFoundError(pattern)
    return files[0]


def trace_table(outdir):
    rows = list(csv.DictReader(open(_one(os.path.join(outdir, "**", "*kernel_stats.csv")))))
    table = []
    for r in rows:
        table.append(dict(name=short_name(r["Name"]), calls=int(r["Calls"]),
                          avg_us=float(r["AverageNs"]) / 1e3,
                          total_ms=float(r["TotalDurationNs"]) / 1e6,
                          pct=float(r["Percentage"])))
    return sorted(table, key=lambda t: -t["total_ms"])


def last_dispatches_us(outdir, kernel, n):
    """Average duration (us) of the last n dispatches of a kernel in a
    --kernel-trace run (the timed steps follow the warm-up)."""
    rows = list(csv.DictReader(open(_one(os.path.join(outdir, "**", "*kernel_trace.csv")))))
    d = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
         for r in rows if short_name(r["Kernel_Name"]).startswith(kernel)]
    d.sort()
    tail = [x[1] for x in d[-n:]]
    return sum(tail) / len(tail) / 1e3, len(tail)


def trace_markdown(outdir, title, cmd, top=16):
    lines = [f"# {title}", "", "Command (from the repository root, on one MI355X):", "",
             "```", cmd, "```", "",
             "| kernel | calls | avg (us) | total (ms) | % |", "|---|---:|---:|---:|---:|"]
    for t in trace_table(outdir)[:top]:
        lines.append(f"| `{t['name']}` | {t['calls']} | {t['avg_us']:.1f} | "
                     f"{t['total_ms']:.1f} | {t['pct']:.1f} |")
    return "\n".join(lines) + "\n"


def counter_values(outdir, counter, kernel):
    """Per-dispatch values (dispatch order) of one counter for kernels whose
    short name starts with `kernel`."""
    rows = list(csv.DictReader(open(_one(os.path.join(outdir, "**", "*counter_collection.csv")))))
    per = {}
    for r in rows:
        if r["Counter_Name"] != counter or not short_name(r["Kernel_Name"]).startswith(kernel):
            continue
        key = int(r["Dispatch_Id"])
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    return [per[k] for k in sorted(per)]


def counter_table(dirs, kernels):
    """Average per dispatch of every counter in the given --pmc runs, per
    kernel (short name with template arguments) whose name starts with one
    of `kernels`."""
    acc = {}
    for d in dirs:
        rows = list(csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))))
        per = {}
        for r in rows:
            name = short_name(r["Kernel_Name"])
            if not any(name.startswith(k) for k in kernels):
                continue
            key = (name, r["Counter_Name"], int(r["Dispatch_Id"]))
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        for (name, counter, _), v in per.items():
            s, n = acc.get((name, counter), (0.0, 0))
            acc[(name, counter)] = (s + v, n + 1)
    out = {}
    for (name, counter), (s, n) in acc.items():
        out.setdefault(name, {})[counter] = (s / n, n)
    return out


def gpu_agent(outdir):
    """SIMD and XCD counts of the GPU agent of a run."""
    for r in csv.DictReader(open(_one(os.path.join(outdir, "**", "*agent_info.csv")))):
        if r["Agent_Type"].strip('"') == "GPU":
            return int(r["Simd_Count"]), int(r["Num_Xcc"])
    raise ValueError("no GPU agent in " + outdir)


def counters_markdown(dirs, kernels, title, cmds):
    """Counter averages per kernel, with the MFMA-busy fraction
    SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / XCDs x SIMDs) (GRBM_GUI_ACTIVE
    sums the busy clocks of every XCD) and the LDS bank-conflict share
    SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE."""
    tab = counter_table(dirs, kernels)
    simds, xcds = gpu_agent(dirs[0])
    counters = sorted({c for v in tab.values() for c in v})
    lines = [f"# {title}", "", "Commands (from the repository root, on one MI355X):", "", "```"]
    lines += list(cmds) + ["```", "",
                           "Averages per dispatch over every dispatch of the run "
                           f"(dispatches in parentheses); {simds} SIMDs in {xcds} XCDs.", ""]
    names = sorted(tab, key=lambda n: -tab[n].get("GRBM_GUI_ACTIVE", (0, 0))[0])
    for name in names:
        v = tab[name]
        lines.append(f"## `{name}`")
        lines.append("")
        lines.append("| counter | average per dispatch |")
        lines.append("|---|---:|")
        for c in counters:
            if c in v:
                lines.append(f"| {c} | {v[c][0]:.4g} ({v[c][1]}) |")
        if "SQ_VALU_MFMA_BUSY_CYCLES" in v and "GRBM_GUI_ACTIVE" in v:
            f = v["SQ_VALU_MFMA_BUSY_CYCLES"][0] / (v["GRBM_GUI_ACTIVE"][0] / xcds * simds)
            lines.append(f"| MFMA busy (derived) | {100 * f:.1f}% |")
        if "SQ_LDS_BANK_CONFLICT" in v and "SQ_LDS_IDX_ACTIVE" in v and v["SQ_LDS_IDX_ACTIVE"][0]:
            f = v["SQ_LDS_BANK_CONFLICT"][0] / v["SQ_LDS_IDX_ACTIVE"][0]
            lines.append(f"| LDS bank-conflict share (derived) | {100 * f:.1f}% |")
        lines.append("")
    return "\n".join(lines) + "\n"


def traffic(kernel, kernel_class, launches, fetch, write, copy_fetch, copy_write, copy_bytes,
            copy_kernel):
    f = counter_values(fetch, "FETCH_SIZE", kernel)[-launches:]
    w = counter_values(write, "WRITE_SIZE", kernel)[-launches:]
    cf = max(counter_values(copy_fetch, "FETCH_SIZE", copy_kernel))
    cw = max(counter_values(copy_write, "WRITE_SIZE", copy_kernel))
    kib = copy_bytes / 1024.0
    ff, fw = cf / kib, cw / kib  # counter KiB per KiB actually moved
    fetch_b = sum(f) / len(f) * 1024.0 / ff
    write_b = sum(w) / len(w) * 1024.0 / fw
    return dict(kernel=kernel, kernel_class=kernel_class, launches=len(f), source_sha=source_sha(),
                fetch_kib_per_dispatch=sum(f) / len(f), write_kib_per_dispatch=sum(w) / len(w),
                copy_bytes=copy_bytes, copy_fetch_factor=ff, copy_write_factor=fw,
                fetch_bytes_per_launch=fetch_b, write_bytes_per_launch=write_b,
                bytes_per_launch=fetch_b + write_b)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="action", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", required=True)
    t.add_argument("--cmd", required=True)
    t.add_argument("--timed-kernel", default="")
    t.add_argument("--timed-launches", type=int, default=0)
    c = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "out"):
        c.add_argument("--" + k.replace("_", "-"), required=True)
    c.add_argument("--kernel", required=True)
    c.add_argument("--kernel-class", required=True)
    c.add_argument("--launches", type=int, required=True)
    c.add_argument("--copy-bytes", type=float, required=True)
    c.add_argument("--copy-kernel", default="")
    k = sub.add_parser("counters")
    k.add_argument("dirs", nargs="+")
    k.add_argument("--kernels", nargs="+", required=True)
    k.add_argument("--title", required=True)
    k.add_argument("--cmd", action="append", default=[])
    a = ap.parse_args(argv)
    if a.action == "counters":
        sys.stdout.write(counters_markdown(a.dirs, a.kernels, a.title, a.cmd))
    elif a.action == "trace":
        sys.stdout.write(trace_markdown(a.dir, a.title, a.cmd))
        if a.timed_kernel:
            us, n = last_dispatches_us(a.dir, a.timed_kernel, a.timed_launches)
            sys.stdout.write(f"\nLast {n} dispatches of `{a.timed_kernel}` (the timed solves): "
                             f"average {us:.1f} us.\n")
    else:
        r = traffic(a.kernel, a.kernel_class, a.launches, a.fetch, a.write, a.copy_fetch, a.copy_write,
                    a.copy_bytes, a.copy_kernel)
        with open(a.out, "w") as f:
            json.dump(r, f, indent=1)
        print(json.dumps(r))


if __name__ == "__main__":
    main()
