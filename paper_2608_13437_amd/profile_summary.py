"""Summarise rocprofv3 output of the update kernel into short text files.

usage:
  python -m paper_2608_13437_amd.profile_summary stats  <kernel_stats.csv> <out.txt> "<command>" [bench.log]
  python -m paper_2608_13437_amd.profile_summary traffic <fetch.csv> <write.csv> <copy_fetch.csv>
         <copy_write.csv> <copy_bytes> <storage> <out.json> "<commands>"
  python -m paper_2608_13437_amd.profile_summary requests <dram.csv> <copy_dram.csv> <copy_bytes>
         <storage> <out.json> "<command>"
The traffic summary scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the
update by the factor the same counter needs on a plain copy of known size.
The requests summary does the same with the DRAM read and write request
counts (TCC_EA0_RDREQ_DRAM_sum, TCC_EA0_WRREQ_DRAM_sum), a cross-check of
the first from another counter.
"""
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the update kernel, its per-cell code, and the population layout and default
# launch shape it runs with
SOURCES = ["paper_2608_13437_amd/csrc/update.hip", "paper_2608_13437_amd/csrc/cnsf_impl.h",
           "paper_2608_13437_amd/csrc/layout.cpp"]


def kernel_hash():
    h = hashlib.sha256()
    for rel in SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


PROBE_UPDATES = 5   # Lattice.placed: one untimed and four timed updates per candidate array


def timed_launches(trace_path, rec):
    """Durations (ms) of the periodic update dispatches of bench.py's timed region
    (first storage): after the placement probe's updates on every candidate
    array and the warmup updates, the next `steps` dispatches."""
    rows = [r for r in csv.DictReader(open(trace_path)) if UPDATE.search(r["Kernel_Name"])]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    placement = rec.get("placement") or {}
    first = rec["config"]["storage"]
    skip = PROBE_UPDATES * len(placement[first]["probe_ms"]) if first in placement else 0
    skip += int(rec["warmup"])
    sel = rows[skip:skip + int(rec["steps"])]
    return [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in sel]


def stats(path, out, command, bench_log=None):
    rows = list(csv.DictReader(open(path)))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}", f"# kernel source hash: {kernel_hash()}"]
    if bench_log:
        # the JSON line bench.py printed in the profiled process itself
        for line in open(bench_log):
            if line.startswith("{") and '"metric"' in line:
                rec = json.loads(line)
                lines.append(f"# bench.py in the same process: ms_per_step {rec['ms_per_step']} "
                             f"(mean of the even and odd launches), {rec['value']} {rec['unit']}")
                trace = os.path.join(os.path.dirname(path), "run_kernel_trace.csv")
                if os.path.exists(trace):
                    # the table below also counts the placement probe's launches on
                    # the candidate arrays and any launches after the timed region
                    d = timed_launches(trace, rec)
                    lines.append(f"# timed region in the kernel trace: the {len(d)} update launches after the "
                                 f"placement probe and warmup, mean {sum(d) / len(d):.4f} ms "
                                 f"(min {min(d):.4f}, max {max(d):.4f})")
    lines.append("")
    lines.append(f"{'calls':>6} {'avg_ms':>10} {'min_ms':>10} {'max_ms':>10} {'pct':>7}  kernel")
    for r in rows:
        lines.append(f"{int(r['Calls']):>6} {float(r['AverageNs']) / 1e6:>10.4f} {float(r['MinNs']) / 1e6:>10.4f} "
                     f"{float(r['MaxNs']) / 1e6:>10.4f} {float(r['Percentage']):>7.2f}  {r['Name'][:110]}")
    open(out, "w").write("\n".join(lines) + "\n")


# the periodic update without the fused diagnostics: k_update<storage, 0, scaled, parity, false>
UPDATE = re.compile(r"k_update<\d, 0, (false|true), [01], false>")
COPY = re.compile(r"k_copy")


def counter(path, pattern):
    return [float(r["Counter_Value"]) for r in csv.DictReader(open(path)) if pattern.search(r["Kernel_Name"])]


def traffic(fetch, write, cfetch, cwrite, copy_bytes, storage, out, command):
    f, w = counter(fetch, UPDATE), counter(write, UPDATE)
    cf, cw = counter(cfetch, COPY), counter(cwrite, COPY)
    copy_bytes = int(copy_bytes)
    ffac = sum(copy_bytes / (x * 1024) for x in cf) / len(cf)
    wfac = sum(copy_bytes / (x * 1024) for x in cw) / len(cw)
    fb = [x * 1024 * ffac for x in f]
    wb = [x * 1024 * wfac for x in w]
    per = [a + b for a, b in zip(fb, wb)]
    rec = json.load(open(out)) if os.path.exists(out) else {}
    rec["kernel_hash"] = kernel_hash()
    rec["copy_factor"] = dict(FETCH_SIZE=round(ffac, 4), WRITE_SIZE=round(wfac, 4))
    rec[storage] = dict(fetch_bytes=[round(x) for x in fb], write_bytes=[round(x) for x in wb],
                        bytes_per_launch=round(sum(per) / len(per)), command=command)
    json.dump(rec, open(out, "w"), indent=1)


def _by_counter(path, pattern):
    out = {}
    for r in csv.DictReader(open(path)):
        if pattern.search(r["Kernel_Name"]):
            out.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return out


def requests(dram, cdram, copy_bytes, storage, out, command):
    u, c = _by_counter(dram, UPDATE), _by_counter(cdram, COPY)
    copy_bytes = int(copy_bytes)
    rd, wr = "TCC_EA0_RDREQ_DRAM_sum", "TCC_EA0_WRREQ_DRAM_sum"
    # a copy reads and writes copy_bytes: bytes per request of each kind
    rsz = copy_bytes / (sum(c[rd]) / len(c[rd]))
    wsz = copy_bytes / (sum(c[wr]) / len(c[wr]))
    per = [a * rsz + b * wsz for a, b in zip(u[rd], u[wr])]
    rec = json.load(open(out)) if os.path.exists(out) else {}
    rec.setdefault(storage, {})["dram_requests"] = dict(
        bytes_per_read=round(rsz, 2), bytes_per_write=round(wsz, 2),
        bytes_per_launch=round(sum(per) / len(per)), launches=len(per), command=command)
    json.dump(rec, open(out, "w"), indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(*sys.argv[2:6])
    elif sys.argv[1] == "requests":
        requests(*sys.argv[2:8])
    else:
        traffic(*sys.argv[2:10])
