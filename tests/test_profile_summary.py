"""Host logic of the rocprofv3 summaries, on synthetic CSV files.

The timed region of a bench.py process is located in the kernel trace after
the placement probe's updates (five per candidate array) and the warmup; the
traffic summary scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by the factor
the same counter needs on a copy of known size.
"""
import csv
import json

import pytest

from paper_2608_13437_amd import profile_summary as ps

UPD = "void cnsf::k_update<{st}, 0, false, {par}, false>(cnsf::Store<{st}>::T*, cnsf::Geom)"
DIAG = "void cnsf::k_update<0, 0, false, 0, true>(cnsf::Store<0>::T*, cnsf::Geom)"
WALL = "void cnsf::k_update<0, 3, false, 1, false>(cnsf::Store<0>::T*, cnsf::Geom)"


def write_trace(path, durations_ns, extra=()):
    cols = ["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    t, rows = 1000, []
    for i, d in enumerate(durations_ns):
        rows.append(dict(Kind="KERNEL_DISPATCH", Kernel_Name=UPD.format(st=0, par=i % 2), Start_Timestamp=t,
                         End_Timestamp=t + d))
        t += d + 10
    for name in extra:
        rows.append(dict(Kind="KERNEL_DISPATCH", Kernel_Name=name, Start_Timestamp=t, End_Timestamp=t + 7))
        t += 20
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=cols)
        w.writeheader()
        w.writerows(rows)


def test_timed_region_follows_probe_and_warmup(tmp_path):
    # 2 candidates x 5 probe updates (ms 9), 2 warmup (ms 8), 4 timed (ms 1..4), 3 later (ms 7)
    probe = [9_000_000] * 10
    warm = [8_000_000] * 2
    timed = [1_000_000, 2_000_000, 3_000_000, 4_000_000]
    later = [7_000_000] * 3
    trace = tmp_path / "run_kernel_trace.csv"
    write_trace(trace, probe + warm + timed + later, extra=[DIAG, WALL])
    rec = {"steps": 4, "warmup": 2, "config": {"storage": "fp32"},
           "placement": {"fp32": {"probe_ms": [9.0, 9.0], "kept": 0}}}
    assert ps.timed_launches(str(trace), rec) == [1.0, 2.0, 3.0, 4.0]
    rec.pop("placement")               # --no-placement: one plain allocation, no probe
    write_trace(trace, warm + timed + later)
    assert ps.timed_launches(str(trace), rec) == [1.0, 2.0, 3.0, 4.0]


def test_update_pattern_takes_only_periodic_plain_updates():
    assert ps.UPDATE.search(UPD.format(st=1, par=1))
    assert not ps.UPDATE.search(DIAG)
    assert not ps.UPDATE.search(WALL)


def write_counters(path, name, kib):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for v in kib:
            w.writerow(dict(Kernel_Name=name, Counter_Value=v))


def test_traffic_scales_counters_by_the_copy_calibration(tmp_path):
    copy_bytes = 2 * 1024 ** 3
    # the copy's FETCH_SIZE reads half its true bytes, WRITE_SIZE all of them
    write_counters(tmp_path / "cf.csv", "cnsf::k_copy(uint4 const*)", [copy_bytes / 2 / 1024] * 2)
    write_counters(tmp_path / "cw.csv", "cnsf::k_copy(uint4 const*)", [copy_bytes / 1024] * 2)
    name = UPD.format(st=0, par=0)
    write_counters(tmp_path / "f.csv", name, [1000.0, 1100.0])
    write_counters(tmp_path / "w.csv", name, [2000.0, 2000.0])
    out = tmp_path / "traffic.json"
    ps.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
               str(tmp_path / "cw.csv"), str(copy_bytes), "fp32", str(out), "cmd")
    rec = json.load(open(out))
    assert rec["copy_factor"] == {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}
    assert rec["fp32"]["fetch_bytes"] == [2_048_000, 2_252_800]
    assert rec["fp32"]["write_bytes"] == [2_048_000, 2_048_000]
    assert rec["fp32"]["bytes_per_launch"] == pytest.approx((2_048_000 + 2_252_800) / 2 + 2_048_000)
    assert rec["kernel_hash"] == ps.kernel_hash()
