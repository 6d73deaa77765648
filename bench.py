"""Throughput of the fused D3Q7 stream-and-collide update on one MI355X.

Workload: the supersonic Taylor-Green vortex at 512^3 (M0 = 1.25, Re = 1600,
Pr = 0.71, mu ~ T^0.76), seeded synthetic initial field, populations stored
FP32 (the headline number) and as FP16 / BF16 deviations (reported beside it).
One step is one in-place pass of the whole update over all 134M cells.

Prints one JSON line:
  value      MLUPS of the FP32-storage update (whole job, inputs resident in HBM)
  roofline   HBM roofline of the update kernel: algorithmic bytes per launch
             (98 populations read + written per cell) / mean launch time from
             HIP events on the launch stream, against 8 TB/s
  cpu_baseline  the FP64 NumPy oracle on a bounded sample (64^3 Taylor-Green)
             on this host's cores
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 512]
                       [--storage all|fp32|fp16|bf16] [--no-cpu] [--batch]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
METRIC = "MLUPS + HBM GB/s (% peak), FP32 vs FP16-storage, supersonic TGV 512^3"
STORAGES = {"fp32": 0, "fp16": 1, "bf16": 2}
BYTES_PER_POP = {"fp32": 4, "fp16": 2, "bf16": 2}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_update_tgv512.json")
from paper_2608_13437_amd.profile_summary import kernel_hash  # noqa: E402


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def tgv_field_device(n, slab=16):
    """The 512^3 Taylor-Green initial conserved field, generated once in host
    slabs and kept in device memory (FP64, 14 x n^3) for every storage run."""
    import torch
    import workloads as W
    prm = W.tgv_params(n)
    t0 = time.perf_counter()
    Q = torch.empty((14, n, n, n), dtype=torch.float64, device="cuda")
    for z0 in range(0, n, slab):
        z1 = min(n, z0 + slab)
        Q[:, z0:z1].copy_(torch.from_numpy(W.tgv_slab(prm, z0, z1)))
    torch.cuda.synchronize()
    log(f"  Taylor-Green field {n}^3: {time.perf_counter() - t0:.1f} s")
    return Q


def load_lattice_tgv(cnsf, n, storage, Qdev, placed=True):
    """The benchmark lattice: by default on the fastest of several probed
    population arrays (Lattice.placed), else on one plain allocation."""
    import torch
    import workloads as W
    prm = W.tgv_params(n, storage=STORAGES[storage])
    L = cnsf.Lattice.placed(prm) if placed else cnsf.Lattice(prm)
    t0 = time.perf_counter()
    L.set_state(Qdev)
    torch.cuda.synchronize()
    log(f"  set_state {n}^3 {storage} from device: {time.perf_counter() - t0:.2f} s")
    return L, prm


def time_update(L, steps, warmup):
    """Mean per-launch time (ms) from HIP events recorded on the launch stream."""
    import torch
    L.step(warmup)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for s in range(steps):
        L.step(1)
        ev[s + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [ev[s].elapsed_time(ev[s + 1]) for s in range(steps)]
    return float(np.mean(per)), float(np.min(per)), wall


SPECTRUM_BYTES_PER_CELL = {"fp32": 400, "fp16": 344, "bf16": 344}


def spectrum_timing(L, storage, reps=3):
    """Shell-averaged velocity spectrum of the current state: mean time of one call
    (velocity readout, three 3D transforms, shell sums), from HIP events on the
    lattice's stream.  Algorithmic bytes per cell: the 28 populations of rho and
    rho u read and u, v, w written (136 B FP32, 80 B 16-bit), 256 B for the axis
    passes, 8 B for the shell sums."""
    import torch
    E = L.spectrum(device=True)          # allocates the workspace
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        E = L.spectrum(device=True)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    gbps = SPECTRUM_BYTES_PER_CELL[storage] * L.ncells / (ms * 1e-3) / 1e9
    return dict(ms=round(ms, 3), shells=int(E.numel()), GBps=round(gbps, 1),
                frac_peak=round(gbps / PEAK_HBM_GBPS, 4), sum_E=float(E.sum().item()))


def diagnostics_timing(L, reps=3):
    """FP64 Eq. (7) diagnostics with spectral derivatives (sums, E_k, eps_s,
    eps_d): mean time of one call, HIP events on the lattice's stream."""
    import torch
    L.diagnostics(spectral=True)         # allocates the workspace
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        L.diagnostics(spectral=True)
    b.record()
    torch.cuda.synchronize()
    return round(a.elapsed_time(b) / reps, 3)


def noslip_timing(cnsf, L, n, storage, Qdev, steps, warmup):
    """The same update with no-slip x-walls (adiabatic and still at x = 0,
    isothermal and moving at x = L) on the same state and in the same
    population array as the periodic timing, so both see one placement."""
    import workloads as W
    prm = W.tgv_wall_params(n, storage=STORAGES[storage])
    Lw = cnsf.Lattice(prm, buf=L.buf)
    Lw.set_state(Qdev)
    ms = time_update(Lw, steps, warmup)[0]
    finite = Lw.diagnostics(spectral=False)["nonfinite"] == 0
    Lw.close()
    del Lw
    return ms, finite


def fused_readout_timing(L, reps=4):
    """Added cost of the same readout when the first update of a step reduces it
    (cnsf_step_diagnostics): one fused call of one step less one plain step,
    HIP events on the lattice's stream; even reps cover both streaming passes."""
    import torch
    L.step_diagnostics(1, spectral=True)
    torch.cuda.synchronize()
    ms = []
    for fn in (lambda: L.step_diagnostics(1, spectral=True), lambda: L.step(1)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b) / reps)
    return round(ms[0] - ms[1], 3)


def copy_bandwidth(cnsf, nbytes=8 << 30, reps=10):
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    s = torch.cuda.current_stream().cuda_stream
    cnsf.cnsf_hbm_copy(dst.data_ptr(), src.data_ptr(), nbytes, s)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        cnsf.cnsf_hbm_copy(dst.data_ptr(), src.data_ptr(), nbytes, s)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(n=64, steps=48, tube_steps=500):
    """The FP64 oracle (NumPy, single-threaded elementwise code) on a bounded sample:
    Taylor-Green (the headline's flow, MLUPS) and, beside it, the two shock tubes
    (Sod 256 cells and Becker 128 cells along x; the oracle runs the y/z-uniform
    tubes on one cell row, bitwise the N x 4 x 4 result)."""
    import warnings
    warnings.simplefilter("ignore", RuntimeWarning)
    import workloads as W
    from oracle import lbm
    case = W.tgv(n)
    f = lbm.init_populations(case.Q0, case.params)
    f = lbm.step(f, case.params)
    t0 = time.perf_counter()
    for _ in range(steps):
        f = lbm.step(f, case.params)
    dt = time.perf_counter() - t0
    tubes = {}
    for name, c in (("sod256", W.sod(256, 1, 1)), ("becker128", W.becker(128, 1, 1))):
        f = lbm.init_populations(c.Q0, c.params)
        t1 = time.perf_counter()
        for _ in range(tube_steps):
            f = lbm.step(f, c.params)
        tt = time.perf_counter() - t1
        tubes[name] = dict(us_per_step=round(tt / tube_steps * 1e6, 1), steps=tube_steps,
                           MLUPS=round(c.params["nx"] * tube_steps / tt / 1e6, 4))
    return dict(value=round(n ** 3 * steps / dt / 1e6, 4), unit="MLUPS", cores=1, kind="oracle",
                host_cpus=os.cpu_count(),
                sample=f"Taylor-Green {n}^3, {steps} steps of the FP64 NumPy oracle ({dt:.1f} s); one core of "
                       f"{os.cpu_count()} (NumPy elementwise code is single-threaded)",
                shock_tubes=tubes)


def shock_tube_timing(cnsf, steps=2000, warmup=100):
    """Sod 256 x 4 x 4 between parity walls and Becker N x 4 x 4 (N = 128 ... 1024)
    with equilibrium ends, FP32: microseconds per step from HIP events around
    one call of `steps` updates on the lattice's stream.  These lattices hold
    4k-16k cells, so each update is one short kernel; the library replays them
    from a captured graph of 32 updates (captured during the warmup)."""
    import torch
    import workloads as W
    out = {}
    cases = [("sod256x4x4", W.sod(256, 4, 4))] + [(f"becker{n}x4x4", W.becker(n, 4, 4)) for n in (128, 256, 512, 1024)]
    for name, c in cases:
        L = cnsf.Lattice(c.params)
        L.set_state(c.Q0)
        L.step(warmup)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        L.step(steps)
        b.record()
        torch.cuda.synchronize()
        us = a.elapsed_time(b) * 1e3 / steps
        finite = L.diagnostics(spectral=False)["nonfinite"] == 0
        out[name] = dict(cells=L.ncells, us_per_step=round(us, 2), MLUPS=round(L.ncells / us, 1), finite=finite)
        L.close()
    return out


def placed_copy_bandwidth(cnsf, L, reps=5):
    """The plain copy kernel between the two halves of a lattice's (placed) population
    array: the attainable streaming rate of that physical memory.  Run after the
    update timing; it overwrites the populations."""
    import torch
    half = (L.nbytes // 2) & ~255
    base = L.buf.data_ptr()
    s = torch.cuda.current_stream().cuda_stream
    cnsf.cnsf_hbm_copy(base + half, base, half, s)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        cnsf.cnsf_hbm_copy(base + half, base, half, s)
    b.record()
    torch.cuda.synchronize()
    return 2 * half / (a.elapsed_time(b) / reps * 1e-3) / 1e9


def traffic_entry(storage, mean_ms):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if current."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    rec = t.get(storage)
    if not rec or t.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


# Bytes between the component runs of the ensemble's population array (the
# component-major batch layout): 1 GiB apart, like a large lattice's regions.
BATCH_SPACING = 1 << 30
BATCH_STEPS = 2000


def run_batch(cnsf, steps, warmup, placed=True):
    """Ensemble of 64 uneven Taylor-Green lattices (FP16 storage): graph replay vs
    per-step launches vs per-member launches.  The population array is placed
    like the single lattices (Batch.placed: the fastest of several probed
    allocations), with its component runs BATCH_SPACING apart; the first
    candidate's probe is the plain-allocation rate."""
    import torch
    import workloads as W
    cases = W.batch_ensemble(materialize=False)
    prms = [c.params for c in cases]
    B = (cnsf.Batch.placed(prms, spacing=BATCH_SPACING) if placed
         else cnsf.Batch(prms, spacing=BATCH_SPACING))
    for j, c in enumerate(cases):
        B.set_state(j, W.tgv_slab(c.params, 0, c.params["nz"]))
    B.autotune(os.path.join(tempfile.gettempdir(), "cnsf_batch_autotune.json"), steps_per_trial=10)
    out = {}
    alg = 98 * 2 * 2 * B.ncells            # FP16: 98 populations read and written, 2 B each
    for name, mode in (("graph", 1), ("launch", 0), ("sequential", 2)):
        B.step(warmup, mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.step(steps, mode)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = round(B.ncells * steps / dt / 1e6, 1)
        if name == "graph":
            out["graph_GBps"] = round(alg * steps / dt / 1e9, 1)
            out["graph_frac_peak"] = round(alg * steps / dt / 1e9 / PEAK_HBM_GBPS, 4)
    out["cells"] = B.ncells
    out["members"] = len(cases)
    out["steps"] = steps
    out["array_bytes"] = B.nbytes
    out["component_spacing_bytes"] = BATCH_SPACING
    if placed:
        ms = B.placement_ms
        out["placement"] = dict(probe_ms=[round(x, 4) for x in ms], kept=B.placement_kept,
                                first_draw_MLUPS=round(B.ncells / (ms[0] * 1e-3) / 1e6, 1))
    out["launch_shape"] = dict(zip(("block", "tile", "grid", "graph_steps"), B.get_launch()))
    B.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--storage", default="all")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-placement", action="store_true",
                    help="one plain allocation per lattice instead of the fastest of several probed arrays")
    ap.add_argument("--no-spectrum", action="store_true", help="skip the shell-spectrum timing")
    ap.add_argument("--no-walls", action="store_true", help="skip the no-slip wall timing")
    ap.add_argument("--no-tubes", action="store_true", help="skip the Sod / Becker shock-tube timing")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched ensemble (the line carries no headline value)")
    ap.add_argument("--copy-only", type=int, default=0, metavar="GIB",
                    help="only run the plain copy kernel on GIB GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU halo-exchange path is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2608_13437_amd as cnsf
    cnsf.library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_only:
        gbps = copy_bandwidth(cnsf, nbytes=args.copy_only << 30, reps=args.steps)
        print(json.dumps({"copy_bytes_per_launch": 2 * (args.copy_only << 30), "copy_GBps": round(gbps, 1),
                          "launches": args.steps + 1}), flush=True)
        return

    if args.batch_only:
        print(json.dumps({"batch": run_batch(cnsf, args.steps, args.warmup, placed=not args.no_placement)}),
              flush=True)
        return

    storages = list(STORAGES) if args.storage == "all" else [args.storage]
    head = "fp32" if "fp32" in storages else storages[0]
    placement = {}
    spectrum = None
    n = args.n
    Qdev = tgv_field_device(n)
    cells = n ** 3
    res = {}
    walls = {}
    placed_copy = None
    for st in storages:
        L, prm = load_lattice_tgv(cnsf, n, st, Qdev, placed=not args.no_placement)
        launch = L.get_launch()
        if not args.no_placement:
            placement[st] = dict(probe_ms=[round(x, 3) for x in L.placement_ms], kept=L.placement_kept)
            log(f"  {st} placement probe: {placement[st]['probe_ms']} ms per update, kept #{L.placement_kept}")
        mean_ms, min_ms, wall = time_update(L, args.steps, args.warmup)
        if st == head and not args.no_spectrum:
            spectrum = spectrum_timing(L, st)
            spectrum["diagnostics_ms"] = diagnostics_timing(L)
            spectrum["fused_diagnostics_ms"] = fused_readout_timing(L)
        d = L.diagnostics(spectral=False)
        alg_bytes = 98 * 2 * BYTES_PER_POP[st] * cells
        res[st] = dict(ms=mean_ms, min_ms=min_ms, wall=wall, mlups=cells / (mean_ms * 1e-3) / 1e6, launch=launch,
                       gbps=alg_bytes / (mean_ms * 1e-3) / 1e9, bytes=alg_bytes, finite=d["nonfinite"] == 0)
        log(f"  {st}: {mean_ms:.3f} ms/step, {res[st]['mlups']:.0f} MLUPS, {res[st]['gbps']:.0f} GB/s")
        if not args.no_walls and st in ("fp32", "fp16"):
            wms, wfin = noslip_timing(cnsf, L, n, st, Qdev, max(2, args.steps // 4), args.warmup)
            walls[st] = dict(ms_per_step=round(wms, 4), MLUPS=round(cells / (wms * 1e-3) / 1e6, 1),
                             GBps=round(alg_bytes / (wms * 1e-3) / 1e9, 1), vs_periodic=round(mean_ms / wms, 4),
                             finite=wfin)
            log(f"  {st} no-slip walls: {wms:.3f} ms/step ({mean_ms / wms:.3f}x the periodic rate)")
        if st == head and not args.no_copy:
            placed_copy = placed_copy_bandwidth(cnsf, L)
            log(f"  copy kernel inside the {st} population array: {placed_copy:.0f} GB/s")
        L.close()
        del L
        torch.cuda.empty_cache()

    del Qdev
    torch.cuda.empty_cache()
    r = res[head]
    copy_gbps = None if args.no_copy else round(copy_bandwidth(cnsf), 1)
    traffic = traffic_entry(head, r["ms"])
    out = {
        "metric": METRIC,
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"supersonic Taylor-Green vortex {n}^3 (M0 1.25, Re 1600), D3Q7 14-component "
                        f"stream-collide, {head} populations, AA in-place",
            "cells": cells, "storage": head,
            "launch": dict(zip(("block", "tile", "grid", "xcd_remap"), r["launch"])),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(r["gbps"], 1),
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": round(r["gbps"] / PEAK_HBM_GBPS, 4),
            "traffic": traffic,
        },
        "hbm_copy_GBps": copy_gbps,
        "hbm_copy_placed_GBps": None if placed_copy is None else round(placed_copy, 1),
        "variants": {st: {"ms_per_step": round(v["ms"], 4), "MLUPS": round(v["mlups"], 1),
                          "GBps": round(v["gbps"], 1), "frac_peak": round(v["gbps"] / PEAK_HBM_GBPS, 4),
                          "speedup_vs_fp32": (round(res["fp32"]["ms"] / v["ms"], 3) if "fp32" in res else None),
                          "launch": dict(zip(("block", "tile", "grid", "xcd_remap"), v["launch"])),
                          "finite": v["finite"]}
                     for st, v in res.items()},
        "kernel_hash": kernel_hash(),
    }
    if spectrum is not None:
        out["spectrum"] = dict(spectrum, storage=head)
    if placement:
        for st, pl in placement.items():
            ms0 = pl["probe_ms"][0]
            gb0 = 98 * 2 * BYTES_PER_POP[st] * cells / (ms0 * 1e-3) / 1e9
            pl["first_draw"] = dict(ms_per_step=ms0, MLUPS=round(cells / (ms0 * 1e-3) / 1e6, 1),
                                    GBps=round(gb0, 1), frac_peak=round(gb0 / PEAK_HBM_GBPS, 4))
        out["placement"] = dict(placement, policy="each lattice on the fastest of up to 8 probed population arrays, "
                                                  "as many as fit in 85% of free memory (Lattice.placed: 4 timed "
                                                  "updates of the cleared state per candidate); value is the full "
                                                  "timed run on the kept array")
    if walls:
        out["noslip_walls"] = dict(walls, note="no-slip x-walls (still adiabatic, moving isothermal): same state "
                                               "and population array as the periodic figure")
    if not args.no_tubes:
        out["shock_tubes"] = shock_tube_timing(cnsf)
    if not args.no_batch:
        # the ensemble configuration's 2,000 steps per member, in each mode
        out["batch"] = run_batch(cnsf, BATCH_STEPS, 4, placed=not args.no_placement)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
