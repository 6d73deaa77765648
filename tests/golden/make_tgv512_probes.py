"""Write FP64 oracle values of the 512^3 Taylor-Green state after 100 steps at probe cubes.

Runs only the oracle and the seeded input generator.  D3Q7 moves each
population one face neighbour per step and the collision is cell-local, so
after n steps a cell depends only on the initial cube of half-width n around
it.  Each probe (edge 2*HALF) starts from a periodic-wrapped crop of edge
2*(HALF + STEPS) of the initial field; after every step the outer layer, the
only one the crop's own wrap reaches, is trimmed off.  The result at the probe
is exactly the full-domain oracle's.

Probe centres are drawn with numpy.random.default_rng(13437); the first three
are fixed (one wraps the periodic x boundary).  The output file is rewritten
after each probe, so an interrupted run keeps the probes it finished, and a
later run with more probes keeps the ones already in the file (same centres,
same time step) and computes only the rest.

usage: python tests/golden/make_tgv512_probes.py [NPROBES]
       python tests/golden/make_tgv512_probes.py NPROBES --only A:B --part PATH
       python tests/golden/make_tgv512_probes.py NPROBES --merge PATH [PATH ...]
--only computes probes A..B-1 of the NPROBES centres into PATH (one process per
range, so ranges can run side by side); --merge adds the probes held in the
part files to the output file, in centre order, and checks every centre.
"""
import os
import sys
import time
import warnings

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import lbm  # noqa: E402

N = 512
STEPS = 100
HALF = 4
FIXED = [(100, 37, 500), (256, 255, 0), (411, 140, 301)]   # (z, y, x)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tgv512_probes_100steps.npz")


def probe_centres(n):
    rng = np.random.default_rng(13437)
    extra = [tuple(int(v) for v in rng.integers(0, N, size=3)) for _ in range(max(0, n - len(FIXED)))]
    return (FIXED + extra)[:n]


def crop_initial(prm, zc, yc, xc, H):
    idx = lambda c: np.arange(c - H, c + H) % N
    planes = [W.tgv_slab(prm, int(z), int(z) + 1)[:, 0] for z in idx(zc)]
    Q = np.stack(planes, axis=1)                      # (14, 2H, N, N)
    return np.ascontiguousarray(Q[:, :, idx(yc)][:, :, :, idx(xc)])


def probe(prm, centre, progress=25):
    H = HALF + STEPS
    f = lbm.init_populations(crop_initial(prm, *centre, H), prm)
    for s in range(STEPS):
        f = np.ascontiguousarray(lbm.step(f, prm)[:, :, 1:-1, 1:-1, 1:-1])
        if progress and (s + 1) % progress == 0:
            print(f"  probe {centre}: step {s + 1}/{STEPS}, crop edge {f.shape[2]}", flush=True)
    assert f.shape[2:] == (2 * HALF,) * 3
    return lbm.moments(f)


def save(path, centres, values, prm):
    np.savez(path, centres=np.array(centres, dtype=np.int64), Q=np.array(values), steps=STEPS, half=HALF,
             dt=prm["dt"])


def main():
    warnings.simplefilter("ignore", RuntimeWarning)
    nprobes = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    prm = W.tgv_params(N, storage=W.STORAGE_FP32)
    want = probe_centres(nprobes)
    if "--only" in sys.argv:
        a, b = (int(v) for v in sys.argv[sys.argv.index("--only") + 1].split(":"))
        part = sys.argv[sys.argv.index("--part") + 1]
        centres, values = [], []
        t0 = time.time()
        for c in want[a:b]:
            values.append(probe(prm, c))
            centres.append(c)
            save(part, centres, values, prm)
            print(f"probe {c} done ({time.time() - t0:.0f} s)", flush=True)
        return
    if "--merge" in sys.argv:
        have = {}
        for path in [OUT] + sys.argv[sys.argv.index("--merge") + 1:]:
            if not os.path.exists(path):
                continue
            d = np.load(path)
            assert float(d["dt"]) == prm["dt"] and int(d["steps"]) == STEPS and int(d["half"]) == HALF, path
            for c, q in zip(d["centres"], d["Q"]):
                have[tuple(int(v) for v in c)] = q
        centres = [c for c in want if c in have]
        assert centres == want[:len(centres)], "the merged probes must be the first centres, in order"
        save(OUT, centres, [have[c] for c in centres], prm)
        print(f"{OUT}: {len(centres)} probes", flush=True)
        return
    centres, values = [], []
    if os.path.exists(OUT):
        old = np.load(OUT)
        have = [tuple(int(v) for v in c) for c in old["centres"]]
        if float(old["dt"]) == prm["dt"] and have == want[:len(have)]:
            centres, values = have, list(old["Q"])
            print(f"keeping {len(have)} probes from {OUT}", flush=True)
    t0 = time.time()
    for c in want[len(centres):]:
        values.append(probe(prm, c))
        centres.append(c)
        save(OUT, centres, values, prm)
        print(f"probe {c} done ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
