"""Write FP64 oracle values of the 512^3 Taylor-Green state between no-slip x-walls
after 100 steps, at probe cubes touching the walls.

Runs only the oracle and the seeded input generator.  After n steps a cell
depends only on cells within n of it, and on the wall it touches.  A probe of
edge 2*HALF against a wall starts from a crop that keeps the real wall: in x,
2*HALF + STEPS cells from the wall inwards; in y and z, a periodic-wrapped
range of edge 2*(HALF + STEPS).  The crop's far x end acts as an artificial
wall.  After every step the layers that its far x end and its y, z wraps
reach are trimmed off, so the result at the probe is exactly the full-domain
oracle's.

usage: python tests/golden/make_tgv512_wall_probes.py
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
# (z centre, y centre, wall): wall 0 at x = 0, wall 1 at x = N
PROBES = [(200, 300, 0), (50, 480, 1)]
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tgv512_wall_probes_100steps.npz")


def crop_initial(prm, zc, yc, wall):
    H = HALF + STEPS
    width = 2 * HALF + STEPS
    xs = np.arange(width) if wall == 0 else np.arange(N - width, N)
    idx = lambda c: np.arange(c - H, c + H) % N
    planes = [W.tgv_slab(prm, int(z), int(z) + 1)[:, 0] for z in idx(zc)]
    Q = np.stack(planes, axis=1)                      # (14, 2H, N, N)
    return np.ascontiguousarray(Q[:, :, idx(yc)][:, :, :, xs])


def probe(prm, zc, yc, wall):
    f = lbm.init_populations(crop_initial(prm, zc, yc, wall), prm)
    for _ in range(STEPS):
        f = lbm.step(f, prm)
        f = f[:, :, 1:-1, 1:-1, :-1] if wall == 0 else f[:, :, 1:-1, 1:-1, 1:]
        f = np.ascontiguousarray(f)
    assert f.shape[2:] == (2 * HALF,) * 3
    return lbm.moments(f)


def main():
    warnings.simplefilter("ignore", RuntimeWarning)
    prm = W.tgv_wall_params(N, storage=W.STORAGE_FP32)
    done, values = [], []
    t0 = time.time()
    for (zc, yc, wall) in PROBES:
        # the crop's own x ends carry the walls; the oracle's step applies the
        # wall of its left end at index 0 and of its right end at index -1
        values.append(probe(prm, zc, yc, wall))
        done.append((zc, yc, wall))
        np.savez(OUT, probes=np.array(done, dtype=np.int64), Q=np.array(values), steps=STEPS, half=HALF,
                 dt=prm["dt"])
        print(f"probe {(zc, yc, wall)} done ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
