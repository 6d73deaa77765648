"""Full-size parity: the 512^3 Taylor-Green update in the benchmark's launch shape.

After n steps a cell depends only on the initial cube of half-width n around it
(D3Q7 streams one face neighbour per step; collision and sensor are
cell-local).  The oracle therefore computes a probe region of edge 2h exactly
from a periodic-wrapped crop of edge 2(h + n) of the initial field; the crop's
own wrap pollutes only its outer n layers.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import lbm

pytestmark = pytest.mark.gpu

N = 512
STEPS = 9          # odd: moments read at odd parity
HALF = 4           # probe edge 2 * HALF
PROBES = [(100, 37, 500), (256, 255, 0), (411, 140, 301)]   # (z, y, x) probe centres


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def crop_initial(prm, zc, yc, xc, H):
    """Initial conserved field on the periodic-wrapped cube of half-width H."""
    idx = lambda c: np.arange(c - H, c + H) % N
    zs, ys, xs = idx(zc), idx(yc), idx(xc)
    planes = [W.tgv_slab(prm, int(z), int(z) + 1)[:, 0] for z in zs]
    Q = np.stack(planes, axis=1)              # (14, 2H, N, N)
    return Q[:, :, ys][:, :, :, xs]


@pytest.mark.parametrize("storage,bound", [(W.STORAGE_FP32, 1e-5), (W.STORAGE_FP16, 2e-3)])
def test_tgv512_probes_match_oracle(storage, bound):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13437_amd as cnsf
    prm = W.tgv_params(N, storage=storage)
    log(f"case tgv512 storage {storage} steps {STEPS}")
    L = cnsf.Lattice(prm)
    log(f"  launch {L.get_launch()}")
    for z0 in range(0, N, 64):
        L.set_state(W.tgv_slab(prm, z0, z0 + 64), z0=z0)
    L.step(STEPS)
    H = HALF + STEPS
    oprm = dict(prm, nx=2 * H, ny=2 * H, nz=2 * H)
    for (zc, yc, xc) in PROBES:
        Qg = L.moments(zc - HALF, 2 * HALF)[:, :, yc - HALF:yc + HALF, :]
        Qg = np.take(Qg, np.arange(xc - HALF, xc + HALF) % N, axis=3)
        Qo = lbm.moments(lbm.run(crop_initial(prm, zc, yc, xc, H), oprm, STEPS))
        Qo = Qo[:, STEPS:STEPS + 2 * HALF, STEPS:STEPS + 2 * HALF, STEPS:STEPS + 2 * HALF]
        rg, ug, _, _, Tg = lbm.primitives(Qg, prm)
        ro, uo, _, _, To = lbm.primitives(Qo, prm)
        err = {k: float(np.linalg.norm(a - b) / np.linalg.norm(b)) for k, a, b in
               (("rho", rg, ro), ("u", ug, uo), ("T", Tg, To))}
        log(f"  probe {(zc, yc, xc)}: rel L2 {err}")
        assert all(v < bound for v in err.values()), err
    d = L.diagnostics(spectral=False)
    assert d["nonfinite"] == 0
    L.close()
