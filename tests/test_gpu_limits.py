"""Largest lattices the library accepts: parity at the top of the 32-bit offset range.

A component's region of 7 population slots is addressed with 32-bit byte
offsets, so the largest cube is 535^3 for FP32 (4.29e9 bytes per region) and
674^3 for FP16.  After n steps a cell depends only on the initial cube of
half-width n around it, so only each probe's neighbourhood must hold the
Taylor-Green field: the lattice is set to the uniform background state, and
the z-planes within reach of a probe to the Taylor-Green field.  The oracle
runs each probe on a periodic crop of the initial field and keeps the interior
that the crop's own wrap cannot reach.  Probes include the last cell of the
lattice, whose populations sit at the highest offsets.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import lbm

pytestmark = pytest.mark.gpu
STEPS = 5
HALF = 4


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def crop_initial(prm, N, zc, yc, xc, H):
    idx = lambda c: np.arange(c - H, c + H) % N
    planes = [W.tgv_slab(prm, int(z), int(z) + 1)[:, 0] for z in idx(zc)]
    Q = np.stack(planes, axis=1)
    return np.ascontiguousarray(Q[:, :, idx(yc)][:, :, :, idx(xc)])


@pytest.mark.parametrize("storage,N,bound", [(W.STORAGE_FP32, 535, 1e-5), (W.STORAGE_FP16, 674, 2e-3)])
def test_largest_lattice_probes_match_oracle(storage, N, bound):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13437_amd as cnsf
    prm = W.tgv_params(N, storage=storage)
    region = 7 * ((N ** 3 + 1023) // 1024 * 1024) * (4 if storage == W.STORAGE_FP32 else 2)
    assert region < 2 ** 32 - 256
    H = HALF + STEPS
    probes = [(N - 1, N - 1, N - 1), (N - 5, 3, N - 2), (0, N - 1, 0), (N // 2, N // 3, N // 5)]
    log(f"case tgv{N} storage {storage} steps {STEPS} region {region} B probes {probes}")
    L = cnsf.Lattice(prm)
    bg = np.array(W.uniform_state(1.0, (0.0, 0.0, 0.0), prm["T_ref"], prm["gamma"]))
    slab = np.broadcast_to(bg[:, None, None, None], (14, 16, N, N)).copy()
    for z0 in range(0, N, 16):
        L.set_state(slab[:, :min(16, N - z0)], z0=z0)
    near = sorted({int(z) % N for (zc, _, _) in probes for z in range(zc - H, zc + H)})
    for z in near:
        L.set_state(W.tgv_slab(prm, z, z + 1), z0=z)
    L.step(STEPS)
    got, ref = [], []
    for (zc, yc, xc) in probes:
        zs, ys, xs = (np.arange(c - HALF, c + HALF) % N for c in (zc, yc, xc))
        Qg = np.concatenate([L.moments(int(z), 1) for z in zs], axis=1)[:, :, ys][:, :, :, xs]
        oprm = dict(prm, nx=2 * H, ny=2 * H, nz=2 * H)
        Qo = lbm.moments(lbm.run(crop_initial(prm, N, zc, yc, xc, H), oprm, STEPS))
        Qo = Qo[:, STEPS:STEPS + 2 * HALF, STEPS:STEPS + 2 * HALF, STEPS:STEPS + 2 * HALF]
        rg, ug, _, _, Tg = lbm.primitives(Qg, prm)
        ro, uo, _, _, To = lbm.primitives(Qo, prm)
        got.append(dict(rho=rg, u=ug, T=Tg))
        ref.append(dict(rho=ro, u=uo, T=To))
        e = {k: float(np.linalg.norm(got[-1][k] - ref[-1][k]) / np.linalg.norm(ref[-1][k])) for k in ref[-1]}
        log(f"  probe {(zc, yc, xc)}: rel L2 {e}")
    pooled = {k: float(np.linalg.norm(np.concatenate([g[k].ravel() for g in got]) -
                                      np.concatenate([r[k].ravel() for r in ref])) /
                       np.linalg.norm(np.concatenate([r[k].ravel() for r in ref]))) for k in ref[0]}
    log(f"  pooled {pooled}")
    assert all(v < bound for v in pooled.values()), pooled
    d = L.diagnostics(spectral=False)
    assert d["nonfinite"] == 0
    L.close()
