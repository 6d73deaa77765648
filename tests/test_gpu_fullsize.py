"""Full-size parity: the 512^3 Taylor-Green update, 100 steps, in the benchmark's launch shape.

The expected values come from tests/golden/make_tgv512_probes.py, which runs
only the FP64 oracle: after n steps a cell depends only on the initial cube of
half-width n around it (D3Q7 streams one face neighbour per step; collision
and sensor are cell-local), so the oracle computes each probe cube exactly
from a cropped initial field.  Bounds: relative L2 on rho, u and T of 1e-5 for
FP32 populations and 2e-3 for 16-bit deviations, FP16 or BF16.  BF16 keeps 8
significant bits against FP16's 11, its errors are about 8x FP16's, and it
misses the bound: that case is a strict expected failure with the errors
measured on MI355X.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import lbm

pytestmark = pytest.mark.gpu
N = 512
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tgv512_probes_100steps.npz")


def fields(Q, prm):
    rho, u, _, _, T = lbm.primitives(Q, prm)
    return {"rho": rho, "u": u, "T": T}


def rel_l2(got, ref):
    return {k: float(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k])) for k in ref}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# tau and q stored x 256 (scale 2^-8): their deviations, 3.5e-4 and 6e-7 rms here, would
# otherwise sit in or near FP16's subnormal range
SCALED = [1.0] * 5 + [2.0 ** -8] * 9


@pytest.mark.parametrize("storage,bound,scale", [
    (W.STORAGE_FP32, 1e-5, None), (W.STORAGE_FP16, 2e-3, None), (W.STORAGE_FP16, 2e-3, SCALED),
    pytest.param(W.STORAGE_BF16, 2e-3, None, marks=pytest.mark.xfail(
        strict=True, reason="BF16 misses the 2e-3 bound (measured on MI355X: rho 2.2e-3, u 5.5e-3, T 1.9e-3)"))],
    ids=["fp32", "fp16", "fp16_scaled", "bf16"])
def test_tgv512_probes_match_oracle(storage, bound, scale):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13437_amd as cnsf
    gold = np.load(GOLDEN)
    steps, half = int(gold["steps"]), int(gold["half"])
    prm = W.tgv_params(N, storage=storage)
    if scale is not None:
        prm["storage_scale"] = scale
    assert prm["dt"] == float(gold["dt"])
    log(f"case tgv512 storage {storage} scale {scale} steps {steps} probes {len(gold['centres'])}")
    L = cnsf.Lattice(prm)
    log(f"  launch {L.get_launch()}")
    for z0 in range(0, N, 64):
        L.set_state(W.tgv_slab(prm, z0, z0 + 64), z0=z0)
    L.step(steps)
    got, ref, qpairs, qpairs_ref = [], [], [], []
    for (zc, yc, xc), Qo in zip(gold["centres"], gold["Q"]):
        zs, ys, xs = (np.arange(c - half, c + half) % N for c in (zc, yc, xc))
        Qg = np.concatenate([L.moments(int(z), 1) for z in zs], axis=1)
        Qg = Qg[:, :, ys][:, :, :, xs]
        got.append(fields(Qg, prm))
        ref.append(fields(Qo, prm))
        qpairs.append({"Q": Qg})
        qpairs_ref.append({"Q": Qo})
        log(f"  probe {(int(zc), int(yc), int(xc))}: rel L2 {rel_l2(got[-1], ref[-1])}")
    # The bound is a relative L2 norm over the field; over sampled cells its
    # estimate pools the samples.  (A single cube near a stagnation point of
    # the vortex has |u| ~ 0.04 and would inflate a per-cube ratio.)
    pooled = rel_l2({k: np.concatenate([g[k].ravel() for g in got]) for k in got[0]},
                    {k: np.concatenate([r[k].ravel() for r in ref]) for k in ref[0]})
    log(f"  pooled over {len(got)} probes: {pooled}")
    # the transported stress and heat flux, per field (reported; the bound is on rho, u, T)
    Qg_all = np.concatenate([g_["Q"].reshape(14, -1) for g_ in qpairs], axis=1)
    Qo_all = np.concatenate([o_["Q"].reshape(14, -1) for o_ in qpairs_ref], axis=1)
    extra = {"tau": float(np.linalg.norm(Qg_all[5:11] - Qo_all[5:11]) / np.linalg.norm(Qo_all[5:11])),
             "q": float(np.linalg.norm(Qg_all[11:14] - Qo_all[11:14]) / np.linalg.norm(Qo_all[11:14])),
             "E": float(np.linalg.norm(Qg_all[4] - Qo_all[4]) / np.linalg.norm(Qo_all[4]))}
    log(f"  pooled over {len(got)} probes, conserved E and transported fields: {extra}")
    assert all(v < bound for v in pooled.values()), pooled
    # and no single cube may hide a local error: each cube's RMS error over
    # the RMS of the field over all cubes
    scale = {k: np.sqrt(np.mean(np.concatenate([r[k].ravel() for r in ref]) ** 2)) for k in ref[0]}
    for (c, g, r) in zip(gold["centres"], got, ref):
        e = {k: float(np.sqrt(np.mean((g[k] - r[k]) ** 2)) / scale[k]) for k in r}
        assert all(v < bound for v in e.values()), (tuple(int(x) for x in c), e)
    d = L.diagnostics(spectral=False)
    assert d["nonfinite"] == 0
    L.close()


WALL_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tgv512_wall_probes_100steps.npz")


@pytest.mark.parametrize("storage,bound", [(W.STORAGE_FP32, 1e-5), (W.STORAGE_FP16, 2e-3)])
def test_tgv512_wall_probes_match_oracle(storage, bound):
    """The 512^3 Taylor-Green state between no-slip x-walls (the benchmark's walled
    configuration), 100 steps, at probe cubes touching each wall; expected values
    from tests/golden/make_tgv512_wall_probes.py (oracle only)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13437_amd as cnsf
    gold = np.load(WALL_GOLDEN)
    steps, half = int(gold["steps"]), int(gold["half"])
    prm = W.tgv_wall_params(N, storage=storage)
    assert prm["dt"] == float(gold["dt"])
    log(f"case tgv512 no-slip walls storage {storage} steps {steps} probes {gold['probes'].tolist()}")
    L = cnsf.Lattice(prm)
    for z0 in range(0, N, 64):
        L.set_state(W.tgv_slab(prm, z0, z0 + 64), z0=z0)
    L.step(steps)
    got, ref, qpairs, qpairs_ref = [], [], [], []
    for (zc, yc, wall), Qo in zip(gold["probes"], gold["Q"]):
        zs, ys = (np.arange(c - half, c + half) % N for c in (zc, yc))
        xs = np.arange(2 * half) if wall == 0 else np.arange(N - 2 * half, N)
        Qg = np.concatenate([L.moments(int(z), 1) for z in zs], axis=1)[:, :, ys][:, :, :, xs]
        got.append(fields(Qg, prm))
        ref.append(fields(Qo, prm))
        qpairs.append({"Q": Qg})
        qpairs_ref.append({"Q": Qo})
        log(f"  probe {(int(zc), int(yc), int(wall))}: rel L2 {rel_l2(got[-1], ref[-1])}")
    pooled = rel_l2({k: np.concatenate([g[k].ravel() for g in got]) for k in got[0]},
                    {k: np.concatenate([r[k].ravel() for r in ref]) for k in ref[0]})
    log(f"  pooled over {len(got)} probes: {pooled}")
    # the transported stress and heat flux, per field (reported; the bound is on rho, u, T)
    Qg_all = np.concatenate([g_["Q"].reshape(14, -1) for g_ in qpairs], axis=1)
    Qo_all = np.concatenate([o_["Q"].reshape(14, -1) for o_ in qpairs_ref], axis=1)
    extra = {"tau": float(np.linalg.norm(Qg_all[5:11] - Qo_all[5:11]) / np.linalg.norm(Qo_all[5:11])),
             "q": float(np.linalg.norm(Qg_all[11:14] - Qo_all[11:14]) / np.linalg.norm(Qo_all[11:14])),
             "E": float(np.linalg.norm(Qg_all[4] - Qo_all[4]) / np.linalg.norm(Qo_all[4]))}
    log(f"  pooled over {len(got)} probes, conserved E and transported fields: {extra}")
    assert all(v < bound for v in pooled.values()), pooled
    assert L.diagnostics(spectral=False)["nonfinite"] == 0
    L.close()


def test_tgv512_fused_readout_at_start_matches_closed_forms():
    """The fused step-and-readout at 512^3 in the benchmark's launch shape reports
    the start level: E_k = 1/8, eps_s = (3/4) mu0 and eps_d = 0 (the Taylor-Green
    start is divergence-free at uniform T), and it equals the separate readout of
    the same level."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13437_amd as cnsf
    prm = W.tgv_params(N, storage=W.STORAGE_FP32)
    log("case tgv512 fused readout at t = 0")
    L = cnsf.Lattice(prm)
    for z0 in range(0, N, 64):
        L.set_state(W.tgv_slab(prm, z0, z0 + 64), z0=z0)
    d = L.diagnostics(spectral=True)
    e = L.step_diagnostics(1, spectral=True)
    log(f"  readout {d}\n  fused   {e}")
    assert L.info()[0] == 1 and e["step"] == 0
    assert abs(e["E_k"] - 0.125) < 1e-7
    assert abs(e["eps_s"] - 0.75 * prm["mu0"]) < 1e-8
    assert abs(e["eps_d"]) < 1e-12
    for k in ("mass", "energy", "E_k", "eps_s"):
        assert abs(e[k] - d[k]) <= 1e-12 * abs(d[k]), k
    for k in ("min_rho", "min_p", "sensor_fraction", "nonfinite"):
        assert e[k] == d[k], k
    L.close()


def test_tgv512_spectrum_start_and_parseval():
    """The 512^3 shell spectrum (512-point lines take the register transform): the
    Taylor-Green start holds 1/8 in shell 2 (|kappa| = sqrt 3) and nothing
    elsewhere (FP32 storage bounds |E[2] - 1/8| by 3e-8); for a seeded
    white-noise velocity field, which fills every shell, the shells are
    non-negative and sum to <|u|^2>/2 of the stored state (Parseval)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13437_amd as cnsf
    prm = W.tgv_params(N, storage=W.STORAGE_FP32)
    log("case tgv512 spectrum at t = 0")
    L = cnsf.Lattice(prm)
    for z0 in range(0, N, 64):
        L.set_state(W.tgv_slab(prm, z0, z0 + 64), z0=z0)
    E = L.spectrum()
    rest = float(np.sum(np.abs(E)) - abs(E[2]))
    log(f"  E[2] = {E[2]!r}, rest {rest:.2e}")
    assert abs(E[2] - 0.125) < 3e-8 and rest < 1e-12
    log("case white noise 512^3 spectrum (seed 13437)")
    gen = torch.Generator(device="cuda").manual_seed(13437)
    P = torch.zeros((14, N, N, N), dtype=torch.float64, device="cuda")
    for k, (c, a) in enumerate(((1.0, 0.1), (0.0, 0.2), (0.0, 0.2), (0.0, 0.2), (1.0, 0.1))):
        P[k] = c + a * (2.0 * torch.rand((N, N, N), generator=gen, dtype=torch.float64, device="cuda") - 1.0)
    L.set_primitive(P)
    del P
    Q = L.moments(device=True)
    u2 = (Q[1] * Q[1] + Q[2] * Q[2] + Q[3] * Q[3]) / (Q[0] * Q[0])
    target = 0.5 * float(u2.mean())
    del Q, u2
    torch.cuda.empty_cache()
    E = L.spectrum()
    log(f"  sum E {E.sum()!r} vs <|u|^2>/2 {target!r}; min shell {E.min():.3e}")
    assert abs(E.sum() - target) < 1e-10 * target and E.min() >= 0.0
    assert np.count_nonzero(E[1:] > 0) == len(E) - 1
    L.close()
