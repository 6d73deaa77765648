"""Full Taylor-Green runs: Eq. (7) histories of the GPU run driver against the FP64 oracle.

The golden histories are written by tests/golden/make_tgv_history.py, which
runs only the oracle:
* tgv64_fmu3.6_history.json: the supersonic case (M0 1.25, Re 1600) at 64^3
  to t_c = 20 (f_mu 3.6; the paper's 1.8 blows up in the oracle itself);
* tgv32_fmu0_M0.5_Re500_history.json: the subsonic verification case of
  Section 3.2 (M0 0.5, Re 500, f_mu 0) at 32^3 to t_c = 10.
paper_2608_13437_amd.runs repeats each case on the GPU, with the diagnostics
every 10 steps; the relative L2 error over the sampled history must stay
within 1% for FP32 populations and 2% for FP16 deviations.  BF16 keeps 8
significant bits against FP16's 11, so its rounding error is 2^3 times larger
and it is held to 8 x 2%: the supersonic histories meet 2% in BF16 too, but
the subsonic eps_d, a quantity three orders below eps_s in this nearly
incompressible flow, carries a 9.6% BF16 error.
"""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CASES = ["tgv64_fmu3.6_history.json", "tgv32_fmu0_M0.5_Re500_history.json"]


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("golden", CASES)
@pytest.mark.parametrize("storage,bound", [(W.STORAGE_FP32, 0.01), (W.STORAGE_FP16, 0.02), (W.STORAGE_BF16, 0.16)])
def test_tgv_history_matches_oracle(golden, storage, bound):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_13437_amd import runs
    ref = json.load(open(os.path.join(GOLDEN, golden)))
    c = ref["case"]
    run = runs.tgv_run(c["n"], steps=ref["steps"], every=ref["every"], storage=storage,
                       M0=c["M0"], Re=c["Re"], f_mu=c["f_mu"])
    assert abs(run["case"]["dt"] - c["dt"]) < 1e-15
    assert run["status"] == "ok" and run["history"]["step"] == ref["history"]["step"]
    err = {k: rel_l2(run["history"][k], ref["history"][k]) for k in ("E_k", "eps_s", "eps_d")}
    print(f"{golden} storage {storage}: history rel L2 {err}", flush=True)
    sys.stdout.flush()
    assert all(v < bound for v in err.values()), err


@pytest.mark.parametrize("storage,bound", [(W.STORAGE_FP32, 1e-5), (W.STORAGE_FP16, 2e-3)])
def test_couette_run_matches_oracle_steady_state(storage, bound):
    """The run driver's Couette flow between no-slip walls (one moving, both
    isothermal) against the oracle's state at the same time (written by
    tests/golden/make_couette_steady.py): relative L2 of u_y and T within the
    parity bound.  For FP32 populations the viscous temperature rise T - T_w
    (about 6e-3, three orders below T) is also held to 100x the bound; FP16
    deviations do not resolve it over 21,061 steps (23% off)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_13437_amd import runs
    gold = json.load(open(os.path.join(GOLDEN, "couette16_steady.json")))
    print(f"case couette{gold['n']} storage {storage} steps {gold['steps']}", flush=True)
    r = runs.couette_run(gold["n"], U=gold["U"], mu=gold["mu"], f_mu=gold["f_mu"], t_end=gold["t_end"],
                         storage=storage)
    assert r["steps"] == gold["steps"]
    e = dict(u_y=rel_l2(r["u"], gold["u_y"]), T=rel_l2(r["T"], gold["T"]),
             rise=rel_l2(np.asarray(r["T"]) - 1.0, np.asarray(gold["T"]) - 1.0))
    print(f"  rel L2 {e}; against the closed form: u {r['err_u']:.2e}, T {r['err_T']:.2e}", flush=True)
    assert e["u_y"] < bound and e["T"] < bound, e
    if storage == W.STORAGE_FP32:
        assert e["rise"] < 100 * bound, e
