"""Full Taylor-Green run: Eq. (7) histories of the HIP path against the FP64 oracle.

The golden history (tests/golden/tgv64_fmu3.6_history.json) is written by
tests/golden/make_tgv_history.py, which runs only the oracle.  The GPU runs the
same seeded case to t_c = 20 with FP64 diagnostics every 10 steps; the
relative L2 error over the sampled history must stay within 1% for FP32
populations and 2% for FP16 deviations.
"""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tgv64_fmu3.6_history.json")


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("storage,bound", [(W.STORAGE_FP32, 0.01), (W.STORAGE_FP16, 0.02), (W.STORAGE_BF16, 0.02)])
def test_tgv64_history_matches_oracle(storage, bound):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13437_amd as cnsf
    ref = json.load(open(GOLDEN))
    c = ref["case"]
    case = W.tgv(c["n"], f_mu=c["f_mu"], storage=storage)
    assert abs(case.params["dt"] - c["dt"]) < 1e-15
    L = cnsf.Lattice(case.params)
    L.set_state(case.Q0)
    every = ref["every"]
    hist = {k: [] for k in ("E_k", "eps_s", "eps_d")}
    nsamp = len(ref["history"]["step"])
    for j in range(nsamp):
        if j:
            L.step(every)
        d = L.diagnostics(spectral=True)
        for k in hist:
            hist[k].append(d[k])
    assert d["nonfinite"] == 0
    err = {k: rel_l2(hist[k], ref["history"][k]) for k in hist}
    print(f"storage {storage}: history rel L2 {err}", flush=True)
    sys.stdout.flush()
    assert err["E_k"] < bound and err["eps_d"] < bound and err["eps_s"] < bound, err
