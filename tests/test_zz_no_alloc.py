"""The no-allocation entry point cnsf_step_diagnostics_static against
cnsf_step_diagnostics (sums only), through the C ABI.

Two calls in a row on the static workspace, the second on a smaller lattice
than the first, so the second reads fewer block partials than the first left
behind.  The first lattice has more update tiles than the workspace holds
partials, so its diagnostic update runs as a persistent grid.  Populations
must be bitwise those of the existing entry point, the FP64 sums equal to
1e-12 relative (their rounding order depends on the block count), minima and
counts exactly.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

SUM_KEYS = ("mass", "energy", "E_k")


def _cnsf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13437_amd as cnsf
    cnsf.library()
    return cnsf


def _pair(cnsf, case, storage):
    prm = dict(case.params, storage=storage)
    a, b = cnsf.Lattice(prm), cnsf.Lattice(prm)
    for L in (a, b):
        L.set_state(case.Q0)
    return a, b


def _check(cnsf, a, b, n):
    da = cnsf._diag_dict(cnsf.cnsf_step_diagnostics(a.h, n, cnsf.CNSF_DIAG_SUMS))
    db = cnsf._diag_dict(cnsf.cnsf_step_diagnostics_static(b.h, n))
    print(f"  existing {da}\n  static   {db}", flush=True)
    assert db["step"] == da["step"] and a.info()[:2] == b.info()[:2]
    for k in SUM_KEYS:
        assert abs(db[k] - da[k]) <= 1e-12 * abs(da[k]), k
    for j in range(3):
        assert abs(db["momentum"][j] - da["momentum"][j]) <= 1e-12 * abs(da["mass"])
    for k in ("min_rho", "min_p", "sensor_fraction", "nonfinite"):
        assert db[k] == da[k], k
    assert db["eps_s"] == 0.0 and db["eps_d"] == 0.0
    assert np.array_equal(a.export_populations()[0], b.export_populations()[0])


@pytest.mark.parametrize("storage", [W.STORAGE_FP32, W.STORAGE_FP16])
def test_static_step_diagnostics_matches_existing_entry_point(storage):
    cnsf = _cnsf()
    big = W.tgv(160)                          # 160^3 / 256-cell tiles: 16,000 > 8,192 blocks
    small = W.smooth_random_case(24, 20, 16, seed=5, sensor=True)
    print(f"case tgv160 storage {storage}: static workspace, persistent first update", flush=True)
    a, b = _pair(cnsf, big, storage)
    _check(cnsf, a, b, 3)
    _check(cnsf, a, b, 2)                     # again, now from an odd time level
    for L in (a, b):
        L.close()
    print(f"case smooth24x20x16 storage {storage}: fewer partials than the previous call left", flush=True)
    a, b = _pair(cnsf, small, storage)
    _check(cnsf, a, b, 5)
    a.close()
    b.close()


def test_static_step_diagnostics_rejects_large_persistent_grid_and_bad_n():
    cnsf = _cnsf()
    case = W.tgv(16)
    L = cnsf.Lattice(case.params)
    L.set_state(case.Q0)
    L.set_launch(256, 256, 2 * 8192, True)
    with pytest.raises(cnsf.CnsfError) as e:
        cnsf.cnsf_step_diagnostics_static(L.h, 1)
    assert e.value.status == cnsf.CNSF_E_SIZE
    L.set_launch(256, 256, 0, True)
    with pytest.raises(cnsf.CnsfError) as e:
        cnsf.cnsf_step_diagnostics_static(L.h, 0)
    assert e.value.status == cnsf.CNSF_E_INVALID
    assert L.info()[0] == 0                   # nothing ran
    L.close()
