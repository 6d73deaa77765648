"""The C-ABI library loads, exports every declared entry point, agrees with the
binding's struct layout and validates parameters, all without a GPU."""
import ctypes
import os
import re
import subprocess
import textwrap

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cnsf.h")


@pytest.fixture(scope="module")
def cnsf():
    import paper_2608_13437_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_2608_13437_amd import build
        build.build()
    m.library()
    return m


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(cnsf_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol(cnsf):
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(cnsf.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layout_matches_header(cnsf, tmp_path):
    fields = [f for f, _ in cnsf.cnsf_params._fields_]
    src = tmp_path / "layout.c"
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "cnsf.h"', "int main(void) {",
             '  printf("%zu\\n", sizeof(cnsf_params));',
             '  printf("%zu\\n", sizeof(cnsf_diag));']
    lines += [f'  printf("%zu\\n", offsetof(cnsf_params, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert out[0] == ctypes.sizeof(cnsf.cnsf_params)
    assert out[1] == ctypes.sizeof(cnsf.cnsf_diag)
    for f, off in zip(fields, out[2:]):
        assert getattr(cnsf.cnsf_params, f).offset == off, f


def test_params_default_and_bytes(cnsf):
    p = cnsf.cnsf_params_default()
    assert p.size == ctypes.sizeof(cnsf.cnsf_params)
    # 14 component regions of 7 slots of the cell count rounded up to groups
    # of 1024 cells
    q = cnsf.make_params(W.tgv_params(512))
    assert cnsf.cnsf_required_bytes(q) == 98 * 512 ** 3 * 4
    q.storage = W.STORAGE_FP16
    assert cnsf.cnsf_required_bytes(q) == 98 * 512 ** 3 * 2
    q = cnsf.make_params(W.random_params(13, 11, 9))
    assert cnsf.cnsf_required_bytes(q) == 14 * 7 * 2048 * 4


def test_batch_layout_bytes(cnsf):
    """Component-major batches take 14 runs of the members' slot counts (each
    member's run rounded to 256 bytes); batches whose runs would pass the
    32-bit region offsets store the members one after another instead."""
    def prm(n, storage):
        q = W.tgv_params(n, storage=storage)
        return cnsf.make_params(q)

    slots = lambda n: 7 * -(-n ** 3 // 1024) * 1024
    for storage, eb in ((W.STORAGE_FP32, 4), (W.STORAGE_FP16, 2)):
        ms = [prm(n, storage) for n in (32, 48, 13)]
        run = sum(-(-slots(n) * eb // 256) * 256 for n in (32, 48, 13))
        assert cnsf.cnsf_batch_required_bytes(ms) == 14 * run
    # three 512^3 FP32 members: 3 x 3.76 GB per component, past 4 GiB
    big = [prm(512, W.STORAGE_FP32)] * 3
    assert cnsf.cnsf_batch_required_bytes(big) == 3 * 98 * 512 ** 3 * 4


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("dt", 0.0), ("dx", -1.0), ("gamma", 1.0), ("tau_R", 0.0), ("tau_q", -1.0),
    ("omega_min", 0.0), ("omega_min", 2.5), ("tau_base_override", 0.4), ("f_mu", -1.0),
    ("visc_law", 7), ("bc_x", 4), ("bc_x", -1), ("storage", 3), ("C_sigma", -1.0), ("prandtl", 0.0),
])
def test_invalid_parameters_rejected(cnsf, field, value):
    prm = W.tgv_params(16)
    prm[field] = value
    with pytest.raises(cnsf.CnsfError) as e:
        cnsf.cnsf_required_bytes(cnsf.make_params(prm))
    assert e.value.status == cnsf.CNSF_E_INVALID


def test_subcharacteristic_bound_and_reference_state(cnsf):
    prm = W.tgv_params(16)
    prm["a_ref"] = 0.51 * prm["dx"] / prm["dt"]
    with pytest.raises(cnsf.CnsfError):
        cnsf.cnsf_required_bytes(cnsf.make_params(prm))
    prm = W.tgv_params(16)
    prm["Q_ref"] = list(prm["Q_ref"])
    prm["Q_ref"][1] = 0.3   # a moving reference state is not supported
    with pytest.raises(cnsf.CnsfError):
        cnsf.cnsf_required_bytes(cnsf.make_params(prm))
    prm = W.tgv_params(16)
    prm["C_sigma"], prm["mu0"] = 10.0, 0.0
    with pytest.raises(cnsf.CnsfError):
        cnsf.cnsf_required_bytes(cnsf.make_params(prm))


@pytest.mark.parametrize("wall_u,wall_T", [
    ([[0.1, 0.0, 0.0], [0.0, 0.0, 0.0]], [1.0, 1.0]),      # normal wall velocity
    ([[0.0, 0.0, 0.0], [0.0, 0.0, -0.2]], [1.0, -1.0]),    # negative temperature
    ([[0.0, float("nan"), 0.0], [0.0] * 3], [0.0, 0.0]),  # non-finite velocity
    ([[0.0] * 3, [0.0] * 3], [float("inf"), 0.0]),         # non-finite temperature
])
def test_invalid_noslip_walls_rejected(cnsf, wall_u, wall_T):
    prm = W.noslip_case(8, 4, 4).params
    prm.update(wall_u=wall_u, wall_T=wall_T)
    with pytest.raises(cnsf.CnsfError) as e:
        cnsf.cnsf_required_bytes(cnsf.make_params(prm))
    assert e.value.status == cnsf.CNSF_E_INVALID


def test_noslip_wall_fields_reach_the_struct(cnsf):
    prm = W.noslip_case(8, 4, 4).params
    p = cnsf.make_params(prm)
    assert p.bc_x == cnsf.CNSF_BC_NOSLIP == W.BC_NOSLIP
    assert [list(p.wall_u[s]) for s in range(2)] == prm["wall_u"] and list(p.wall_T) == prm["wall_T"]
    assert cnsf.cnsf_required_bytes(p) > 0


def test_lattice_too_large_for_32bit_offsets(cnsf):
    prm = W.default_params(1024, 1024, 1024)
    with pytest.raises(cnsf.CnsfError):
        cnsf.cnsf_required_bytes(cnsf.make_params(prm))


@pytest.mark.parametrize("storage,elem,cube,last", [(W.STORAGE_FP32, 4, 535, 153_391_104),
                                                     (W.STORAGE_FP16, 2, 674, 306_783_232),
                                                     (W.STORAGE_BF16, 2, 674, 306_783_232)])
def test_largest_accepted_lattice(cnsf, storage, elem, cube, last):
    """A component's 7 slots (cells rounded up to groups of 1024) stay below
    2^32 - 256 bytes: the documented limits are exact."""
    assert 7 * last * elem < 2 ** 32 - 256 <= 7 * (last + 1024) * elem and last % 1024 == 0

    def bytes_for(nx, ny, nz):
        prm = dict(W.default_params(nx, ny, nz), storage=storage)
        return cnsf.cnsf_required_bytes(cnsf.make_params(prm))

    assert bytes_for(last, 1, 1) == 98 * last * elem
    with pytest.raises(cnsf.CnsfError) as e:
        bytes_for(last + 1, 1, 1)
    assert e.value.status == cnsf.CNSF_E_INVALID
    assert bytes_for(cube, cube, cube) == 14 * 7 * ((cube ** 3 + 1023) // 1024 * 1024) * elem
    with pytest.raises(cnsf.CnsfError):
        bytes_for(cube + 1, cube + 1, cube + 1)


def test_status_strings(cnsf):
    assert cnsf.cnsf_status_string(0) == "ok"
    assert "HIP" in cnsf.cnsf_status_string(3)
