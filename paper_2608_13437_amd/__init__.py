"""Python binding of the cnsf HIP library (D3Q7 compressible NSF lattice Boltzmann).

Argument marshalling only: every step of the method runs in the HIP kernels of
``libcnsf.so``.  PyTorch supplies device memory (the population array is a
torch uint8 tensor) and the HIP stream (torch's current stream), nothing else.

The module-level functions carry the names of the C ABI (``cnsf_create``,
``cnsf_step``, ...); :class:`Lattice` and :class:`Batch` wrap them for use
with NumPy arrays and torch tensors.  Importing this package never falls back
to another implementation: if the library is missing the first call raises.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcnsf.so")

NCOMP, NVEL, NPOP = 14, 7, 98
CNSF_OK, CNSF_E_INVALID, CNSF_E_NOMEM, CNSF_E_DEVICE, CNSF_E_STATE, CNSF_E_SIZE = range(6)
CNSF_HOST, CNSF_DEVICE = 0, 1
CNSF_BC_PERIODIC, CNSF_BC_WALL, CNSF_BC_DIRICHLET, CNSF_BC_NOSLIP = 0, 1, 2, 3
CNSF_DIAG_SUMS, CNSF_DIAG_SPECTRAL = 0, 1

D14 = C.c_double * NCOMP


class cnsf_params(C.Structure):
    _fields_ = [
        ("size", C.c_uint32),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("dx", C.c_double), ("dt", C.c_double),
        ("gamma", C.c_double), ("mu0", C.c_double), ("T_ref", C.c_double),
        ("visc_law", C.c_int32), ("visc_param", C.c_double),
        ("prandtl", C.c_double),
        ("tau_R", C.c_double), ("tau_q", C.c_double),
        ("f_mu", C.c_double), ("tau_base_override", C.c_double),
        ("C_sigma", C.c_double), ("J_min", C.c_double), ("omega_min", C.c_double),
        ("bc_x", C.c_int32),
        ("Q_left", D14), ("Q_right", D14),
        ("storage", C.c_int32),
        ("Q_ref", D14),
        ("storage_scale", D14),
        ("a_ref", C.c_double),
        ("wall_u", (C.c_double * 3) * 2),
        ("wall_T", C.c_double * 2),
    ]


class cnsf_diag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("time", C.c_double),
        ("mass", C.c_double), ("momentum", C.c_double * 3), ("energy", C.c_double),
        ("E_k", C.c_double), ("eps_s", C.c_double), ("eps_d", C.c_double),
        ("min_rho", C.c_double), ("min_p", C.c_double),
        ("sensor_fraction", C.c_double), ("nonfinite", C.c_int64),
    ]


class CnsfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"cnsf status {status}: {message}")
        self.status = status


_lib = None


def library():
    """Load libcnsf.so (in-tree build); raise if it is missing.

    torch is imported first: its wheel carries its own HIP runtime under the
    same soname as the system one, and loading the library first would put
    the system runtime in the process beside torch's (two runtimes, one of
    which then finds no device).  Loaded after torch, the library binds to
    torch's runtime, so torch's memory and streams are the library's."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2608_13437_amd.build`")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = C.CDLL(LIB_PATH)
        vp, i32, i64, sz, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.POINTER(C.c_double)
        pp = C.POINTER(cnsf_params)
        sig = {
            "cnsf_params_default": [pp],
            "cnsf_required_bytes": [pp, C.POINTER(sz)],
            "cnsf_create": [pp, vp, sz, vp, C.POINTER(vp)],
            "cnsf_destroy": [vp],
            "cnsf_set_state": [vp, dp, i32, i32, i32],
            "cnsf_step": [vp, i64],
            "cnsf_get_moments": [vp, dp, i32, i32, i32],
            "cnsf_set_primitive": [vp, dp, i32, i32, i32],
            "cnsf_get_primitives": [vp, dp, i32, i32, i32],
            "cnsf_diagnostics": [vp, i32, C.POINTER(cnsf_diag)],
            "cnsf_step_diagnostics": [vp, i64, i32, C.POINTER(cnsf_diag)],
            "cnsf_step_diagnostics_static": [vp, i64, C.POINTER(cnsf_diag)],
            "cnsf_probe_update_ms": [vp, i32, C.POINTER(C.c_double)],
            "cnsf_spectrum_shells": [vp, C.POINTER(i32)],
            "cnsf_spectrum": [vp, dp, i32, i32],
            "cnsf_get_info": [vp, C.POINTER(i64), C.POINTER(i32), C.POINTER(sz)],
            "cnsf_export_populations": [vp, vp, sz, C.POINTER(i64), C.POINTER(i32)],
            "cnsf_import_populations": [vp, vp, sz, i64, i32],
            "cnsf_hbm_copy": [vp, vp, sz, vp],
            "cnsf_set_launch": [vp, i32, i32, i32, i32],
            "cnsf_get_launch": [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
            "cnsf_batch_required_bytes": [pp, i32, C.POINTER(sz)],
            "cnsf_batch_create": [pp, i32, vp, sz, vp, C.POINTER(vp)],
            "cnsf_batch_destroy": [vp],
            "cnsf_batch_set_state": [vp, i32, dp, i32],
            "cnsf_batch_step": [vp, i64, i32],
            "cnsf_batch_get_moments": [vp, i32, dp, i32],
            "cnsf_batch_set_launch": [vp, i32, i32, i32, i32],
            "cnsf_batch_get_launch": [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
            "cnsf_batch_autotune": [vp, C.c_char_p, i32],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = C.c_int
        lib.cnsf_last_error.restype = C.c_char_p
        lib.cnsf_status_string.restype = C.c_char_p
        lib.cnsf_status_string.argtypes = [C.c_int]
        _lib = lib
    return _lib


def _check(status):
    if status != CNSF_OK:
        raise CnsfError(status, library().cnsf_last_error().decode())
    return status


# ---------------------------------------------------------------- C ABI names
def cnsf_params_default() -> cnsf_params:
    p = cnsf_params()
    _check(library().cnsf_params_default(C.byref(p)))
    return p


def cnsf_required_bytes(p: cnsf_params) -> int:
    n = C.c_size_t()
    _check(library().cnsf_required_bytes(C.byref(p), C.byref(n)))
    return n.value


def cnsf_create(p: cnsf_params, dev_buf: int, nbytes: int, stream: int) -> C.c_void_p:
    h = C.c_void_p()
    _check(library().cnsf_create(C.byref(p), C.c_void_p(dev_buf), nbytes, C.c_void_p(stream), C.byref(h)))
    return h


def cnsf_destroy(h):
    _check(library().cnsf_destroy(h))


def cnsf_set_state(h, Q_ptr: int, z0: int, nzs: int, where: int):
    _check(library().cnsf_set_state(h, C.cast(C.c_void_p(Q_ptr), C.POINTER(C.c_double)), z0, nzs, where))


def cnsf_step(h, n: int):
    _check(library().cnsf_step(h, n))


def cnsf_get_moments(h, out_ptr: int, z0: int, nzs: int, where: int):
    _check(library().cnsf_get_moments(h, C.cast(C.c_void_p(out_ptr), C.POINTER(C.c_double)), z0, nzs, where))


def cnsf_probe_update_ms(h, steps: int) -> float:
    ms = C.c_double()
    _check(library().cnsf_probe_update_ms(h, steps, C.byref(ms)))
    return ms.value


def _diag_dict(d: cnsf_diag) -> dict:
    return dict(step=d.step, time=d.time, mass=d.mass, momentum=list(d.momentum), energy=d.energy,
                E_k=d.E_k, eps_s=d.eps_s, eps_d=d.eps_d, min_rho=d.min_rho, min_p=d.min_p,
                sensor_fraction=d.sensor_fraction, nonfinite=d.nonfinite)


def cnsf_step_diagnostics(h, n: int, flags: int) -> cnsf_diag:
    d = cnsf_diag()
    _check(library().cnsf_step_diagnostics(h, n, flags, C.byref(d)))
    return d


def cnsf_step_diagnostics_static(h, n: int) -> cnsf_diag:
    d = cnsf_diag()
    _check(library().cnsf_step_diagnostics_static(h, n, C.byref(d)))
    return d


def cnsf_set_primitive(h, P_ptr: int, z0: int, nzs: int, where: int):
    _check(library().cnsf_set_primitive(h, C.cast(C.c_void_p(P_ptr), C.POINTER(C.c_double)), z0, nzs, where))


def cnsf_get_primitives(h, out_ptr: int, z0: int, nzs: int, where: int):
    _check(library().cnsf_get_primitives(h, C.cast(C.c_void_p(out_ptr), C.POINTER(C.c_double)), z0, nzs, where))


def cnsf_spectrum_shells(h) -> int:
    n = C.c_int32()
    _check(library().cnsf_spectrum_shells(h, C.byref(n)))
    return n.value


def cnsf_spectrum(h, E_ptr: int, nshells: int, where: int) -> None:
    _check(library().cnsf_spectrum(h, C.cast(C.c_void_p(E_ptr), C.POINTER(C.c_double)), nshells, where))


def cnsf_diagnostics(h, flags: int) -> cnsf_diag:
    d = cnsf_diag()
    _check(library().cnsf_diagnostics(h, flags, C.byref(d)))
    return d


def cnsf_get_info(h):
    s, par, nb = C.c_int64(), C.c_int32(), C.c_size_t()
    _check(library().cnsf_get_info(h, C.byref(s), C.byref(par), C.byref(nb)))
    return s.value, par.value, nb.value


def cnsf_export_populations(h, host_ptr: int, nbytes: int):
    s, par = C.c_int64(), C.c_int32()
    _check(library().cnsf_export_populations(h, C.c_void_p(host_ptr), nbytes, C.byref(s), C.byref(par)))
    return s.value, par.value


def cnsf_import_populations(h, host_ptr: int, nbytes: int, step: int, parity: int):
    _check(library().cnsf_import_populations(h, C.c_void_p(host_ptr), nbytes, step, parity))


def cnsf_hbm_copy(dst: int, src: int, nbytes: int, stream: int):
    _check(library().cnsf_hbm_copy(C.c_void_p(dst), C.c_void_p(src), nbytes, C.c_void_p(stream)))


def cnsf_set_launch(h, block: int, tile: int, grid: int, xcd_remap: int):
    _check(library().cnsf_set_launch(h, block, tile, grid, xcd_remap))


def cnsf_get_launch(h):
    v = [C.c_int32() for _ in range(4)]
    _check(library().cnsf_get_launch(h, *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)


def cnsf_status_string(s: int) -> str:
    return library().cnsf_status_string(s).decode()


# ---------------------------------------------------------------- helpers
def make_params(prm: dict) -> cnsf_params:
    """cnsf_params from a dict with the struct's field names (missing fields keep defaults)."""
    p = cnsf_params_default()
    for name, _ in cnsf_params._fields_:
        if name == "size" or name not in prm:
            continue
        v = prm[name]
        if name in ("Q_left", "Q_right", "Q_ref", "storage_scale"):
            arr = getattr(p, name)
            for k in range(NCOMP):
                arr[k] = float(v[k])
        elif name == "wall_u":
            for s in range(2):
                for a in range(3):
                    p.wall_u[s][a] = float(v[s][a])
        elif name == "wall_T":
            for s in range(2):
                p.wall_T[s] = float(v[s])
        elif name in ("nx", "ny", "nz", "visc_law", "bc_x", "storage"):
            setattr(p, name, int(v))
        else:
            setattr(p, name, float(v))
    return p


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Lattice:
    """One lattice on the current HIP device; populations in a torch-owned buffer."""

    def __init__(self, prm: dict, *, device="cuda", stream=None, buf=None):
        """buf: optional uint8 CUDA tensor of at least the required bytes to hold the
        populations (e.g. another lattice's, whose state this one then overwrites)."""
        torch = _torch()
        self.prm = dict(prm)
        self.p = make_params(prm)
        self.nbytes = cnsf_required_bytes(self.p)
        self.device = torch.device(device) if buf is None else buf.device
        if buf is not None:
            if buf.dtype != torch.uint8 or not buf.is_cuda or buf.numel() < self.nbytes or not buf.is_contiguous():
                raise ValueError(f"buf must be a contiguous uint8 CUDA tensor of >= {self.nbytes} bytes")
            self.buf = buf
        else:
            self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream
        self.h = cnsf_create(self.p, self.buf.data_ptr(), self.nbytes, _stream_handle(stream))
        self.shape = (self.p.nz, self.p.ny, self.p.nx)

    @classmethod
    def placed(cls, prm: dict, *, candidates: int | None = None, probe_steps: int = 4, device="cuda", stream=None):
        """A lattice whose population array is the fastest of `candidates` allocations
        (default: as many as fit in 85% of the free device memory, at most 8).

        The same update runs at one of two speeds (about 20% apart on large
        arrays) depending on the physical memory behind the array, and an
        allocation keeps its speed for its lifetime.  Each candidate array is
        created (cleared), timed over `probe_steps` updates of its cleared
        state after one untimed update, and kept alive until all are timed, so
        that each gets different memory; the fastest is kept and the others
        freed.  The returned lattice is freshly created on that array (cleared,
        step 0).  Candidates that no longer fit in memory are skipped.
        ``placement_ms`` holds each candidate's mean time per update and
        ``placement_kept`` the index kept."""
        torch = _torch()
        # each candidate its own exact-size device allocation, not a piece of a
        # larger block cached by torch: on MI355X the first half of 52.6 GB
        # buffers ran fast 0 of 20 times for a 26.3 GB array, exact-size
        # allocations 9 of 24
        torch.cuda.empty_cache()
        if candidates is None:
            free = torch.cuda.mem_get_info(torch.device(device))[0]
            candidates = min(8, int(0.85 * free) // max(1, cnsf_required_bytes(make_params(prm))))
        lats, ms = [], []
        for _ in range(max(1, int(candidates))):
            try:
                L = cls(prm, device=device, stream=stream)
            except torch.cuda.OutOfMemoryError:
                if not lats:
                    raise
                break
            ms.append(cnsf_probe_update_ms(L.h, probe_steps))
            lats.append(L)
        best = min(range(len(ms)), key=ms.__getitem__)
        buf = lats[best].buf
        for L in lats:
            L.close()
        del lats, L
        torch.cuda.empty_cache()      # return the slower arrays to the device
        out = cls(prm, device=device, stream=stream, buf=buf)
        out.placement_ms, out.placement_kept = ms, best
        return out

    def close(self):
        if getattr(self, "h", None):
            cnsf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ncells(self):
        return self.p.nx * self.p.ny * self.p.nz

    def _fields_arg(self, F):
        """(pointer, nzs, where, keep) of a (14, nzs, ny, nx) FP64 field: a NumPy array
        (host) or a CUDA tensor on this lattice's device (converted on the current
        stream, which the lattice's stream then waits for)."""
        torch = _torch()
        if isinstance(F, torch.Tensor):
            if not F.is_cuda or F.device != self.buf.device:
                raise ValueError(f"field tensor on {F.device}, lattice on {self.buf.device}")
            if F.dim() != 4 or F.shape[0] != NCOMP or tuple(F.shape[2:]) != self.shape[1:]:
                raise ValueError(f"field shape {tuple(F.shape)} is not (14, nzs, {self.shape[1]}, {self.shape[2]})")
            F = F.to(dtype=torch.float64).contiguous()
            if self.stream is not None:
                self.stream.wait_stream(torch.cuda.current_stream(F.device))
            return F.data_ptr(), F.shape[1], CNSF_DEVICE, F
        F = np.ascontiguousarray(F, dtype=np.float64)
        if F.ndim != 4 or F.shape[0] != NCOMP or F.shape[2:] != self.shape[1:]:
            raise ValueError(f"field shape {F.shape} is not (14, nzs, {self.shape[1]}, {self.shape[2]})")
        return F.ctypes.data, F.shape[1], CNSF_HOST, F

    def set_state(self, Q, z0: int = 0):
        """Q: float64 (14, nzs, ny, nx) NumPy array (host) or torch CUDA tensor (device)."""
        ptr, nzs, where, keep = self._fields_arg(Q)
        cnsf_set_state(self.h, ptr, z0, nzs, where)

    def set_primitive(self, P, z0: int = 0):
        """P: float64 (14, nzs, ny, nx): rho, u (3), p, tau (6), q (3); host array or CUDA tensor."""
        ptr, nzs, where, keep = self._fields_arg(P)
        cnsf_set_primitive(self.h, ptr, z0, nzs, where)

    def primitives(self, z0: int = 0, nzs: int | None = None):
        """(6, nzs, ny, nx) FP64: rho, u_x, u_y, u_z, p, T of the current time level."""
        if nzs is None:
            nzs = self.p.nz - z0
        out = np.empty((6, nzs, self.p.ny, self.p.nx), dtype=np.float64)
        cnsf_get_primitives(self.h, out.ctypes.data, z0, nzs, CNSF_HOST)
        return out

    def step(self, n: int = 1):
        cnsf_step(self.h, int(n))

    def moments(self, z0: int = 0, nzs: int | None = None, device: bool = False):
        if nzs is None:
            nzs = self.p.nz - z0
        if device:
            torch = _torch()
            out = torch.empty((NCOMP, nzs, self.p.ny, self.p.nx), dtype=torch.float64, device=self.device)
            cnsf_get_moments(self.h, out.data_ptr(), z0, nzs, CNSF_DEVICE)
            return out
        out = np.empty((NCOMP, nzs, self.p.ny, self.p.nx), dtype=np.float64)
        cnsf_get_moments(self.h, out.ctypes.data, z0, nzs, CNSF_HOST)
        return out

    def diagnostics(self, spectral: bool = True) -> dict:
        d = cnsf_diagnostics(self.h, CNSF_DIAG_SPECTRAL if spectral else CNSF_DIAG_SUMS)
        return _diag_dict(d)

    def step_diagnostics(self, n: int, spectral: bool = True) -> dict:
        """Advance n steps; return the diagnostics of the level at entry (one population read)."""
        return _diag_dict(cnsf_step_diagnostics(self.h, int(n), CNSF_DIAG_SPECTRAL if spectral else CNSF_DIAG_SUMS))

    def spectrum(self, device: bool = False):
        """Shell-averaged velocity spectrum E[k], k = 0 .. 1 + nint(sqrt(3) n / 2) - 1 (FP64)."""
        k = cnsf_spectrum_shells(self.h)
        if device:
            torch = _torch()
            out = torch.empty(k, dtype=torch.float64, device=self.device)
            cnsf_spectrum(self.h, out.data_ptr(), k, CNSF_DEVICE)
            return out
        out = np.empty(k, dtype=np.float64)
        cnsf_spectrum(self.h, out.ctypes.data, k, CNSF_HOST)
        return out

    def info(self):
        return cnsf_get_info(self.h)

    def export_populations(self):
        _, _, nb = self.info()
        buf = np.empty(nb, dtype=np.uint8)
        step, parity = cnsf_export_populations(self.h, buf.ctypes.data, nb)
        return buf, step, parity

    def import_populations(self, buf: np.ndarray, step: int, parity: int):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        cnsf_import_populations(self.h, buf.ctypes.data, buf.nbytes, step, parity)

    def set_launch(self, block: int = 256, tile: int | None = None, grid: int = 0, xcd_remap: bool = True):
        cnsf_set_launch(self.h, block, block if tile is None else tile, grid, int(bool(xcd_remap)))

    def get_launch(self):
        """(block, tile, grid, xcd_remap) of the update launch."""
        return cnsf_get_launch(self.h)


# ---------------------------------------------------------------- batch
def cnsf_batch_required_bytes(members) -> int:
    arr = (cnsf_params * len(members))(*members)
    n = C.c_size_t()
    _check(library().cnsf_batch_required_bytes(arr, len(members), C.byref(n)))
    return n.value


def cnsf_batch_create(members, dev_buf: int, nbytes: int, stream: int):
    arr = (cnsf_params * len(members))(*members)
    h = C.c_void_p()
    _check(library().cnsf_batch_create(arr, len(members), C.c_void_p(dev_buf), nbytes, C.c_void_p(stream),
                                       C.byref(h)))
    return h


def cnsf_batch_destroy(h):
    _check(library().cnsf_batch_destroy(h))


def cnsf_batch_set_state(h, j: int, Q_ptr: int, where: int):
    _check(library().cnsf_batch_set_state(h, j, C.cast(C.c_void_p(Q_ptr), C.POINTER(C.c_double)), where))


def cnsf_batch_step(h, n: int, mode: int):
    _check(library().cnsf_batch_step(h, n, mode))


def cnsf_batch_get_moments(h, j: int, out_ptr: int, where: int):
    _check(library().cnsf_batch_get_moments(h, j, C.cast(C.c_void_p(out_ptr), C.POINTER(C.c_double)), where))


def cnsf_batch_set_launch(h, block: int, tile: int, grid: int, graph_steps: int):
    _check(library().cnsf_batch_set_launch(h, block, tile, grid, graph_steps))


def cnsf_batch_get_launch(h):
    v = [C.c_int32() for _ in range(4)]
    _check(library().cnsf_batch_get_launch(h, *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)


def cnsf_batch_autotune(h, cache_path: str | None, steps_per_trial: int):
    _check(library().cnsf_batch_autotune(h, cache_path.encode() if cache_path else None, steps_per_trial))


class Batch:
    """An ensemble of independent periodic lattices stepped together."""

    MODE_LAUNCH, MODE_GRAPH, MODE_SEQUENTIAL = 0, 1, 2

    def __init__(self, prms, *, device="cuda", stream=None, buf=None, spacing: int = 0):
        """buf: optional uint8 CUDA tensor of at least the required bytes for the
        members' populations (e.g. another batch's, whose state this one then
        overwrites).  spacing: bytes between the runs of consecutive components
        in the component-major layout (the library's minimum if 0); the array
        then takes NCOMP * spacing bytes (capped by buf's size when buf is
        given).  About 1 GiB lets MI355X run an ensemble of small members at
        a large lattice's rate; results do not depend on it."""
        torch = _torch()
        self.prms = [dict(p) for p in prms]
        self.ps = [make_params(p) for p in prms]
        need = cnsf_batch_required_bytes(self.ps)
        self.nbytes = max(need, NCOMP * int(spacing))
        if buf is not None:
            if buf.dtype != torch.uint8 or not buf.is_cuda or buf.numel() < need or not buf.is_contiguous():
                raise ValueError(f"buf must be a contiguous uint8 CUDA tensor of >= {need} bytes")
            self.buf = buf
            self.nbytes = min(self.nbytes, buf.numel())
        else:
            self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=torch.device(device))
        self.stream = stream
        self.h = cnsf_batch_create(self.ps, self.buf.data_ptr(), self.nbytes, _stream_handle(stream))

    @classmethod
    def placed(cls, prms, *, candidates: int | None = None, probe_steps: int = 4, device="cuda", stream=None,
               spacing: int = 0):
        """A batch whose population array is the fastest of `candidates` allocations
        (default: as many as fit in 85% of the free device memory, at most 8),
        by the policy of Lattice.placed: each candidate batch is created
        (cleared) and timed over `probe_steps` launch-per-step updates after one
        untimed update (HIP events on the batch's stream); all stay alive until
        every one is timed; the fastest array is kept and the returned batch is
        freshly created on it (cleared, step 0).  ``placement_ms`` holds each
        candidate's mean time per step and ``placement_kept`` the index kept."""
        torch = _torch()
        torch.cuda.empty_cache()
        need = max(cnsf_batch_required_bytes([make_params(p) for p in prms]), NCOMP * int(spacing))
        if candidates is None:
            free = torch.cuda.mem_get_info(torch.device(device))[0]
            candidates = min(8, int(0.85 * free) // max(1, need))
        bs, ms = [], []
        s = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        for _ in range(max(1, int(candidates))):
            try:
                B = cls(prms, device=device, stream=stream, spacing=spacing)
            except torch.cuda.OutOfMemoryError:
                if not bs:
                    raise
                break
            B.step(1, cls.MODE_LAUNCH)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            B.step(probe_steps, cls.MODE_LAUNCH)
            b.record(s)
            b.synchronize()
            ms.append(a.elapsed_time(b) / probe_steps)
            bs.append(B)
        best = min(range(len(ms)), key=ms.__getitem__)
        buf = bs[best].buf
        for B in bs:
            B.close()
        del bs, B
        torch.cuda.empty_cache()
        out = cls(prms, device=device, stream=stream, buf=buf, spacing=spacing)
        out.placement_ms, out.placement_kept = ms, best
        return out

    def close(self):
        if getattr(self, "h", None):
            cnsf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ncells(self):
        return sum(p.nx * p.ny * p.nz for p in self.ps)

    def set_state(self, j: int, Q):
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        cnsf_batch_set_state(self.h, j, Q.ctypes.data, CNSF_HOST)

    def step(self, n: int, mode: int = 1):
        cnsf_batch_step(self.h, int(n), int(mode))

    def moments(self, j: int):
        p = self.ps[j]
        out = np.empty((NCOMP, p.nz, p.ny, p.nx), dtype=np.float64)
        cnsf_batch_get_moments(self.h, j, out.ctypes.data, CNSF_HOST)
        return out

    def set_launch(self, block=256, tile=256, grid=0, graph_steps=20):
        cnsf_batch_set_launch(self.h, block, tile, grid, graph_steps)

    def get_launch(self):
        """(block, tile, grid, graph_steps) of the batched update."""
        return cnsf_batch_get_launch(self.h)

    def autotune(self, cache_path=None, steps_per_trial=10):
        cnsf_batch_autotune(self.h, cache_path, steps_per_trial)
