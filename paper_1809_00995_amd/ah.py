"""ctypes binding of ``libah.so`` (include/ah.h), argument marshalling only.

PyTorch supplies device memory (one tensor of 15 or 20 planes per realization) and
the stream; every step of the method runs in the library's HIP kernels.  If
the library has not been built this module raises on load: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libah.so")

AH_OK, AH_E_INVALID, AH_E_NOMEM, AH_E_HIP, AH_E_DOMAIN, AH_E_STATE, AH_E_NONFINITE = \
    0, -1, -2, -3, -4, -5, -6
AH_FP64, AH_FP32 = 0, 1
AH_INIT_RANDOM_PHASE, AH_INIT_VACUUM, AH_INIT_NONE = 0, 1, 2
AH_KERNEL_AUTO, AH_KERNEL_PLAIN, AH_KERNEL_TILED, AH_KERNEL_TILED2 = 0, 1, 2, 3
AH_LAYOUT_15, AH_LAYOUT_20 = 0, 1

FIELDS = ("phi_re", "phi_im", "pi_re", "pi_im", "ax", "ay", "az", "ex", "ey", "ez")
AH_NOALLOC_MAX_REAL = 64

EXPORTED = ("ah_error_string", "ah_last_error", "ah_init", "ah_step", "ah_measure",
            "ah_measure_noalloc", "ah_gauss_residual", "ah_current_planes", "ah_current_step",
            "ah_set_kernel", "ah_set_launch", "ah_autotune", "ah_free")


class AHError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("precision", C.c_int32),
                ("dx", C.c_double), ("dt", C.c_double),
                ("tau0", C.c_double), ("tau_ref", C.c_double),
                ("era_p", C.c_double), ("s", C.c_double),
                ("lambda0", C.c_double), ("e0", C.c_double), ("sigma", C.c_double),
                ("seed", C.c_uint64), ("init", C.c_int32), ("layout", C.c_int32),
                ("step0", C.c_int64), ("n_end", C.c_int64),
                ("s_late", C.c_double), ("tau_s", C.c_double),
                ("z_halo", C.c_int32), ("reserved", C.c_int32)]


class _Buffers(C.Structure):
    _fields_ = [("planes", C.c_void_p)]


class _Obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("tau", C.c_double), ("a", C.c_double),
                ("n_wind", C.c_int64), ("n_wind_dir", C.c_int64 * 3),
                ("net_wind_dir", C.c_int64 * 3), ("n_pierced", C.c_int64),
                ("length", C.c_double), ("xi_w", C.c_double),
                ("sum_lag", C.c_double), ("xi_l", C.c_double),
                ("num", C.c_double * 3), ("den", C.c_double * 3), ("v2", C.c_double * 3),
                ("kin", C.c_double), ("grad", C.c_double), ("elec", C.c_double),
                ("mag", C.c_double), ("pot", C.c_double), ("energy", C.c_double),
                ("pres", C.c_double), ("pres_lag", C.c_double), ("rho_lag", C.c_double),
                ("v2_eos", C.c_double), ("nonfinite", C.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libah.so (no GPU call is made by loading)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1809_00995_amd/build.py "
                           "(there is no CPU fallback)")
    lib = C.CDLL(path)
    P = C.POINTER
    lib.ah_error_string.restype = C.c_char_p
    lib.ah_error_string.argtypes = [C.c_int]
    lib.ah_last_error.restype = C.c_char_p
    lib.ah_last_error.argtypes = [C.c_void_p]
    lib.ah_init.argtypes = [P(C.c_void_p), C.c_int32, P(_Params), P(_Buffers), C.c_void_p]
    lib.ah_step.argtypes = [C.c_void_p, C.c_int64, C.c_int32, P(_Obs), C.c_int64, P(C.c_int64)]
    lib.ah_measure.argtypes = [C.c_void_p, P(_Obs), C.c_void_p]
    lib.ah_measure_noalloc.argtypes = [C.c_int32, P(_Params), P(_Buffers), C.c_void_p,
                                       C.c_void_p, C.c_void_p]
    lib.ah_gauss_residual.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
    lib.ah_current_planes.argtypes = [C.c_void_p, C.c_int32, P(C.c_int32)]
    lib.ah_current_step.argtypes = [C.c_void_p, C.c_int32, P(C.c_int64)]
    lib.ah_set_kernel.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
    lib.ah_set_launch.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
    lib.ah_autotune.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32)]
    lib.ah_free.argtypes = [C.c_void_p]
    for name in EXPORTED:
        if name != "ah_error_string" and name != "ah_last_error":
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


@dataclass
class Params:
    """Problem statement of one realization (mirrors ah_params)."""
    nx: int
    ny: int
    nz: int
    precision: int = AH_FP64
    dx: float = 0.5
    dt: float = 0.1
    tau0: float = 0.0
    tau_ref: float = 1.0
    era_p: float = 1.0
    s: float = 1.0
    lambda0: float = 2.0
    e0: float = 1.0
    sigma: float = 1.0
    seed: int = 1
    init: int = AH_INIT_RANDOM_PHASE
    step0: int = 0
    n_end: int = 0
    s_late: float = 1.0
    tau_s: float = 0.0
    # the 20-plane layout: unmeasured steps go two per pass (the library's fastest
    # path); AH_LAYOUT_15 needs 60 instead of 80 B/site (FP32) of field storage
    layout: int = AH_LAYOUT_20
    z_halo: int = 0

    def _c(self) -> _Params:
        return _Params(self.nx, self.ny, self.nz, self.precision, self.dx, self.dt, self.tau0,
                       self.tau_ref, self.era_p, self.s, self.lambda0, self.e0, self.sigma,
                       self.seed & 0xFFFFFFFFFFFFFFFF, self.init, self.layout, self.step0,
                       self.n_end, self.s_late, self.tau_s, self.z_halo, 0)

    @property
    def planes(self) -> int:
        return 20 if self.layout == AH_LAYOUT_20 else 15

    @property
    def dtype(self):
        return torch.float64 if self.precision == AH_FP64 else torch.float32

    @property
    def nz_stored(self) -> int:
        """z-planes held per field plane: nz, plus the halo planes of a slab."""
        return self.nz + 2 * self.z_halo

    @property
    def sites(self) -> int:
        """Stored sites per field plane."""
        return self.nx * self.ny * self.nz_stored


@dataclass
class Obs:
    step: int
    tau: float
    a: float
    n_wind: int
    n_wind_dir: list
    net_wind_dir: list
    n_pierced: int
    length: float
    xi_w: float
    sum_lag: float
    xi_l: float
    num: list
    den: list
    v2: list
    kin: float
    grad: float
    elec: float
    mag: float
    pot: float
    energy: float
    pres: float
    pres_lag: float
    rho_lag: float
    v2_eos: float
    nonfinite: int

    @staticmethod
    def _from(o: _Obs) -> "Obs":
        d = {}
        for k, _ in _Obs._fields_:
            v = getattr(o, k)
            d[k] = list(v) if not isinstance(v, (int, float)) else v
        return Obs(**d)


class ObsRecords:
    """Undecoded observations of one ah_step call: n_slots measured states of n_real
    realizations each."""

    def __init__(self, records, n_slots: int, n_real: int):
        self.records, self.n_slots, self.n_real = records, n_slots, n_real

    def __len__(self) -> int:
        return self.n_slots

    def decode(self) -> list:
        """The observations as a list of per-slot lists of Obs."""
        flat = _obs_list(self.records, self.n_slots * self.n_real)
        return [flat[j * self.n_real:(j + 1) * self.n_real] for j in range(self.n_slots)]


def _obs_list(records, n: int) -> list:
    """The first n ah_obs of a ctypes array as Obs, read in one pass (a field-by-field
    ctypes read costs tens of microseconds per record)."""
    if n <= 0:
        return []
    rows = np.ctypeslib.as_array(records)[:n].tolist()
    return [Obs(*[v.tolist() if isinstance(v, np.ndarray) else v for v in row]) for row in rows]


def alloc_planes(p: Params, device="cuda") -> torch.Tensor:
    """Caller-owned field storage: 15 or 20 planes by layout (see include/ah.h), shape
    (planes, nz + 2 z_halo, ny, nx)."""
    return torch.empty((p.planes, p.nz_stored, p.ny, p.nx), dtype=p.dtype, device=device)


OBS_BYTES = C.sizeof(_Obs)


def measure_noalloc(params: Sequence[Params], planes: Sequence[torch.Tensor], out: torch.Tensor,
                    wind: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None):
    """ah_measure_noalloc: the diagnostics of S_{step0} held in planes 0-9 of each tensor,
    without a context and without any allocation in the library.  ``out`` is a caller-owned
    uint8 device tensor of at least ``len(params) * OBS_BYTES`` bytes that receives the
    ah_obs records; ``wind`` None or an int8 device tensor as for ``Context.measure``.
    Asynchronous on ``stream`` (default: the current stream); decode ``out`` with
    ``obs_from_bytes`` once the stream has reached this call."""
    lib = load_library()
    n = len(params)
    if n != len(planes) or out.dtype != torch.uint8 or not out.is_cuda or \
            out.numel() < n * OBS_BYTES or not out.is_contiguous():
        raise ValueError("one planes tensor per realization and a contiguous uint8 device "
                         "tensor of n_real * OBS_BYTES bytes are required")
    st = stream if stream is not None else torch.cuda.current_stream()
    cp = (_Params * n)(*[p._c() for p in params])
    cb = (_Buffers * n)(*[_Buffers(t.data_ptr()) for t in planes])
    rc = lib.ah_measure_noalloc(n, cp, cb, C.c_void_p(out.data_ptr()),
                                C.c_void_p(wind.data_ptr()) if wind is not None else None,
                                C.c_void_p(st.cuda_stream))
    _check(lib, None, rc)
    return out


def obs_from_bytes(raw, n: int) -> list:
    """Decode n ah_obs records from host bytes (or a CPU uint8 tensor)."""
    if isinstance(raw, torch.Tensor):
        raw = raw.cpu().numpy().tobytes()
    return [Obs._from(_Obs.from_buffer_copy(raw, k * OBS_BYTES)) for k in range(n)]


def _check(lib, ctx, rc):
    if rc != AH_OK:
        msg = lib.ah_last_error(ctx).decode() or lib.ah_error_string(rc).decode()
        raise AHError(rc, msg)


class Context:
    """One ah_ctx: n_real realizations advanced together on one stream."""

    def __init__(self, params: Sequence[Params], planes: Sequence[torch.Tensor],
                 stream: torch.cuda.Stream | None = None):
        self.lib = load_library()
        self.params = list(params)
        self.planes = list(planes)
        if len(self.params) != len(self.planes) or not self.params:
            raise ValueError("one planes tensor per realization is required")
        for p, t in zip(self.params, self.planes):
            if (not t.is_cuda or t.dtype != p.dtype or not t.is_contiguous()
                    or t.numel() != p.planes * p.sites):
                raise ValueError("planes must be contiguous device tensors of 15 (or 20 with "
                                 "AH_LAYOUT_20) planes of nx*ny*nz elements of the "
                                 "realization's precision")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        n = len(self.params)
        cp = (_Params * n)(*[p._c() for p in self.params])
        cb = (_Buffers * n)(*[_Buffers(t.data_ptr()) for t in self.planes])
        self._ctx = C.c_void_p()
        rc = self.lib.ah_init(C.byref(self._ctx), n, cp, cb, C.c_void_p(self.stream.cuda_stream))
        _check(self.lib, None, rc)

    @property
    def n_real(self) -> int:
        return len(self.params)

    def step(self, nsteps: int, measure_every: int = 0, out_cap: int | None = None,
             decode: bool = True):
        """Advance nsteps; returns the observations (list of per-slot lists) when measuring.
        With decode=False the records come back undecoded (an ObsRecords; its decode()
        gives the same lists), which keeps Python object construction out of the call."""
        if measure_every <= 0:
            rc = self.lib.ah_step(self._ctx, nsteps, 0, None, 0, None)
            _check(self.lib, self._ctx, rc)
            return []
        cap = out_cap if out_cap is not None else nsteps // measure_every + 2
        out = (_Obs * (cap * self.n_real))()
        n_out = C.c_int64()
        rc = self.lib.ah_step(self._ctx, nsteps, measure_every, out, cap, C.byref(n_out))
        if rc == AH_E_NONFINITE:
            raise AHError(rc, self.lib.ah_last_error(self._ctx).decode())
        _check(self.lib, self._ctx, rc)
        rec = ObsRecords(out, n_out.value, self.n_real)
        return rec.decode() if decode else rec

    def measure(self, wind: bool = False):
        """Observations of the current state; with wind=True also the W maps (int8, device)."""
        out = (_Obs * self.n_real)()
        wmap = None
        if wind:
            # cleared on the library's stream, which ah_measure synchronises
            with torch.cuda.stream(self.stream):
                wmap = torch.zeros(sum(3 * p.sites for p in self.params), dtype=torch.int8,
                                   device=self.planes[0].device)
        rc = self.lib.ah_measure(self._ctx, out,
                                 C.c_void_p(wmap.data_ptr()) if wmap is not None else None)
        _check(self.lib, self._ctx, rc)
        obs = _obs_list(out, self.n_real)
        if not wind:
            return obs
        maps, off = [], 0
        for p in self.params:
            n = 3 * p.sites
            maps.append(wmap[off:off + n].view(3, p.nz_stored, p.ny, p.nx))
            off += n
        return obs, maps

    def gauss_residual(self):
        n = self.n_real
        mx, rms = (C.c_double * n)(), (C.c_double * n)()
        rc = self.lib.ah_gauss_residual(self._ctx, mx, rms)
        _check(self.lib, self._ctx, rc)
        return list(mx), list(rms)

    def current_planes(self, r: int = 0):
        arr = (C.c_int32 * 10)()
        _check(self.lib, self._ctx, self.lib.ah_current_planes(self._ctx, r, arr))
        return list(arr)

    def current_step(self, r: int = 0) -> int:
        n = C.c_int64()
        _check(self.lib, self._ctx, self.lib.ah_current_step(self._ctx, r, C.byref(n)))
        return n.value

    def fields(self, r: int = 0) -> torch.Tensor:
        """The current state S_n of realization r as a (10, nz + 2 z_halo, ny, nx) tensor (a
        copy)."""
        planes = self.current_planes(r)
        # copied on the library's stream, after its work; the caller's current
        # stream then waits for the copy
        with torch.cuda.stream(self.stream):
            idx = torch.tensor(planes, device=self.planes[r].device)
            out = self.planes[r].index_select(0, idx)
        torch.cuda.current_stream(self.planes[r].device).wait_stream(self.stream)
        return out

    def set_kernel(self, kernel: int, tile_y: int = 0, chunk_z: int = 0):
        _check(self.lib, self._ctx, self.lib.ah_set_kernel(self._ctx, kernel, tile_y, chunk_z))

    def set_launch(self, batched: bool = False, graph_steps: int = 0):
        _check(self.lib, self._ctx, self.lib.ah_set_launch(self._ctx, int(batched), graph_steps))

    def autotune(self):
        """Time tile heights and z-chunks on scratch lattices; returns (tile_y, [chunk_z])."""
        ty = C.c_int32()
        cz = (C.c_int32 * self.n_real)()
        _check(self.lib, self._ctx, self.lib.ah_autotune(self._ctx, C.byref(ty), cz))
        return ty.value, list(cz)

    def close(self):
        if self._ctx:
            rc = self.lib.ah_free(self._ctx)
            self._ctx = C.c_void_p()
            _check(self.lib, None, rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if getattr(self, "_ctx", None):
                self.lib.ah_free(self._ctx)
        except Exception:
            pass
