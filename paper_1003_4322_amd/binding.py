"""Thin ctypes binding of libps.so (C ABI in include/ps.h).

Argument marshalling only: shapes, dtypes and devices are checked here, then
the tensors' device pointers and torch's current HIP stream are handed to the
library, where every step runs in hand-written gfx950 kernels.  PyTorch
provides device memory and streams; nothing here computes.  If the library is
missing the import raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence, Tuple, Union

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libps.so")

PS_F32, PS_F64 = 0, 1
PS_NS, PS_MHD = 0, 1
_STATUS = {0: "PS_OK", -1: "PS_ERR_ARG", -2: "PS_ERR_SIZE", -3: "PS_ERR_NOMEM",
           -4: "PS_ERR_HIP", -5: "PS_ERR_STATE", -6: "PS_ERR_DIVERGED"}

# (name, restype, argtypes) of every exported function, in header order
_vp, _sz, _i, _d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
_SIGS = [
    ("ps_plan_create", _i, [ctypes.POINTER(_vp), _i, _i, _i]),
    ("ps_plan_create_batch", _i, [ctypes.POINTER(_vp), _i, ctypes.POINTER(_i), _i, _i]),
    ("ps_plan_create_grid", _i, [ctypes.POINTER(_vp), _i, _i, _i, _i, _i]),
    ("ps_plan_destroy", _i, [_vp]),
    ("ps_plan_set_stream", _i, [_vp, _vp]),
    ("ps_plan_workspace_bytes", _sz, [_vp]),
    ("ps_plan_set_workspace", _i, [_vp, _vp, _sz]),
    ("ps_plan_box_offsets", _i, [_vp, _i, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    ("ps_num_shells", _i, [_vp, _i]),
    ("ps_fft_r2c", _i, [_vp, _vp, _vp]),
    ("ps_fft_c2r", _i, [_vp, _vp, _vp]),
    ("ps_nonlinear_ns", _i, [_vp, _vp, _vp]),
    ("ps_nonlinear_mhd", _i, [_vp, _vp, _vp]),
    ("ps_rk2_step", _i, [_vp, _vp, _i, _d, _d, _d, _i]),
    ("ps_plan_set_monitor", _i, [_vp, _i, _d]),
    ("ps_plan_set_rotation", _i, [_vp, _d, _d, _d]),
    ("ps_plan_set_box", _i, [_vp, _d, _d, _d]),
    ("ps_energy_spectrum", _i, [_vp, _vp, _i, _vp, _vp]),
    ("ps_energy_spectrum_static", _i, [_vp, _vp, _i, _vp, _vp]),
    ("ps_mhd_spectrum", _i, [_vp, _vp, _vp, _vp]),
    ("ps_plan_set_variant", _i, [_vp, ctypes.c_char_p, _i]),
    ("ps_plan_get_variant", _i, [_vp, ctypes.c_char_p]),
    ("ps_plan_variant_count", _i, [_vp, ctypes.c_char_p]),
    ("ps_plan_autotune", _i, [_vp, _vp, _i, _i]),
    ("ps_plan_autotune_timed", _i, [_vp]),
    ("ps_plan_set_timing", _i, [_vp, _i]),
    ("ps_plan_set_graphs", _i, [_vp, _i]),
    ("ps_plan_timing_reset", _i, [_vp]),
    ("ps_plan_timing_count", _i, [_vp]),
    ("ps_plan_timing_get", _i, [_vp, _i, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(_d),
                                ctypes.POINTER(ctypes.c_long), ctypes.POINTER(_d)]),
    ("ps_status_string", ctypes.c_char_p, [_i]),
    ("ps_last_error", ctypes.c_char_p, []),
    ("ps_build_hash", ctypes.c_char_p, []),
]
SYMBOLS = [s[0] for s in _SIGS]

_lib: Optional[ctypes.CDLL] = None


class PsError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {_STATUS.get(code, code)} ({detail})")
        self.code = code


def lib() -> ctypes.CDLL:
    """The in-tree libps.so (built by paper_1003_4322_amd.build).  Raises if it
    is missing or was built from other sources than the ones beside it."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1003_4322_amd/build.py "
                              "(there is no non-HIP fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        from . import build as _build
        have, want = L.ps_build_hash().decode(), _build.src_hash()
        if have != want:
            raise ImportError(f"{LIB_PATH} was built from other sources (hash {have}, sources "
                              f"{want}): rebuild it with paper_1003_4322_amd/build.py")
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != 0:
        raise PsError(rc, where, lib().ps_last_error().decode(errors="replace"))


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


_CDT = {PS_F32: torch.complex64, PS_F64: torch.complex128}
_RDT = {PS_F32: torch.float32, PS_F64: torch.float64}


def dtype_code(dtype: Union[str, torch.dtype, int]) -> int:
    if dtype in (PS_F32, "f32", "float32", torch.float32, torch.complex64):
        return PS_F32
    if dtype in (PS_F64, "f64", "float64", torch.float64, torch.complex128):
        return PS_F64
    raise ValueError(f"unsupported dtype {dtype!r}")


class Plan:
    """A plan for one N^3 box (``N`` an int), an ensemble (``N`` a list) or
    one nx x ny x nz box (``grid=(nx, ny, nz)``, ``N`` ignored)."""

    def __init__(self, N: Union[int, Sequence[int], None] = None, nfields: int = 3, dtype="f32",
                 device: Union[int, str, torch.device, None] = None, workspace: bool = True,
                 grid: Optional[Sequence[int]] = None):
        self.dtype = dtype_code(dtype)
        self.nfields = int(nfields)
        if grid is not None:
            self.dims = [tuple(int(n) for n in grid)]
            if len(self.dims[0]) != 3:
                raise ValueError("grid must be (nx, ny, nz)")
        else:
            if N is None:
                raise ValueError("Plan needs N (an int or a list) or grid=(nx, ny, nz)")
            sizes = [int(N)] if isinstance(N, int) else [int(n) for n in N]
            self.dims = [(n, n, n) for n in sizes]
        self.sizes = [d[0] for d in self.dims]
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        L = lib()
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            if grid is not None:
                _check(L.ps_plan_create_grid(ctypes.byref(h), *self.dims[0], self.nfields,
                                             self.dtype), "ps_plan_create_grid")
            elif len(self.sizes) == 1:
                _check(L.ps_plan_create(ctypes.byref(h), self.sizes[0], self.nfields, self.dtype),
                       "ps_plan_create")
            else:
                arr = (ctypes.c_int * len(self.sizes))(*self.sizes)
                _check(L.ps_plan_create_batch(ctypes.byref(h), len(self.sizes), arr, self.nfields,
                                              self.dtype), "ps_plan_create_batch")
        self._h = h
        self.ws: Optional[torch.Tensor] = None
        self.real_off, self.cplx_off = [], []
        for b in range(len(self.sizes)):
            r, c = ctypes.c_size_t(), ctypes.c_size_t()
            _check(L.ps_plan_box_offsets(h, b, ctypes.byref(r), ctypes.byref(c)), "box_offsets")
            self.real_off.append(r.value)
            self.cplx_off.append(c.value)
        self.nshells = [L.ps_num_shells(h, b) for b in range(len(self.sizes))]
        if workspace:
            self.allocate_workspace()

    # -- plumbing ------------------------------------------------------------
    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise RuntimeError("plan is closed")
        return self._h

    def workspace_bytes(self) -> int:
        return int(lib().ps_plan_workspace_bytes(self.handle))

    def allocate_workspace(self):
        n = self.workspace_bytes()
        self.ws = torch.empty(max(n, 256), dtype=torch.uint8, device=self.device)
        _check(lib().ps_plan_set_workspace(self.handle, _ptr(self.ws), self.ws.numel()),
               "ps_plan_set_workspace")

    def _stream(self):
        s = torch.cuda.current_stream(self.device)
        _check(lib().ps_plan_set_stream(self.handle, ctypes.c_void_p(s.cuda_stream)), "set_stream")

    def close(self):
        if self._h is not None:
            lib().ps_plan_destroy(self._h)
            self._h = None
            self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def complex_dtype(self):
        return _CDT[self.dtype]

    @property
    def real_dtype(self):
        return _RDT[self.dtype]

    def spectral_shape(self, nf: Optional[int] = None):
        assert len(self.dims) == 1, "ensembles use flat buffers"
        nx, ny, nz = self.dims[0]
        return (nf or self.nfields, nz, ny, nx // 2 + 1)

    def real_shape(self):
        assert len(self.dims) == 1, "ensembles use flat buffers"
        nx, ny, nz = self.dims[0]
        return (self.nfields, nz, ny, nx)

    def n_complex(self) -> int:
        return sum(self.nfields * nz * ny * (nx // 2 + 1) for nx, ny, nz in self.dims)

    def n_real(self) -> int:
        return sum(self.nfields * nx * ny * nz for nx, ny, nz in self.dims)

    def _need(self, t: torch.Tensor, kind: str, name: str, numel: Optional[int] = None):
        want = self.complex_dtype if kind == "c" else self.real_dtype
        if not isinstance(t, torch.Tensor) or t.dtype != want:
            raise TypeError(f"{name}: expected a {want} tensor")
        if t.device != self.device:
            raise ValueError(f"{name}: tensor on {t.device}, plan on {self.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: tensor must be contiguous")
        n = numel if numel is not None else (self.n_complex() if kind == "c" else self.n_real())
        if t.numel() != n:
            raise ValueError(f"{name}: expected {n} elements, got {t.numel()}")

    def _empty(self, kind: str, like_shape=None):
        if len(self.sizes) == 1:
            shape = self.spectral_shape() if kind == "c" else self.real_shape()
        else:
            shape = (self.n_complex() if kind == "c" else self.n_real(),)
        dt = self.complex_dtype if kind == "c" else self.real_dtype
        return torch.empty(shape, dtype=dt, device=self.device)

    # -- API -------------------------------------------------------------------
    def fft_r2c(self, real: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._need(real, "r", "real")
        out = self._empty("c") if out is None else out
        self._need(out, "c", "out")
        self._stream()
        _check(lib().ps_fft_r2c(self.handle, _ptr(real), _ptr(out)), "ps_fft_r2c")
        return out

    def fft_c2r(self, cplx: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._need(cplx, "c", "cplx")
        out = self._empty("r") if out is None else out
        self._need(out, "r", "out")
        self._stream()
        _check(lib().ps_fft_c2r(self.handle, _ptr(cplx), _ptr(out)), "ps_fft_c2r")
        return out

    def nonlinear_ns(self, uhat: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._need(uhat, "c", "uhat")
        out = self._empty("c") if out is None else out
        self._need(out, "c", "out")
        self._stream()
        _check(lib().ps_nonlinear_ns(self.handle, _ptr(uhat), _ptr(out)), "ps_nonlinear_ns")
        return out

    def nonlinear_mhd(self, zhat: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._need(zhat, "c", "zhat")
        out = self._empty("c") if out is None else out
        self._need(out, "c", "out")
        self._stream()
        _check(lib().ps_nonlinear_mhd(self.handle, _ptr(zhat), _ptr(out)), "ps_nonlinear_mhd")
        return out

    def rk2_step(self, state: torch.Tensor, model: int, nu: float, eta: float, dt: float,
                 nsteps: int = 1) -> torch.Tensor:
        """In place on ``state``; returns it."""
        self._need(state, "c", "state")
        self._stream()
        _check(lib().ps_rk2_step(self.handle, _ptr(state), int(model), float(nu), float(eta),
                                 float(dt), int(nsteps)), "ps_rk2_step")
        return state

    def energy_spectrum(self, fhat: torch.Tensor, nfields: Optional[int] = None
                        ) -> Tuple[torch.Tensor, torch.Tensor]:
        """Device FP64 (spectrum, totals[E, Z, maxdiv]); ensembles: concatenated."""
        nf = nfields or self.nfields
        if fhat.dtype != self.complex_dtype or fhat.device != self.device or not fhat.is_contiguous():
            raise TypeError("fhat: contiguous complex tensor of the plan's dtype and device")
        spec = torch.empty(sum(self.nshells), dtype=torch.float64, device=self.device)
        tot = torch.empty(3 * len(self.sizes), dtype=torch.float64, device=self.device)
        self._stream()
        _check(lib().ps_energy_spectrum(self.handle, _ptr(fhat), nf, _ptr(spec), _ptr(tot)),
               "ps_energy_spectrum")
        return spec, tot

    def energy_spectrum_static(self, fhat: torch.Tensor, nfields: Optional[int] = None
                               ) -> Tuple[torch.Tensor, torch.Tensor]:
        """energy_spectrum through the allocation-free entry point (no
        workspace needed; the partials live in the library's device scratch).
        The output tensors are allocated here, by torch, not by the library."""
        nf = nfields or self.nfields
        if fhat.dtype != self.complex_dtype or fhat.device != self.device or not fhat.is_contiguous():
            raise TypeError("fhat: contiguous complex tensor of the plan's dtype and device")
        spec = torch.empty(sum(self.nshells), dtype=torch.float64, device=self.device)
        tot = torch.empty(3 * len(self.sizes), dtype=torch.float64, device=self.device)
        self._stream()
        _check(lib().ps_energy_spectrum_static(self.handle, _ptr(fhat), nf, _ptr(spec), _ptr(tot)),
               "ps_energy_spectrum_static")
        return spec, tot

    def mhd_spectrum(self, zhat: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
        """Device FP64 (spectra [Eu(s)], [Eb(s)], [Hc(s)] per box, totals
        [Eu, Eb, Hc] per box) of an Elsasser state; one box: shapes (3, nshell)
        and (3,)."""
        self._need(zhat, "c", "zhat")
        spec = torch.empty(3 * sum(self.nshells), dtype=torch.float64, device=self.device)
        tot = torch.empty(3 * len(self.sizes), dtype=torch.float64, device=self.device)
        self._stream()
        _check(lib().ps_mhd_spectrum(self.handle, _ptr(zhat), _ptr(spec), _ptr(tot)),
               "ps_mhd_spectrum")
        if len(self.sizes) == 1:
            return spec.view(3, self.nshells[0]), tot
        return spec, tot

    def set_monitor(self, every: int, growth: float = 1e3):
        """Blow-up monitor of rk2_step: energy checked every ``every`` steps;
        PsError with code -6 (PS_ERR_DIVERGED) when it is not finite or grew by
        more than ``growth``.  every = 0 switches it off."""
        _check(lib().ps_plan_set_monitor(self.handle, int(every), float(growth)), "set_monitor")

    def set_rotation(self, ox: float, oy: float, oz: float):
        """Rotating frame for rk2_step: Coriolis term -P(k)(2 Omega x u)."""
        _check(lib().ps_plan_set_rotation(self.handle, float(ox), float(oy), float(oz)),
               "set_rotation")

    def set_box(self, Lx: float, Ly: float, Lz: float):
        """Box lengths (default 2 pi each): physical wavenumbers 2 pi n / L."""
        _check(lib().ps_plan_set_box(self.handle, float(Lx), float(Ly), float(Lz)), "set_box")

    # -- variants and autotuning ---------------------------------------------------
    KINDS = ("y", "z", "z_curl", "z_epi", "x_prod", "batch", "prune", "form", "pipe", "overlap")

    def set_variant(self, kind: str, v: int):
        _check(lib().ps_plan_set_variant(self.handle, kind.encode(), int(v)), "set_variant")

    def variant(self, kind: str) -> int:
        return int(lib().ps_plan_get_variant(self.handle, kind.encode()))

    def variant_count(self, kind: str) -> int:
        return int(lib().ps_plan_variant_count(self.handle, kind.encode()))

    def variants(self) -> Dict[str, int]:
        return {k: self.variant(k) for k in self.KINDS}

    def autotune(self, state: torch.Tensor, model: int, reps: int = 3) -> Dict[str, int]:
        self._need(state, "c", "state")
        self._stream()
        _check(lib().ps_plan_autotune(self.handle, _ptr(state), int(model), int(reps)), "autotune")
        return self.variants()

    def autotune_timed(self) -> int:
        """Timing launches of the last autotune (0: taken from PS_TUNE_CACHE)."""
        return int(lib().ps_plan_autotune_timed(self.handle))

    # -- timing ----------------------------------------------------------------
    def set_timing(self, on: bool):
        _check(lib().ps_plan_set_timing(self.handle, int(bool(on))), "set_timing")

    def set_graphs(self, on: bool):
        _check(lib().ps_plan_set_graphs(self.handle, int(bool(on))), "set_graphs")

    def timing_reset(self):
        _check(lib().ps_plan_timing_reset(self.handle), "timing_reset")

    def timings(self) -> Dict[str, Dict[str, float]]:
        L = lib()
        n = L.ps_plan_timing_count(self.handle)
        if n < 0:
            _check(n, "timing_count")
        out = {}
        for i in range(n):
            name = ctypes.c_char_p()
            ms, bpl = ctypes.c_double(), ctypes.c_double()
            cnt = ctypes.c_long()
            _check(L.ps_plan_timing_get(self.handle, i, ctypes.byref(name), ctypes.byref(ms),
                                        ctypes.byref(cnt), ctypes.byref(bpl)), "timing_get")
            out[name.value.decode()] = {"total_ms": ms.value, "launches": cnt.value,
                                        "bytes_per_launch": bpl.value}
        return out
