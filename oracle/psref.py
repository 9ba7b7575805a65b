"""FP64 CPU oracle for the pseudospectral step -- Python binding.

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this module.  The product path
(the HIP library and its binding) never imports it.

The arithmetic lives in ``psref.c`` (plain C, FP64); this module only builds
and loads that library and marshals numpy arrays.  Every array is C-contiguous:
real fields ``float64[nf, N, N, N]`` ([f][z][y][x]) and half spectra
``complex128[nf, N, N, N//2+1]`` ([f][kz][ky][kx]).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "psref.c")
LIB = os.path.join(HERE, "libpsref.so")

NS, MHD = 0, 1


def build(mutant: int = 0, out: Optional[str] = None, openmp: bool = True) -> str:
    """Compile psref.c with gcc.  ``mutant`` > 0 plants the numbered mistake
    (used only by the mutation tests).  Returns the path of the library."""
    out = out or LIB
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-Wno-unused-parameter", f"-DPSREF_MUTANT={int(mutant)}", SRC, "-o", out, "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


class Oracle:
    """ctypes wrapper around one build of the oracle library."""

    def __init__(self, path: Optional[str] = None):
        path = path or LIB
        if not os.path.exists(path):
            if path != LIB:
                raise FileNotFoundError(path)
            build()
        self.lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L = self.lib
        L.psref_set_threads.argtypes = [ctypes.c_int]
        L.psref_fft_r2c.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.psref_fft_c2r.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.psref_dft_at.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ip, ip, dp]
        L.psref_curl.argtypes = [ctypes.c_int, dp, dp]
        L.psref_nonlinear_ns.argtypes = [ctypes.c_int, dp, dp]
        L.psref_nonlinear_mhd.argtypes = [ctypes.c_int, dp, dp]
        L.psref_nonlinear_at.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ip, ip,
                                         ip, dp]
        L.psref_rk2_step.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.psref_rk2_step_rot.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.psref_set_box.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.psref_num_shells.argtypes = [ctypes.c_int]
        L.psref_energy_spectrum.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]

    # -- helpers -----------------------------------------------------------
    @staticmethod
    def _p(a: np.ndarray):
        assert a.flags.c_contiguous
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    @staticmethod
    def _ip(a: np.ndarray):
        assert a.flags.c_contiguous and a.dtype == np.int32
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))

    @staticmethod
    def _spec(a, N: int, nf: Optional[int] = None) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.complex128)
        if a.ndim == 3:
            a = a[None]
        if a.shape[1:] != (N, N, N // 2 + 1) or (nf is not None and a.shape[0] != nf):
            raise ValueError(f"bad spectral shape {a.shape} for N={N}")
        return a

    @staticmethod
    def _check(rc: int, what: str):
        if rc != 0:
            raise RuntimeError(f"{what} failed with code {rc}")

    # -- API ---------------------------------------------------------------
    def set_threads(self, n: int) -> int:
        return int(self.lib.psref_set_threads(int(n)))

    def fft_r2c(self, u: np.ndarray) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64)
        squeeze = u.ndim == 3
        if squeeze:
            u = u[None]
        nf, N = u.shape[0], u.shape[1]
        out = np.empty((nf, N, N, N // 2 + 1), np.complex128)
        self._check(self.lib.psref_fft_r2c(N, nf, self._p(u), self._p(out)), "fft_r2c")
        return out[0] if squeeze else out

    def fft_c2r(self, X: np.ndarray) -> np.ndarray:
        squeeze = X.ndim == 3
        N = X.shape[-2]
        X = self._spec(X, N)
        nf = X.shape[0]
        out = np.empty((nf, N, N, N), np.float64)
        self._check(self.lib.psref_fft_c2r(N, nf, self._p(X), self._p(out)), "fft_c2r")
        return out[0] if squeeze else out

    def dft_at(self, u: np.ndarray, kx, ky, kz) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64)
        N = u.shape[-1]
        kx, ky, kz = (np.ascontiguousarray(k, dtype=np.int32) for k in (kx, ky, kz))
        out = np.empty(len(kx), np.complex128)
        self._check(self.lib.psref_dft_at(N, self._p(u), len(kx), self._ip(kx), self._ip(ky),
                                          self._ip(kz), self._p(out)), "dft_at")
        return out

    def curl(self, uhat: np.ndarray) -> np.ndarray:
        N = uhat.shape[-2]
        uhat = self._spec(uhat, N, 3)
        out = np.empty_like(uhat)
        self._check(self.lib.psref_curl(N, self._p(uhat), self._p(out)), "curl")
        return out

    def nonlinear_ns(self, uhat: np.ndarray) -> np.ndarray:
        N = uhat.shape[-2]
        uhat = self._spec(uhat, N, 3)
        out = np.empty_like(uhat)
        self._check(self.lib.psref_nonlinear_ns(N, self._p(uhat), self._p(out)), "nonlinear_ns")
        return out

    def nonlinear_mhd(self, zhat: np.ndarray) -> np.ndarray:
        N = zhat.shape[-2]
        zhat = self._spec(zhat, N, 6)
        out = np.empty_like(zhat)
        self._check(self.lib.psref_nonlinear_mhd(N, self._p(zhat), self._p(out)),
                    "nonlinear_mhd")
        return out

    def nonlinear_at(self, fhat: np.ndarray, model: int, kx, ky, kz) -> np.ndarray:
        N = fhat.shape[-2]
        nf = 3 if model == NS else 6
        fhat = self._spec(fhat, N, nf)
        kx, ky, kz = (np.ascontiguousarray(k, dtype=np.int32) for k in (kx, ky, kz))
        out = np.empty((len(kx), nf), np.complex128)
        self._check(self.lib.psref_nonlinear_at(N, model, self._p(fhat), len(kx), self._ip(kx),
                                                self._ip(ky), self._ip(kz), self._p(out)),
                    "nonlinear_at")
        return out

    def rk2_step(self, state: np.ndarray, model: int, nu: float, eta: float, dt: float,
                 nsteps: int = 1, omega=None) -> np.ndarray:
        """Returns a new array (the argument is not modified).  omega: the
        frame's rotation vector (Coriolis term), or None."""
        N = state.shape[-2]
        nf = 3 if model == NS else 6
        z = self._spec(state, N, nf).copy()
        if omega is None:
            rc = self.lib.psref_rk2_step(N, model, self._p(z), float(nu), float(eta), float(dt),
                                         int(nsteps))
        else:
            om = np.ascontiguousarray(omega, dtype=np.float64).reshape(3)
            rc = self.lib.psref_rk2_step_rot(N, model, self._p(z), float(nu), float(eta),
                                             float(dt), int(nsteps), self._p(om))
        self._check(rc, "rk2_step")
        return z

    def set_box(self, Lx: float = 2 * math.pi, Ly: float = 2 * math.pi, Lz: float = 2 * math.pi):
        """Box lengths for every later call (process-wide; default 2 pi)."""
        self._check(self.lib.psref_set_box(float(Lx), float(Ly), float(Lz)), "set_box")

    def num_shells(self, N: int) -> int:
        return int(self.lib.psref_num_shells(N))

    def energy_spectrum(self, fhat: np.ndarray):
        N = fhat.shape[-2]
        fhat = self._spec(fhat, N)
        nf = fhat.shape[0]
        spec = np.empty(self.num_shells(N), np.float64)
        tot = np.empty(3, np.float64)
        self._check(self.lib.psref_energy_spectrum(N, nf, self._p(fhat), self._p(spec),
                                                   self._p(tot)), "energy_spectrum")
        return spec, tot


_default: Optional[Oracle] = None


def oracle() -> Oracle:
    """The default (unmutated) oracle, built on first use if absent."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default
