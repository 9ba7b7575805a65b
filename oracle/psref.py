"""FP64 CPU oracle for the pseudospectral step -- Python binding.

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this module.  The product path
(the HIP library and its binding) never imports it.

The arithmetic lives in ``psref.c`` (plain C, FP64); this module only builds
and loads that library and marshals numpy arrays.  Every array is C-contiguous:
real fields ``float64[nf, nz, ny, nx]`` ([f][z][y][x]) and half spectra
``complex128[nf, nz, ny, nx//2+1]`` ([f][kz][ky][kx]); the cube is nx = ny = nz.
"""
from __future__ import annotations

import ctypes
import hashlib
import math
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "psref.c")
LIB = os.path.join(HERE, "libpsref.so")

NS, MHD = 0, 1


def src_hash() -> str:
    """SHA-256 (16 hex digits) of psref.c and psref.h."""
    h = hashlib.sha256()
    for f in (SRC, os.path.join(HERE, "psref.h")):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(mutant: int = 0, out: Optional[str] = None, openmp: bool = True) -> str:
    """Compile psref.c with gcc.  ``mutant`` > 0 plants the numbered mistake
    (used only by the mutation tests).  Returns the path of the library."""
    out = out or LIB
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-Wno-unused-parameter", f"-DPSREF_MUTANT={int(mutant)}",
           f'-DPSREF_SRC_HASH="{src_hash()}"', SRC, "-o", out, "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


class Oracle:
    """ctypes wrapper around one build of the oracle library.  Grid sizes are
    taken from the array shapes: real fields ``[nf, nz, ny, nx]``, half
    spectra ``[nf, nz, ny, nx//2+1]`` (nx even)."""

    def __init__(self, path: Optional[str] = None):
        path = path or LIB
        if not os.path.exists(path):
            if path != LIB:
                raise FileNotFoundError(path)
            build()
        self.lib = ctypes.CDLL(path)
        self.lib.psref_build_hash.restype = ctypes.c_char_p
        have, want = self.lib.psref_build_hash().decode(), src_hash()
        if have != want:
            raise RuntimeError(f"{path} was built from other sources (hash {have}, sources {want}):"
                               " rebuild it with oracle.psref.build()")
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i = ctypes.c_int
        d = ctypes.c_double
        L = self.lib
        L.psref_set_threads.argtypes = [i]
        L.psref_fft_r2c.argtypes = [i, i, i, i, dp, dp]
        L.psref_fft_c2r.argtypes = [i, i, i, i, dp, dp]
        L.psref_dft_at.argtypes = [i, i, i, dp, i, ip, ip, ip, dp]
        L.psref_curl.argtypes = [i, i, i, dp, dp]
        L.psref_nonlinear_ns.argtypes = [i, i, i, dp, dp]
        L.psref_nonlinear_mhd.argtypes = [i, i, i, dp, dp]
        L.psref_nonlinear_at.argtypes = [i, i, i, i, dp, i, ip, ip, ip, dp]
        L.psref_rk2_step.argtypes = [i, i, i, i, dp, d, d, d, i]
        L.psref_rk2_step_rot.argtypes = [i, i, i, i, dp, d, d, d, i, dp]
        L.psref_set_box.argtypes = [d, d, d]
        L.psref_num_shells.argtypes = [i, i, i]
        L.psref_energy_spectrum.argtypes = [i, i, i, i, dp, dp, dp]
        L.psref_mhd_spectrum.argtypes = [i, i, i, dp, dp, dp]

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
    def _spec(a, nf: Optional[int] = None):
        """(array [nf, nz, ny, H], (nx, ny, nz)) with nx = 2 (H - 1)."""
        a = np.ascontiguousarray(a, dtype=np.complex128)
        if a.ndim == 3:
            a = a[None]
        if a.ndim != 4 or a.shape[-1] < 2 or (nf is not None and a.shape[0] != nf):
            raise ValueError(f"bad spectral shape {a.shape}")
        nz, ny, H = a.shape[1:]
        return a, (2 * (H - 1), ny, nz)

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
        nf, nz, ny, nx = u.shape
        out = np.empty((nf, nz, ny, nx // 2 + 1), np.complex128)
        self._check(self.lib.psref_fft_r2c(nx, ny, nz, nf, self._p(u), self._p(out)), "fft_r2c")
        return out[0] if squeeze else out

    def fft_c2r(self, X: np.ndarray) -> np.ndarray:
        squeeze = X.ndim == 3
        X, (nx, ny, nz) = self._spec(X)
        nf = X.shape[0]
        out = np.empty((nf, nz, ny, nx), np.float64)
        self._check(self.lib.psref_fft_c2r(nx, ny, nz, nf, self._p(X), self._p(out)), "fft_c2r")
        return out[0] if squeeze else out

    def dft_at(self, u: np.ndarray, kx, ky, kz) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64)
        nz, ny, nx = u.shape[-3:]
        kx, ky, kz = (np.ascontiguousarray(k, dtype=np.int32) for k in (kx, ky, kz))
        out = np.empty(len(kx), np.complex128)
        self._check(self.lib.psref_dft_at(nx, ny, nz, self._p(u), len(kx), self._ip(kx),
                                          self._ip(ky), self._ip(kz), self._p(out)), "dft_at")
        return out

    def curl(self, uhat: np.ndarray) -> np.ndarray:
        uhat, n = self._spec(uhat, 3)
        out = np.empty_like(uhat)
        self._check(self.lib.psref_curl(*n, self._p(uhat), self._p(out)), "curl")
        return out

    def nonlinear_ns(self, uhat: np.ndarray) -> np.ndarray:
        uhat, n = self._spec(uhat, 3)
        out = np.empty_like(uhat)
        self._check(self.lib.psref_nonlinear_ns(*n, self._p(uhat), self._p(out)), "nonlinear_ns")
        return out

    def nonlinear_mhd(self, zhat: np.ndarray) -> np.ndarray:
        zhat, n = self._spec(zhat, 6)
        out = np.empty_like(zhat)
        self._check(self.lib.psref_nonlinear_mhd(*n, self._p(zhat), self._p(out)),
                    "nonlinear_mhd")
        return out

    def nonlinear_at(self, fhat: np.ndarray, model: int, kx, ky, kz) -> np.ndarray:
        nf = 3 if model == NS else 6
        fhat, n = self._spec(fhat, nf)
        kx, ky, kz = (np.ascontiguousarray(k, dtype=np.int32) for k in (kx, ky, kz))
        out = np.empty((len(kx), nf), np.complex128)
        self._check(self.lib.psref_nonlinear_at(*n, model, self._p(fhat), len(kx), self._ip(kx),
                                                self._ip(ky), self._ip(kz), self._p(out)),
                    "nonlinear_at")
        return out

    def rk2_step(self, state: np.ndarray, model: int, nu: float, eta: float, dt: float,
                 nsteps: int = 1, omega=None) -> np.ndarray:
        """Returns a new array (the argument is not modified).  omega: the
        frame's rotation vector (Coriolis term), or None."""
        nf = 3 if model == NS else 6
        z, n = self._spec(state, nf)
        z = z.copy()
        if omega is None:
            rc = self.lib.psref_rk2_step(*n, model, self._p(z), float(nu), float(eta), float(dt),
                                         int(nsteps))
        else:
            om = np.ascontiguousarray(omega, dtype=np.float64).reshape(3)
            rc = self.lib.psref_rk2_step_rot(*n, model, self._p(z), float(nu), float(eta),
                                             float(dt), int(nsteps), self._p(om))
        self._check(rc, "rk2_step")
        return z

    def set_box(self, Lx: float = 2 * math.pi, Ly: float = 2 * math.pi, Lz: float = 2 * math.pi):
        """Box lengths for every later call (process-wide; default 2 pi)."""
        self._check(self.lib.psref_set_box(float(Lx), float(Ly), float(Lz)), "set_box")

    def num_shells(self, nx: int, ny: Optional[int] = None, nz: Optional[int] = None) -> int:
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        return int(self.lib.psref_num_shells(nx, ny, nz))

    def energy_spectrum(self, fhat: np.ndarray):
        fhat, n = self._spec(fhat)
        nf = fhat.shape[0]
        spec = np.empty(self.num_shells(*n), np.float64)
        tot = np.empty(3, np.float64)
        self._check(self.lib.psref_energy_spectrum(*n, nf, self._p(fhat), self._p(spec),
                                                   self._p(tot)), "energy_spectrum")
        return spec, tot

    def mhd_spectrum(self, zhat: np.ndarray):
        """(spec[3, nshell] = [Eu(s), Eb(s), Hc(s)], totals [Eu, Eb, Hc]) of an
        Elsasser state (6 fields)."""
        zhat, n = self._spec(zhat, 6)
        ns = self.num_shells(*n)
        spec = np.empty(3 * ns, np.float64)
        tot = np.empty(3, np.float64)
        self._check(self.lib.psref_mhd_spectrum(*n, self._p(zhat), self._p(spec), self._p(tot)),
                    "mhd_spectrum")
        return spec.reshape(3, ns), tot


_default: Optional[Oracle] = None


def oracle() -> Oracle:
    """The default (unmutated) oracle, built on first use if absent."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default
