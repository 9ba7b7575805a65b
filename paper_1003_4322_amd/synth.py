"""Seeded synthetic inputs: random-phase solenoidal fields and closed-form flows.

This module produces *input data* only.  It is shared by the tests, the
benchmark and the oracle-side checks, and it contains none of the step's
arithmetic: no transform, no curl, no projection operator, no dealiasing of a
computed term and no time stepping.  Solenoidal random fields are made as
``k x a`` of a random complex vector ``a`` (divergence-free by construction),
not with the projector the step uses.

Spectral arrays are half spectra ``[f][kz][ky][kx]``, kx = 0..N/2, holding the
normalised Fourier coefficients u(x) = sum_k u_k exp(i k.x) on [0, 2 pi)^3.

Random numbers come from a counter-based generator: SplitMix64 (Steele, Lea &
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) evaluated
at a counter, 53-bit uniforms, and the Box-Muller transform.  A mode's value
therefore depends only on (seed, storage index, component), never on the order
in which modes are generated or on how much of the spectrum is materialised.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Iterable, Sequence, Tuple

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_mix(z: np.ndarray) -> np.ndarray:
    """The SplitMix64 output function (finaliser) on uint64 values."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform53(seed: int, ctr: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1): SplitMix64 state seed' + (ctr+1) * gamma,
    with seed' = mix(seed), top 53 bits."""
    s0 = splitmix64_mix(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]
    ctr = np.asarray(ctr, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = splitmix64_mix(s0 + (ctr + np.uint64(1)) * _GAMMA)
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def box_muller(u1: np.ndarray, u2: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    r = np.sqrt(-2.0 * np.log1p(-u1))  # 1 - u1 in (0, 1]
    t = 2.0 * math.pi * u2
    return r * np.cos(t), r * np.sin(t)


def shape_spectrum(s: np.ndarray, k0: float) -> np.ndarray:
    """Target shell energy shape E(s) ~ s^4 exp(-2 (s/k0)^2)."""
    s = np.asarray(s, dtype=np.float64)
    return s ** 4 * np.exp(-2.0 * (s / k0) ** 2)


def shell_index(k2: np.ndarray) -> np.ndarray:
    """round(|k|) in exact integer arithmetic: smallest s with 4 k2 < (2s+1)^2."""
    k2 = np.asarray(k2, dtype=np.int64)
    s = np.floor(np.sqrt(k2.astype(np.float64))).astype(np.int64)
    s = np.where((s > 0) & (4 * k2 < (2 * s - 1) ** 2), s - 1, s)
    s = np.where(4 * k2 >= (2 * s + 1) ** 2, s + 1, s)
    return s


@dataclass
class SparseField:
    """A half-spectrum vector field given on a cube of low wavenumbers.

    kx in [0, K], ky and kz in [-K, K]; ``values[c, iz, iy, ix]`` with
    iz = kz + K, iy = ky + K, ix = kx.  Every mode outside the cube is zero.
    """

    N: int
    K: int
    values: np.ndarray  # complex128 [ncomp, 2K+1, 2K+1, K+1]

    def dense(self, dtype=np.complex128) -> np.ndarray:
        N, K = self.N, self.K
        out = np.zeros((self.values.shape[0], N, N, N // 2 + 1), dtype=dtype)
        kk = np.arange(-K, K + 1) % N
        out[:, kk[:, None], kk[None, :], : K + 1] = self.values.astype(dtype)
        return out

    def dense_xyz(self, nx: int, ny: int, nz: int, dtype=np.complex128) -> np.ndarray:
        """The same modes scattered into an nx x ny x nz grid's half spectrum
        [c][kz][ky][kx] (each axis long enough to hold them)."""
        K = self.K
        if 2 * K >= min(nx, ny, nz) or K > nx // 2:
            raise ValueError("grid too small for the field's modes")
        out = np.zeros((self.values.shape[0], nz, ny, nx // 2 + 1), dtype=dtype)
        kr = np.arange(-K, K + 1)
        out[:, (kr % nz)[:, None], (kr % ny)[None, :], : K + 1] = self.values.astype(dtype)
        return out

    def index_arrays(self):
        """(iz, iy, ix) storage indices of the cube, for scattering elsewhere."""
        K, N = self.K, self.N
        kk = np.arange(-K, K + 1) % N
        return kk, kk, np.arange(K + 1)

    def __add__(self, other: "SparseField") -> "SparseField":
        assert self.N == other.N and self.K == other.K
        return SparseField(self.N, self.K, self.values + other.values)

    def __sub__(self, other: "SparseField") -> "SparseField":
        assert self.N == other.N and self.K == other.K
        return SparseField(self.N, self.K, self.values - other.values)


def _last_nonzero_shell(k0: float, smax: int) -> int:
    s = np.arange(smax + 1)
    nz = np.nonzero(shape_spectrum(s, k0) > 0)[0]
    return int(nz[-1]) if len(nz) else 0


def random_solenoidal(N: int, seed: int, k0: float, energy: float = 0.5) -> SparseField:
    """Random-phase, divergence-free, zero-mean field on the kept sphere
    9|k|^2 < N^2, with shell energies E(s) = C s^4 exp(-2 (s/k0)^2) and total
    energy 1/2 <|u|^2> = ``energy``.

    Steps: complex Gaussian vector a(k) per mode from (seed, storage index,
    component); v = k x a; the kx = 0 plane replaced by its Hermitian part;
    k = 0 and modes outside the sphere zeroed; each shell rescaled to its
    target energy.
    """
    if N < 4 or N % 2:
        raise ValueError("N must be even and >= 4")
    H = N // 2 + 1
    kmax_sphere = (N - 1) // 3  # |k_i| < N/3 on the kept sphere
    # largest shell present in the kept sphere
    s_sphere = int(shell_index(np.array([(N * N - 1) // 9]))[0])
    s_last = _last_nonzero_shell(k0, s_sphere)
    K = max(1, min(kmax_sphere, s_last))
    kr = np.arange(-K, K + 1)
    KZ, KY, KX = np.meshgrid(kr, kr, np.arange(K + 1), indexing="ij")
    # counters from the storage index in the full N-grid
    m = ((KZ % N) * N + (KY % N)) * H + KX
    a = np.empty((3,) + KZ.shape, np.complex128)
    for c in range(3):
        ctr = (m.astype(np.uint64) * np.uint64(3) + np.uint64(c)) * np.uint64(2)
        re, im = box_muller(uniform53(seed, ctr), uniform53(seed, ctr + np.uint64(1)))
        a[c] = re + 1j * im
    kx, ky, kz = KX.astype(np.float64), KY.astype(np.float64), KZ.astype(np.float64)
    v = np.empty_like(a)
    v[0] = ky * a[2] - kz * a[1]
    v[1] = kz * a[0] - kx * a[2]
    v[2] = kx * a[1] - ky * a[0]
    # kx = 0 plane: Hermitian part, v(0,ky,kz) = conj(v(0,-ky,-kz))
    p0 = v[:, :, :, 0]
    v[:, :, :, 0] = 0.5 * (p0 + np.conj(p0[:, ::-1, ::-1]))
    k2 = KX * KX + KY * KY + KZ * KZ
    keep = (9 * k2 < N * N) & (k2 > 0)
    v *= keep
    # shell rescaling
    w = np.where(KX == 0, 1.0, 2.0)
    e_mode = 0.5 * w * np.sum(np.abs(v) ** 2, axis=0)
    shell = shell_index(k2)
    nshell = int(shell.max()) + 1
    e_raw = np.bincount(shell.ravel(), weights=e_mode.ravel(), minlength=nshell)
    # normalisation over every shell of the kept sphere
    s_all = np.arange(1, s_sphere + 1)
    C = energy / np.sum(shape_spectrum(s_all, k0))
    target = C * shape_spectrum(np.arange(nshell), k0)
    target[0] = 0.0
    scale = np.zeros(nshell)
    ok = e_raw > 0
    scale[ok] = np.sqrt(target[ok] / e_raw[ok])
    v *= scale[shell]
    return SparseField(N, K, v)


def random_grid(nx: int, ny: int, nz: int, seed: int, k0: float, energy: float = 0.5,
                dtype=np.complex128) -> np.ndarray:
    """Dense random-phase, divergence-free, zero-mean field [3][kz][ky][kx] on
    an nx x ny x nz grid, filling the kept region (3kx/nx)^2 + (3ky/ny)^2 +
    (3kz/nz)^2 < 1 with amplitudes |k| exp(-(|k|/k0)^2) (|k| of the index) and
    total energy 1/2 <|u|^2> = ``energy``.

    Steps as in random_solenoidal: complex Gaussian a(k) from (seed, storage
    index, component); v = k x a; the kx = 0 plane replaced by its Hermitian
    part; k = 0 and modes outside the kept region zeroed; then scaled.
    """
    H = nx // 2 + 1
    kz = np.where(np.arange(nz) < nz // 2, np.arange(nz), np.arange(nz) - nz)
    ky = np.where(np.arange(ny) < ny // 2, np.arange(ny), np.arange(ny) - ny)
    KZ, KY, KX = np.meshgrid(kz, ky, np.arange(H), indexing="ij")
    m = (np.arange(nz)[:, None, None] * ny + np.arange(ny)[None, :, None]) * H + np.arange(H)
    a = np.empty((3,) + KZ.shape, np.complex128)
    for c in range(3):
        ctr = (m.astype(np.uint64) * np.uint64(3) + np.uint64(c)) * np.uint64(2)
        re, im = box_muller(uniform53(seed, ctr), uniform53(seed, ctr + np.uint64(1)))
        a[c] = re + 1j * im
    fx, fy, fz = KX.astype(np.float64), KY.astype(np.float64), KZ.astype(np.float64)
    v = np.empty_like(a)
    v[0] = fy * a[2] - fz * a[1]
    v[1] = fz * a[0] - fx * a[2]
    v[2] = fx * a[1] - fy * a[0]
    # Hermitian part of the kx = 0 plane: v(0, ky, kz) = conj(v(0, -ky, -kz))
    iy, iz = (-np.arange(ny)) % ny, (-np.arange(nz)) % nz
    p0 = v[:, :, :, 0]
    v[:, :, :, 0] = 0.5 * (p0 + np.conj(p0[:, iz[:, None], iy[None, :]]))
    # kept region in exact integers: 9 (kx^2 (ny nz)^2 + ...) < (nx ny nz)^2,
    # below 2^63 for axis lengths up to 1024
    X, Y, Z = np.int64(nx), np.int64(ny), np.int64(nz)
    KX64, KY64, KZ64 = KX.astype(np.int64), KY.astype(np.int64), KZ.astype(np.int64)
    q = 9 * (KX64 ** 2 * (Y * Z) ** 2 + KY64 ** 2 * (X * Z) ** 2 + KZ64 ** 2 * (X * Y) ** 2)
    k2 = KX * KX + KY * KY + KZ * KZ
    keep = (q < (X * Y * Z) ** 2) & (k2 > 0)
    kk = np.sqrt(k2.astype(np.float64))
    v *= keep * np.exp(-(kk / k0) ** 2)
    w = np.where(KX == 0, 1.0, 2.0)
    w[..., -1] = 1.0
    e = 0.5 * np.sum(w * np.sum(np.abs(v) ** 2, axis=0))
    v *= math.sqrt(energy / e)
    return v.astype(dtype)


def target_spectrum(N: int, k0: float, energy: float = 0.5) -> np.ndarray:
    """Shell energies the generator aims at, for shells 0..s(3 (N/2)^2)."""
    s_sphere = int(shell_index(np.array([(N * N - 1) // 9]))[0])
    nsh = int(shell_index(np.array([3 * (N // 2) ** 2]))[0]) + 1
    C = energy / np.sum(shape_spectrum(np.arange(1, s_sphere + 1), k0))
    t = C * shape_spectrum(np.arange(nsh), k0)
    t[0] = 0.0
    t[s_sphere + 1:] = 0.0
    return t


def random_ns(N: int, seed: int, k0: float, energy: float = 0.5,
              dtype=np.complex128) -> np.ndarray:
    """Dense NS velocity state [3][kz][ky][kx]."""
    return random_solenoidal(N, seed, k0, energy).dense(dtype)


def mhd_sparse(N: int, seed_u: int, seed_b: int, k0: float, eu: float = 0.5,
               eb: float = 0.5) -> SparseField:
    """Elsasser state z+ = u + b (components 0..2), z- = u - b (3..5)."""
    u = random_solenoidal(N, seed_u, k0, eu)
    b = random_solenoidal(N, seed_b, k0, eb)
    return SparseField(N, u.K, np.concatenate([(u + b).values, (u - b).values]))


def random_mhd(N: int, seed_u: int, seed_b: int, k0: float, eu: float = 0.5, eb: float = 0.5,
               dtype=np.complex128) -> np.ndarray:
    return mhd_sparse(N, seed_u, seed_b, k0, eu, eb).dense(dtype)


def ensemble_k0(seed: int) -> float:
    """k0 drawn uniformly in [2, 5] from the box's own seed."""
    return 2.0 + 3.0 * float(uniform53(seed, np.array([2 ** 40], dtype=np.uint64))[0])


# ---------------------------------------------------------------------------
# Closed-form flows written as sums of complex exponentials.
# ---------------------------------------------------------------------------

def _trig_terms(factors: Sequence[Tuple[str, int]]):
    """Expand prod_axis f_axis(k_axis * x_axis), f in {sin, cos}, over (x, y, z)
    into complex exponentials: yields (kx, ky, kz, coefficient)."""
    per_axis = []
    for kind, k in factors:
        if k == 0:
            per_axis.append([(0, 1.0 + 0j)] if kind == "cos" else [])
        elif kind == "cos":
            per_axis.append([(k, 0.5 + 0j), (-k, 0.5 + 0j)])
        else:  # sin t = (e^{it} - e^{-it}) / (2i)
            per_axis.append([(k, -0.5j), (-k, 0.5j)])
    if any(len(p) == 0 for p in per_axis):
        return
    for ax, ca in per_axis[0]:
        for ay, cb in per_axis[1]:
            for az, cc in per_axis[2]:
                yield ax, ay, az, ca * cb * cc


def trig_field(N: int, components: Iterable[Iterable[Tuple[float, Sequence[Tuple[str, int]]]]],
               dtype=np.complex128) -> np.ndarray:
    """Half spectrum of a real vector field given per component as a sum of
    amp * f(kx x) g(ky y) h(kz z).  Terms with kx < 0 are the conjugate
    partners of stored ones and are not stored."""
    comps = list(components)
    out = np.zeros((len(comps), N, N, N // 2 + 1), np.complex128)
    for c, terms in enumerate(comps):
        for amp, factors in terms:
            for kx, ky, kz, coef in _trig_terms(factors):
                if kx < 0:
                    continue
                out[c, kz % N, ky % N, kx] += amp * coef
    return out.astype(dtype)


def abc_flow(N: int, A: float = 1.0, B: float = 1.0, C: float = 1.0, k: int = 1,
             dtype=np.complex128) -> np.ndarray:
    """Arnold-Beltrami-Childress flow at wavenumber k:
    u = (A sin kz + C cos ky, B sin kx + A cos kz, C sin ky + B cos kx)."""
    return trig_field(N, [
        [(A, [("cos", 0), ("cos", 0), ("sin", k)]), (C, [("cos", 0), ("cos", k), ("cos", 0)])],
        [(B, [("sin", k), ("cos", 0), ("cos", 0)]), (A, [("cos", 0), ("cos", 0), ("cos", k)])],
        [(C, [("cos", 0), ("sin", k), ("cos", 0)]), (B, [("cos", k), ("cos", 0), ("cos", 0)])],
    ], dtype)


def taylor_green(N: int, dtype=np.complex128) -> np.ndarray:
    """u = (sin x cos y cos z, -cos x sin y cos z, 0)."""
    return trig_field(N, [
        [(1.0, [("sin", 1), ("cos", 1), ("cos", 1)])],
        [(-1.0, [("cos", 1), ("sin", 1), ("cos", 1)])],
        [],
    ], dtype)


def band_limited(N: int, seed: int, kmax: int, energy: float = 0.5) -> SparseField:
    """Random solenoidal field supported on |k| <= kmax with a flat shell
    spectrum (used to embed a small-grid problem exactly in a large grid)."""
    H = N // 2 + 1
    K = kmax
    kr = np.arange(-K, K + 1)
    KZ, KY, KX = np.meshgrid(kr, kr, np.arange(K + 1), indexing="ij")
    m = ((KZ % N) * N + (KY % N)) * H + KX
    a = np.empty((3,) + KZ.shape, np.complex128)
    for c in range(3):
        ctr = (m.astype(np.uint64) * np.uint64(3) + np.uint64(c)) * np.uint64(2)
        re, im = box_muller(uniform53(seed, ctr), uniform53(seed, ctr + np.uint64(1)))
        a[c] = re + 1j * im
    kx, ky, kz = KX.astype(np.float64), KY.astype(np.float64), KZ.astype(np.float64)
    v = np.stack([ky * a[2] - kz * a[1], kz * a[0] - kx * a[2], kx * a[1] - ky * a[0]])
    p0 = v[:, :, :, 0]
    v[:, :, :, 0] = 0.5 * (p0 + np.conj(p0[:, ::-1, ::-1]))
    k2 = KX * KX + KY * KY + KZ * KZ
    v *= (k2 <= kmax * kmax) & (k2 > 0)
    w = np.where(KX == 0, 1.0, 2.0)
    e = 0.5 * np.sum(w * np.sum(np.abs(v) ** 2, axis=0))
    v *= math.sqrt(energy / e)
    return SparseField(N, K, v)


def _flat_group(N: int, seed: int, kz: int, kyr: np.ndarray, kxr: np.ndarray) -> np.ndarray:
    """v = k x a / |k| at storage plane kz, rows ky in kyr (storage indices) and
    columns kx in kxr: a complex Gaussian 3-vector a per mode from (seed,
    storage index, component), so every mode has the same expected size."""
    H = N // 2 + 1
    KY, KX = np.meshgrid(kyr, kxr, indexing="ij")
    m = (np.int64(kz) * N + KY) * H + KX
    a = np.empty((3,) + KY.shape, np.complex128)
    for c in range(3):
        ctr = (m.astype(np.uint64) * np.uint64(3) + np.uint64(c)) * np.uint64(2)
        re, im = box_muller(uniform53(seed, ctr), uniform53(seed, ctr + np.uint64(1)))
        a[c] = re + 1j * im
    wz = kz if kz < N // 2 else kz - N
    ky = np.where(KY < N // 2, KY, KY - N).astype(np.float64)
    kx = KX.astype(np.float64)
    kn = np.sqrt(kx * kx + ky * ky + float(wz * wz))
    kn[kn == 0] = 1.0
    return np.stack([ky * a[2] - wz * a[1], wz * a[0] - kx * a[2], kx * a[1] - ky * a[0]]) / kn


def flat_solenoidal(N: int, seed: int, groups: int = 1, energy: float = 0.5,
                    dtype=np.complex128) -> np.ndarray:
    """Dense field [3 groups][kz][ky][kx] of solenoidal 3-vectors whose modes
    fill the kept sphere 9|k|^2 < N^2 (k != 0) with the same expected
    amplitude at every |k| (a flat spectrum up to the 2/3 edge), zero outside;
    the kx = 0 plane is replaced by its Hermitian part.  Group g uses seed + g
    and is scaled to total energy ``energy``.  Only the planes |kz| < N/3 are
    generated (the others are zero), one plane at a time."""
    H = N // 2 + 1
    K = (N - 1) // 3                      # |k_i| <= K inside the sphere
    kr = np.concatenate([np.arange(0, K + 1), np.arange(N - K, N)])   # storage rows
    kxr = np.arange(K + 1)
    out = np.zeros((3 * groups, N, N, H), dtype=dtype)
    wy = np.where(kr < N // 2, kr, kr - N)
    for g in range(groups):
        e = 0.0
        for kz in kr:
            wz = kz if kz < N // 2 else kz - N
            v = _flat_group(N, seed + g, int(kz), kr, kxr)
            # Hermitian part of the kx = 0 column: v(0, ky, kz) = conj v(0, -ky, -kz)
            mz = (-int(kz)) % N
            mrow = (-kr) % N
            w0 = _flat_group(N, seed + g, mz, mrow, np.array([0]))[..., 0]
            v[..., 0] = 0.5 * (v[..., 0] + np.conj(w0))
            k2 = wy[:, None] ** 2 + kxr[None, :] ** 2 + wz * wz
            keep = (9 * k2 < N * N) & (k2 > 0)
            v *= keep
            w = np.where(kxr == 0, 1.0, 2.0)[None, :]
            e += 0.5 * float(np.sum(w * np.sum(np.abs(v) ** 2, axis=0)))
            out[3 * g:3 * g + 3, kz, kr[:, None], kxr[None, :]] = v.astype(dtype)
        out[3 * g:3 * g + 3] *= np.asarray(math.sqrt(energy / e), dtype=np.float64).astype(
            out.real.dtype)
    return out


def embed(f: SparseField, N: int) -> SparseField:
    """The same low-wavenumber coefficients on a grid of size N."""
    assert f.K < N // 3 or f.K < N // 2
    return SparseField(N, f.K, f.values.copy())
