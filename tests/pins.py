"""Pins for the FP64 oracle: checks against what the mathematics fixes.

Every function here takes an oracle instance and raises AssertionError when
the oracle disagrees with a definition written out directly (a literal DFT
sum, a literal triad sum), a closed form (ABC and Taylor-Green flows, a single
Fourier mode), an invariant (energy, helicity and Elsasser-energy
conservation of the dealiased quadratic term, solenoidality), a library
special case (numpy's real FFT) or a convergence order.  The same functions
run against deliberately broken builds of the oracle in the mutation tests,
which check that every planted mistake trips at least one pin.

The paper prints no worked numerical example, so no pin quotes a number from
it; each pin names the passage whose mathematics it checks.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from oracle.psref import MHD, NS
from paper_1003_4322_amd import synth

TWO_PI = 2.0 * math.pi


def _rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = max(np.linalg.norm(b.ravel()), 1e-300)
    return float(np.linalg.norm((a - b).ravel()) / den)


def _hweights(N: int) -> np.ndarray:
    w = np.full(N // 2 + 1, 2.0)
    w[0] = 1.0
    w[-1] = 1.0
    return w


def _wavenumbers(N: int):
    """Signed wavenumber grids (KZ, KY, KX) over the half-spectrum storage."""
    k = np.where(np.arange(N) < N // 2, np.arange(N), np.arange(N) - N)
    return np.meshgrid(k, k, np.arange(N // 2 + 1), indexing="ij")


def _grid(N: int):
    x = TWO_PI * np.arange(N) / N
    return np.meshgrid(x, x, x, indexing="ij")  # Z, Y, X


def _random_half(rng, nf, N):
    s = (nf, N, N, N // 2 + 1)
    return rng.standard_normal(s) + 1j * rng.standard_normal(s)


# ---------------------------------------------------------------------------
# Transforms (Sec. 2: FFT of real N^3 data into an (N/2+1) x N x N half
# spectrum, Fig. 1).
# ---------------------------------------------------------------------------

def brute_r2c(u: np.ndarray) -> np.ndarray:
    """X(k) = sum_x u(x) exp(-i k.x), literally: every k against every x
    (u is [nz, ny, nx]; the phase of each axis is taken modulo its length)."""
    nz, ny, nx = u.shape
    H = nx // 2 + 1
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(H), indexing="ij")
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ph = (np.outer(kx.ravel(), x.ravel()) % nx / nx + np.outer(ky.ravel(), y.ravel()) % ny / ny
          + np.outer(kz.ravel(), z.ravel()) % nz / nz)
    return (np.exp(-1j * TWO_PI * ph) @ u.ravel()).reshape(nz, ny, H)


def brute_c2r(X: np.ndarray) -> np.ndarray:
    """The inverse in pass order: inverse sums along z and y on every kx plane,
    then u = Re Y_0 + 2 sum_{0<k<nx/2} Re(Y_k e^{ikx}) + Re Y_{nx/2} (-1)^x."""
    nz, ny, H = X.shape
    nx = 2 * (H - 1)

    def einv(n):  # [x, k]
        j = np.arange(n)
        return np.exp(1j * TWO_PI * (np.outer(j, j) % n) / n)

    Y = np.einsum("zc,cbk->zbk", einv(nz), X)   # along kz
    Y = np.einsum("yb,zbk->zyk", einv(ny), Y)   # along ky
    j = np.arange(nx)
    u = np.real(Y[..., 0])[..., None] * np.ones(nx)
    for k in range(1, nx // 2):
        u = u + 2.0 * np.real(Y[..., k][..., None] * np.exp(1j * TWO_PI * k * j / nx))
    u = u + np.real(Y[..., nx // 2])[..., None] * ((-1.0) ** j)
    return u


def pin_fft_brute(o):
    rng = np.random.default_rng(11)
    for N in (6, 8, 12):
        u = rng.standard_normal((N, N, N))
        got = o.fft_r2c(u)
        ref = brute_r2c(u)
        assert _rel(got, ref) < 1e-13, (N, _rel(got, ref))
        X = _random_half(rng, 1, N)[0]  # not Hermitian on the kx=0, N/2 planes
        got = o.fft_c2r(X)
        ref = brute_c2r(X)
        assert _rel(got, ref) < 1e-13, (N, _rel(got, ref))


def pin_fft_numpy(o):
    """numpy's rfftn/irfftn use the same sign, storage and pass conventions."""
    rng = np.random.default_rng(12)
    for N in (16, 24, 18):
        u = rng.standard_normal((2, N, N, N))
        assert _rel(o.fft_r2c(u), np.fft.rfftn(u, axes=(1, 2, 3))) < 1e-13
        X = _random_half(rng, 2, N)
        ref = np.fft.irfftn(X, s=(N, N, N), axes=(1, 2, 3)) * N ** 3
        assert _rel(o.fft_c2r(X), ref) < 1e-13


def pin_fft_parseval_roundtrip(o):
    rng = np.random.default_rng(13)
    N = 16
    u = rng.standard_normal((N, N, N))
    X = o.fft_r2c(u)
    lhs = np.sum(u * u)
    rhs = np.sum(_hweights(N) * np.abs(X) ** 2) / N ** 3
    assert abs(lhs - rhs) / lhs < 1e-13
    assert _rel(o.fft_c2r(X), N ** 3 * u) < 1e-13


def pin_fft_single_mode(o):
    N = 16
    Z, Y, X = _grid(N)
    k = (3, -5, 2)  # (kx, ky, kz)
    u = np.cos(k[0] * X + k[1] * Y + k[2] * Z + 0.7)
    F = o.fft_r2c(u)
    expect = np.zeros_like(F)
    expect[k[2] % N, k[1] % N, k[0]] = 0.5 * N ** 3 * np.exp(1j * 0.7)
    assert np.abs(F - expect).max() < 1e-10 * N ** 3


def pin_dft_at(o):
    rng = np.random.default_rng(14)
    N = 8
    u = rng.standard_normal((N, N, N))
    ref = brute_r2c(u)
    kx = np.array([0, 1, 4, 3]); ky = np.array([0, 7, 4, 2]); kz = np.array([5, 0, 4, 6])
    got = o.dft_at(u, kx, ky, kz)
    assert np.abs(got - ref[kz, ky, kx]).max() < 1e-12


# ---------------------------------------------------------------------------
# Spectral curl (derivatives of the Fourier expansion, Sec. 2)
# ---------------------------------------------------------------------------

def pin_curl_abc(o):
    """ABC flows are Beltrami fields: curl u = k u at wavenumber k."""
    N = 16
    for k in (1, 3):
        u = synth.abc_flow(N, 1.0, 0.7, 0.4, k=k)
        assert np.abs(o.curl(u) - k * u).max() < 1e-14


def pin_curl_single_modes(o):
    """u = a cos(k.x + phi) differentiates exactly; checked on the grid."""
    N = 16
    Z, Y, X = _grid(N)
    rng = np.random.default_rng(15)
    for _ in range(4):
        k = rng.integers(-7, 8, size=3)
        a = rng.standard_normal(3)
        ph = rng.uniform(0, TWO_PI)
        arg = k[0] * X + k[1] * Y + k[2] * Z + ph
        u = np.stack([a[c] * np.cos(arg) for c in range(3)])
        uhat = np.fft.rfftn(u, axes=(1, 2, 3)) / N ** 3
        w = np.fft.irfftn(o.curl(uhat), s=(N, N, N), axes=(1, 2, 3)) * N ** 3
        s = -np.sin(arg)  # d/dx_j cos(k.x+ph) = -k_j sin(.)
        ex = np.stack([(k[1] * a[2] - k[2] * a[1]) * s, (k[2] * a[0] - k[0] * a[2]) * s,
                       (k[0] * a[1] - k[1] * a[0]) * s])
        assert np.abs(w - ex).max() < 1e-12, (k, np.abs(w - ex).max())


def pin_curl_nyquist(o):
    """cos(N y / 2) is (-1)^j on the grid, where its derivative vanishes:
    the spectral derivative of the Nyquist mode must be zero there."""
    N = 12
    Z, Y, X = _grid(N)
    u = np.stack([np.cos(N // 2 * Y) * np.cos(X), np.zeros_like(X), np.cos(N // 2 * Z) * np.sin(2 * X)])
    uhat = np.fft.rfftn(u, axes=(1, 2, 3)) / N ** 3
    w = np.fft.irfftn(o.curl(uhat), s=(N, N, N), axes=(1, 2, 3)) * N ** 3
    ex = np.stack([np.zeros_like(X), -2 * np.cos(N // 2 * Z) * np.cos(2 * X),
                   np.zeros_like(X)])  # only d/dx of the second term survives
    assert np.abs(w - ex).max() < 1e-12


# ---------------------------------------------------------------------------
# Nonlinear term (Eq. 1-2 in rotational form, projected and dealiased)
# ---------------------------------------------------------------------------

def _effective_full(F: np.ndarray):
    """All modes of the full spectrum with |k_a| < n_a/2 as seen by the inverse
    transform (Hermitian part of the kx = 0 plane): returns (K [M,3], V [nf,M])."""
    nf, nz, ny, H = F.shape
    nx = 2 * (H - 1)
    ks, vals = [], []
    for kz in range(-(nz // 2) + 1, nz // 2):
        for ky in range(-(ny // 2) + 1, ny // 2):
            for kx in range(-(nx // 2) + 1, nx // 2):
                sx, sy, sz = (kx, ky, kz) if kx >= 0 else (-kx, -ky, -kz)
                a = F[:, sz % nz, sy % ny, sx]
                if sx == 0:
                    a = 0.5 * (a + np.conj(F[:, (-sz) % nz, (-sy) % ny, 0]))
                if kx < 0:
                    a = np.conj(a)
                if np.any(a != 0):
                    ks.append((kx, ky, kz))
                    vals.append(a)
    return np.array(ks, dtype=np.int64).reshape(-1, 3), np.array(vals).T.reshape(nf, -1)


def _in_ellipsoid(n, k) -> bool:
    """The 2/3 rule on grid n = (nx, ny, nz): (3 kx/nx)^2 + (3 ky/ny)^2 +
    (3 kz/nz)^2 < 1 in exact rational arithmetic (the sphere 9|k|^2 < N^2 of
    the cube)."""
    return sum(Fraction(3 * int(k[a]), n[a]) ** 2 for a in range(3)) < 1


def _signed(i, n):
    return i if i < n // 2 else i - n


def _kept_outputs(n):
    nx, ny, nz = n
    out = []
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx // 2 + 1):
                k = np.array([kx, _signed(ky, ny), _signed(kz, nz)])
                if int(k @ k) > 0 and _in_ellipsoid(n, k):
                    out.append(((kz, ky, kx), k))
    return out


def brute_triads(F: np.ndarray, model: int) -> np.ndarray:
    """Dealiased, projected quadratic term as a literal sum over triads
    p + q = k of Fourier coefficients (Galerkin convolution)."""
    n = (2 * (F.shape[3] - 1), F.shape[2], F.shape[1])
    K, V = _effective_full(F)
    index = {tuple(k): i for i, k in enumerate(K)}
    out = np.zeros(F.shape, np.complex128)
    if model == NS:
        U = V
    else:
        U = 0.5 * (V[:3] + V[3:])
        B = 0.5 * (V[:3] - V[3:])

    def icross(k, v):  # i k x v, k [M,3], v [3,M]
        return 1j * np.stack([k[:, 1] * v[2] - k[:, 2] * v[1], k[:, 2] * v[0] - k[:, 0] * v[2],
                              k[:, 0] * v[1] - k[:, 1] * v[0]])

    def cross(a, b):
        return np.stack([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],
                         a[0] * b[1] - a[1] * b[0]])

    for (sz, sy, sx), k in _kept_outputs(n):
        q = k[None, :] - K
        qi = np.array([index.get(tuple(x), -1) for x in q])
        m = qi >= 0
        if not np.any(m):
            continue
        p_idx = np.nonzero(m)[0]
        qq = q[m]
        q_idx = qi[m]
        if model == NS:
            aL = cross(U[:, p_idx], icross(qq, U[:, q_idx])).sum(axis=1)
        else:
            aL = (cross(U[:, p_idx], icross(qq, U[:, q_idx]))
                  + cross(icross(K[p_idx], B[:, p_idx]), B[:, q_idx])).sum(axis=1)
            aE = cross(U[:, p_idx], B[:, q_idx]).sum(axis=1)
        k2 = float(k @ k)
        proj = aL - k * (k @ aL) / k2
        if model == NS:
            out[:, sz, sy, sx] = proj
        else:
            ce = icross(k[None, :], aE[:, None])[:, 0]
            out[:3, sz, sy, sx] = proj + ce
            out[3:, sz, sy, sx] = proj - ce
    return out


def pin_ns_abc_zero(o):
    N = 16
    u = synth.abc_flow(N, 1.0, 0.8, 0.6)
    assert np.abs(o.nonlinear_ns(u)).max() < 1e-14


def pin_ns_taylor_green(o):
    """For u = (sin x cos y cos z, -cos x sin y cos z, 0):
    P(u x w) = -1/8 (sin 2x cos 2z, sin 2y cos 2z, -(cos 2x + cos 2y) sin 2z)."""
    for N in (16, 32):
        n = o.nonlinear_ns(synth.taylor_green(N))
        Z, Y, X = _grid(N)
        ex = -0.125 * np.stack([np.sin(2 * X) * np.cos(2 * Z), np.sin(2 * Y) * np.cos(2 * Z),
                                -(np.cos(2 * X) + np.cos(2 * Y)) * np.sin(2 * Z)])
        got = np.fft.irfftn(n, s=(N, N, N), axes=(1, 2, 3)) * N ** 3
        assert np.abs(got - ex).max() < 1e-14, np.abs(got - ex).max()


def _inner(a, b, N):
    return float(np.sum(_hweights(N) * np.real(np.conj(a) * b)))


def pin_ns_invariants(o):
    """Energy and helicity are conserved by the dealiased term; k.N = 0."""
    N = 24
    u = synth.random_ns(N, 7, 3.0)
    n = o.nonlinear_ns(u)
    w = o.curl(u)
    nn = math.sqrt(_inner(n, n, N))
    assert abs(_inner(u, n, N)) / (math.sqrt(_inner(u, u, N)) * nn) < 1e-14
    assert abs(_inner(w, n, N)) / (math.sqrt(_inner(w, w, N)) * nn) < 1e-14
    KZ, KY, KX = _wavenumbers(N)
    div = KX * n[0] + KY * n[1] + KZ * n[2]
    assert np.abs(div).max() < 1e-14 * np.abs(n).max() * N


def pin_ns_triad_brute(o):
    N = 12
    u = synth.random_ns(N, 5, 2.0)
    ref = brute_triads(u, NS)
    assert _rel(o.nonlinear_ns(u), ref) < 1e-13


def pin_mhd_equal_fields(o):
    """u = b (z- = 0): u x w + j x b = 0 and u x b = 0 pointwise."""
    N = 16
    u = synth.random_ns(N, 21, 2.5)
    z = np.concatenate([2 * u, np.zeros_like(u)])
    assert np.abs(o.nonlinear_mhd(z)).max() < 1e-14 * np.abs(z).max()


def pin_mhd_reduces_to_ns(o):
    N = 16
    u = synth.random_ns(N, 22, 2.5)
    nm = o.nonlinear_mhd(np.concatenate([u, u]))
    ns = o.nonlinear_ns(u)
    assert _rel(nm[:3], ns) < 1e-14 and _rel(nm[3:], ns) < 1e-14


def pin_mhd_invariants(o):
    """Elsasser energies are conserved separately: sum Re(z+-* . N+-) = 0."""
    N = 24
    z = synth.random_mhd(N, 3, 4, 3.0)
    n = o.nonlinear_mhd(z)
    for s in (0, 3):
        a, b = z[s:s + 3], n[s:s + 3]
        assert abs(_inner(a, b, N)) / math.sqrt(_inner(a, a, N) * _inner(b, b, N)) < 1e-14


def pin_mhd_triad_brute(o):
    N = 12
    z = synth.random_mhd(N, 31, 32, 2.0)
    ref = brute_triads(z, MHD)
    assert _rel(o.nonlinear_mhd(z), ref) < 1e-13


def pin_nonlinear_at(o):
    """The oracle's triad-sum entry agrees with the literal triad sum."""
    N = 12
    for model, f in ((NS, synth.random_ns(N, 41, 2.0)), (MHD, synth.random_mhd(N, 42, 43, 2.0))):
        ref = brute_triads(f, model)
        kz = np.array([1, 0, 11, 3]); ky = np.array([2, 1, 10, 0]); kx = np.array([0, 3, 1, 2])
        got = o.nonlinear_at(f, model, kx, ky, kz)
        assert np.abs(got.T - ref[:, kz, ky, kx]).max() < 1e-13 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# Time advance (the main time-advance loop, Sec. 4; explicit midpoint RK2)
# ---------------------------------------------------------------------------

def pin_rk2_abc_decay(o):
    """ABC has zero nonlinear term, so each step multiplies it by the RK2
    stability polynomial R(-a) = 1 - a + a^2/2, a = nu |k|^2 dt."""
    N = 16
    nu, dt, k = 0.1, 0.1, 2
    u = synth.abc_flow(N, 1.0, 0.9, 0.5, k=k)
    got = o.rk2_step(u, NS, nu, 0.0, dt, 3)
    a = nu * k * k * dt
    assert _rel(got, (1 - a + 0.5 * a * a) ** 3 * u) < 1e-14


def pin_rk2_taylor_green_energy(o):
    """E(t) = 1/8 - (3/4) nu t + (9/4) nu^2 t^2 + O(t^3) for Taylor-Green:
    E0 = 1/8, Z0 = 3/8, P0 = 9/8 and the t = 0 nonlinear term lives on modes
    absent from u."""
    N = 16
    nu, dt, n = 0.05, 2e-4, 10
    u = o.rk2_step(synth.taylor_green(N), NS, nu, 0.0, dt, n)
    _, tot = o.energy_spectrum(u)
    t = n * dt
    second = (tot[0] - (0.125 - 0.75 * nu * t)) / (2.25 * nu * nu * t * t)
    assert abs(second - 1.0) < 0.05, second


def pin_rk2_second_order(o):
    N = 16
    nu, T = 0.02, 0.2
    u0 = synth.random_ns(N, 3, 2.0)
    ref = o.rk2_step(u0, NS, nu, 0.0, T / 64, 64)
    errs = [_rel(o.rk2_step(u0, NS, nu, 0.0, T / m, m), ref) for m in (4, 8, 16)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.4 < r1 < 4.6 and 3.4 < r2 < 4.6, errs


def pin_rk2_mhd_second_order(o):
    N = 12
    T = 0.2
    z0 = synth.random_mhd(N, 5, 6, 2.0)
    ref = o.rk2_step(z0, MHD, 0.02, 0.01, T / 64, 64)
    errs = [_rel(o.rk2_step(z0, MHD, 0.02, 0.01, T / m, m), ref) for m in (4, 8, 16)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.4 < r1 < 4.6 and 3.4 < r2 < 4.6, errs


def pin_rk2_divergence_free(o):
    N = 16
    u = o.rk2_step(synth.random_ns(N, 9, 2.0), NS, 0.01, 0.0, 0.01, 5)
    KZ, KY, KX = _wavenumbers(N)
    div = KX * u[0] + KY * u[1] + KZ * u[2]
    kk = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    assert np.abs(div).max() < 1e-14 * np.max(kk * np.abs(u).max(axis=0))


# ---------------------------------------------------------------------------
# Spectra and global quantities (Sec. 3: reductions)
# ---------------------------------------------------------------------------

def pin_spectrum_brute(o):
    """Shell energies by a plain loop: shell = round(|k|), weight 1 on the
    kx = 0 and kx = N/2 planes, 2 elsewhere."""
    N = 8
    rng = np.random.default_rng(16)
    F = _random_half(rng, 3, N)
    ns = o.num_shells(N)
    spec = np.zeros(ns)
    Z = 0.0
    maxdiv = 0.0
    for kz in range(N):
        for ky in range(N):
            for kx in range(N // 2 + 1):
                k = (kx, ky if ky < N // 2 else ky - N, kz if kz < N // 2 else kz - N)
                k2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
                s = 0
                while not (4 * k2 < (2 * s + 1) ** 2):
                    s += 1
                w = 1.0 if kx in (0, N // 2) else 2.0
                e = sum(abs(F[c, kz, ky, kx]) ** 2 for c in range(3))
                spec[s] += 0.5 * w * e
                Z += 0.5 * w * k2 * e
                kd = [0 if 2 * abs(v) == N else v for v in k]
                maxdiv = max(maxdiv, abs(sum(kd[c] * F[c, kz, ky, kx] for c in range(3))))
    got, tot = o.energy_spectrum(F)
    assert ns == int(math.floor(math.sqrt(3 * (N // 2) ** 2) + 0.5)) + 1
    assert _rel(got, spec) < 1e-14
    assert abs(tot[0] - spec.sum()) < 1e-13 * spec.sum()
    assert abs(tot[1] - Z) < 1e-13 * Z
    assert abs(tot[2] - maxdiv) < 1e-13 * maxdiv


def _mhd_brute(Z: np.ndarray):
    """Eu(s), Eb(s), Hc(s) and their totals by a plain loop over the stored
    modes: u = (z+ + z-)/2, b = (z+ - z-)/2, shell = round(|k|) found by
    counting, weight 1 on the kx = 0 and kx = N/2 planes and 2 elsewhere."""
    N = Z.shape[-2]
    nsh = int(math.floor(math.sqrt(3 * (N // 2) ** 2) + 0.5)) + 1
    out = np.zeros((3, nsh))
    for kz in range(N):
        for ky in range(N):
            for kx in range(N // 2 + 1):
                k = (kx, ky if ky < N // 2 else ky - N, kz if kz < N // 2 else kz - N)
                k2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
                s = 0
                while not (4 * k2 < (2 * s + 1) ** 2):
                    s += 1
                w = 1.0 if kx in (0, N // 2) else 2.0
                for c in range(3):
                    u = 0.5 * (Z[c, kz, ky, kx] + Z[3 + c, kz, ky, kx])
                    b = 0.5 * (Z[c, kz, ky, kx] - Z[3 + c, kz, ky, kx])
                    out[0, s] += 0.5 * w * abs(u) ** 2
                    out[1, s] += 0.5 * w * abs(b) ** 2
                    out[2, s] += 0.5 * w * (u * np.conj(b)).real
    return out


def pin_mhd_spectrum_brute(o):
    """Sec. 3 / Sec. 5: kinetic and magnetic energy and cross-helicity spectra
    of an Elsasser state against a plain loop over the modes (8^3, random
    coefficients, Hermitian planes not symmetrised: the weights alone decide)."""
    N = 8
    Z = _random_half(np.random.default_rng(21), 6, N)
    spec, tot = o.mhd_spectrum(Z)
    want = _mhd_brute(Z)
    assert spec.shape == want.shape
    assert _rel(spec, want) < 1e-14
    for q in range(3):
        assert abs(tot[q] - want[q].sum()) <= 1e-13 * np.abs(want[q]).sum()


def pin_mhd_spectrum_physical(o):
    """Parseval through numpy's real FFT: for real fields u(x), b(x) with
    normalised half spectra rfftn(.)/N^3 and z+- = u +- b, the totals are the
    box averages 1/2 <|u|^2>, 1/2 <|b|^2> and 1/2 <u . b>."""
    N = 12
    rng = np.random.default_rng(22)
    u = rng.standard_normal((3, N, N, N))
    b = 0.3 * u + rng.standard_normal((3, N, N, N))  # correlated: H_c far from 0
    uh = np.fft.rfftn(u, axes=(1, 2, 3)) / N ** 3
    bh = np.fft.rfftn(b, axes=(1, 2, 3)) / N ** 3
    _, tot = o.mhd_spectrum(np.concatenate([uh + bh, uh - bh]))
    want = [0.5 * np.mean(np.sum(u * u, axis=0)), 0.5 * np.mean(np.sum(b * b, axis=0)),
            0.5 * np.mean(np.sum(u * b, axis=0))]
    for q in range(3):
        assert abs(tot[q] - want[q]) < 1e-13 * abs(want[q]), (q, tot[q], want[q])


def pin_mhd_spectrum_special(o):
    """b = u (z- = 0): Eu = Eb = Hc shell by shell; b = -u (z+ = 0): Hc = -Eu;
    b = 0 (z+ = z- = u): Eb = Hc = 0 and Eu(s) is the energy spectrum of u."""
    N = 16
    U = synth.random_ns(N, 23, 3.0)
    spec, tot = o.mhd_spectrum(np.concatenate([2 * U, 0 * U]))
    assert _rel(spec[1], spec[0]) < 1e-15 and _rel(spec[2], spec[0]) < 1e-15
    assert abs(tot[0] - 0.5) < 1e-14
    spec, tot = o.mhd_spectrum(np.concatenate([0 * U, 2 * U]))
    assert _rel(spec[2], -spec[0]) < 1e-15 and abs(tot[2] + 0.5) < 1e-14
    spec, tot = o.mhd_spectrum(np.concatenate([U, U]))
    assert np.abs(spec[1:]).max() == 0.0 and tot[1] == 0.0 and tot[2] == 0.0
    e, _ = o.energy_spectrum(U)
    assert _rel(spec[0], e) < 1e-15


def _helical_mode(N: int, k, s: int):
    """One helical Fourier mode h e^{ik.x} + c.c. (kx > 0), h = e1 + i s e2 with
    e1 perpendicular to k and e2 = k^ x e1, so that k^ x h = -i s h and
    curl u = s|k| u (a Beltrami field: u x w = 0 pointwise)."""
    kv = np.array(k, dtype=np.float64)
    kh = kv / np.linalg.norm(kv)
    t = np.array([1.0, 0.0, 0.0]) if abs(kh[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(kh, t)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(kh, e1)
    h = e1 + 1j * s * e2
    U = np.zeros((3, N, N, N // 2 + 1), np.complex128)
    U[:, k[2] % N, k[1] % N, k[0]] = h
    return U, kh


def _rk2_factor(lam: complex, dt: float) -> complex:
    """Midpoint RK2 applied to u' = lam u multiplies u by 1 + x + x^2/2, x = lam dt."""
    x = lam * dt
    return 1 + x + x * x / 2


def pin_rk2_rotation_inertial_wave(o):
    """Rotation: a helical mode has no nonlinear term and is an eigenvector of
    the projected Coriolis operator, P(2 W x h) = 2 (W.k^)(k^ x h) = -2 i s (W.k^) h
    (the part of W across k gives a vector along k, which P removes).  So
    u' = (2 i s W.k^ - nu |k|^2) u exactly, and two RK2 steps multiply the
    mode by the closed-form factor squared (W generic, not along k)."""
    N, k, nu, dt = 16, (2, 1, 2), 0.01, 0.05
    om = np.array([0.3, -0.7, 1.1])
    for s in (1, -1):
        U, kh = _helical_mode(N, k, s)
        lam = 2j * s * float(om @ kh) - nu * 9.0
        want = U * _rk2_factor(lam, dt) ** 2
        got = o.rk2_step(U, NS, nu, 0.0, dt, 2, omega=om)
        assert _rel(got, want) < 1e-13, (s, _rel(got, want))
    # zero rotation is the plain step
    U, _ = _helical_mode(N, k, 1)
    a = o.rk2_step(U, NS, nu, 0.0, dt, 1, omega=np.zeros(3))
    b = o.rk2_step(U, NS, nu, 0.0, dt, 1)
    assert _rel(a, b) < 1e-15


def pin_rk2_rotation_mhd(o):
    """MHD in a rotating frame: the Coriolis term acts on u = (z+ + z-)/2 only.
    With b = 0 (z+ = z- = u) both Elsasser fields follow the NS inertial wave;
    with u = 0 (z+ = b, z- = -b, b helical) there is no nonlinear term and no
    Coriolis term, only (nu = eta) viscous decay."""
    N, k, nu, dt = 16, (2, 1, 2), 0.01, 0.05
    om = np.array([0.3, -0.7, 1.1])
    U, kh = _helical_mode(N, k, 1)
    lam = 2j * float(om @ kh) - nu * 9.0
    got = o.rk2_step(np.concatenate([U, U]), MHD, nu, nu, dt, 2, omega=om)
    want = np.concatenate([U, U]) * _rk2_factor(lam, dt) ** 2
    assert _rel(got, want) < 1e-13, _rel(got, want)
    got = o.rk2_step(np.concatenate([U, -U]), MHD, nu, nu, dt, 2, omega=om)
    want = np.concatenate([U, -U]) * _rk2_factor(-nu * 9.0, dt) ** 2
    assert _rel(got, want) < 1e-13, _rel(got, want)


def pin_rk2_mhd_resistive_coupling(o):
    """MHD with nu != eta in Elsasser variables: with u and b both multiples
    of one ABC (Beltrami) field every quadratic term vanishes (u x w, j x b and
    u x b are all zero), so the step is linear and, in the primitive variables,
    diagonal: u decays at rate nu |k|^2 and b at rate eta |k|^2, each RK2 step
    multiplying them by R(-nu |k|^2 dt) and R(-eta |k|^2 dt), R(x) = 1 + x + x^2/2.
    Checked for b = 0, u = 0 and a mixed state, so the viscosity and the
    resistivity cannot trade places anywhere in the coupled Elsasser update."""
    N, k, nu, eta, dt = 16, 2, 0.1, 0.03, 0.1
    A = synth.abc_flow(N, 1.0, 0.9, 0.5, k=k)
    ru, rb = _rk2_factor(-nu * k * k, dt), _rk2_factor(-eta * k * k, dt)
    for cu, cb in ((1.0, 0.0), (0.0, 1.0), (1.0, 0.6), (0.4, -1.3)):
        u, b = cu * A, cb * A
        got = o.rk2_step(np.concatenate([u + b, u - b]), MHD, nu, eta, dt, 3)
        uw, bw = u * ru ** 3, b * rb ** 3
        assert _rel(got, np.concatenate([uw + bw, uw - bw])) < 1e-14, (cu, cb)


def pin_box_mhd_resistive_coupling(o):
    """The same in a (2 pi, 4 pi, 6 pi) box with the ABC flow of physical
    wavenumber 1 (|k|^2 = 1 in the box's metric at indices 1, 2, 3)."""
    N, nu, eta, dt = 16, 0.07, 0.02, 0.1
    L = (2 * math.pi, 4 * math.pi, 6 * math.pi)
    A = box_abc(N, L)
    ru, rb = _rk2_factor(-nu, dt), _rk2_factor(-eta, dt)
    o.set_box(*L)
    try:
        u, b = 0.8 * A, -0.5 * A
        got = o.rk2_step(np.concatenate([u + b, u - b]), MHD, nu, eta, dt, 2)
        uw, bw = u * ru ** 2, b * rb ** 2
        assert _rel(got, np.concatenate([uw + bw, uw - bw])) < 1e-14
    finally:
        o.set_box()


def box_abc(N: int, L, A=1.0, B=0.7, C=0.4) -> np.ndarray:
    """ABC flow of physical wavenumber 1 on a box of lengths L (each a whole
    multiple of 2 pi), as normalised half-spectrum coefficients: a Beltrami
    field (curl u = u) whose three sinusoids sit at different indices."""
    x, y, z = (L[i] * np.arange(N) / N for i in range(3))
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    u = np.stack([A * np.sin(Z) + C * np.cos(Y), B * np.sin(X) + A * np.cos(Z),
                  C * np.sin(Y) + B * np.cos(X)])
    return np.fft.rfftn(u, axes=(1, 2, 3)) / N ** 3


def pin_box_aspect_ratio(o):
    """A non-cubic box (2 pi, 4 pi, 6 pi): the ABC flow of physical wavenumber 1
    has its modes at indices 1, 2 and 3 along x, y and z.  With the box's
    factors 2 pi / L in the derivatives it is still Beltrami (curl u = u, no
    nonlinear term), every mode has |k|^2 = 1, so the step is pure decay by the
    RK2 factor of -nu dt, the enstrophy equals the energy and the divergence is
    zero; MHD with b = u / 2 likewise only decays."""
    N, L, nu, dt = 16, (2 * math.pi, 4 * math.pi, 6 * math.pi), 0.05, 0.1
    U = box_abc(N, L)
    o.set_box(*L)
    try:
        assert _rel(o.curl(U), U) < 1e-13
        assert np.abs(o.nonlinear_ns(U)).max() < 1e-14 * np.abs(U).max()
        r = _rk2_factor(-nu, dt) ** 2
        assert _rel(o.rk2_step(U, NS, nu, 0.0, dt, 2), U * r) < 1e-13
        _, tot = o.energy_spectrum(U)
        assert abs(tot[1] - tot[0]) < 1e-13 * tot[0] and tot[2] < 1e-13
        Z = np.concatenate([1.5 * U, 0.5 * U])
        assert _rel(o.rk2_step(Z, MHD, nu, nu, dt, 2), Z * r) < 1e-13
    finally:
        o.set_box()


def pin_box_inertial_wave(o):
    """Rotation in a non-cubic box: the inertial-wave closed form with the
    physical wavenumber k = (2 pi / L) n in the helical basis, the Coriolis
    eigenvalue and the viscous rate."""
    N, n, nu, dt = 16, (2, 1, 2), 0.01, 0.05
    L = (2 * math.pi, 3 * math.pi, 4 * math.pi)
    kp = np.array([2 * math.pi / L[i] * n[i] for i in range(3)])
    om = np.array([0.3, -0.7, 1.1])
    U, kh = _helical_mode(N, n, 1)            # helical basis of the index vector
    kh = kp / np.linalg.norm(kp)              # rebuild it for the physical one
    t = np.array([1.0, 0.0, 0.0]) if abs(kh[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(kh, t)
    e1 /= np.linalg.norm(e1)
    h = e1 + 1j * np.cross(kh, e1)
    U[:, n[2], n[1], n[0]] = h
    lam = 2j * float(om @ kh) - nu * float(kp @ kp)
    o.set_box(*L)
    try:
        got = o.rk2_step(U, NS, nu, 0.0, dt, 2, omega=om)
        assert _rel(got, U * _rk2_factor(lam, dt) ** 2) < 1e-13, _rel(got, U * _rk2_factor(lam, dt) ** 2)
    finally:
        o.set_box()


# ---------------------------------------------------------------------------
# Grids whose axis lengths differ (Sec. 5: domains of non-unit aspect ratio;
# the grid (nx, ny, nz) replaces the cube N^3 in every definition)
# ---------------------------------------------------------------------------

def _random_grid_half(rng, nf, n):
    nx, ny, nz = n
    s = (nf, nz, ny, nx // 2 + 1)
    return rng.standard_normal(s) + 1j * rng.standard_normal(s)


def pin_grid_fft_brute(o):
    """Literal DFT sums on grids with three different axis lengths."""
    rng = np.random.default_rng(51)
    for nx, ny, nz in ((6, 4, 8), (8, 12, 6)):
        u = rng.standard_normal((nz, ny, nx))
        assert _rel(o.fft_r2c(u), brute_r2c(u)) < 1e-13, (nx, ny, nz)
        X = _random_grid_half(rng, 1, (nx, ny, nz))[0]
        assert _rel(o.fft_c2r(X), brute_c2r(X)) < 1e-13, (nx, ny, nz)
        kx = np.array([0, 1, nx // 2, 2]); ky = np.array([0, ny - 1, 2, ny // 2])
        kz = np.array([nz - 1, 0, 3, nz // 2])
        assert np.abs(o.dft_at(u, kx, ky, kz) - brute_r2c(u)[kz, ky, kx]).max() < 1e-12


def pin_grid_fft_numpy(o):
    """numpy's rfftn/irfftn on grids with different axis lengths."""
    rng = np.random.default_rng(52)
    for nz, ny, nx in ((12, 16, 24), (24, 8, 18)):
        u = rng.standard_normal((2, nz, ny, nx))
        assert _rel(o.fft_r2c(u), np.fft.rfftn(u, axes=(1, 2, 3))) < 1e-13
        X = _random_grid_half(rng, 2, (nx, ny, nz))
        ref = np.fft.irfftn(X, s=(nz, ny, nx), axes=(1, 2, 3)) * (nx * ny * nz)
        assert _rel(o.fft_c2r(X), ref) < 1e-13


def _random_in_ellipsoid(rng, nf, n):
    """Random half spectrum, zero outside the 2/3-rule ellipsoid of grid n (an
    input with no aliases reaching a kept mode)."""
    F = _random_grid_half(rng, nf, n)
    nx, ny, nz = n
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx // 2 + 1):
                if not _in_ellipsoid(n, (kx, _signed(ky, ny), _signed(kz, nz))):
                    F[:, kz, ky, kx] = 0
    return F


def pin_grid_triad_brute(o):
    """The dealiased, projected nonlinear terms (NS and MHD) on grids with
    different axis lengths equal the literal triad sum with the stretched
    2/3-rule mask, and the oracle's triad-sum entry agrees."""
    rng = np.random.default_rng(53)
    for n in ((12, 8, 16), (16, 12, 10)):
        u = _random_in_ellipsoid(rng, 3, n)
        ref = brute_triads(u, NS)
        assert _rel(o.nonlinear_ns(u), ref) < 1e-13, n
        z = _random_in_ellipsoid(rng, 6, n)
        ref = brute_triads(z, MHD)
        assert _rel(o.nonlinear_mhd(z), ref) < 1e-13, n
        kz = np.array([1, 0, n[2] - 2, 3]); ky = np.array([1, 1, n[1] - 1, 0])
        kx = np.array([0, 2, 1, 1])
        got = o.nonlinear_at(z, MHD, kx, ky, kz)
        assert np.abs(got.T - ref[:, kz, ky, kx]).max() < 1e-13 * np.abs(ref).max()


def _low(F, K):
    """Coefficients of a half spectrum on the cube |k_a| <= K, and the norm of
    everything outside it."""
    nz, ny = F.shape[1], F.shape[2]
    kr = np.arange(-K, K + 1)
    iz, iy = (kr % nz)[:, None], (kr % ny)[None, :]
    low = F[:, iz, iy, : K + 1]
    rest = F.copy()
    rest[:, iz, iy, : K + 1] = 0
    return low, float(np.linalg.norm(rest.ravel()))


def pin_grid_embedding(o):
    """A field with modes |k| <= 2 evolves identically on any grid that keeps
    every mode it reaches: one RK2 step (support |k| <= 8) on 32^3 and on
    grids with different axis lengths, NS and MHD, rotating, in a box."""
    K, nu, dt = 8, 0.01, 0.02
    om = np.array([0.4, -0.3, 0.9])
    u = synth.band_limited(32, 61, 2)
    b = synth.band_limited(32, 62, 2)
    zsp = synth.SparseField(32, 2, np.concatenate([(u.values + b.values), (u.values - b.values)]))
    o.set_box(2 * math.pi, 3 * math.pi, 4 * math.pi)
    try:
        ref_ns = o.rk2_step(u.dense(), NS, nu, 0.0, dt, 1, omega=om)
        ref_mhd = o.rk2_step(zsp.dense(), MHD, nu, 0.5 * nu, dt, 1, omega=om)
        ref_nl = o.nonlinear_mhd(zsp.dense())
        for n in ((32, 48, 64), (64, 32, 48)):
            for got, ref in ((o.rk2_step(u.dense_xyz(*n), NS, nu, 0.0, dt, 1, omega=om), ref_ns),
                             (o.rk2_step(zsp.dense_xyz(*n), MHD, nu, 0.5 * nu, dt, 1, omega=om),
                              ref_mhd),
                             (o.nonlinear_mhd(zsp.dense_xyz(*n)), ref_nl)):
                gl, grest = _low(got, K)
                rl, rrest = _low(ref, K)
                scale = np.linalg.norm(rl.ravel())
                assert grest < 1e-13 * scale and rrest < 1e-13 * scale, n
                assert _rel(gl, rl) < 1e-13, (n, _rel(gl, rl))
    finally:
        o.set_box()


def pin_grid_spectrum_brute(o):
    """Shell energies on a grid with different axis lengths by a plain loop:
    weight 1 on the kx = 0 and kx = nx/2 planes, shells round(|k|) of the
    index."""
    nx, ny, nz = 8, 6, 10
    rng = np.random.default_rng(54)
    F = _random_grid_half(rng, 3, (nx, ny, nz))
    ns = o.num_shells(nx, ny, nz)
    spec = np.zeros(ns)
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx // 2 + 1):
                k2 = kx ** 2 + _signed(ky, ny) ** 2 + _signed(kz, nz) ** 2
                s = 0
                while not (4 * k2 < (2 * s + 1) ** 2):
                    s += 1
                w = 1.0 if kx in (0, nx // 2) else 2.0
                spec[s] += 0.5 * w * sum(abs(F[c, kz, ky, kx]) ** 2 for c in range(3))
    got, tot = o.energy_spectrum(F)
    assert ns == int(math.floor(math.sqrt((nx // 2) ** 2 + (ny // 2) ** 2 + (nz // 2) ** 2) + 0.5)) + 1
    assert _rel(got, spec) < 1e-14
    assert abs(tot[0] - spec.sum()) < 1e-13 * spec.sum()


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
