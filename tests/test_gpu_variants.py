"""Every kernel variant (tile width, split and direct forms, occupancy hint,
radix-16 schedule, rows per workgroup) against the FP64 oracle at 256^3, the
smallest size with variants.

The nonlinear-term inputs are flat up to the 2/3 sphere (every kept mode of
the same expected size), so the sphere-boundary tiles, the tails of the disk
tile lists and the high-ky/kz workgroup ranges all carry real data; each
result is checked in relative L2 and shell by shell (max error in the shell /
max reference value in the shell), and modes the 2/3 rule removes must come
out exactly zero.

Tolerances: transforms as in the main parity suite; nonlinear terms 1e-12
(FP64) and 2e-5 (FP32) in relative L2, and per shell 1e-12 (FP64) and 5e-5
(FP32): a value of a length-N^3 transform carries about eps log2(N^3) of the
RMS of its shell (6e-8 x 24 = 1.4e-6 in FP32), two transform sets and a
product about twice that, and the largest of ~10^7 values a few times more.
"""
import numpy as np
import pytest
import torch

from gpu_util import (DEV, host, rel_l2, rel_l2_w, rel_l2_w_dev, rounded, say, shell_err_dev,
                      to_dev)
from paper_1003_4322_amd import synth

pytestmark = pytest.mark.gpu
N = 256
TOL_FFT = {"f64": 1e-13, "f32": 2e-6}
TOL_NL = {"f64": 1e-12, "f32": 2e-5}
TOL_SHELL = {"f64": 1e-12, "f32": 5e-5}


@pytest.fixture(scope="module")
def B():
    from paper_1003_4322_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def fft_case(ref):
    rng = np.random.default_rng(7)
    u = rng.standard_normal((3, N, N, N))
    s = (3, N, N, N // 2 + 1)
    X = rng.standard_normal(s) + 1j * rng.standard_normal(s)
    return u, X


def _flat_case(ref, groups, fn):
    out = {}
    v = synth.flat_solenoidal(N, 11 if groups == 1 else 12, groups=groups)
    for dt in ("f32", "f64"):
        x = rounded(v, dt)
        out[dt] = (x, torch.from_numpy(fn(x)).to(DEV))
    return out


@pytest.fixture(scope="module")
def ns_case(ref):
    return _flat_case(ref, 1, ref.nonlinear_ns)


@pytest.fixture(scope="module")
def mhd_case(ref):
    return _flat_case(ref, 2, ref.nonlinear_mhd)


def check_nl(got, want, dt, what):
    e = rel_l2_w_dev(got, want)
    es, s, outside = shell_err_dev(got, want)
    say(what, f"rel-L2 {e:.2e}, worst shell {s}: {es:.2e}, outside {outside:.1e}")
    assert e < TOL_NL[dt], (what, e)
    assert es < TOL_SHELL[dt], (what, s, es)
    assert outside == 0.0, (what, outside)


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("kind", ["y", "z"])
def test_fft_variants(B, ref, fft_case, kind, dt):
    u, X = fft_case
    u, X = rounded(u, dt), rounded(X, dt)
    want_c = ref.fft_r2c(u)
    want_r = ref.fft_c2r(X)
    p = B.Plan(N, 3, dt)
    ud, xd = to_dev(u, dt, "r"), to_dev(X, dt)
    for v in range(p.variant_count(kind)):
        say("fft variant", kind, v, dt)
        p.set_variant(kind, v)
        e1 = rel_l2(host(p.fft_r2c(ud)), want_c)
        e2 = rel_l2(host(p.fft_c2r(xd)), want_r)
        assert e1 < TOL_FFT[dt] and e2 < TOL_FFT[dt], (kind, v, e1, e2)


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prune", [0, 1])
@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("kind", ["y", "z_curl", "x_prod", "z_epi", "pipe"])
def test_nonlinear_ns_variants(B, ns_case, kind, dt, prune, form):
    u, want = ns_case[dt]
    p = B.Plan(N, 3, dt)
    p.set_variant("prune", prune)
    p.set_variant("form", form)
    ud = to_dev(u, dt)
    out = torch.full(ud.shape, 1e30, dtype=ud.dtype, device=DEV)
    for v in range(p.variant_count(kind)):
        say("ns variant", kind, v, dt, prune, form)
        p.set_variant(kind, v)
        check_nl(p.nonlinear_ns(ud, out), want, dt, (kind, v))


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prune", [0, 1])
@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("kind", ["y", "z_curl", "x_prod", "z_epi", "pipe"])
def test_nonlinear_mhd_variants(B, mhd_case, kind, dt, prune, form):
    z, want = mhd_case[dt]
    p = B.Plan(N, 6, dt)
    p.set_variant("prune", prune)
    p.set_variant("form", form)
    zd = to_dev(z, dt)
    out = torch.full(zd.shape, 1e30, dtype=zd.dtype, device=DEV)
    for v in range(p.variant_count(kind)):
        say("mhd variant", kind, v, dt, prune, form)
        p.set_variant(kind, v)
        check_nl(p.nonlinear_mhd(zd, out), want, dt, (kind, v))


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_autotuned_step_matches_default(B, dt):
    """The autotuned plan gives the same step as the default one (same
    arithmetic up to rounding order), and so does the divergence form on this
    solenoidal, truncated state."""
    z = rounded(synth.random_mhd(N, 14, 15, 3.0), dt)
    a, b, c = to_dev(z, dt), to_dev(z, dt), to_dev(z, dt)
    p0 = B.Plan(N, 6, dt)
    p1 = B.Plan(N, 6, dt)
    p1.set_variant("prune", 1)
    say("autotune", dt, p1.autotune(b, B.PS_MHD, 2))
    p2 = B.Plan(N, 6, dt)
    p2.set_variant("prune", 1)
    p2.set_variant("form", 1)
    say("autotune form 1", dt, p2.autotune(c, B.PS_MHD, 2))
    p0.rk2_step(a, B.PS_MHD, 5e-4, 5e-4, 1e-3, 2)
    p1.rk2_step(b, B.PS_MHD, 5e-4, 5e-4, 1e-3, 2)
    p2.rk2_step(c, B.PS_MHD, 5e-4, 5e-4, 1e-3, 2)
    e = rel_l2_w(host(b), host(a))
    assert e < (1e-14 if dt == "f64" else 1e-6), e
    e = rel_l2_w(host(c), host(a))
    assert e < (1e-13 if dt == "f64" else 1e-6), e
