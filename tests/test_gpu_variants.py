"""Every kernel variant (tile width, split and direct forms, occupancy hint, radix-16
schedule, rows per workgroup) against the FP64 oracle at 256^3, the smallest
size with variants.  Same tolerances as the main parity suite."""
import numpy as np
import pytest

from gpu_util import host, rel_l2, rel_l2_w, rounded, say, to_dev
from paper_1003_4322_amd import synth

pytestmark = pytest.mark.gpu
N = 256
TOL_FFT = {"f64": 1e-13, "f32": 2e-6}
TOL_NL = {"f64": 1e-12, "f32": 2e-5}


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


@pytest.fixture(scope="module")
def ns_case(ref):
    u = synth.random_ns(N, 11, 4.0)
    return {dt: (rounded(u, dt), ref.nonlinear_ns(rounded(u, dt))) for dt in ("f32", "f64")}


@pytest.fixture(scope="module")
def mhd_case(ref):
    z = synth.random_mhd(N, 12, 13, 3.0)
    return {dt: (rounded(z, dt), ref.nonlinear_mhd(rounded(z, dt))) for dt in ("f32", "f64")}


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
    for v in range(p.variant_count(kind)):
        say("ns variant", kind, v, dt, prune, form)
        p.set_variant(kind, v)
        e = rel_l2_w(host(p.nonlinear_ns(ud)), want)
        assert e < TOL_NL[dt], (kind, v, e)


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
    for v in range(p.variant_count(kind)):
        say("mhd variant", kind, v, dt, prune, form)
        p.set_variant(kind, v)
        e = rel_l2_w(host(p.nonlinear_mhd(zd)), want)
        assert e < TOL_NL[dt], (kind, v, e)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_autotuned_step_matches_default(B, dt):
    """The autotuned plan gives the same step as the default one (same
    arithmetic up to rounding order)."""
    z = rounded(synth.random_mhd(N, 14, 15, 3.0), dt)
    a, b = to_dev(z, dt), to_dev(z, dt)
    p0 = B.Plan(N, 6, dt)
    p1 = B.Plan(N, 6, dt)
    p1.set_variant("prune", 1)
    say("autotune", dt, p1.autotune(b, B.PS_MHD, 2))
    p0.rk2_step(a, B.PS_MHD, 5e-4, 5e-4, 1e-3, 2)
    p1.rk2_step(b, B.PS_MHD, 5e-4, 5e-4, 1e-3, 2)
    e = rel_l2_w(host(b), host(a))
    assert e < (1e-14 if dt == "f64" else 1e-6), e
