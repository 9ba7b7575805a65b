"""Flat-spectrum parity at the radix-3 lengths and the large sizes.

Inputs are flat up to the 2/3 sphere (synth.flat_solenoidal: every kept mode
of the same expected size).  FP64 runs take the field as generated (solenoidal
to rounding, as the divergence form requires); FP32 runs take it rounded to
FP32 and are compared with the oracle's result for those same values (the
rounding leaves a divergence of ~6e-8 relative, which the divergence form
turns into a difference of that order, well inside the FP32 bars).  Each
result is compared element by element, shell by
shell (max |gpu - oracle| in a shell / max |oracle| in it), on two pass sets:
the defaults (rotational form, nothing pruned) and the benchmark's (the
divergence form with dealias pruning).  768^3 is beyond the oracle's full
step; there the nonlinear term is checked at modes on and near the sphere
edge against the oracle's direct triad sums, and the transforms against
direct DFT sums and the round trip.

Tolerances as in the variant suite (nonlinear terms per shell 1e-12 FP64,
5e-5 FP32; relative L2 1e-12 and 2e-5); one RK2 step per shell 1e-12 (FP64)
and 1e-5 (FP32: the state's own rounding, 6e-8, plus dt times the nonlinear
term's error, with dt |N| ~ 0.1 |u| here).
"""
import numpy as np
import pytest
import torch

from gpu_util import DEV, host, rel_l2_w_dev, rounded, say, shell_err_dev, to_dev
from oracle.psref import MHD, NS
from paper_1003_4322_amd import synth

pytestmark = pytest.mark.gpu

TOL_NL = {"f64": 1e-12, "f32": 2e-5}
TOL_SHELL = {"f64": 1e-12, "f32": 5e-5}
TOL_STEP_SHELL = {"f64": 1e-12, "f32": 1e-5}
TOL_STEP = {"f64": 1e-12, "f32": 2e-6}
PASS_SETS = [(0, 0), (1, 1)]  # (prune, form)


@pytest.fixture(scope="module")
def B():
    from paper_1003_4322_amd import binding
    binding.lib()
    return binding


def flat(N, seed, groups, dt):
    """The flat field as generated (f64) or rounded to FP32 and promoted back."""
    v = synth.flat_solenoidal(N, seed, groups=groups)
    return rounded(v, dt)


def check(got, want, tol_l2, tol_shell, what, bad):
    """Records a failure in `bad` instead of raising, so that one run reports
    every pass set and precision."""
    e = rel_l2_w_dev(got, want)
    es, s, outside = shell_err_dev(got, want)
    say(what, f"rel-L2 {e:.2e}, worst shell {s}: {es:.2e}, outside {outside:.1e}")
    if not (e < tol_l2 and es < tol_shell):
        bad.append((what, e, s, es))
    return outside


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("model", ["ns", "mhd"])
@pytest.mark.parametrize("N", [96, 192, 384])
def test_flat_nonlinear(B, ref, N, model, dt):
    say("flat nonlinear", N, model, dt)
    mhd = model == "mhd"
    x = flat(N, 50 + N, 2 if mhd else 1, dt)
    want = torch.from_numpy(ref.nonlinear_mhd(x) if mhd else ref.nonlinear_ns(x)).to(DEV)
    p = B.Plan(N, 6 if mhd else 3, dt)
    xd = to_dev(x, dt)
    out = torch.full(xd.shape, 1e30, dtype=xd.dtype, device=DEV)
    bad = []
    for prune, form in PASS_SETS:
        p.set_variant("prune", prune)
        p.set_variant("form", form)
        got = p.nonlinear_mhd(xd, out) if mhd else p.nonlinear_ns(xd, out)
        outside = check(got, want, TOL_NL[dt], TOL_SHELL[dt], (N, model, dt, prune, form), bad)
        assert outside == 0.0
    p.close()
    assert not bad, bad


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("model", ["ns", "mhd"])
@pytest.mark.parametrize("N", [96, 192])
def test_flat_rk2_step(B, ref, N, model, dt):
    """One RK2 step of the flat state (nu = eta = 1e-3, dt = 2e-3): every mode
    of the sphere moves, the viscous factor reaches |k|^2 ~ (N/3)^2."""
    say("flat rk2", N, model, dt)
    mhd = model == "mhd"
    x = flat(N, 60 + N, 2 if mhd else 1, dt)
    want = torch.from_numpy(ref.rk2_step(x, MHD if mhd else NS, 1e-3, 1e-3, 2e-3, 1)).to(DEV)
    p = B.Plan(N, 6 if mhd else 3, dt)
    bad = []
    for prune, form in PASS_SETS:
        p.set_variant("prune", prune)
        p.set_variant("form", form)
        s = to_dev(x, dt)
        p.rk2_step(s, B.PS_MHD if mhd else B.PS_NS, 1e-3, 1e-3, 2e-3, 1)
        check(s, want, TOL_STEP[dt], TOL_STEP_SHELL[dt], (N, model, dt, prune, form), bad)
    p.close()
    assert not bad, bad


# modes on and near the 2/3 sphere (9|k|^2 < 768^2 keeps |k| <= 255) across
# tiles, ky and kz ranges, one inside-out (Nyquist row) and one outside
SAMPLE768 = [(255, 0, 0), (0, 255, 0), (0, 0, 513), (150, 150, 100), (1, 767, 1), (180, 600, 20),
             (250, 30, 740), (3, 5, 7), (64, 700, 600), (128, 384, 0)]


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_flat_nonlinear_768_sampled(B, ref, dt):
    N = 768
    say("flat nonlinear 768 sampled: input and triad sums", dt)
    x = flat(N, 71, 1, dt)
    kx = np.array([s[0] for s in SAMPLE768]); ky = np.array([s[1] for s in SAMPLE768])
    kz = np.array([s[2] for s in SAMPLE768])
    want = ref.nonlinear_at(x, NS, kx, ky, kz)           # [mode][field]
    xd = to_dev(x, dt)
    del x
    p = B.Plan(N, 3, dt)
    for prune, form in PASS_SETS:
        p.set_variant("prune", prune)
        p.set_variant("form", form)
        got = host(p.nonlinear_ns(xd)[:, kz, ky, kx]).T
        scale = np.abs(want).max(axis=1)                 # per mode
        live = scale > 0
        err = (np.abs(got - want).max(axis=1)[live] / scale[live]).max()
        say(dt, prune, form, f"worst mode error {err:.2e}")
        assert err < TOL_SHELL[dt], err
        assert np.abs(got[~live]).max() == 0.0
    p.close()


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_fft768_sampled_and_roundtrip(B, ref, dt):
    N = 768
    say("fft768", dt)
    rdt = torch.float32 if dt == "f32" else torch.float64
    g = torch.Generator(device=DEV).manual_seed(9)
    u = torch.randn((3, N, N, N), generator=g, device=DEV, dtype=torch.float64).to(rdt)
    p = B.Plan(N, 3, dt)
    X = p.fft_r2c(u)
    kx = np.array([0, 1, 384, 255]); ky = np.array([0, 767, 384, 600]); kz = np.array([0, 5, 384, 700])
    want = ref.dft_at(host(u[1]), kx, ky, kz)
    got = host(X[1, kz, ky, kx])
    scale = np.sqrt(N ** 3)  # |X| ~ sqrt(N^3) for unit white noise
    assert np.abs(got - want).max() / scale < (2e-5 if dt == "f32" else 1e-11)
    back = p.fft_c2r(X)
    err = float(((back / N ** 3 - u).norm() / u.norm()).item())
    assert err < (2e-6 if dt == "f32" else 1e-13), err
    p.close()


# sampled modes of a 512^3 box: on and near the 2/3 sphere (|k| <= 170), low
# modes, negative ky/kz, one outside the sphere
SAMPLE512 = [(170, 0, 0), (0, 170, 0), (0, 0, 342), (100, 100, 60), (1, 511, 1), (120, 400, 20),
             (160, 30, 500), (3, 5, 7), (40, 470, 400), (128, 256, 0)]


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_xprod_variants_512_flat(B, ref, dt):
    """Every product-pass variant (including the packed forms, whose 512-point
    transforms span whole waves) at 512^3 on a flat MHD input, both forms,
    pruned: against the oracle's triad sums at sampled modes and, over the
    whole field, against the default variant (itself checked the same way)."""
    N = 512
    say("x_prod variants 512 flat: input and triad sums", dt)
    x = flat(N, 91, 2, dt)
    kx = np.array([s[0] for s in SAMPLE512]); ky = np.array([s[1] for s in SAMPLE512])
    kz = np.array([s[2] for s in SAMPLE512])
    want = ref.nonlinear_at(x, MHD, kx, ky, kz)           # [mode][field]
    scale = np.abs(want).max(axis=1)
    live = scale > 0
    xd = to_dev(x, dt)
    del x
    p = B.Plan(N, 6, dt)
    p.set_variant("prune", 1)
    bad = []
    for form in (0, 1):
        p.set_variant("form", form)
        p.set_variant("x_prod", 0)
        base = p.nonlinear_mhd(xd).clone()
        for v in range(p.variant_count("x_prod")):
            p.set_variant("x_prod", v)
            got_d = p.nonlinear_mhd(xd)
            got = host(got_d[:, kz, ky, kx]).T
            err = (np.abs(got - want).max(axis=1)[live] / scale[live]).max()
            e0 = rel_l2_w_dev(got_d, base)
            say(dt, "form", form, "x_prod", v, f"worst mode {err:.2e}, vs variant 0 {e0:.2e}")
            if not (err < TOL_SHELL[dt] and e0 < TOL_NL[dt] and np.abs(got[~live]).max() == 0.0):
                bad.append((form, v, err, e0))
    p.close()
    assert not bad, bad
