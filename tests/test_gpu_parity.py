"""HIP path against the FP64 oracle, element by element, at sizes the oracle
finishes in seconds (several tiles and a ragged kx tail in every pass).

Tolerances (relative L2 over all stored values):
  FP64: 1e-13 for transforms, 1e-12 for nonlinear terms and RK2 steps
        (the bar the method's FP64 form is held to);
  FP32: transforms 2e-6 (rounding eps32 = 6e-8 times O(log N) butterfly
        levels with headroom), nonlinear terms 2e-5 (two transforms and a
        product; the term is a difference of O(1) quantities), RK2 state after
        one step 2e-6 from identical FP32 inputs.
"""
import numpy as np
import pytest
import torch

from gpu_util import CDT, DEV, host, rel_l2, rel_l2_w, rounded, say, to_dev
from oracle.psref import MHD, NS
from paper_1003_4322_amd import synth

pytestmark = pytest.mark.gpu

TOL_FFT = {"f64": 1e-13, "f32": 2e-6}
TOL_NL = {"f64": 1e-12, "f32": 2e-5}
TOL_STEP = {"f64": 1e-12, "f32": 2e-6}

FFT_SIZES = [8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 384]


@pytest.fixture(scope="module")
def B():
    from paper_1003_4322_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("N", FFT_SIZES)
def test_fft_r2c(B, ref, N, dt):
    say("fft_r2c", N, dt)
    rng = np.random.default_rng(100 + N)
    u = rounded(rng.standard_normal((3, N, N, N)), dt)
    p = B.Plan(N, 3, dt)
    got = host(p.fft_r2c(to_dev(u, dt, "r")))
    want = ref.fft_r2c(u)
    assert rel_l2(got, want) < TOL_FFT[dt], rel_l2(got, want)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("N", FFT_SIZES)
def test_fft_c2r(B, ref, N, dt):
    say("fft_c2r", N, dt)
    rng = np.random.default_rng(200 + N)
    s = (3, N, N, N // 2 + 1)
    X = rounded(rng.standard_normal(s) + 1j * rng.standard_normal(s), dt)  # not Hermitian
    p = B.Plan(N, 3, dt)
    xd = to_dev(X, dt)
    got = host(p.fft_c2r(xd))
    want = ref.fft_c2r(X)
    assert rel_l2(got, want) < TOL_FFT[dt], rel_l2(got, want)
    assert np.array_equal(host(xd), X)  # input preserved


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prune", [0, 1])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("N", [8, 16, 24, 32, 48, 64])
def test_nonlinear_ns(B, ref, N, dt, prune, form):
    """form 1 (divergence form, products u_i u_j) against the oracle's
    rotational form: equal up to rounding for solenoidal inputs."""
    say("nonlinear_ns", N, dt, prune, form)
    u = rounded(synth.random_ns(N, 1000 + N, 2.0 if N < 32 else 3.0), dt)
    p = B.Plan(N, 3, dt)
    p.set_variant("prune", prune)
    p.set_variant("form", form)
    out = torch.full(u.shape, 1e30, dtype=CDT[dt], device=DEV)
    got = host(p.nonlinear_ns(to_dev(u, dt), out))
    want = ref.nonlinear_ns(u)
    assert rel_l2_w(got, want) < TOL_NL[dt], rel_l2_w(got, want)


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prune", [0, 1])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("N", [8, 16, 24, 32, 48])
def test_nonlinear_mhd(B, ref, N, dt, prune, form):
    """form 1 (Elsasser divergence form) against the oracle's rotational form:
    equal up to rounding for the solenoidal inputs used here."""
    say("nonlinear_mhd", N, dt, prune, form)
    z = rounded(synth.random_mhd(N, 2000 + N, 3000 + N, 2.0), dt)
    p = B.Plan(N, 6, dt)
    p.set_variant("prune", prune)
    p.set_variant("form", form)
    out = torch.full(z.shape, 1e30, dtype=CDT[dt], device=DEV)
    got = host(p.nonlinear_mhd(to_dev(z, dt), out))
    want = ref.nonlinear_mhd(z)
    assert rel_l2_w(got, want) < TOL_NL[dt], rel_l2_w(got, want)


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prune", [0, 1])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_rk2_ns_32_one_step(B, ref, dt, prune, form):
    """NS 32^3, nu = 0.02, dt = 1e-3, seed 1, k0 = 2, E = 0.5: one RK2 step."""
    say("rk2 ns 32", dt, prune, form)
    u0 = rounded(synth.random_ns(32, 1, 2.0), dt)
    p = B.Plan(32, 3, dt)
    p.set_variant("prune", prune)
    p.set_variant("form", form)
    s = to_dev(u0, dt)
    p.rk2_step(s, B.PS_NS, 0.02, 0.0, 1e-3, 1)
    got = host(s)
    want = ref.rk2_step(u0, NS, 0.02, 0.0, 1e-3, 1)
    assert rel_l2_w(got, want) < TOL_STEP[dt], rel_l2_w(got, want)
    # increment error, informational bar: the change over the step itself
    inc = rel_l2_w(got - u0, want - u0)
    assert inc < (1e-10 if dt == "f64" else 1e-3), inc


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prune", [0, 1])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("graphs", [True, False])
def test_rk2_mhd_steps(B, ref, dt, graphs, prune, form):
    say("rk2 mhd 24", dt, graphs, prune, form)
    N = 24
    z0 = rounded(synth.random_mhd(N, 3, 4, 2.0), dt)
    p = B.Plan(N, 6, dt)
    p.set_graphs(graphs)
    p.set_variant("prune", prune)
    p.set_variant("form", form)
    s = to_dev(z0, dt)
    p.rk2_step(s, B.PS_MHD, 0.02, 0.01, 2e-3, 3)
    got = host(s)
    want = ref.rk2_step(z0, MHD, 0.02, 0.01, 2e-3, 3)
    assert rel_l2_w(got, want) < 3 * TOL_STEP[dt], rel_l2_w(got, want)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("N", [8, 16, 32, 48])
def test_spectrum(B, ref, N, dt):
    say("spectrum", N, dt)
    rng = np.random.default_rng(300 + N)
    s = (3, N, N, N // 2 + 1)
    F = rounded(rng.standard_normal(s) + 1j * rng.standard_normal(s), dt)
    p = B.Plan(N, 3, dt)
    spec, tot = p.energy_spectrum(to_dev(F, dt))
    ws, wt = ref.energy_spectrum(F)
    assert np.allclose(host(spec), ws, rtol=1e-13, atol=0)
    assert np.allclose(host(tot), wt, rtol=1e-12, atol=0)


# ---------------------------------------------------------------- rotation
OMEGA = (1.5, -2.0, 3.0)


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prune", [0, 1])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_rk2_ns_rotation(B, ref, dt, prune, form):
    """Rotating frame: two RK2 steps of NS 32^3 with a Coriolis term strong
    enough to matter (|2 Omega| dt ~ 0.04) against the oracle."""
    say("rk2 ns rotation", dt, prune, form)
    u0 = rounded(synth.random_ns(32, 1, 2.0), dt)
    p = B.Plan(32, 3, dt)
    p.set_variant("prune", prune)
    p.set_variant("form", form)
    p.set_rotation(*OMEGA)
    s = to_dev(u0, dt)
    p.rk2_step(s, B.PS_NS, 0.02, 0.0, 5e-3, 2)
    got = host(s)
    want = ref.rk2_step(u0, NS, 0.02, 0.0, 5e-3, 2, omega=OMEGA)
    assert rel_l2_w(got, want) < TOL_STEP[dt], rel_l2_w(got, want)
    # the rotation changed the result well beyond the tolerance
    plain = ref.rk2_step(u0, NS, 0.02, 0.0, 5e-3, 2)
    assert rel_l2_w(plain, want) > 1e3 * TOL_STEP[dt]


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prune", [0, 1])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_rk2_mhd_rotation(B, ref, dt, prune, form):
    say("rk2 mhd rotation", dt, prune, form)
    N = 24
    z0 = rounded(synth.random_mhd(N, 3, 4, 2.0), dt)
    p = B.Plan(N, 6, dt)
    p.set_variant("prune", prune)
    p.set_variant("form", form)
    p.set_rotation(*OMEGA)
    s = to_dev(z0, dt)
    p.rk2_step(s, B.PS_MHD, 0.02, 0.01, 5e-3, 2)
    got = host(s)
    want = ref.rk2_step(z0, MHD, 0.02, 0.01, 5e-3, 2, omega=OMEGA)
    assert rel_l2_w(got, want) < 3 * TOL_STEP[dt], rel_l2_w(got, want)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_rotation_inertial_wave_closed_form(B, dt):
    """GPU step against the closed form directly: a helical mode (no
    nonlinear term) is an eigenvector of the projected Coriolis operator, so
    each RK2 step multiplies it by 1 + x + x^2/2, x = (2 i s W.k^ - nu|k|^2) dt."""
    import pins
    say("inertial wave", dt)
    N, k, nu, step = 16, (2, 1, 2), 0.01, 0.05
    om = np.array([0.3, -0.7, 1.1])
    for s_ in (1, -1):
        U, kh = pins._helical_mode(N, k, s_)
        lam = 2j * s_ * float(om @ kh) - nu * 9.0
        want = U * pins._rk2_factor(lam, step) ** 3
        p = B.Plan(N, 3, dt)
        p.set_rotation(*om)
        d = to_dev(U, dt)
        p.rk2_step(d, B.PS_NS, nu, 0.0, step, 3)
        assert rel_l2(host(d), want) < (1e-13 if dt == "f64" else 2e-6)


def test_rotation_change_drops_graph(B, ref):
    """A step captured without rotation is not replayed after set_rotation."""
    say("rotation graph")
    u0 = synth.random_ns(16, 5, 2.0)
    p = B.Plan(16, 3, "f64")
    s = to_dev(u0, "f64")
    p.rk2_step(s, B.PS_NS, 0.02, 0.0, 5e-3, 1)       # captures the plain step
    p.set_rotation(*OMEGA)
    p.rk2_step(s, B.PS_NS, 0.02, 0.0, 5e-3, 1)
    want = ref.rk2_step(ref.rk2_step(u0, NS, 0.02, 0.0, 5e-3, 1), NS, 0.02, 0.0, 5e-3, 1,
                        omega=OMEGA)
    assert rel_l2_w(host(s), want) < TOL_STEP["f64"]
    with pytest.raises(B.PsError):
        p.set_rotation(float("nan"), 0.0, 0.0)


# ---------------------------------------------------------------- non-cubic box
BOX = (2 * np.pi, 3 * np.pi, 5 * np.pi)


def box_solenoidal(z, L):
    """Remove the divergence of each 3-vector group in the box's metric
    (physical wavenumbers 2 pi n / L): states of a stretched box must be
    solenoidal there for the two MHD forms to agree."""
    N = z.shape[-2]
    n = np.fft.fftfreq(N, 1.0 / N)
    k = [2 * np.pi / L[0] * np.arange(N // 2 + 1)[None, None, :],
         2 * np.pi / L[1] * n[None, :, None], 2 * np.pi / L[2] * n[:, None, None]]
    k2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
    k2[0, 0, 0] = 1.0
    out = z.copy()
    for g in range(0, z.shape[0], 3):
        kv = sum(k[c] * z[g + c] for c in range(3))
        for c in range(3):
            out[g + c] = z[g + c] - k[c] * kv / k2
    return out


@pytest.fixture
def boxed(ref):
    ref.set_box(*BOX)
    yield ref
    ref.set_box()


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prune", [0, 1])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_box_nonlinear_ns(B, boxed, dt, prune, form):
    say("box nonlinear ns", dt, prune, form)
    N = 24
    u = rounded(box_solenoidal(synth.random_ns(N, 41, 2.0), BOX), dt)
    p = B.Plan(N, 3, dt)
    p.set_variant("prune", prune)
    p.set_variant("form", form)
    p.set_box(*BOX)
    got = host(p.nonlinear_ns(to_dev(u, dt)))
    assert rel_l2_w(got, boxed.nonlinear_ns(u)) < TOL_NL[dt]


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prune", [0, 1])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_box_rk2_mhd_rotation(B, boxed, dt, prune, form):
    """Everything at once: stretched box, rotation, MHD in both forms."""
    say("box rk2 mhd rotation", dt, prune, form)
    N = 24
    z0 = rounded(box_solenoidal(synth.random_mhd(N, 43, 44, 2.0), BOX), dt)
    p = B.Plan(N, 6, dt)
    p.set_variant("prune", prune)
    p.set_variant("form", form)
    p.set_box(*BOX)
    p.set_rotation(*OMEGA)
    s = to_dev(z0, dt)
    p.rk2_step(s, B.PS_MHD, 0.02, 0.01, 5e-3, 2)
    want = boxed.rk2_step(z0, MHD, 0.02, 0.01, 5e-3, 2, omega=OMEGA)
    assert rel_l2_w(host(s), want) < 3 * TOL_STEP[dt], rel_l2_w(host(s), want)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_box_spectrum(B, boxed, dt):
    say("box spectrum", dt)
    N = 32
    u = rounded(synth.random_ns(N, 45, 3.0), dt)
    p = B.Plan(N, 3, dt)
    p.set_box(*BOX)
    spec, tot = p.energy_spectrum(to_dev(u, dt))
    ws, wt = boxed.energy_spectrum(u)
    spec, tot = spec.cpu().numpy(), tot.cpu().numpy()
    assert np.abs(spec - ws).max() <= 1e-12 * ws.max()
    assert abs(tot[0] - wt[0]) <= 1e-12 * wt[0] and abs(tot[1] - wt[1]) <= 1e-12 * wt[1]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_box_abc_closed_form(B, dt):
    """GPU against the closed form: the ABC flow of physical wavenumber 1 in
    a (2 pi, 4 pi, 6 pi) box only decays, by the RK2 factor of -nu dt."""
    import pins
    say("box abc", dt)
    N, L, nu, step = 16, (2 * np.pi, 4 * np.pi, 6 * np.pi), 0.05, 0.1
    U = pins.box_abc(N, L)
    p = B.Plan(N, 3, dt)
    p.set_box(*L)
    d = to_dev(U, dt)
    p.rk2_step(d, B.PS_NS, nu, 0.0, step, 2)
    want = U * pins._rk2_factor(-nu, step) ** 2
    assert rel_l2(host(d), want) < (1e-13 if dt == "f64" else 2e-6)
    with pytest.raises(B.PsError):
        p.set_box(0.0, 1.0, 1.0)


# ---------------------------------------------------------------- slab pipeline
@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("pipe", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_rk2_pipe(B, ref, pipe, graphs):
    """The y / x / y passes split into z-slabs: 2^pipe over three helper
    streams (1..3) or in order on the plan's stream (4..6), or 2^(pipe-3) as
    two chains on two helper streams (7..9); at N = 24, 32 and 64 slabs
    exceed the planes (one plane per slab).  Captured into the step's graph
    or launched directly, every setting gives the same step."""
    say("rk2 pipe", pipe, graphs)
    for model, N, nf in ((NS, 32, 3), (MHD, 24, 6)):
        z0 = synth.random_ns(N, 7, 2.0) if model == NS else synth.random_mhd(N, 8, 9, 2.0)
        p = B.Plan(N, nf, "f64")
        p.set_graphs(graphs)
        p.set_variant("prune", 1)
        p.set_variant("pipe", pipe)
        s = to_dev(z0, "f64")
        pm = B.PS_NS if model == NS else B.PS_MHD
        p.rk2_step(s, pm, 0.02, 0.01, 2e-3, 3)
        want = ref.rk2_step(z0, model, 0.02, 0.01, 2e-3, 3)
        assert rel_l2_w(host(s), want) < 3 * TOL_STEP["f64"], (model, rel_l2_w(host(s), want))
