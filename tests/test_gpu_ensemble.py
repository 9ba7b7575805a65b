"""Ensembles of independent boxes of uneven size in one plan: every box
against the FP64 oracle, with one launch per pass for each run of equal-size
boxes (batch variant 0) and with one launch per box (batch variant 1)."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, host, rel_l2, rel_l2_w, rounded, say
from oracle.psref import MHD, NS
from paper_1003_4322_amd import synth

pytestmark = pytest.mark.gpu
SIZES = [16, 16, 24, 32, 32, 16, 12]
TOL = {"f64": 1e-12, "f32": 2e-6}


@pytest.fixture(scope="module")
def B():
    from paper_1003_4322_amd import binding
    binding.lib()
    return binding


def pack(plan, fields, cdt):
    flat = torch.empty(plan.n_complex(), dtype=cdt, device=DEV)
    for b, f in enumerate(fields):
        n = f.size
        flat[plan.cplx_off[b]:plan.cplx_off[b] + n] = torch.from_numpy(f.ravel()).to(DEV, cdt)
    return flat


def unpack(plan, flat, shapes):
    h = host(flat)
    return [h[plan.cplx_off[b]:plan.cplx_off[b] + int(np.prod(s))].reshape(s) for b, s in enumerate(shapes)]


@pytest.mark.parametrize("batch", [0, 1])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_ensemble_rk2_ns(B, ref, dt, batch):
    say("ensemble ns", dt, batch)
    cdt = torch.complex128 if dt == "f64" else torch.complex64
    fields = [rounded(synth.random_ns(N, 1000 + i, synth.ensemble_k0(1000 + i)), dt)
              for i, N in enumerate(SIZES)]
    p = B.Plan(SIZES, 3, dt)
    p.set_variant("batch", batch)
    st = pack(p, fields, cdt)
    p.rk2_step(st, B.PS_NS, 5e-3, 0.0, 2e-3, 2)
    got = unpack(p, st, [f.shape for f in fields])
    for i, f in enumerate(fields):
        want = ref.rk2_step(f, NS, 5e-3, 0.0, 2e-3, 2)
        assert rel_l2_w(got[i], want) < 2 * TOL[dt], (i, rel_l2_w(got[i], want))


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_ensemble_rk2_mhd(B, ref, dt):
    say("ensemble mhd", dt)
    cdt = torch.complex128 if dt == "f64" else torch.complex64
    sizes = [16, 24, 24, 16]
    fields = [rounded(synth.random_mhd(N, 2000 + i, 3000 + i, 2.0), dt) for i, N in enumerate(sizes)]
    p = B.Plan(sizes, 6, dt)
    st = pack(p, fields, cdt)
    p.rk2_step(st, B.PS_MHD, 5e-3, 2e-3, 2e-3, 1)
    got = unpack(p, st, [f.shape for f in fields])
    for i, f in enumerate(fields):
        want = ref.rk2_step(f, MHD, 5e-3, 2e-3, 2e-3, 1)
        assert rel_l2_w(got[i], want) < TOL[dt], (i, rel_l2_w(got[i], want))


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_ensemble_fft_and_spectrum(B, ref, dt):
    say("ensemble fft", dt)
    rdt = torch.float64 if dt == "f64" else torch.float32
    rng = np.random.default_rng(9)
    us = [rounded(rng.standard_normal((3, N, N, N)), dt) for N in SIZES]
    p = B.Plan(SIZES, 3, dt)
    real = torch.empty(p.n_real(), dtype=rdt, device=DEV)
    for b, u in enumerate(us):
        real[p.real_off[b]:p.real_off[b] + u.size] = torch.from_numpy(u.ravel()).to(DEV, rdt)
    X = p.fft_r2c(real)
    Xs = unpack(p, X, [(3, N, N, N // 2 + 1) for N in SIZES])
    back = host(p.fft_c2r(X))
    spec, tot = p.energy_spectrum(X)
    spec, tot = host(spec), host(tot)
    so = 0
    for b, (N, u) in enumerate(zip(SIZES, us)):
        want = ref.fft_r2c(u)
        assert rel_l2(Xs[b], want) < (1e-13 if dt == "f64" else 2e-6)
        rb = back[p.real_off[b]:p.real_off[b] + u.size].reshape(u.shape)
        assert rel_l2(rb, N ** 3 * u) < (1e-13 if dt == "f64" else 2e-6)
        ws, wt = ref.energy_spectrum(Xs[b])
        ns = len(ws)
        assert np.allclose(spec[so:so + ns], ws, rtol=1e-12, atol=0)
        assert np.allclose(tot[3 * b:3 * b + 3], wt, rtol=1e-12, atol=0)
        so += ns
