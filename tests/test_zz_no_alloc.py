"""The allocation-free spectrum entry point (ps_energy_spectrum_static),
called through the C ABI, against ps_energy_spectrum: bit-identical results
(the same kernels in the same order), on calls in a row whose second input is
smaller than the first, on plans with and without a workspace, and on an
ensemble whose boxes reuse the scratch one after another."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import DEV, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1003_4322_amd import binding
    binding.lib()
    return binding


def random_half(N, nf, seed, cdt):
    g = torch.Generator(device=DEV).manual_seed(seed)
    re = torch.randn((nf, N, N, N // 2 + 1), generator=g, device=DEV, dtype=torch.float64)
    im = torch.randn((nf, N, N, N // 2 + 1), generator=g, device=DEV, dtype=torch.float64)
    return torch.complex(re, im).to(cdt)


def static_call(B, plan, f, nf):
    """ps_energy_spectrum_static straight through the C ABI; outputs
    pre-filled with NaN so that a value it does not write is seen."""
    L = B.lib()
    spec = torch.full((sum(plan.nshells),), float("nan"), dtype=torch.float64, device=DEV)
    tot = torch.full((3 * len(plan.sizes),), float("nan"), dtype=torch.float64, device=DEV)
    s = torch.cuda.current_stream(DEV)
    assert L.ps_plan_set_stream(plan.handle, ctypes.c_void_p(s.cuda_stream)) == 0
    rc = L.ps_energy_spectrum_static(plan.handle, ctypes.c_void_p(f.data_ptr()), int(nf),
                                     ctypes.c_void_p(spec.data_ptr()), ctypes.c_void_p(tot.data_ptr()))
    assert rc == 0, L.ps_last_error()
    torch.cuda.synchronize()
    return spec, tot


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_static_matches_workspace_entry_point(B, dt):
    cdt = torch.complex128 if dt == "f64" else torch.complex64
    # the second call has the smaller input (fewer modes and fewer fields)
    for N, nf, seed in ((96, 3, 1), (32, 2, 2)):
        say("no-alloc spectrum", dt, N, nf)
        p = B.Plan(N, 3, dt)
        f = random_half(N, 3, seed, cdt)
        want_s, want_t = p.energy_spectrum(f, nf)
        got_s, got_t = static_call(B, p, f, nf)
        assert torch.equal(got_s, want_s) and torch.equal(got_t, want_t)
        p.close()


def test_static_needs_no_workspace(B):
    say("no-alloc spectrum without workspace")
    p = B.Plan(24, 3, "f64", workspace=False)
    f = random_half(24, 3, 3, torch.complex128)
    with pytest.raises(B.PsError):
        p.energy_spectrum(f)            # the workspace entry point needs one
    got_s, got_t = static_call(B, p, f, 3)
    q = B.Plan(24, 3, "f64")
    want_s, want_t = q.energy_spectrum(f)
    assert torch.equal(got_s, want_s) and torch.equal(got_t, want_t)


def test_static_ensemble(B):
    say("no-alloc spectrum ensemble")
    sizes = [32, 16, 16, 24]
    p = B.Plan(sizes, 3, "f64")
    f = torch.complex(torch.randn(p.n_complex(), dtype=torch.float64, device=DEV),
                      torch.randn(p.n_complex(), dtype=torch.float64, device=DEV))
    want_s, want_t = p.energy_spectrum(f)
    got_s, got_t = static_call(B, p, f, 3)
    assert torch.equal(got_s, want_s) and torch.equal(got_t, want_t)
    assert not torch.isnan(got_s).any()
