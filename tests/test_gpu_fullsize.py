"""Parity at the benchmark's full sizes and launch configuration (autotuned
variants), where the oracle cannot run the whole step:

* 512^3 MHD nonlinear terms of the benchmark's random-phase input at sampled
  modes, against the oracle's direct Galerkin triad sums;
* 512^3 MHD and 1024^3 NS RK2 steps by exact embedding: a field supported on
  |k| <= 4 evolves identically on a 64^3 grid (oracle) and on the full grid
  (the quadratic terms of two steps reach |k| <= 16, inside both 2/3 spheres);
* 512^3 transform bins against direct DFT sums, the round trip, and the
  shell spectrum against the oracle;
* the full 68-box ensemble plan, a box of each size against the oracle.
"""
import numpy as np
import pytest
import torch

from gpu_util import DEV, host, rel_l2, rel_l2_w, rounded, say
from oracle.psref import MHD, NS
from paper_1003_4322_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def B():
    from paper_1003_4322_amd import binding
    binding.lib()
    return binding


def sparse_to_dev(sf, cdt):
    N = sf.N
    st = torch.zeros((sf.values.shape[0], N, N, N // 2 + 1), dtype=cdt, device=DEV)
    iz, iy, ix = sf.index_arrays()
    vals = torch.from_numpy(np.ascontiguousarray(sf.values)).to(DEV, cdt)
    fi = torch.arange(sf.values.shape[0], device=DEV).view(-1, 1, 1, 1)
    st.index_put_((fi, torch.as_tensor(iz, device=DEV).view(1, -1, 1, 1),
                   torch.as_tensor(iy, device=DEV).view(1, 1, -1, 1),
                   torch.as_tensor(ix, device=DEV).view(1, 1, 1, -1)), vals)
    return st


def cube_of(full, N, K):
    """Coefficients of |k_i| <= K from a half spectrum: [f][kz][ky][kx<=K]."""
    kk = np.arange(-K, K + 1) % N
    return full[:, kk[:, None], kk[None, :], :K + 1]


SAMPLE = [(0, 1, 0), (3, 2, 1), (5, 507, 4), (17, 30, 501), (40, 2, 9), (2, 100, 3),
          (60, 60, 60), (1, 511, 511), (113, 0, 0), (9, 9, 500)]


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_mhd512_nonlinear_sampled(B, ref, dt, form):
    N = 512
    say("mhd512 nonlinear sampled", dt, form)
    cdt = torch.complex64 if dt == "f32" else torch.complex128
    sf = synth.mhd_sparse(N, 3, 4, 3.0)
    if dt == "f32":
        sf = synth.SparseField(N, sf.K, sf.values.astype(np.complex64).astype(np.complex128))
    z = sparse_to_dev(sf, cdt)
    p = B.Plan(N, 6, dt)
    p.set_variant("prune", 1)
    p.set_variant("form", form)
    say("autotune", p.autotune(z, B.PS_MHD, 2))
    out = p.nonlinear_mhd(z)
    kx = np.array([s[0] for s in SAMPLE]); ky = np.array([s[1] for s in SAMPLE])
    kz = np.array([s[2] for s in SAMPLE])
    got = host(out[:, kz, ky, kx]).T                      # [mode][field]
    zh = sf.dense()                                       # FP64 values the GPU started from
    want = ref.nonlinear_at(zh, MHD, kx, ky, kz)
    scale = np.abs(want).max()
    err = np.abs(got - want).max() / scale
    assert err < (1e-5 if dt == "f32" else 1e-12), err
    del out, z


@pytest.mark.parametrize("case", [("mhd", 512, "f64", 0), ("mhd", 512, "f32", 0), ("mhd", 512, "f64", 1),
                                  ("mhd", 512, "f32", 1), ("ns", 1024, "f32", 0), ("ns", 1024, "f64", 0),
                                  ("mhd", 1024, "f32", 1), ("ns", 1024, "f32", 1)])
def test_rk2_embedding(B, ref, case):
    model, N, dt, form = case
    say("embedding", model, N, dt, form)
    cdt = torch.complex64 if dt == "f32" else torch.complex128
    K, n0 = 4, 64
    if model == "mhd":
        u, b = synth.band_limited(n0, 21, K), synth.band_limited(n0, 22, K)
        small = synth.SparseField(n0, K, np.concatenate([(u + b).values, (u - b).values]))
        nf, pm, nu, eta = 6, B.PS_MHD, 5e-4, 5e-4
    else:
        small = synth.band_limited(n0, 23, K)
        nf, pm, nu, eta = 3, B.PS_NS, 2e-4, 0.0
    vals = small.values if dt == "f64" else small.values.astype(np.complex64).astype(np.complex128)
    small = synth.SparseField(n0, K, vals)
    big = synth.SparseField(N, K, vals.copy())
    dtime, steps = 2e-3, 2
    want_full = ref.rk2_step(small.dense(), MHD if model == "mhd" else NS, nu, eta, dtime, steps)
    z = sparse_to_dev(big, cdt)
    p = B.Plan(N, nf, dt)
    p.set_variant("prune", 1)
    p.set_variant("form", form)
    say("autotune", p.autotune(z, pm, 2))
    p.rk2_step(z, pm, nu, eta, dtime, steps)
    Kc = 4 * K  # support after two steps
    got = host(z[:, np.arange(-Kc, Kc + 1) % N][:, :, np.arange(-Kc, Kc + 1) % N][..., :Kc + 1])
    want = cube_of(want_full, n0, Kc)
    err = rel_l2(got, want)
    assert err < (2e-6 if dt == "f32" else 1e-12), err
    # and nothing outside the support beyond rounding: energy there <= tol^2
    tol = 2e-6 if dt == "f32" else 1e-12
    tot = float(z.abs().double().pow(2).sum().item())
    inside = float(np.sum(np.abs(got) ** 2))
    assert tot - inside <= tol * tol * tot + 1e-15 * tot, (tot, inside)
    del z, p


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_fft512_sampled_and_roundtrip(B, ref, dt):
    N = 512
    say("fft512", dt)
    rdt = torch.float32 if dt == "f32" else torch.float64
    g = torch.Generator(device=DEV).manual_seed(5)
    u = torch.randn((3, N, N, N), generator=g, device=DEV, dtype=torch.float64).to(rdt)
    p = B.Plan(N, 3, dt)
    X = p.fft_r2c(u)
    kx = np.array([0, 1, 256, 77]); ky = np.array([0, 511, 3, 256]); kz = np.array([0, 5, 256, 400])
    u0 = host(u[0])
    want = ref.dft_at(u0, kx, ky, kz)
    got = host(X[0, kz, ky, kx])
    scale = np.sqrt(N ** 3)  # |X| ~ sqrt(N^3) for unit white noise
    assert np.abs(got - want).max() / scale < (2e-5 if dt == "f32" else 1e-11)
    back = p.fft_c2r(X)
    err = float(((back / N ** 3 - u).norm() / u.norm()).item())
    assert err < (2e-6 if dt == "f32" else 1e-13), err
    # spectrum of field 0..2 against the oracle on the host copy
    spec, tot = p.energy_spectrum(X)
    Xh = host(X)
    ws, wt = ref.energy_spectrum(Xh)
    assert np.allclose(host(spec), ws, rtol=1e-12, atol=1e-300)
    assert np.allclose(host(tot), wt, rtol=1e-12)


def test_ensemble_full_config(B, ref):
    say("ensemble full config")
    sizes = [64] * 48 + [96] * 16 + [128] * 4
    p = B.Plan(sizes, 3, "f32")
    p.set_variant("prune", 1)
    st = torch.empty(p.n_complex(), dtype=torch.complex64, device=DEV)
    fields = {}
    for i, N in enumerate(sizes):
        f = synth.random_ns(N, 1000 + i, synth.ensemble_k0(1000 + i), dtype=np.complex64)
        if i in (0, 47, 48, 63, 64, 67):
            fields[i] = f.astype(np.complex128)
        st[p.cplx_off[i]:p.cplx_off[i] + f.size] = torch.from_numpy(f.ravel()).to(DEV)
    say("autotune", p.autotune(st, B.PS_NS, 2))
    p.rk2_step(st, B.PS_NS, 5e-3, 0.0, 2e-3, 1)
    h = host(st)
    for i, f in fields.items():
        got = h[p.cplx_off[i]:p.cplx_off[i] + f.size].reshape(f.shape)
        want = ref.rk2_step(f, NS, 5e-3, 0.0, 2e-3, 1)
        assert rel_l2_w(got, want) < 2e-6, (i, rel_l2_w(got, want))


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_mhd512_slab_settings_bitwise(B, dt):
    """At the benchmark's size, the tuned in-order slabs (16) and the two
    overlapping chains of 32 and 64 slabs give the same two steps bit for bit
    (each plane's chain is the same arithmetic whichever slab or stream runs
    it)."""
    cdt = torch.complex64 if dt == "f32" else torch.complex128
    s0 = sparse_to_dev(synth.mhd_sparse(512, 3, 4, 3.0), cdt)
    p = B.Plan(512, 6, dt)
    p.set_variant("prune", 1)
    p.set_variant("form", 1)
    ref = None
    for pipe in (4, 8, 9):
        say("mhd512 slab settings", dt, "pipe", pipe)
        p.set_variant("pipe", pipe)
        s = s0.clone()
        p.rk2_step(s, B.PS_MHD, 5e-4, 5e-4, 1e-3, 2)
        torch.cuda.synchronize()
        if ref is None:
            ref = s
        else:
            iv = torch.int32 if dt == "f32" else torch.int64
            assert torch.equal(torch.view_as_real(s).view(iv), torch.view_as_real(ref).view(iv)), pipe
            del s
    p.close()
