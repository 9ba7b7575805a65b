"""The boundary's documented contract on the GPU.

* Default variants compute the documented (rotational) function on ANY
  input: not solenoidal, not dealiased, not even Hermitian.  The divergence
  form is opt-in; on such an input it computes a different function.
* The blow-up monitor of ps_rk2_step (PS_ERR_DIVERGED), and that it does not
  change a step it does not stop.
* The persistent autotune cache (PS_TUNE_CACHE).
* MHD diagnostics (kinetic and magnetic energy, cross-helicity) against the
  oracle.
"""
import numpy as np
import pytest
import torch

from gpu_util import DEV, host, rel_l2_w, rounded, say, to_dev
from oracle.psref import MHD, NS
from paper_1003_4322_amd import synth

pytestmark = pytest.mark.gpu
TOL_NL = {"f64": 1e-12, "f32": 2e-5}
TOL_STEP = {"f64": 1e-12, "f32": 2e-6}


@pytest.fixture(scope="module")
def B():
    from paper_1003_4322_amd import binding
    binding.lib()
    return binding


def general_input(N, nf, seed):
    """Complex Gaussian coefficients at every stored mode: no symmetry, no
    solenoidality, no truncation (Nyquist planes included)."""
    rng = np.random.default_rng(seed)
    s = (nf, N, N, N // 2 + 1)
    return 0.05 * (rng.standard_normal(s) + 1j * rng.standard_normal(s))


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("model", ["ns", "mhd"])
@pytest.mark.parametrize("N", [24, 32])
def test_defaults_on_general_input(B, ref, N, model, dt):
    say("general input", N, model, dt)
    mhd = model == "mhd"
    x = rounded(general_input(N, 6 if mhd else 3, 400 + N), dt)
    p = B.Plan(N, 6 if mhd else 3, dt)
    assert p.variant("form") == 0 and p.variant("prune") == 0
    xd = to_dev(x, dt)
    got = host(p.nonlinear_mhd(xd) if mhd else p.nonlinear_ns(xd))
    want = ref.nonlinear_mhd(x) if mhd else ref.nonlinear_ns(x)
    assert rel_l2_w(got, want) < TOL_NL[dt], rel_l2_w(got, want)
    # one RK2 step of the same state
    nu, eta, step = 0.02, 0.01, 1e-3
    p.rk2_step(xd, B.PS_MHD if mhd else B.PS_NS, nu, eta, step, 1)
    want_s = ref.rk2_step(x, MHD if mhd else NS, nu, eta, step, 1)
    assert rel_l2_w(host(xd), want_s) < TOL_STEP[dt], rel_l2_w(host(xd), want_s)
    # the divergence form is another function on such an input
    p.set_variant("form", 1)
    other = host(p.nonlinear_mhd(to_dev(x, dt)) if mhd else p.nonlinear_ns(to_dev(x, dt)))
    assert rel_l2_w(other, want) > 0.01, rel_l2_w(other, want)


@pytest.mark.parametrize("graphs", [True, False])
def test_monitor_stops_a_blowup(B, graphs):
    """dt = 1 on a random field is far beyond the explicit step's stability
    limit: the energy explodes (finite values at first, then overflow) and the
    monitor stops the run with PS_ERR_DIVERGED."""
    say("monitor blowup", graphs)
    N = 32
    u = synth.random_ns(N, 7, 3.0)
    p = B.Plan(N, 3, "f64")
    p.set_graphs(graphs)
    p.set_monitor(1, 100.0)
    s = to_dev(u, "f64")
    with pytest.raises(B.PsError) as ei:
        p.rk2_step(s, B.PS_NS, 0.0, 0.0, 1.0, 50)
    assert ei.value.code == -6
    assert "energy" in str(ei.value)


@pytest.mark.parametrize("graphs", [True, False])
def test_monitor_leaves_a_normal_step_alone(B, graphs):
    say("monitor normal", graphs)
    N = 32
    u = synth.random_ns(N, 8, 2.0)
    a, b = to_dev(u, "f64"), to_dev(u, "f64")
    p0 = B.Plan(N, 3, "f64")
    p1 = B.Plan(N, 3, "f64")
    p0.set_graphs(graphs)
    p1.set_graphs(graphs)
    p1.set_monitor(2, 1.5)
    p0.rk2_step(a, B.PS_NS, 0.02, 0.0, 1e-3, 5)
    p1.rk2_step(b, B.PS_NS, 0.02, 0.0, 1e-3, 5)
    assert torch.equal(a, b)
    with pytest.raises(B.PsError):
        p1.set_monitor(1, 1.0)
    with pytest.raises(B.PsError):
        p1.set_monitor(-1, 2.0)
    p1.set_monitor(0, 0.0)  # off


def test_pipe_settings_bitwise_equal(B):
    """Every slab-pipeline setting (concurrent and serial slabs, and more
    slabs than planes) computes the same step bit for bit: each plane's chain
    of passes is the same arithmetic whichever slab it falls in."""
    say("pipe settings bitwise")
    N = 192
    z = to_dev(synth.flat_solenoidal(N, 31, groups=2), "f32")
    p = B.Plan(N, 6, "f32")
    p.set_variant("prune", 1)
    p.set_variant("form", 1)
    ref = None
    for v in range(p.variant_count("pipe")):
        p.set_variant("pipe", v)
        s = z.clone()
        p.rk2_step(s, B.PS_MHD, 1e-3, 5e-4, 1e-3, 2)
        if ref is None:
            ref = s
        else:
            assert torch.equal(s, ref), v
    p.close()


@pytest.mark.parametrize("kind", ["ensemble", "grid"])
def test_pipe_settings_bitwise_other_plans(B, kind):
    """Every slab-pipeline setting on an ensemble of uneven boxes (NS) and on
    an nx x ny x nz grid (MHD) computes the same two steps bit for bit as one
    slab (slab counts are capped at each box's planes)."""
    say("pipe settings bitwise", kind)
    if kind == "ensemble":
        sizes = [16, 24, 32, 16]
        p = B.Plan(sizes, 3, "f64")
        z = torch.zeros(p.n_complex(), dtype=torch.complex128, device=DEV)
        for b, n in enumerate(sizes):
            f = synth.random_ns(n, 600 + b, synth.ensemble_k0(600 + b))
            z[p.cplx_off[b]:p.cplx_off[b] + f.size] = torch.from_numpy(np.ascontiguousarray(f).ravel()).to(DEV)
        model, nu, eta, dt = B.PS_NS, 1e-3, 0.0, 2e-3
    else:
        n = (32, 48, 64)
        p = B.Plan(nfields=6, dtype="f32", grid=n)
        u, b_ = synth.random_grid(*n, 41, 2.0), synth.random_grid(*n, 42, 2.0)
        z = to_dev(np.concatenate([u + b_, u - b_]), "f32")
        model, nu, eta, dt = B.PS_MHD, 1e-3, 5e-4, 1e-3
    p.set_variant("prune", 1)
    ref = None
    for v in range(p.variant_count("pipe")):
        p.set_variant("pipe", v)
        s = z.clone()
        p.rk2_step(s, model, nu, eta, dt, 2)
        r = torch.view_as_real(s)
        bits = r.view(torch.int64 if r.dtype == torch.float64 else torch.int32)
        if ref is None:
            ref = bits.clone()
        else:
            assert torch.equal(bits, ref), (kind, v)
    p.close()


def test_autotune_cache(B, tmp_path, monkeypatch):
    say("autotune cache")
    path = tmp_path / "tune.txt"
    path.write_text("garbage line without a tab\nother\tz_curl=1\n")
    monkeypatch.setenv("PS_TUNE_CACHE", str(path))
    N = 256
    u = to_dev(synth.random_ns(N, 2, 4.0), "f32")
    p1 = B.Plan(N, 3, "f32")
    p1.set_variant("prune", 1)
    v1 = p1.autotune(u, B.PS_NS, 1)
    assert p1.autotune_timed() > 0
    lines = path.read_text().splitlines()
    assert len(lines) == 3 and "\t" in lines[-1] and "pipe=" in lines[-1]
    p2 = B.Plan(N, 3, "f32")
    p2.set_variant("prune", 1)
    assert p2.autotune_timed() == -1
    v2 = p2.autotune(u, B.PS_NS, 1)
    assert p2.autotune_timed() == 0 and v2 == v1
    assert len(path.read_text().splitlines()) == 3
    p3 = B.Plan(N, 3, "f32")            # another key (prune differs): timed again
    p3.autotune(u, B.PS_NS, 1)
    assert p3.autotune_timed() > 0
    assert len(path.read_text().splitlines()) == 4


def test_autotune_overlap(B, tmp_path, monkeypatch):
    """With "overlap" 1 the autotuner may also choose the two-chain slab
    settings; whatever it chooses computes the one-slab step bit for bit, and
    the tuning cache keeps overlap-tuned and in-order-tuned entries apart."""
    say("autotune overlap")
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("PS_TUNE_CACHE", str(path))
    N = 256
    z = to_dev(synth.random_mhd(N, 3, 4, 3.0), "f32")

    def plan(overlap):
        p = B.Plan(N, 6, "f32")
        p.set_variant("prune", 1)
        p.set_variant("form", 1)
        p.set_variant("overlap", overlap)
        return p

    p1 = plan(1)
    v1 = p1.autotune(z, B.PS_MHD, 1)
    assert p1.autotune_timed() > 0 and v1["overlap"] == 1
    assert v1["pipe"] in (0, 4, 5, 6, 7, 8, 9), v1
    s = z.clone()
    p1.rk2_step(s, B.PS_MHD, 5e-4, 5e-4, 1e-3, 2)
    p1.set_variant("pipe", 0)
    s0 = z.clone()
    p1.rk2_step(s0, B.PS_MHD, 5e-4, 5e-4, 1e-3, 2)
    assert torch.equal(torch.view_as_real(s).view(torch.int32), torch.view_as_real(s0).view(torch.int32))
    p2 = plan(0)                          # another key: timed again, in-order settings only
    v2 = p2.autotune(z, B.PS_MHD, 1)
    assert p2.autotune_timed() > 0 and v2["pipe"] in (0, 4, 5, 6), v2
    p3 = plan(1)                          # the overlap entry again: from the file
    assert p3.autotune(z, B.PS_MHD, 1) == v1 and p3.autotune_timed() == 0
    assert len(path.read_text().splitlines()) == 2
    for p in (p1, p2, p3):
        p.close()


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("N", [16, 32])
def test_mhd_spectrum(B, ref, N, dt):
    say("mhd spectrum", N, dt)
    rng = np.random.default_rng(500 + N)
    s = (6, N, N, N // 2 + 1)
    z = rounded(rng.standard_normal(s) + 1j * rng.standard_normal(s), dt)
    p = B.Plan(N, 6, dt)
    spec, tot = p.mhd_spectrum(to_dev(z, dt))
    ws, wt = ref.mhd_spectrum(z)
    spec, tot = host(spec), host(tot)
    scale = ws[0] + ws[1]                     # per shell: Eu + Eb >= 2 |Hc|
    assert np.abs(spec - ws).max(axis=0).max() <= 1e-13 * scale.max()
    assert (np.abs(spec - ws) <= 1e-13 * scale[None, :] + 1e-300).all()
    assert np.abs(tot - wt).max() <= 1e-13 * (wt[0] + wt[1])
    # E(z+) + E(z-) = 2 (Eu + Eb) through the energy spectrum
    e, et = p.energy_spectrum(to_dev(z, dt))
    assert abs(host(et)[0] - 2 * (tot[0] + tot[1])) <= 1e-12 * host(et)[0]


def test_spectra_bitwise_reproducible(B):
    """Fixed-order sums: the same state gives the same bits, call after call."""
    say("spectra reproducible")
    N = 96
    z = synth.random_mhd(N, 41, 42, 6.0)
    p = B.Plan(N, 6, "f64")
    zd = to_dev(z, "f64")
    a = [t.clone() for t in p.mhd_spectrum(zd)]
    b = p.mhd_spectrum(zd)
    assert all(torch.equal(x, y) for x, y in zip(a, b))
    a = [t.clone() for t in p.energy_spectrum(zd)]
    b = p.energy_spectrum(zd)
    assert all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_mhd_spectrum_384(B, ref, dt):
    """333 shells: more than one round of shells per workgroup."""
    say("mhd spectrum 384", dt)
    N = 384
    rng = np.random.default_rng(777)
    s = (6, N, N, N // 2 + 1)
    z = rounded(rng.standard_normal(s) + 1j * rng.standard_normal(s), dt)
    p = B.Plan(N, 6, dt)
    spec, tot = p.mhd_spectrum(to_dev(z, dt))
    ws, wt = ref.mhd_spectrum(z)
    del z
    spec, tot = host(spec), host(tot)
    scale = ws[0] + ws[1]
    assert ws.shape[1] > 256
    assert (np.abs(spec - ws) <= 1e-13 * scale[None, :] + 1e-300).all()
    assert np.abs(tot - wt).max() <= 1e-13 * (wt[0] + wt[1])
    p.close()


def test_mhd_spectrum_ensemble(B, ref):
    say("mhd spectrum ensemble")
    sizes = [16, 16, 24]
    p = B.Plan(sizes, 6, "f64")
    zs = [synth.random_mhd(n, 80 + i, 90 + i, 3.0) for i, n in enumerate(sizes)]
    st = torch.empty(p.n_complex(), dtype=torch.complex128, device=DEV)
    for i, z in enumerate(zs):
        st[p.cplx_off[i]:p.cplx_off[i] + z.size] = torch.from_numpy(z.ravel()).to(DEV)
    spec, tot = p.mhd_spectrum(st)
    spec, tot = host(spec), host(tot)
    so = 0
    for i, z in enumerate(zs):
        ws, wt = ref.mhd_spectrum(z)
        n = p.nshells[i]
        got = spec[3 * so:3 * (so + n)].reshape(3, n)
        assert np.abs(got - ws).max() <= 1e-13 * (ws[0] + ws[1]).max()
        assert np.abs(tot[3 * i:3 * i + 3] - wt).max() <= 1e-13 * (wt[0] + wt[1])
        so += n
