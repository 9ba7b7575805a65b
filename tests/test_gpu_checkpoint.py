"""Resume from a checkpoint reproduces the uninterrupted run bit for bit:
ten RK2 steps in one go against five steps, save, a new plan (made from the
checkpoint's header) and a new state buffer loaded from the file, and five
more steps.  Cubes run on the benchmark's launch configuration (divergence
form, dealias pruning, autotuned variants, which the checkpoint carries to
the new plan); an ensemble of uneven boxes and an nx x ny x nz grid on the
default plan."""
import numpy as np
import pytest
import torch

from gpu_util import CDT, DEV, rounded, say, to_dev
from paper_1003_4322_amd import checkpoint as ck
from paper_1003_4322_amd import synth

pytestmark = pytest.mark.gpu

RECIPES = {  # nfields, nu, eta, dt
    "mhd": (6, 5e-4, 5e-4, 1e-3),
    "ns": (3, 1e-3, 0.0, 2e-3),
}


@pytest.fixture(scope="module")
def B():
    from paper_1003_4322_amd import binding
    binding.lib()
    return binding


def _bits(t: torch.Tensor) -> torch.Tensor:
    r = torch.view_as_real(t)
    return r.view(torch.int32 if r.dtype == torch.float32 else torch.int64)


def _resume_matches(B, tmp_path, name, make_plan, s0, pm, nf, nu, eta, step, boxes, tune):
    """10 steps straight against 5 + save + load into a new plan + 5."""
    say("checkpoint", name, "ten steps straight")
    p = make_plan()
    if tune:
        p.set_variant("prune", 1)
        p.set_variant("form", 1)
        p.autotune(s0.clone(), pm, 2)
    variants = p.variants()
    s = s0.clone()
    p.rk2_step(s, pm, nu, eta, step, 10)
    torch.cuda.synchronize()
    p.close()

    say("checkpoint", name, "five steps, save")
    q = make_plan()
    for k, v in variants.items():
        q.set_variant(k, v)
    s1 = s0.clone()
    q.rk2_step(s1, pm, nu, eta, step, 5)
    path = str(tmp_path / f"{name}.ckpt")
    ck.save(path, s1, nfields=nf, t=5 * step, step=5, nu=nu, eta=eta, dt=step, seed=name,
            variants=q.variants(), **boxes)
    q.close()
    del s1

    say("checkpoint", name, "load, five more steps")
    s2, h = ck.load(path, device=DEV)
    assert h["step"] == 5 and h["t"] == 5 * step and h["seed"] == name
    r = B.Plan(**ck.plan_args(h))
    assert ck.apply_variants(r, h) == variants
    r.rk2_step(s2, pm, h["nu"], h["eta"], h["dt"], 10 - h["step"])
    torch.cuda.synchronize()
    r.close()
    assert torch.isfinite(torch.view_as_real(s)).all()
    diff = int((_bits(s) != _bits(s2)).sum())
    say("differing words", diff)
    assert diff == 0


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("model,N", [("mhd", 64), ("ns", 128)])
def test_resume_bitwise(B, tmp_path, model, N, dt):
    nf, nu, eta, step = RECIPES[model]
    pm = B.PS_MHD if model == "mhd" else B.PS_NS
    x = rounded(synth.random_mhd(N, 3, 4, 3.0) if model == "mhd" else synth.random_ns(N, 2, 4.0), dt)
    _resume_matches(B, tmp_path, f"{model}{N}{dt}", lambda: B.Plan(N, nf, dt), to_dev(x, dt), pm,
                    nf, nu, eta, step, {"sizes": N}, tune=True)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_resume_ensemble_bitwise(B, tmp_path, dt):
    sizes = [16, 24, 32, 16]
    nf, nu, eta, step = RECIPES["ns"]
    p = B.Plan(sizes, nf, dt)
    flat = torch.empty(p.n_complex(), dtype=CDT[dt], device=DEV)
    for b, n in enumerate(sizes):
        f = rounded(synth.random_ns(n, 500 + b, synth.ensemble_k0(500 + b)), dt)
        flat[p.cplx_off[b]:p.cplx_off[b] + f.size] = torch.from_numpy(np.ascontiguousarray(f).ravel()).to(
            DEV, CDT[dt])
    p.close()
    _resume_matches(B, tmp_path, f"ensemble{dt}", lambda: B.Plan(sizes, nf, dt), flat, B.PS_NS, nf, nu,
                    eta, step, {"sizes": sizes}, tune=False)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_resume_grid_bitwise(B, tmp_path, dt):
    n = (32, 48, 64)
    nf, nu, eta, step = RECIPES["mhd"]
    u = synth.random_grid(*n, 11, 2.0)
    b = synth.random_grid(*n, 12, 2.0)
    x = rounded(np.concatenate([u + b, u - b]), dt)
    _resume_matches(B, tmp_path, f"grid{dt}", lambda: B.Plan(nfields=nf, dtype=dt, grid=n), to_dev(x, dt),
                    B.PS_MHD, nf, nu, eta, step, {"grid": n}, tune=False)
