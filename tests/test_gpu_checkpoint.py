"""Resume from a checkpoint reproduces the uninterrupted run bit for bit:
ten RK2 steps in one go against five steps, save, a new plan and a new
state buffer loaded from the file, and five more steps.  Runs on the
benchmark's launch configuration (divergence form, dealias pruning,
autotuned variants, which the checkpoint carries to the new plan)."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, rounded, say, to_dev
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


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("model,N", [("mhd", 64), ("ns", 128)])
def test_resume_bitwise(B, tmp_path, model, N, dt):
    nf, nu, eta, step = RECIPES[model]
    pm = B.PS_MHD if model == "mhd" else B.PS_NS
    x = rounded(synth.random_mhd(N, 3, 4, 3.0) if model == "mhd" else synth.random_ns(N, 2, 4.0), dt)

    say("checkpoint", model, N, dt, "ten steps straight")
    p = B.Plan(N, nf, dt)
    p.set_variant("prune", 1)
    p.set_variant("form", 1)
    s = to_dev(x, dt)
    variants = p.autotune(s, pm, 2)
    s = to_dev(x, dt)
    p.rk2_step(s, pm, nu, eta, step, 10)
    torch.cuda.synchronize()
    p.close()

    say("checkpoint", model, N, dt, "five steps, save")
    q = B.Plan(N, nf, dt)
    for k, v in variants.items():
        q.set_variant(k, v)
    s1 = to_dev(x, dt)
    q.rk2_step(s1, pm, nu, eta, step, 5)
    path = str(tmp_path / f"{model}{N}{dt}.ckpt")
    ck.save(path, s1, sizes=N, nfields=nf, t=5 * step, step=5, nu=nu, eta=eta, dt=step,
            seed=[3, 4] if model == "mhd" else 2, variants=q.variants(), extra={"model": model})
    q.close()
    del s1

    say("checkpoint", model, N, dt, "load, five more steps")
    s2, h = ck.load(path, device=DEV)
    assert h["step"] == 5 and h["t"] == 5 * step and h["extra"]["model"] == model
    r = B.Plan(h["sizes"], h["nfields"], dt)
    assert ck.apply_variants(r, h) == variants
    r.rk2_step(s2, pm, h["nu"], h["eta"], h["dt"], 10 - h["step"])
    torch.cuda.synchronize()
    r.close()
    assert torch.isfinite(torch.view_as_real(s)).all()
    diff = int((_bits(s) != _bits(s2)).sum())
    say("differing words", diff)
    assert diff == 0
