#!/usr/bin/env python3
"""Benchmark of the pseudospectral RK2 hot path on one MI355X.

Default workload: incompressible MHD in Elsasser variables on a 512^3 box,
6 fields batched, nu = eta = 5e-4, dt = 1e-3; u and b independent
random-phase solenoidal fields (seeds 3 and 4) with E(k) ~ k^4 exp(-2 (k/3)^2)
and E_u = E_b = 1/2.  The FP32 form is the headline; the FP64 form runs the
same steps from the same (FP32-representable) initial state, and the relative
L2 distance between the two is reported.

One JSON line goes to stdout; progress goes to stderr.  The timed region is
K RK2 steps as the library runs them (a HIP graph replay per step) bracketed
by torch.cuda.synchronize(); K more steps with a HIP event pair around every
kernel on its stream give the per-kernel average durations, which with the
library's algorithmic byte counts give the achieved GB/s per pass.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RK2 steps/s + FFT GB/s (%HBM peak) at 512^3, FP32 vs FP64 at stated L2 err"
HBM_PEAK_GBS = 8000.0
ALU_PEAK_TFS = 78.6  # FP32 vector without packed instructions: 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz

WORKLOADS = {
    # name: (N, model, nu, eta, dt, seeds, k0)
    "mhd512": dict(N=512, model="mhd", nu=5e-4, eta=5e-4, dt=1e-3, seeds=(3, 4), k0=3.0),
    "ns256": dict(N=256, model="ns", nu=1e-3, eta=0.0, dt=2e-3, seeds=(2,), k0=4.0),
    "ns1024": dict(N=1024, model="ns", nu=2e-4, eta=0.0, dt=5e-4, seeds=(5,), k0=4.0),
    "ns32": dict(N=32, model="ns", nu=0.02, eta=0.0, dt=1e-3, seeds=(1,), k0=2.0),
    "ns512": dict(N=512, model="ns", nu=5e-4, eta=0.0, dt=1e-3, seeds=(3,), k0=3.0),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _code_only(text: str) -> str:
    """Source text without comments, whitespace runs collapsed."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def src_hash() -> str:
    """Hash of the device-side code (kernels, their configurations and
    launchers; comments excluded) that committed traffic counters belong to:
    host-only code (ps_api.cpp) does not change a kernel's traffic."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1003_4322_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            h.update(_code_only(open(os.path.join(d, f), encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def initial_state(w, dtype_c, device):
    """Sparse low-wavenumber cube from the generator, scattered on the GPU."""
    import numpy as np
    import torch

    from paper_1003_4322_amd import synth

    N = w["N"]
    if w["model"] == "mhd":
        sf = synth.mhd_sparse(N, w["seeds"][0], w["seeds"][1], w["k0"])
    else:
        sf = synth.random_solenoidal(N, w["seeds"][0], w["k0"])
    nf = sf.values.shape[0]
    st = torch.zeros((nf, N, N, N // 2 + 1), dtype=dtype_c, device=device)
    iz, iy, ix = sf.index_arrays()
    vals = torch.from_numpy(np.ascontiguousarray(sf.values)).to(device=device, dtype=dtype_c)
    fi = torch.arange(nf, device=device).view(-1, 1, 1, 1)
    zi = torch.as_tensor(iz, device=device).view(1, -1, 1, 1)
    yi = torch.as_tensor(iy, device=device).view(1, 1, -1, 1)
    xi = torch.as_tensor(ix, device=device).view(1, 1, 1, -1)
    st.index_put_((fi, zi, yi, xi), vals)
    return st, sf


def rel_l2_w(a, b):
    import torch
    N = a.shape[-2]
    w = torch.full((N // 2 + 1,), 2.0, dtype=torch.float64, device=a.device)
    w[0] = 1.0
    w[-1] = 1.0
    d = (a.to(torch.complex128) - b.to(torch.complex128)).abs() ** 2
    n = b.to(torch.complex128).abs() ** 2
    return math.sqrt(float((d * w).sum() / (n * w).sum()))


def run_timed(plan, state, model, w, steps, warmup):
    """Warmup, then the timed region: `steps` RK2 steps as the library runs
    them by default (one HIP graph replay per step), bracketed by
    synchronisations.  Then `steps` more with a HIP event pair around every
    kernel on the plan's stream (graphs off while timing) for the per-kernel
    table; the events cost a few microseconds per launch, so that region is
    reported beside the timed one, not as it.
    Returns (ms_per_step, per-kernel stats, ms_per_step of the event region)."""
    import torch

    plan.set_timing(False)
    plan.rk2_step(state, model, w["nu"], w["eta"], w["dt"], warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.rk2_step(state, model, w["nu"], w["eta"], w["dt"], steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    plan.set_timing(True)
    plan.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.rk2_step(state, model, w["nu"], w["eta"], w["dt"], steps)
    torch.cuda.synchronize()
    ms_events = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    stats = plan.timings()
    plan.set_timing(False)
    return ms, stats, ms_events


def pipe_slabs(pipe, nz):
    """z-slabs of slab-pipeline setting `pipe` (2^pipe for 1..6, 2^(pipe-3)
    for the two-chain settings 7..9), at most one per plane."""
    if pipe <= 0:
        return 1
    return min(2 ** (pipe - 3 if pipe >= 7 else pipe), nz)


def overlapped_slabs(plan, state0, model, w, steps, warmup, tuned):
    """The opt-in slab settings whose two chains of z-slabs overlap on two
    helper streams (pipe 7, 8, 9: 16, 32, 64 slabs), timed by graph replay
    beside the tuned in-order setting, in two interleaved rounds (best of
    each).  The autotuner does not choose them: their launches share the
    chip, so a launch's duration is no longer its own."""
    import torch

    base = (tuned or {}).get("pipe", plan.variant("pipe"))
    best = {}
    for _ in range(2):
        for pipe in (base, 7, 8, 9):
            plan.set_variant("pipe", pipe)
            s = state0.clone()
            plan.rk2_step(s, model, w["nu"], w["eta"], w["dt"], warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.rk2_step(s, model, w["nu"], w["eta"], w["dt"], steps)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
            best[pipe] = min(best.get(pipe, 1e30), ms)
            del s
    plan.set_variant("pipe", base)
    top = min((7, 8, 9), key=lambda v: best[v])
    return {"pipe": top, "slabs": pipe_slabs(top, 1 << 30), "steps_per_s": round(1e3 / best[top], 3),
            "ms_per_step": round(best[top], 4), "in_order_pipe": base,
            "in_order_ms_per_step": round(best[base], 4),
            "ms_per_step_by_pipe": {str(k): round(v, 4) for k, v in sorted(best.items())}}


def pass_table(stats):
    out = {}
    for k, s in stats.items():
        avg = s["total_ms"] / max(s["launches"], 1)
        gbs = s["bytes_per_launch"] / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
        out[k] = {"avg_ms": round(avg, 5), "launches": s["launches"],
                  "GB_per_launch": round(s["bytes_per_launch"] / 1e9, 6),
                  "GB/s": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                  "share_of_time": None}
    tot = sum(s["total_ms"] for s in stats.values()) or 1.0
    for k, s in stats.items():
        out[k]["share_of_time"] = round(s["total_ms"] / tot, 4)
    return out


def load_traffic(kernel_kind, workload, dtype, variants=None):
    """HBM traffic per launch from committed rocprofv3 counter runs, only if
    the kernel sources are unchanged since the counters were taken and the
    counters were taken in the same slab-pipeline setting (a launch covers
    the whole box or one slab)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    key = f"{workload}/{dtype}/{kernel_kind}"
    r = rec.get(key)
    if not r or r.get("src_hash") != src_hash():
        return None
    if r.get("pipe") != (variants or {}).get("pipe"):
        return None
    return r.get("bytes_per_launch")


def device_copy(nbytes: int = 1 << 31, reps: int = 10):
    """A plain device-to-device copy of known size (torch copy kernel): the
    practical HBM rate on this device and the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    n = nbytes // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    torch.cuda.empty_cache()
    return {"bytes_read": nbytes, "bytes_written": nbytes, "ms": round(ms, 4),
            "GB/s": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


def ensemble_run(steps: int = 100, warmup: int = 5):
    """48 NS boxes of 64^3 + 16 of 96^3 + 4 of 128^3, FP32, nu = 5e-3,
    dt = 2e-3, each seeded separately (seed 1000 + i, k0 uniform in [2, 5]):
    autotuned class-batched launches vs one box per launch, both replayed
    from captured graphs."""
    import numpy as np
    import torch

    from paper_1003_4322_amd import binding, synth

    sizes = [64] * 48 + [96] * 16 + [128] * 4
    plan = binding.Plan(sizes, 3, "f32", device="cuda:0")
    plan.set_variant("prune", PRUNE)
    plan.set_variant("form", FORM)
    st = torch.empty(plan.n_complex(), dtype=torch.complex64, device="cuda:0")
    for i, N in enumerate(sizes):
        f = synth.random_ns(N, 1000 + i, synth.ensemble_k0(1000 + i), dtype=np.complex64)
        st[plan.cplx_off[i]:plan.cplx_off[i] + f.size] = torch.from_numpy(f.ravel()).to("cuda:0")
    out = {"boxes": "48 x 64^3 + 16 x 96^3 + 4 x 128^3 NS FP32", "steps": steps}
    tuned = plan.autotune(st, binding.PS_NS, 3)
    for mode, name in ((0, "batched"), (1, "per_box")):
        plan.set_variant("batch", mode)
        s = st.clone()
        plan.rk2_step(s, binding.PS_NS, 5e-3, 0.0, 2e-3, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.rk2_step(s, binding.PS_NS, 5e-3, 0.0, 2e-3, steps)
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t0
        out[name] = {"steps_per_s": round(steps / dt_, 2), "ms_per_step": round(dt_ * 1e3 / steps, 4)}
    # per-kernel timing of the batched mode
    plan.set_variant("batch", 0)
    plan.set_timing(True)
    plan.timing_reset()
    s = st.clone()
    plan.rk2_step(s, binding.PS_NS, 5e-3, 0.0, 2e-3, 10)
    torch.cuda.synchronize()
    out["passes_batched"] = pass_table(plan.timings())
    plan.set_timing(False)
    out["variants"] = tuned
    out["speedup_batched_vs_per_box"] = round(out["batched"]["steps_per_s"] / out["per_box"]["steps_per_s"], 3)
    bytes_step = sum(v["GB_per_launch"] * v["launches"] for v in out["passes_batched"].values()) / 10
    out["GB_per_step"] = round(bytes_step, 4)
    out["effective_GB/s_batched"] = round(bytes_step * out["batched"]["steps_per_s"], 1)
    plan.close()
    return out


# the synthetic states are solenoidal and zero outside the 2/3 sphere, and
# the step keeps them so: the divergence form and dealias pruning apply
PRUNE = 1
FORM = 1


def form_for(model: str, dtype: str) -> int:
    """The divergence form, except for FP64 Navier-Stokes, whose product pass
    is faster in the rotational form at 1024^3 (measured; same result)."""
    return 0 if (FORM == 0 or (model == "ns" and dtype == "f64")) else 1


def grid_run(ms_cube: float, steps: int = 10):
    """MHD (Elsasser form) on a 512 x 512 x 1024 grid in a (2 pi, 2 pi, 4 pi)
    box rotating about z, FP32, autotuned: steps/s, the passes, and the time
    per grid point relative to the 512^3 headline step (1.0 = the same)."""
    import numpy as np
    import torch

    from paper_1003_4322_amd import binding, synth

    n = (512, 512, 1024)
    w = WORKLOADS["mhd512"]
    dev = torch.device("cuda:0")
    sf = synth.mhd_sparse(512, w["seeds"][0], w["seeds"][1], w["k0"])
    nx, ny, nz = n
    K = sf.K
    st = torch.zeros((6, nz, ny, nx // 2 + 1), dtype=torch.complex64, device=dev)
    kr = np.arange(-K, K + 1)
    st.index_put_((torch.arange(6, device=dev).view(-1, 1, 1, 1),
                   torch.as_tensor(kr % nz, device=dev).view(1, -1, 1, 1),
                   torch.as_tensor(kr % ny, device=dev).view(1, 1, -1, 1),
                   torch.arange(K + 1, device=dev).view(1, 1, 1, -1)),
                  torch.from_numpy(np.ascontiguousarray(sf.values)).to(dev, torch.complex64))
    plan = binding.Plan(nfields=6, dtype="f32", device=dev, grid=n)
    plan.set_variant("prune", PRUNE)
    plan.set_variant("form", FORM)
    plan.set_box(2 * np.pi, 2 * np.pi, 4 * np.pi)
    plan.set_rotation(0.0, 0.0, 2.0)
    tuned = plan.autotune(st, binding.PS_MHD, 2)
    plan.rk2_step(st, binding.PS_MHD, w["nu"], w["eta"], w["dt"], 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.rk2_step(st, binding.PS_MHD, w["nu"], w["eta"], w["dt"], steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan.set_timing(True)
    plan.timing_reset()
    plan.rk2_step(st, binding.PS_MHD, w["nu"], w["eta"], w["dt"], 2)
    torch.cuda.synchronize()
    passes = pass_table(plan.timings())
    plan.set_timing(False)
    ms = el * 1e3 / steps
    out = {"grid": list(n), "box": "(2 pi, 2 pi, 4 pi)", "omega": [0.0, 0.0, 2.0], "dtype": "f32",
           "steps": steps, "steps_per_s": round(1e3 / ms, 3), "ms_per_step": round(ms, 3),
           "time_per_point_vs_512^3": round(ms / (2.0 * ms_cube), 3),
           "variants": tuned, "passes": passes,
           "energy_after": float(plan.energy_spectrum(st)[1][0].item())}
    plan.close()
    del st
    torch.cuda.empty_cache()
    return out


def precision_pair(wname: str, steps: int, warmup: int = 2, spectra_every: int = 0):
    """FP32 and FP64 forms of a workload from the same FP32-representable
    initial state: steps/s of each and the FP32-vs-FP64 distance; optional
    energy spectra every few steps (FP64, deterministic)."""
    import torch

    from paper_1003_4322_amd import binding

    w = WORKLOADS[wname]
    dev = torch.device("cuda:0")
    model = binding.PS_MHD if w["model"] == "mhd" else binding.PS_NS
    nf = 6 if w["model"] == "mhd" else 3
    s32, _ = initial_state(w, torch.complex64, dev)
    res = {"N": w["N"], "fields": nf, "steps": steps}
    finals = {}
    for dt in ("f32", "f64"):
        s = s32.clone() if dt == "f32" else s32.to(torch.complex128)
        plan = binding.Plan(w["N"], nf, dt, device=dev)
        plan.set_variant("prune", PRUNE)
        plan.set_variant("form", form_for(w["model"], dt))
        tuned = plan.autotune(s, model, 2)
        one = s.clone()  # one step from the identical initial state
        plan.rk2_step(one, model, w["nu"], w["eta"], w["dt"], 1)
        plan.rk2_step(s, model, w["nu"], w["eta"], w["dt"], warmup)
        torch.cuda.synchronize()
        spectra = []
        t0 = time.perf_counter()
        if spectra_every:
            done = 0
            while done < steps:
                k = min(spectra_every, steps - done)
                plan.rk2_step(s, model, w["nu"], w["eta"], w["dt"], k)
                done += k
                spectra.append(plan.energy_spectrum(s))
        else:
            plan.rk2_step(s, model, w["nu"], w["eta"], w["dt"], steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        r = {"steps_per_s": round(steps / el, 3), "ms_per_step": round(el * 1e3 / steps, 3),
             "variants": tuned}
        if spectra:
            r["energy_every_%d_steps" % spectra_every] = [float(t[1][0].item()) for t in spectra]
            r["spectrum_last_first_16_shells"] = [float(x) for x in spectra[-1][0][:16].cpu()]
        finals[dt] = (s, one)
        res[dt] = r
        del plan
        torch.cuda.empty_cache()
    a, b = finals["f32"], finals["f64"]
    res["l2_f32_vs_f64_one_step"] = rel_l2_w(a[1], b[1])
    del s32
    res[f"l2_f32_vs_f64_after_{warmup + steps}_steps"] = rel_l2_w(a[0], b[0])
    res["tolerance_per_step"] = 2e-6
    return res


def host_info():
    """Cores this process may use, the CPU model and the host's memory."""
    info = {"nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        for line in open("/proc/meminfo"):
            k, v = line.split(":", 1)
            if k in ("MemTotal", "MemAvailable"):
                info[k + "_GB"] = round(float(v.split()[0]) * 1024 / 1e9, 1)
    except OSError:
        pass
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        keep = ("CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)", "NUMA node(s)",
                "CPU max MHz", "L3 cache")
        info["lscpu"] = {k.strip(): v.strip() for k, v in (l.split(":", 1) for l in out.splitlines() if ":" in l)
                         if k.strip() in keep}
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return info


def model_step_bytes(N: int, nf: int, real_bytes: int = 8) -> float:
    """Bytes of one RK2 step in the fused-pipeline byte model (93 half-spectrum
    fields for NS, 186 for MHD, unpruned), the yardstick the oracle's rate is
    quoted on."""
    sc = N * N * (N // 2 + 1) * 2.0 * real_bytes
    return (186 if nf == 6 else 93) * sc


def oracle_step_bytes(N: int, nf: int) -> float:
    """Host memory of one oracle RK2 step (FP64): the state, its copy, z* and
    the right-hand side (4 x nf half spectra), the nonlinear term's spectral
    temporaries (3 x 3 + 1 fields) and its physical fields (6 or 12 of N^3)."""
    sc = N * N * (N // 2 + 1) * 16.0
    return 4 * nf * sc + 10 * sc + (12 if nf == 6 else 6) * N ** 3 * 8.0


def cpu_baseline(w, sample_N: int = 0, single_N: int = 128):
    """The FP64 oracle, as it stands, timed on this host: one RK2 step of the
    workload's recipe on all cores at the workload's own size when the host
    has the memory (else at sample_N), and one step on a single thread at
    single_N.  Measured values only: nothing is scaled to another size."""
    import numpy as np

    from oracle.psref import MHD, NS, oracle
    from paper_1003_4322_amd import synth

    o = oracle()
    host = host_info()
    mhd = w["model"] == "mhd"
    nf = 6 if mhd else 3
    N = w["N"]
    avail = host.get("MemAvailable_GB", 0.0) * 1e9
    if not sample_N:
        sample_N = N if avail > 1.3 * oracle_step_bytes(N, nf) + 8e9 else 256

    def recipe(n):
        if mhd:
            sf = synth.mhd_sparse(n, w["seeds"][0], w["seeds"][1], w["k0"])
        else:
            sf = synth.random_solenoidal(n, w["seeds"][0], w["k0"])
        # the FP32-representable values the GPU's FP32 run starts from
        return synth.SparseField(n, sf.K, sf.values.astype(np.complex64).astype(np.complex128)).dense()

    def one_step(n, threads):
        z = recipe(n)
        used = o.set_threads(threads)
        t0 = time.perf_counter()
        o.rk2_step(z, MHD if mhd else NS, w["nu"], w["eta"], w["dt"], 1)
        return time.perf_counter() - t0, used

    t_all, cores = one_step(sample_N, len(os.sched_getaffinity(0)))
    t_one, _ = one_step(single_N, 1)
    o.set_threads(cores)
    what = f"{'MHD' if mhd else 'NS'} {sample_N}^3"
    res = {"value": 1.0 / t_all, "unit": "steps/s", "cores": cores, "kind": "oracle",
           "sample": f"one FP64 RK2 step (the first of the run) of the {what} recipe on {cores} "
                     f"threads: {t_all:.2f} s, measured" +
                     ("" if sample_N == N else f"; the {N}^3 step does not fit this host's memory, "
                                               f"so the value is the {sample_N}^3 rate, not scaled"),
           "measured": {"N": sample_N, "threads": cores, "s_per_step": round(t_all, 3),
                        "steps_per_s": round(1.0 / t_all, 5),
                        "GB_per_s_byte_model": round(model_step_bytes(sample_N, nf) / t_all / 1e9, 3)},
           "single_thread": {"N": single_N, "threads": 1, "s_per_step": round(t_one, 3),
                             "steps_per_s": round(1.0 / t_one, 5),
                             "GB_per_s_byte_model": round(model_step_bytes(single_N, nf) / t_one / 1e9, 3)},
           "host": host}
    return res


def diagnostics(plan, state, nf):
    """FP64 global quantities of the state (deterministic compensated sums):
    MHD kinetic and magnetic energy and cross-helicity, or NS energy,
    enstrophy and max |k . u|."""
    if nf == 6:
        _, t = plan.mhd_spectrum(state)
        t = t.cpu().tolist()
        return {"E_u": t[0], "E_b": t[1], "H_c": t[2]}
    _, t = plan.energy_spectrum(state)
    t = t.cpu().tolist()
    return {"E": t[0], "Z": t[1], "maxdiv": t[2]}


def run_primary(args, w, model, nf, N, dev):
    """The headline workload: FP32 timed region (+ FP64 side by side)."""
    import torch

    from paper_1003_4322_amd import binding

    s32, _ = initial_state(w, torch.complex64, dev)
    s32_0 = s32.clone()
    plan32 = binding.Plan(N, nf, "f32", device=dev)
    plan32.set_variant("prune", PRUNE)
    plan32.set_variant("form", FORM)
    log("fp32 plan ready, workspace GB", plan32.workspace_bytes() / 1e9)
    diag = {"initial": diagnostics(plan32, s32, nf)}
    tuned32 = None if args.no_tune else plan32.autotune(s32, model, 3)
    log("fp32 variants", tuned32)
    ms, stats, ms_events = run_timed(plan32, s32, model, w, args.steps, args.warmup)
    passes32 = pass_table(stats)
    log(f"fp32: {ms:.3f} ms/step (with per-kernel events {ms_events:.3f})")
    overlap = {}
    if not args.no_extras:
        overlap["f32"] = overlapped_slabs(plan32, s32_0, model, w, args.steps, args.warmup, tuned32)
        log("fp32 overlapped slab chains", overlap["f32"])
    diag[f"after_{args.warmup + 2 * args.steps}_steps"] = diagnostics(plan32, s32, nf)
    log("fp32 diagnostics", diag)

    dom = max(stats, key=lambda k: stats[k]["total_ms"])
    d = passes32[dom]
    traffic = load_traffic(dom, args.workload, "f32", tuned32)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": d["GB/s"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(d["GB/s"] / HBM_PEAK_GBS, 4),
                "traffic": traffic}
    if dom == "x_prod":
        # the same launch against the vector ALU: real transforms of length N
        # per grid row (inverse inputs + forward products), 2.5 N log2 N flops
        # each, over N^2 rows; FP32 without packed instructions peaks at
        # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz = 78.6 TFLOP/s
        nt = (8 if FORM == 1 else 9) if nf == 3 else (14 if FORM == 1 else 18)
        # a launch covers one z-slab of the box under the slab pipeline
        slabs = pipe_slabs((tuned32 or {}).get("pipe", 0), N)
        flops = nt * N * N * 2.5 * N * math.log2(N) / slabs
        tf = flops / (d["avg_ms"] * 1e-3) / 1e12
        roofline["alu_view"] = {"bound": "alu", "achieved": round(tf, 2), "peak": ALU_PEAK_TFS,
                                "unit": "TFLOP/s", "frac": round(tf / ALU_PEAK_TFS, 4),
                                "flops_per_launch": flops}

    fp64 = None
    if not args.no_fp64:
        s64 = s32_0.to(torch.complex128)
        s64_0 = s64.clone()
        del plan32
        torch.cuda.empty_cache()
        plan64 = binding.Plan(N, nf, "f64", device=dev)
        plan64.set_variant("prune", PRUNE)
        plan64.set_variant("form", form_for(w["model"], "f64"))
        tuned64 = None if args.no_tune else plan64.autotune(s64, model, 3)
        log("fp64 variants", tuned64)
        ms64, stats64, ms64_events = run_timed(plan64, s64, model, w, args.steps, args.warmup)
        log(f"fp64: {ms64:.3f} ms/step (with per-kernel events {ms64_events:.3f})")
        if not args.no_extras:
            overlap["f64"] = overlapped_slabs(plan64, s64_0, model, w, args.steps, args.warmup, tuned64)
            log("fp64 overlapped slab chains", overlap["f64"])
        # same number of steps from the same initial state in both precisions
        l2_run = rel_l2_w(s32, s64)
        # one step from the identical initial state
        a, b = s32_0.clone(), s64_0.clone()
        plan64.rk2_step(b, model, w["nu"], w["eta"], w["dt"], 1)
        del plan64
        torch.cuda.empty_cache()
        plan32 = binding.Plan(N, nf, "f32", device=dev)
        plan32.set_variant("prune", PRUNE)
        plan32.set_variant("form", FORM)
        for k, v in (tuned32 or {}).items():
            plan32.set_variant(k, v)
        plan32.rk2_step(a, model, w["nu"], w["eta"], w["dt"], 1)
        torch.cuda.synchronize()
        l2_1 = rel_l2_w(a, b)
        inc = rel_l2_w(a.to(torch.complex128) - s64_0, b - s64_0)
        fp64 = {"steps_per_s": round(1e3 / ms64, 3), "ms_per_step": round(ms64, 3),
                "ms_per_step_events": round(ms64_events, 3), "passes": pass_table(stats64),
                "variants": tuned64,
                "l2_f32_vs_f64_one_step": l2_1,
                "l2_f32_vs_f64_increment_one_step": inc,
                f"l2_f32_vs_f64_after_{args.warmup + 2 * args.steps}_steps": l2_run,
                "tolerance_per_step": 2e-6}
        log(f"fp32 vs fp64: one step {l2_1:.3e}, increment {inc:.3e}, run {l2_run:.3e}")

    return ms, ms_events, tuned32, passes32, roofline, fp64, diag, overlap


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mhd512", choices=sorted(WORKLOADS))
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="size of the oracle's all-core step (0: the workload's own if it fits)")
    ap.add_argument("--copy-only", action="store_true",
                    help="only the reference device copy (for counter scaling)")
    ap.add_argument("--no-tune", action="store_true", help="default kernel variants")
    ap.add_argument("--no-prune", action="store_true",
                    help="transform every pencil (no dealias-sphere pruning)")
    ap.add_argument("--rotational", action="store_true",
                    help="the rotational form of the nonlinear term instead of the divergence form")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 256^3, 1024^3, ensemble, 32^3 and 512x512x1024 workloads")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the hot path keeps the whole box on one device "
              f"and has no multi-GPU path (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1003_4322_amd import binding

    global PRUNE, FORM
    PRUNE = 0 if args.no_prune else 1
    FORM = 0 if args.rotational else 1
    w = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_only:
        print(json.dumps({"device_copy": device_copy()}), flush=True)
        return
    copy_ref = device_copy()
    log(f"device copy: {copy_ref['GB/s']} GB/s")
    model = binding.PS_MHD if w["model"] == "mhd" else binding.PS_NS
    nf = 6 if w["model"] == "mhd" else 3
    N = w["N"]
    log(f"workload {args.workload}: N={N} fields={nf} steps={args.steps} warmup={args.warmup}")

    ms, ms_events, tuned32, passes32, roofline, fp64, diag, overlap = run_primary(args, w, model, nf, N, dev)
    torch.cuda.empty_cache()

    extras = None
    if not args.no_extras:
        extras = {}
        log("extra: NS 256^3 FP32/FP64, 50 steps, spectra every 10")
        extras["ns256"] = precision_pair("ns256", 50, spectra_every=10)
        log("extra: NS 1024^3 FP32 vs FP64, 10 steps")
        extras["ns1024"] = precision_pair("ns1024", 10)
        log("extra: ensemble")
        extras["ensemble"] = ensemble_run()
        log("extra: NS 32^3 FP64 latency")
        extras["ns32"] = precision_pair("ns32", 200)
        log("extra: MHD 512 x 512 x 1024 FP32, rotating, (2 pi, 2 pi, 4 pi) box")
        extras["mhd_grid"] = grid_run(ms)

    cpu = None
    if not args.no_cpu:
        log("cpu baseline: the oracle, one step on all cores and one on a single thread")
        cpu = cpu_baseline(w, args.cpu_sample)
        log(f"cpu baseline: {cpu['sample']}")

    line = {
        "metric": METRIC, "value": round(1e3 / ms, 3), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{'MHD Elsasser' if nf == 6 else 'NS'} {N}^3 RK2, {nf} fields "
                               f"batched, nu={w['nu']}, eta={w['eta']}, dt={w['dt']}, "
                               f"random-phase k0={w['k0']} seeds {list(w['seeds'])}",
                   "N": N, "fields": nf, "workload_key": args.workload,
                   "prune": PRUNE,
                   "form": "divergence" if FORM == 1 else "rotational"},
        "ms_per_step_events": round(ms_events, 4),
        "variants": tuned32,
        "passes": passes32,
        "device_copy": copy_ref,
        "roofline": roofline,
        "fp64": fp64,
        "overlapped_slab_chains": overlap or None,
        "diagnostics": diag,
        "extras": extras,
        "cpu_baseline": cpu,
        "src_hash": src_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
