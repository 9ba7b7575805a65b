"""Helpers shared by the GPU tests: device transfer, error norms, flushed
progress lines naming each case before it runs on the GPU."""
import os
import sys

import numpy as np
import torch

DEV = "cuda:0"
CDT = {"f32": torch.complex64, "f64": torch.complex128}
RDT = {"f32": torch.float32, "f64": torch.float64}
NPC = {"f32": np.complex64, "f64": np.complex128}
NPR = {"f32": np.float32, "f64": np.float64}


def say(*a):
    """Progress line naming the case (flushed before the GPU work it names);
    also appended to the file PS_TEST_LOG names, if any, so that the values
    passing tests measured are kept."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()
    path = os.environ.get("PS_TEST_LOG")
    if path:
        with open(path, "a") as f:
            print("[case]", *a, file=f)


def to_dev(a: np.ndarray, dt: str, kind: str = "c") -> torch.Tensor:
    npdt = NPC[dt] if kind == "c" else NPR[dt]
    return torch.from_numpy(np.ascontiguousarray(a.astype(npdt))).to(DEV)


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def rounded(a: np.ndarray, dt: str) -> np.ndarray:
    """The values a GPU run of precision dt starts from, promoted to FP64."""
    if dt == "f64":
        return np.ascontiguousarray(a)
    return a.astype(NPC[dt] if np.iscomplexobj(a) else NPR[dt]).astype(
        np.complex128 if np.iscomplexobj(a) else np.float64)


def hweights(N: int) -> np.ndarray:
    w = np.full(N // 2 + 1, 2.0)
    w[0] = 1.0
    w[-1] = 1.0
    return w


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def rel_l2_w(a: np.ndarray, b: np.ndarray) -> float:
    """Hermitian-weighted relative L2 over half spectra (= physical-space L2)."""
    w = np.full(a.shape[-1], 2.0)  # kx = 0 and kx = nx/2 count once
    w[0] = 1.0
    w[-1] = 1.0
    num = np.sum(w * np.abs(a - b) ** 2)
    den = np.sum(w * np.abs(b) ** 2)
    return float(np.sqrt(num / (den if den > 0 else 1.0)))


_SHELLS = {}


def shells_of(N: int):
    """(order, starts, shell ids): the half-spectrum storage indices of an N^3
    box sorted by shell round(|k|) (exact integer rule: smallest s with
    4|k|^2 < (2s+1)^2), the first position of every shell in that order and
    the shell of each run."""
    if N not in _SHELLS:
        from paper_1003_4322_amd import synth
        k = np.where(np.arange(N) < N // 2, np.arange(N), np.arange(N) - N).astype(np.int64)
        k2 = (k[:, None, None] ** 2 + k[None, :, None] ** 2 +
              np.arange(N // 2 + 1, dtype=np.int64)[None, None, :] ** 2)
        sh = synth.shell_index(k2).ravel()
        order = np.argsort(sh, kind="stable")
        ss = sh[order]
        starts = np.concatenate([[0], np.nonzero(np.diff(ss))[0] + 1])
        _SHELLS[N] = (order, starts, ss[starts])
    return _SHELLS[N]


def shell_err(got: np.ndarray, want: np.ndarray):
    """Per-shell element-wise error: for every shell s where the reference is
    not zero, max_{k in s} |got - want| / max_{k in s} |want| (over all
    fields).  Returns (worst value, its shell, max |got| where want is zero)."""
    N = want.shape[-2]
    order, starts, ids = shells_of(N)
    d = np.abs(got - want).max(axis=0).ravel()
    r = np.abs(want).max(axis=0).ravel()
    dm = np.maximum.reduceat(d[order], starts)
    rm = np.maximum.reduceat(r[order], starts)
    live = rm > 0
    ratio = np.where(live, dm / np.where(live, rm, 1.0), 0.0)
    i = int(np.argmax(ratio))
    zero = r == 0
    outside = float(np.abs(got).max(axis=0).ravel()[zero].max()) if np.any(zero) else 0.0
    return float(ratio[i]), int(ids[i]), outside


_SHELLS_DEV = {}


def shell_err_dev(got: torch.Tensor, want: torch.Tensor):
    """shell_err on device tensors (same definition, computed with torch on
    the GPU: the reference values were made by the oracle on the host)."""
    N = want.shape[-2]
    key = (N, str(want.device))
    if key not in _SHELLS_DEV:
        order, starts, ids = shells_of(N)
        sh = np.empty(order.size, np.int64)
        sh[order] = np.repeat(ids, np.diff(np.concatenate([starts, [order.size]])))
        _SHELLS_DEV[key] = torch.from_numpy(sh).to(want.device)
    sh = _SHELLS_DEV[key]
    ns = int(sh.max().item()) + 1
    w = want.to(torch.complex128)
    d = (got.to(torch.complex128) - w).abs().amax(dim=0).flatten()
    r = w.abs().amax(dim=0).flatten()
    z = torch.zeros(ns, dtype=torch.float64, device=want.device)
    dm = z.clone().scatter_reduce_(0, sh, d, reduce="amax")
    rm = z.clone().scatter_reduce_(0, sh, r, reduce="amax")
    ratio = torch.where(rm > 0, dm / torch.where(rm > 0, rm, torch.ones_like(rm)), z)
    i = int(torch.argmax(ratio).item())
    zero = r == 0
    outside = float(got.abs().amax(dim=0).flatten()[zero].max().item()) if bool(zero.any()) else 0.0
    return float(ratio[i].item()), i, outside


def rel_l2_w_dev(a: torch.Tensor, b: torch.Tensor) -> float:
    """rel_l2_w on device tensors."""
    w = torch.full((a.shape[-1],), 2.0, dtype=torch.float64, device=a.device)
    w[0] = 1.0
    w[-1] = 1.0
    bb = b.to(torch.complex128)
    num = ((a.to(torch.complex128) - bb).abs() ** 2 * w).sum()
    den = (bb.abs() ** 2 * w).sum()
    return float(torch.sqrt(num / torch.clamp(den, min=1e-300)).item())
