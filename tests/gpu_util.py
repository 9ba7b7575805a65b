"""Helpers shared by the GPU tests: device transfer, error norms, flushed
progress lines naming each case before it runs on the GPU."""
import sys

import numpy as np
import torch

DEV = "cuda:0"
CDT = {"f32": torch.complex64, "f64": torch.complex128}
RDT = {"f32": torch.float32, "f64": torch.float64}
NPC = {"f32": np.complex64, "f64": np.complex128}
NPR = {"f32": np.float32, "f64": np.float64}


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


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
