"""Checkpoint and resume of a run's spectral state.

The paper's code writes its fields with parallel MPI I/O and writes nothing
in benchmark mode (Sec. 4); here a run saves the spectral state (the half
spectra ps_rk2_step advances, layout [box][f][kz][ky][kx <= nx/2]) with a JSON
header of what is needed to continue it, and resumes from it bit for bit.

File layout (one file, little-endian):
    b"PSCKPT1\\n"                   magic
    8-byte unsigned length L
    L bytes of UTF-8 JSON           header (see save)
    the state's bytes               complex64 or complex128, C order

The header also records the plan's kernel variants: the variants differ in
their order of rounding, so a resumed run reproduces the uninterrupted one
bit for bit only on the same variants (apply_variants sets them on a new
plan).  The header records the shape, the element type, the payload's size
and its SHA-256; load checks all of them and raises ValueError on any mismatch, so a
truncated or altered file is refused rather than resumed.  Nothing in a
checkpoint is executed: the header is JSON and the payload raw numbers.
Writes go to a temporary file in the same folder, then replace the target,
so a crash mid-write leaves any earlier checkpoint intact.
"""
from __future__ import annotations

import hashlib
import json
import os
import struct
from typing import Any, Dict, Optional, Sequence, Tuple, Union

import numpy as np
import torch

MAGIC = b"PSCKPT1\n"
_DTYPES = {torch.complex64: "complex64", torch.complex128: "complex128"}


def save(path: str, state: torch.Tensor, *, nfields: int, t: float, step: int, nu: float, eta: float,
         dt: float, sizes: Union[int, Sequence[int], None] = None, grid: Optional[Sequence[int]] = None,
         seed: Optional[Any] = None, variants: Optional[Dict[str, int]] = None,
         extra: Optional[Dict[str, Any]] = None) -> Dict[str, Any]:
    """Write `state` (a complex tensor on any device) and its header to `path`.

    Exactly one of sizes (the plan's box size N, or a list of sizes for an
    ensemble) and grid (nx, ny, nz) names the plan's boxes.
    t, step: the simulation time and step count reached;
    nu, eta, dt: the step's parameters; seed: whatever made the initial state;
    variants: the plan's kernel variants (Plan.variants()); extra: further
    JSON-serialisable fields.  Returns the header written."""
    if state.dtype not in _DTYPES:
        raise ValueError(f"state must be complex64 or complex128, not {state.dtype}")
    if (sizes is None) == (grid is None):
        raise ValueError("give exactly one of sizes and grid")
    if grid is not None and len(grid) != 3:
        raise ValueError("grid must be (nx, ny, nz)")
    host = state.detach().contiguous().to("cpu")
    payload = memoryview(np.ascontiguousarray(host.numpy())).cast("B")  # no copy
    header = {
        "format": "pseudospectral-state",
        "version": 1,
        "sizes": None if sizes is None else [int(n) for n in sizes] if isinstance(sizes, (list, tuple))
        else int(sizes),
        "grid": None if grid is None else [int(n) for n in grid],
        "nfields": int(nfields),
        "dtype": _DTYPES[state.dtype],
        "shape": list(host.shape),
        "t": float(t),
        "step": int(step),
        "nu": float(nu),
        "eta": float(eta),
        "dt": float(dt),
        "seed": seed,
        "variants": {str(k): int(v) for k, v in (variants or {}).items()},
        "payload_bytes": payload.nbytes,
        "sha256": hashlib.sha256(payload).hexdigest(),
    }
    if extra:
        header["extra"] = extra
    text = json.dumps(header, sort_keys=True).encode("utf-8")
    folder = os.path.dirname(os.path.abspath(path))
    tmp = os.path.join(folder, f".{os.path.basename(path)}.tmp{os.getpid()}")
    with open(tmp, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<Q", len(text)))
        f.write(text)
        f.write(payload)
        f.flush()
        os.fsync(f.fileno())
    os.replace(tmp, path)
    return header


def read_header(path: str) -> Dict[str, Any]:
    """The header of a checkpoint, without reading its payload."""
    with open(path, "rb") as f:
        return _header(f)


def _header(f) -> Dict[str, Any]:
    if f.read(len(MAGIC)) != MAGIC:
        raise ValueError("not a checkpoint of this format (bad magic)")
    raw = f.read(8)
    if len(raw) != 8:
        raise ValueError("checkpoint truncated in its header")
    (n,) = struct.unpack("<Q", raw)
    if n > 1 << 20:
        raise ValueError("checkpoint header implausibly long")
    text = f.read(n)
    if len(text) != n:
        raise ValueError("checkpoint truncated in its header")
    header = json.loads(text.decode("utf-8"))
    if header.get("format") != "pseudospectral-state" or header.get("version") != 1:
        raise ValueError("unknown checkpoint format or version")
    return header


def load(path: str, device: Union[str, torch.device, None] = None) -> Tuple[torch.Tensor, Dict[str, Any]]:
    """Read a checkpoint: (state on `device` (CPU if None), header).  Raises
    ValueError if the file is truncated, altered or of another format."""
    with open(path, "rb") as f:
        header = _header(f)
        dtype = {"complex64": np.complex64, "complex128": np.complex128}.get(header["dtype"])
        if dtype is None:
            raise ValueError(f"unknown element type {header['dtype']!r}")
        shape = tuple(int(s) for s in header["shape"])
        nbytes = int(np.prod(shape)) * np.dtype(dtype).itemsize
        if nbytes != header["payload_bytes"]:
            raise ValueError("checkpoint shape does not match its payload size")
        arr = np.empty(shape, dtype=dtype)  # the payload is read straight into it
        view = memoryview(arr).cast("B")
        got = 0
        while got < nbytes:  # a single read may return less (about 2 GB per system call)
            n = f.readinto(view[got:])
            if not n:
                break
            got += n
        if got != nbytes or f.read(1):
            raise ValueError(f"checkpoint payload is not the {nbytes} bytes its header says")
    if hashlib.sha256(view).hexdigest() != header["sha256"]:
        raise ValueError("checkpoint payload does not match its SHA-256")
    state = torch.from_numpy(arr)
    if device is not None:
        state = state.to(device)
    return state, header


def plan_args(header: Dict[str, Any]) -> Dict[str, Any]:
    """Keyword arguments of binding.Plan that recreate the checkpoint's boxes,
    fields and element type."""
    dtype = {"complex64": "f32", "complex128": "f64"}[header["dtype"]]
    boxes = {"grid": tuple(header["grid"])} if header.get("grid") else {"N": header["sizes"]}
    return {**boxes, "nfields": header["nfields"], "dtype": dtype}


def apply_variants(plan, header: Dict[str, Any]) -> Dict[str, int]:
    """Set the kernel variants a checkpoint recorded on `plan`; returns them.
    Raises ValueError if the plan's element type, field count or state size
    differs from the checkpoint's."""
    if _DTYPES[plan.complex_dtype] != header["dtype"] or plan.nfields != header["nfields"]:
        raise ValueError(f"plan ({_DTYPES[plan.complex_dtype]}, {plan.nfields} fields) does not match "
                         f"the checkpoint ({header['dtype']}, {header['nfields']} fields)")
    if plan.n_complex() != int(np.prod(header["shape"])):
        raise ValueError(f"plan holds {plan.n_complex()} spectral values, checkpoint "
                         f"{int(np.prod(header['shape']))}")
    v = header.get("variants") or {}
    for kind, value in v.items():
        plan.set_variant(kind, int(value))
    return dict(v)
