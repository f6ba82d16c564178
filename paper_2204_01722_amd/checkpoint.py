"""Checkpoint and resume of load stepping.

The load is applied in n equal increments (pseudo-time t = k / n, Section III-A); after
every converged load level the displacement, the level k and a fingerprint of the run
go to an ``.npz`` file, written to a temporary name and renamed so that a file is always
whole.  A run given an existing checkpoint of the same fingerprint continues after the
saved level; the linearisation needs no saving, since every load step starts by
evaluating the residual (and storing the state) at its starting point.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np
import torch

FORMAT = 1


def fingerprint(*arrays, extra="") -> str:
    """sha256 over the bytes of host copies of ``arrays`` (tensors or numpy) and ``extra``."""
    h = hashlib.sha256(extra.encode())
    for a in arrays:
        if a is None:
            h.update(b"none")
            continue
        a = a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else np.asarray(a)
        h.update(str(a.dtype).encode() + str(a.shape).encode())
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def save(path: str, u: torch.Tensor, level: int, n_steps: int, tag: str) -> None:
    """Writes the checkpoint of load level ``level`` (of ``n_steps``) atomically."""
    tmp = f"{path}.tmp.npz"
    try:
        np.savez(tmp, u=u.detach().cpu().numpy(), level=np.int64(level), n_steps=np.int64(n_steps),
                 tag=np.array(tag), format=np.int64(FORMAT))
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.remove(tmp)
        raise


def load(path: str, shape, n_steps: int, tag: str):
    """Reads a checkpoint and checks it belongs to this run; returns (u, level)."""
    with np.load(path, allow_pickle=False) as z:
        if int(z["format"]) != FORMAT:
            raise ValueError(f"{path}: checkpoint format {int(z['format'])}, expected {FORMAT}")
        if int(z["n_steps"]) != n_steps:
            raise ValueError(f"{path}: written for {int(z['n_steps'])} load steps, not {n_steps}")
        if str(z["tag"]) != tag:
            raise ValueError(f"{path}: written for another problem (fingerprint differs)")
        u = z["u"]
        level = int(z["level"])
    if tuple(u.shape) != tuple(shape):
        raise ValueError(f"{path}: displacement of shape {u.shape}, expected {tuple(shape)}")
    if not 0 <= level <= n_steps:
        raise ValueError(f"{path}: load level {level} outside 0..{n_steps}")
    return u, level


def run_load_steps(step, u: torch.Tensor, n_steps: int, path: str | None = None, tag: str = "",
                   stop_after: int | None = None):
    """Runs load levels k = 1..n_steps with ``step(k, u)``, which must leave ``u`` (updated
    in place) at the converged state of level k and may return per-step statistics.

    With ``path`` the state is saved after every level, and a checkpoint already there
    (same ``n_steps`` and ``tag``) makes the run continue after its level.  With
    ``stop_after`` the run stops once that level is reached (a job split over several
    allocations).  Returns ``(u, first_level_run, level_reached, stats_per_level)``."""
    if n_steps < 1:
        raise ValueError("n_steps must be at least 1")
    start = 0
    if path is not None and os.path.exists(path):
        saved, start = load(path, u.shape, n_steps, tag)
        u.copy_(torch.from_numpy(saved).to(device=u.device, dtype=u.dtype))
    last = n_steps if stop_after is None else min(n_steps, int(stop_after))
    stats = []
    level = start
    for k in range(start + 1, last + 1):
        stats.append(step(k, u))
        level = k
        if path is not None:
            save(path, u, k, n_steps, tag)
    return u, start + 1, level, stats
