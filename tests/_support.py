"""Shared helpers for the tests: building meshes, moving them to the device and
computing oracle references on the same seeded inputs."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2204_01722_amd import inputs  # noqa: E402

MU, LAM = inputs.lame(1.0, 0.3)


def ensure_built():
    """Builds the library if (and only if) it is not there yet."""
    from paper_2204_01722_amd import binding, build
    if not os.path.exists(binding.LIB_PATH):
        build.build()


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


def rel(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rel_max(a, b):
    """Max-norm relative error ``max|a - b| / max|b|``."""
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    mb = np.abs(b).max() if b.size else 0.0
    return np.abs(a - b).max() / (mb if mb > 0 else 1.0) if a.size else 0.0


def report(name, got, ref):
    """Relative errors of ``got`` against ``ref`` in the 2-norm and, element by element, in
    the max-norm (both printed); returns the larger, which the caller holds to the
    tolerance, so that both norms meet it."""
    e2, einf = rel(got, ref), rel_max(got, ref)
    print(f"  {name}: rel 2-norm {e2:.2e}, rel max-norm {einf:.2e}", flush=True)
    return max(e2, einf)


def t2n(t):
    return t.detach().double().cpu().numpy()


def incident_elements(elem_nodes, nodes):
    """Indices of the elements that contain any of ``nodes``."""
    return np.nonzero(np.isin(elem_nodes, nodes).any(axis=1))[0]


def print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
