"""Moves a box mesh to the device and builds the operator hierarchy of a p-multigrid
solve (fine operator plus coarse operators on the same elements and quadrature)."""
from __future__ import annotations

import numpy as np
import torch

from . import inputs
from .binding import Operator


class Hierarchy:
    """Level operators for orders ``orders[0] > orders[1] > ...`` on one box mesh."""

    def __init__(self, mesh: inputs.BoxMesh, orders, faces: dict | None = None, mu=None, lam=None,
                 mu_e=None, lam_e=None, q=None, device="cuda"):
        if orders[0] != mesh.p:
            raise ValueError("orders[0] must be the mesh order")
        self.mesh = mesh
        self.orders = list(orders)
        self.device = torch.device(device)
        Q = mesh.P if q is None else q
        self.coords = torch.from_numpy(mesh.coords).to(self.device)
        self.ops, self.masks, self.topos = [], [], []
        if mu is None:
            mu, lam = inputs.lame(1.0, 0.3)
        self.mu_e_t = None if mu_e is None else torch.from_numpy(np.asarray(mu_e, np.float64)).to(self.device)
        self.lam_e_t = None if lam_e is None else torch.from_numpy(np.asarray(lam_e, np.float64)).to(self.device)
        for l, p in enumerate(self.orders):
            topo = mesh.elem_nodes if l == 0 else inputs.box_topology(mesh.n, p)
            nn = int(np.prod([p * n + 1 for n in mesh.n]))
            mask = None
            if faces:
                mask = inputs.face_mask(None, faces, p=p, n=mesh.n) if l else inputs.face_mask(mesh, faces)
            en = torch.from_numpy(np.ascontiguousarray(topo, np.int32)).to(self.device)
            mk = None if mask is None else torch.from_numpy(np.ascontiguousarray(mask)).to(self.device)
            op = Operator(p + 1, Q, en, nn, mk, fine=None if l == 0 else self.ops[0])
            if l == 0:
                op.set_material(mu, lam, self.mu_e_t, self.lam_e_t)
            self.ops.append(op)
            self.masks.append(mask)
            self.topos.append(topo)
        self.ops[0].qdata_setup(self.coords.reshape(-1, 3))

    @property
    def fine(self) -> Operator:
        return self.ops[0]

    def seeds(self, seed=7):
        """Rough start vectors (uniform(-1, 1) on free components) for each smoothed level."""
        out = []
        for l in range(len(self.ops) - 1):
            v = inputs.rough_seed(self.ops[l].n_nodes, self.masks[l], seed + l)
            out.append(torch.from_numpy(v).to(self.device))
        return out
