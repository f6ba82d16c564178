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
                 mu_e=None, lam_e=None, q=None, device="cuda", rediscretize=False):
        """``rediscretize=False``: coarse operators share the fine quadrature and state
        (Galerkin).  ``True``: each coarse level is an operator of its own order on its
        own (p + 1)^3 Gauss points, with its geometry from the coarse nodes (which are
        fine nodes: nested node sets) and its state stored at the injected field."""
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
            if l == 0 or not rediscretize:
                op = Operator(p + 1, Q, en, nn, mk, fine=None if l == 0 else self.ops[0])
                if l == 0:
                    op.set_material(mu, lam, self.mu_e_t, self.lam_e_t)
            else:
                op = Operator(p + 1, p + 1, en, nn, mk, fine=None)
                op.set_material(mu, lam, self.mu_e_t, self.lam_e_t)
                xc = _nested_nodes(mesh.coords, mesh.elem_nodes, mesh.P, topo, p + 1, nn)
                op.qdata_setup(torch.from_numpy(xc).to(self.device))
            self.ops.append(op)
            self.masks.append(mask)
            self.topos.append(topo)
        self.rediscretize = bool(rediscretize)
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


def _nested_nodes(xf, topo_f, Pf, topo_c, Pc, Nc):
    """Values at the coarse nodes of a field given at the fine nodes when the coarse node
    set is a subset of the fine one (coarse local node (a1, a2, a3) of an element is its
    fine local node (s a1, s a2, s a3), s = (Pf - 1) / (Pc - 1))."""
    if (Pf - 1) % (Pc - 1):
        raise ValueError("rediscretised levels need nested node sets")
    s = (Pf - 1) // (Pc - 1)
    a = np.arange(Pc)
    A1, A2, A3 = np.meshgrid(a, a, a, indexing="ij")
    loc_c = (A1 + Pc * (A2 + Pc * A3)).transpose(2, 1, 0).reshape(-1)
    loc_f = (s * A1 + Pf * (s * A2 + Pf * s * A3)).transpose(2, 1, 0).reshape(-1)
    out = np.zeros((Nc,) + np.asarray(xf).shape[1:])
    out[np.asarray(topo_c)[:, loc_c].reshape(-1)] = np.asarray(xf)[np.asarray(topo_f)[:, loc_f].reshape(-1)]
    return out
