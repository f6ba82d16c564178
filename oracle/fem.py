"""Oracle: geometry, Neo-Hookean residual, tangent, energy and adjoint on Q_p hexahedra.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section II-A (strain energy, Green-Euler strain, weak form, Kirchhoff stress,
Jacobian form) and Section II-B (discrete residual and Jacobian action), written in the
textbook initial-configuration form:

* ``F = I + H`` with ``H = grad_X u``; ``J - 1`` from the exact expansion of
  ``det(I + H)`` (no cancellation) and ``log J = log1p(J - 1)``;
* first Piola stress ``P = mu (F - F^{-T}) + lambda log J F^{-T}``, which equals
  ``tau F^{-T}`` for the paper's Kirchhoff stress ``tau = 2 mu e + lambda log J I``;
* tangent ``A_{iJkL} = dP_{iJ}/dF_{kL}
  = mu d_ik d_JL + (mu - lambda log J) Finv_{Jk} Finv_{Li} + lambda Finv_{Ji} Finv_{Lk}``;
* residual ``r_{a,i} = sum_e sum_q W P_{iJ} dphi_a/dX_J`` (internal force);
* external dead loads (eq. variational-form, right-hand side): body force
  ``int v . rho0 g dV`` and traction ``int v . t dA`` on reference element faces, both
  constant in u, so the Jacobian is unchanged;
* energy ``Psi = sum W psi``, ``psi = lambda/2 (log J)^2 - mu log J + mu tr e`` with
  ``e = (H + H^T + H H^T)/2``.

Dirichlet convention (the paper leaves it to the solver): with a mask ``m`` (1 =
constrained component) the residual's constrained rows are zero, the Jacobian operator is
``M K M + (I - M)`` with ``M = diag(1 - m)``, and the diagonal is 1 on constrained rows.

Arrays: L-vectors ``[N][3]`` (degree of freedom ``3*node + component``), materials as
scalars or per-element arrays ``[E]``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .basis import gauss, gll_nodes, lagrange, tensor_3d


@dataclass
class Disc:
    """A mesh with its dense reference tables (one order, one quadrature)."""
    coords: np.ndarray      # [N][3]
    elem_nodes: np.ndarray  # [E][P^3]
    P: int
    Q: int
    T: dict

    @property
    def n_elem(self):
        return self.elem_nodes.shape[0]

    @property
    def n_nodes(self):
        return self.coords.shape[0]


def make_disc(coords, elem_nodes, P: int, Q: int | None = None) -> Disc:
    Q = P if Q is None else Q
    return Disc(np.asarray(coords, np.float64), np.asarray(elem_nodes, np.int64), P, Q,
                tensor_3d(P, Q))


def _mat(v, E):
    v = np.asarray(v, dtype=np.float64)
    return np.full(E, float(v)) if v.ndim == 0 else v


def _chunks(E, size):
    for s in range(0, E, size):
        yield slice(s, min(E, s + size))


# --------------------------------------------------------------------------------------
# Geometry (Section II-B: W = det(grad_xi X) w_hat, and the map grad_X xi)
# --------------------------------------------------------------------------------------
def geometry(disc: Disc, sl=slice(None)):
    """``W [e][q]``, ``dxi/dX [e][q][d][J]`` and physical basis gradients
    ``gradphi [e][q][J][a]`` for the elements in ``sl``.  Raises on ``det <= 0``."""
    T = disc.T
    Xe = disc.coords[disc.elem_nodes[sl]]                       # [e][a][i]
    dXdxi = np.einsum("eai,dqa->eqid", Xe, T["dPhi"])           # [e][q][i][d]
    det = np.linalg.det(dXdxi)
    if np.any(det <= 0.0):
        raise ValueError("non-positive element Jacobian determinant")
    W = det * T["w3"][None, :]
    dxidX = np.linalg.inv(dXdxi)                                # [e][q][d][J]
    gradphi = np.einsum("dqa,eqdJ->eqJa", T["dPhi"], dxidX)     # [e][q][J][a]
    return W, dxidX, gradphi


def qdata(disc: Disc):
    """Per-quadrature-point ``W`` and ``dxi/dX`` for every element."""
    W, dxidX, _ = geometry(disc)
    return W, dxidX


# --------------------------------------------------------------------------------------
# Pointwise constitutive law (Section II-A)
# --------------------------------------------------------------------------------------
def j_minus_1(H):
    """``det(I + H) - 1 = tr H + ((tr H)^2 - tr(H^2))/2 + det H``, evaluated without
    forming ``det(I + H)`` so small strains keep full relative accuracy."""
    tr = np.trace(H, axis1=-2, axis2=-1)
    tr2 = np.einsum("...ij,...ji->...", H, H)
    return tr + 0.5 * (tr * tr - tr2) + np.linalg.det(H)


def piola(H, mu, lam):
    """First Piola stress ``P = mu (F - F^-T) + lambda log J F^-T`` of the compressible
    Neo-Hookean model; ``mu``, ``lam`` broadcast against the leading axes of ``H``.

    ``F - F^-T`` is formed as ``H + H^T F^-T`` (from ``F^-1 = I - F^-1 H``), so the
    identities cancel analytically and small strains keep full relative accuracy, as
    the Kirchhoff stress written with ``e`` in terms of ``grad u`` does (Section II-A)."""
    F = np.eye(3) + H
    Finv = np.linalg.inv(F)
    FinvT = np.swapaxes(Finv, -1, -2)
    logJ = np.log1p(j_minus_1(H))
    F_minus_FinvT = H + np.swapaxes(H, -1, -2) @ FinvT
    return mu[..., None, None] * F_minus_FinvT + (lam * logJ)[..., None, None] * FinvT


def tangent(H, mu, lam):
    """``A[..., i, J, k, L] = dP_{iJ}/dF_{kL}``."""
    F = np.eye(3) + H
    Fi = np.linalg.inv(F)
    logJ = np.log1p(j_minus_1(H))
    d = np.eye(3)
    A = mu[..., None, None, None, None] * np.einsum("ik,JL->iJkL", d, d)
    A = A + (mu - lam * logJ)[..., None, None, None, None] * np.einsum("...Jk,...Li->...iJkL", Fi, Fi)
    A = A + lam[..., None, None, None, None] * np.einsum("...Ji,...Lk->...iJkL", Fi, Fi)
    return A


def energy_density(H, mu, lam):
    """``psi = lambda/2 (log J)^2 - mu log J + mu tr e``."""
    logJ = np.log1p(j_minus_1(H))
    tr_e = np.trace(H, axis1=-2, axis2=-1) + 0.5 * np.einsum("...ij,...ij->...", H, H)
    return 0.5 * lam * logJ ** 2 - mu * logJ + mu * tr_e


# --------------------------------------------------------------------------------------
# Discrete operators (Section II-B, eqs. residual-discrete and Jacobian-discrete-ref)
# --------------------------------------------------------------------------------------
def _gradient(gradphi, ve):
    """``G[e][q][i][J] = sum_a v[e][a][i] dphi_a/dX_J``."""
    return np.einsum("eai,eqJa->eqiJ", ve, gradphi)


def _free(mask, N):
    if mask is None:
        return np.ones((N, 3))
    return 1.0 - np.asarray(mask, dtype=np.float64).reshape(N, 3)


def residual(disc: Disc, u, mu, lam, mask=None, chunk=4096):
    """``r(u)`` as an L-vector ``[N][3]``; constrained rows are zero."""
    E, N = disc.n_elem, disc.n_nodes
    mu, lam = _mat(mu, E), _mat(lam, E)
    u = np.asarray(u, np.float64).reshape(N, 3)
    r = np.zeros((N, 3))
    for sl in _chunks(E, chunk):
        W, _, gp = geometry(disc, sl)
        H = _gradient(gp, u[disc.elem_nodes[sl]])
        Pk = piola(H, mu[sl][:, None], lam[sl][:, None])
        re = np.einsum("eq,eqiJ,eqJa->eai", W, Pk, gp)
        np.add.at(r, disc.elem_nodes[sl], re)
    return r * _free(mask, N)


def jacobian_apply(disc: Disc, u, du, mu, lam, mask=None, chunk=4096):
    """``y = (M K(u) M + I - M) du`` matrix-free with dense element tables."""
    E, N = disc.n_elem, disc.n_nodes
    mu, lam = _mat(mu, E), _mat(lam, E)
    u = np.asarray(u, np.float64).reshape(N, 3)
    fr = _free(mask, N)
    dv = np.asarray(du, np.float64).reshape(N, 3)
    dm = dv * fr
    y = np.zeros((N, 3))
    for sl in _chunks(E, chunk):
        W, _, gp = geometry(disc, sl)
        H = _gradient(gp, u[disc.elem_nodes[sl]])
        A = tangent(H, mu[sl][:, None], lam[sl][:, None])
        dH = _gradient(gp, dm[disc.elem_nodes[sl]])
        dP = np.einsum("eqiJkL,eqkL->eqiJ", A, dH)
        ye = np.einsum("eq,eqiJ,eqJa->eai", W, dP, gp)
        np.add.at(y, disc.elem_nodes[sl], ye)
    return y * fr + dv * (1.0 - fr)


def element_matrices(disc: Disc, u, mu, lam, sl=slice(None), grad_override=None):
    """Dense element tangents ``K_e[(a,i),(b,k)] = sum_q W dphi_a/dX_J A_{iJkL}
    dphi_b/dX_L``, returned as ``[e][P^3*3][P^3*3]`` with local dof ``3a + i``."""
    E = disc.n_elem
    mu, lam = _mat(mu, E)[sl], _mat(lam, E)[sl]
    u = np.asarray(u, np.float64).reshape(disc.n_nodes, 3)
    W, _, gp = geometry(disc, sl)
    H = _gradient(gp, u[disc.elem_nodes[sl]])
    A = tangent(H, mu[:, None], lam[:, None])
    gq = gp if grad_override is None else grad_override
    K = np.einsum("eq,eqJa,eqiJkL,eqLb->eaibk", W, gq, A, gq, optimize=True)
    n = gq.shape[-1] * 3
    return K.reshape(K.shape[0], n, n)


def assemble(elem_nodes, Ke, n_nodes):
    """Sum element matrices into a global CSR matrix ``[3N][3N]``."""
    elem_nodes = np.asarray(elem_nodes, np.int64)
    E, P3 = elem_nodes.shape
    dofs = (3 * elem_nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(E, 3 * P3)
    rows = np.repeat(dofs[:, :, None], 3 * P3, axis=2)
    cols = np.repeat(dofs[:, None, :], 3 * P3, axis=1)
    K = sp.coo_matrix((Ke.reshape(-1), (rows.reshape(-1), cols.reshape(-1))),
                      shape=(3 * n_nodes, 3 * n_nodes))
    return K.tocsr()


def tangent_matrix(disc: Disc, u, mu, lam):
    """Assembled ``K(u)`` without boundary conditions."""
    return assemble(disc.elem_nodes, element_matrices(disc, u, mu, lam), disc.n_nodes)


def apply_bc(K, mask):
    """``M K M + (I - M)`` for a ``[N][3]`` mask (1 = constrained)."""
    n = K.shape[0]
    if mask is None:
        return K.tocsr()
    fr = 1.0 - np.asarray(mask, np.float64).reshape(-1)
    M = sp.diags(fr)
    return (M @ K @ M + sp.diags(1.0 - fr)).tocsr()


def diagonal(disc: Disc, u, mu, lam, mask=None):
    """Diagonal of the Dirichlet-modified tangent, as ``[N][3]``."""
    K = apply_bc(tangent_matrix(disc, u, mu, lam), mask)
    return K.diagonal().reshape(-1, 3)


def energy(disc: Disc, u, mu, lam, chunk=4096):
    """Total strain energy ``Psi(u)``."""
    E, N = disc.n_elem, disc.n_nodes
    mu, lam = _mat(mu, E), _mat(lam, E)
    u = np.asarray(u, np.float64).reshape(N, 3)
    tot = 0.0
    for sl in _chunks(E, chunk):
        W, _, gp = geometry(disc, sl)
        H = _gradient(gp, u[disc.elem_nodes[sl]])
        tot += float(np.sum(W * energy_density(H, mu[sl][:, None], lam[sl][:, None])))
    return tot


def residual_vjp(disc: Disc, u, w, mu, lam, mask=None, chunk=4096):
    """Vector-Jacobian product of the (masked) residual ``r(u; mu_e, lambda_e)``:
    returns ``(u_bar, mu_bar, lambda_bar)`` with ``u_bar = (dr/du)^T w`` written as the
    explicit transpose contraction ``sum W (grad w)_{iJ} A_{iJkL} dphi_b/dX_L`` and
    ``mu_bar_e = sum_q W grad(w):(F - F^{-T})``,
    ``lambda_bar_e = sum_q W log J grad(w):F^{-T}`` (P is linear in mu and lambda)."""
    E, N = disc.n_elem, disc.n_nodes
    mu, lam = _mat(mu, E), _mat(lam, E)
    u = np.asarray(u, np.float64).reshape(N, 3)
    wm = np.asarray(w, np.float64).reshape(N, 3) * _free(mask, N)
    ub = np.zeros((N, 3))
    mub = np.zeros(E)
    lamb = np.zeros(E)
    for sl in _chunks(E, chunk):
        W, _, gp = geometry(disc, sl)
        H = _gradient(gp, u[disc.elem_nodes[sl]])
        Gw = _gradient(gp, wm[disc.elem_nodes[sl]])
        A = tangent(H, mu[sl][:, None], lam[sl][:, None])
        T = np.einsum("eqiJ,eqiJkL->eqkL", Gw, A)
        ube = np.einsum("eq,eqkL,eqLb->ebk", W, T, gp)
        np.add.at(ub, disc.elem_nodes[sl], ube)
        F = np.eye(3) + H
        FinvT = np.swapaxes(np.linalg.inv(F), -1, -2)
        logJ = np.log1p(j_minus_1(H))
        mub[sl] = np.einsum("eq,eqiJ,eqiJ->e", W, Gw, F - FinvT)
        lamb[sl] = np.einsum("eq,eq,eqiJ,eqiJ->e", W, logJ, Gw, FinvT)
    return ub, mub, lamb


# --------------------------------------------------------------------------------------
# External dead loads (eq. variational-form, right-hand side)
# --------------------------------------------------------------------------------------
def body_force_load(disc: Disc, rho_g):
    """``b_{a,i} = int phi_a (rho0 g)_i dV`` over the reference volume, ``[N][3]``, for a
    constant body force per unit reference volume ``rho_g`` (3-vector)."""
    W, _, _ = geometry(disc)                                   # [e][q]
    per = np.einsum("eq,qa->ea", W, disc.T["Phi"])             # int phi_a dV per element
    out = np.zeros((disc.n_nodes, 3))
    np.add.at(out, disc.elem_nodes.reshape(-1), per.reshape(-1)[:, None] * np.asarray(rho_g)[None, :])
    return out


# Local faces of a hexahedron: (reference direction held fixed, its value).
FACES = [(0, -1.0), (0, 1.0), (1, -1.0), (1, 1.0), (2, -1.0), (2, 1.0)]


def traction_load(coords, elem_nodes, P, Q, faces, t):
    """``b_{a,i} = int phi_a t_i dA`` over the listed element faces of the reference
    configuration, ``[N][3]``: ``faces`` holds ``(element, local face)`` pairs with
    local faces 0..5 = xi_1 = -1, +1, xi_2 = -1, +1, xi_3 = -1, +1; ``t`` is a constant
    traction per unit reference area.  The area element is ``|dX/dxi_s x dX/dxi_r|``
    for the two in-face directions (s, r), Gauss rule with ``Q`` points per direction."""
    nodes = gll_nodes(P)
    xq, wq = gauss(Q)
    coords = np.asarray(coords, np.float64)
    out = np.zeros((coords.shape[0], 3))
    for e, f in faces:
        d, v = FACES[f]
        s_dir, r_dir = [k for k in range(3) if k != d]
        Le, _ = lagrange(nodes, np.array([v]))                 # 1D values at the fixed end
        Xe = coords[np.asarray(elem_nodes[e])]                 # [P^3][3]
        for i in range(Q):
            for j in range(Q):
                xi = np.zeros(3)
                xi[d], xi[s_dir], xi[r_dir] = v, xq[i], xq[j]
                val = np.ones(P ** 3)
                der = {s_dir: np.ones(P ** 3), r_dir: np.ones(P ** 3)}
                for k in range(3):
                    Lk, Dk = lagrange(nodes, np.array([xi[k]]))
                    idx = np.arange(P ** 3)
                    ak = (idx // P ** k) % P
                    val = val * Lk[0, ak]
                    for m in (s_dir, r_dir):
                        der[m] = der[m] * (Dk[0, ak] if m == k else Lk[0, ak])
                ts = der[s_dir] @ Xe
                tr = der[r_dir] @ Xe
                dA = np.linalg.norm(np.cross(ts, tr)) * wq[i] * wq[j]
                np.add.at(out, np.asarray(elem_nodes[e]), val[:, None] * np.asarray(t)[None, :] * dA)
    return out
