"""Oracle: p-multigrid transfer, Chebyshev/Jacobi smoothing, eigenvalue estimate,
V-cycle, Jacobi-PCG, flexible CG, the Newton load-stepping driver, and limited-memory
BFGS with the V-cycle as initial inverse Hessian.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section III-A (Newton-Krylov with a critical-point line search, Lanczos
estimates from the CG recurrence) and Section III-B (the V-cycle of Fig.
multigrid_algorithm with Galerkin coarse operators, restriction = transpose of
prolongation, Chebyshev/Jacobi smoothing on [0.1, 1.1] lambda_max with lambda_max
from 10 Lanczos iterations on a rough vector, prolongation by coarse-to-fine
interpolation).  All operators are assembled scipy matrices: tiny meshes only.

Readings taken where the paper is silent:
* prolongation: the fine nodal value is the coarse finite-element function evaluated
  at the fine node (its plain definition; continuity makes it element independent);
* the eigenvalue estimate runs Jacobi-preconditioned CG from ``x0 = 0`` on the rough
  right-hand side and reads the Lanczos tridiagonal from its coefficients;
* Chebyshev is the three-term semi-iteration for ``D^{-1} A`` on ``[a, b]`` whose
  degree counts operator applications (first one on the initial residual);
* the coarsest level is solved by Jacobi-PCG (relative 2-norm tolerance, ``x0 = 0``),
  optionally for a fixed number of iterations;
* the outer solver is flexible CG with the Polak-Ribiere form of beta; inside Newton it
  stops at a direction of non-positive curvature and returns the iterate so far (the
  preconditioned residual before the first step), as truncated Newton does;
* Newton stops on the 2-norm of the residual relative to the load step's first one;
  the line search takes one secant step for ``F(u + a du)^T du = 0`` from ``a = 0, 1``
  and clips ``a`` to ``[0.1, 1.5]`` (``a = 1`` if the secant slope is not positive);
* a rediscretised coarse level evaluates the operator of its own order on its own
  (p_c + 1)^3 Gauss points at the coarse interpolant of u (the fine field evaluated at
  the coarse nodes), instead of the Galerkin product;
* L-BFGS (Section III-A: the V-cycle as "initial inverse Hessian", same critical-point
  line search) uses the textbook two-loop recursion over the last ``memory`` pairs
  ``s = u_new - u``, ``y = F(u_new) - F(u)``, skips pairs with ``y^T s <= 0``, and
  builds the V-cycle once per load step, at the lifted starting point.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem
from .basis import eval_3d, node_positions_3d


# --------------------------------------------------------------------------------------
# Transfer (Section III-B, eq. mg_prolong)
# --------------------------------------------------------------------------------------
def prolongation(elem_f, Pf, Nf, elem_c, Pc, Nc):
    """``[3 Nf][3 Nc]`` interpolation from order ``Pc - 1`` to order ``Pf - 1`` on the
    same elements: row ``3 n_f + i`` holds the coarse basis functions evaluated at fine
    node ``n_f`` (component ``i``)."""
    vals = eval_3d(Pc, node_positions_3d(Pf))            # [Pf^3][Pc^3]
    elem_f = np.asarray(elem_f, np.int64)
    elem_c = np.asarray(elem_c, np.int64)
    rows = np.repeat(elem_f[:, :, None], elem_c.shape[1], axis=2).reshape(-1)
    cols = np.repeat(elem_c[:, None, :], elem_f.shape[1], axis=1).reshape(-1)
    v = np.broadcast_to(vals[None], (elem_f.shape[0],) + vals.shape).reshape(-1)
    # Each (fine node, coarse node) pair is visited once per shared element with the
    # same value; keep one copy.
    key = rows * Nc + cols
    _, first = np.unique(key, return_index=True)
    rows, cols, v = rows[first], cols[first], v[first]
    keep = v != 0.0
    rows, cols, v = rows[keep], cols[keep], v[keep]
    R = np.concatenate([3 * rows + i for i in range(3)])
    C = np.concatenate([3 * cols + i for i in range(3)])
    V = np.concatenate([v, v, v])
    return sp.csr_matrix((V, (R, C)), shape=(3 * Nf, 3 * Nc))


def inject(u_f, elem_f, Pf, elem_c, Pc, Nc):
    """Coarse nodal values of a fine field for a rediscretised coarse level: the fine
    finite-element function evaluated at each coarse node (its plain definition; for
    nested node sets it is the fine value at the coinciding node).  ``[Nc][3]``."""
    vals = eval_3d(Pf, node_positions_3d(Pc))            # [Pc^3][Pf^3]
    u_f = np.asarray(u_f, np.float64).reshape(-1, 3)
    out = np.zeros((Nc, 3))
    for e in range(len(elem_f)):
        out[np.asarray(elem_c[e])] = vals @ u_f[np.asarray(elem_f[e])]
    return out


def galerkin(K_f, Pm):
    """Coarse operator ``P^T K_f P``."""
    return (Pm.T @ K_f @ Pm).tocsr()


# --------------------------------------------------------------------------------------
# Krylov pieces (Section III-A)
# --------------------------------------------------------------------------------------
def pcg_jacobi(A, dinv, b, rtol=1e-3, maxit=10000, fixed_its=None):
    """Jacobi-preconditioned CG from ``x0 = 0``.  Returns ``x, its, alphas, betas``.
    Stops when ``||b - A x||_2 <= rtol ||b||_2``, or after ``fixed_its`` iterations."""
    x = np.zeros_like(b)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    alphas, betas = [], []
    its = 0
    limit = fixed_its if fixed_its is not None else maxit
    if fixed_its is None and bn == 0.0:
        return x, 0, alphas, betas
    while its < limit:
        q = A @ p
        pq = p @ q
        if pq <= 0.0:
            break
        a = rz / pq
        x += a * p
        r -= a * q
        its += 1
        alphas.append(a)
        if fixed_its is None and np.linalg.norm(r) <= rtol * bn:
            break
        z = dinv * r
        rz_new = r @ z
        beta = rz_new / rz
        betas.append(beta)
        p = z + beta * p
        rz = rz_new
    return x, its, alphas, betas


def lanczos_tridiagonal(alphas, betas):
    """Tridiagonal matrix implied by the CG coefficients."""
    k = len(alphas)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return T


def estimate_lambda_max(A, dinv, seed, its=10):
    """Largest Ritz value of ``D^{-1} A`` from ``its`` Jacobi-PCG steps on the seed."""
    _, _, al, be = pcg_jacobi(A, dinv, seed, fixed_its=its)
    T = lanczos_tridiagonal(al, be[: max(len(al) - 1, 0)])
    return float(np.linalg.eigvalsh(T).max())


def chebyshev(A, dinv, b, x, lam_max, degree, lo=0.1, hi=1.1):
    """``degree`` steps of Chebyshev semi-iteration for ``D^{-1} A`` on
    ``[lo, hi] * lam_max`` (Saad, Iterative Methods, 2nd ed., Alg. 12.1), from ``x``."""
    a, bb = lo * lam_max, hi * lam_max
    theta, delta = 0.5 * (bb + a), 0.5 * (bb - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = x.copy()
    r = dinv * (b - A @ x)
    d = r / theta
    for k in range(degree):
        x += d
        if k + 1 == degree:
            break
        r -= dinv * (A @ d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * r
        rho = rho_new
    return x


class VCycle:
    """p-multigrid V-cycle (Fig. multigrid_algorithm) on assembled level operators.

    ``ops[0]`` is the finest Dirichlet-modified operator; ``prolongs[l]`` maps level
    ``l+1`` to level ``l``; ``masks[l]`` are the level masks.  Coarse operators are
    Galerkin products with the masks re-applied (identity on constrained rows), or the
    given rediscretised operators ``coarse_raw`` (levels 1, 2, ...)."""

    def __init__(self, K_fine_raw, prolongs, masks, seeds, degree=3, lo=0.1, hi=1.1,
                 lanczos_its=10, coarse_rtol=1e-3, coarse_maxit=10000, coarse_fixed=None,
                 lam_override=None, coarse_raw=None):
        self.prolongs = prolongs
        self.masks = [None if m is None else np.asarray(m, np.float64).reshape(-1) for m in masks]
        raw = [K_fine_raw.tocsr()]
        if coarse_raw is not None:       # rediscretised coarse operators, one per level
            raw += [K.tocsr() for K in coarse_raw]
        else:
            for Pm in prolongs:
                raw.append(galerkin(raw[-1], Pm))
        self.ops = [fem.apply_bc(K, None if m is None else m.reshape(-1, 3))
                    for K, m in zip(raw, self.masks)]
        self.dinv = [1.0 / K.diagonal() for K in self.ops]
        self.degree, self.lo, self.hi = degree, lo, hi
        self.coarse_rtol, self.coarse_maxit, self.coarse_fixed = coarse_rtol, coarse_maxit, coarse_fixed
        self.lam = []
        for l in range(len(self.ops) - 1):
            if lam_override is not None:
                self.lam.append(float(lam_override[l]))
            else:
                self.lam.append(estimate_lambda_max(self.ops[l], self.dinv[l],
                                                    seeds[l].reshape(-1), lanczos_its))
        self.coarse_its = []

    def _fr(self, l):
        m = self.masks[l]
        return 1.0 if m is None else 1.0 - m

    def cycle(self, l, b):
        A, dinv = self.ops[l], self.dinv[l]
        if l == len(self.ops) - 1:
            x, its, _, _ = pcg_jacobi(A, dinv, b, self.coarse_rtol, self.coarse_maxit,
                                      self.coarse_fixed)
            self.coarse_its.append(its)
            return x
        x = chebyshev(A, dinv, b, np.zeros_like(b), self.lam[l], self.degree, self.lo, self.hi)
        r = b - A @ x
        rc = (self.prolongs[l].T @ r) * self._fr(l + 1)
        e = self.cycle(l + 1, rc)
        x = x + (self.prolongs[l] @ e) * self._fr(l)
        x = chebyshev(A, dinv, b, x, self.lam[l], self.degree, self.lo, self.hi)
        return x

    def __call__(self, r):
        return self.cycle(0, np.asarray(r, np.float64).reshape(-1))


def fcg(A, prec, b, rtol=1e-8, maxit=500, x0=None, norm="2"):
    """Flexible CG (Polak-Ribiere beta) for ``A x = b``.  ``norm="2"`` stops when
    ``||b - A x||_2 <= rtol ||b - A x0||_2``; ``norm="natural"`` measures the residual
    in the natural norm of the preconditioned system (Section III-A),
    ``sqrt(r^T prec(r))``, relative to its value at x0.  Returns
    ``x, its, final_relres``."""
    if norm not in ("2", "natural"):
        raise ValueError(norm)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    z = prec(r)
    rz = r @ z
    r0 = np.sqrt(abs(rz)) if norm == "natural" else np.linalg.norm(r)
    if r0 == 0.0:
        return x, 0, 0.0
    p = z.copy()
    its = 0
    rel = 1.0
    while its < maxit:
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r_new = r - a * q
        its += 1
        z = prec(r_new)
        rz_new = r_new @ z
        rel = (np.sqrt(abs(rz_new)) if norm == "natural" else np.linalg.norm(r_new)) / r0
        if rel <= rtol:
            break
        beta = (z @ (r_new - r)) / rz
        rz = rz_new
        p = z + beta * p
        r = r_new
    return x, its, rel


def fcg_truncated(A, prec, b, rtol=1e-8, maxit=500, norm="2"):
    """Flexible CG as ``fcg`` (same ``norm`` choice) from x0 = 0, stopped at a direction of non-positive
    curvature (p^T A p <= 0, possible when the Newton tangent is indefinite): the iterate
    reached so far is returned, or the preconditioned residual when it happens before the
    first step, so that a Newton step can still move along a descent direction (the
    truncated-Newton treatment of negative curvature).  Returns
    ``x, its, final_relres, broke``."""
    if norm not in ("2", "natural"):
        raise ValueError(norm)
    x = np.zeros_like(b)
    r = b.copy()
    if not np.any(r):
        return x, 0, 0.0, False
    z = prec(r)
    rz = r @ z
    r0 = np.sqrt(abs(rz)) if norm == "natural" else np.linalg.norm(r)
    if r0 == 0.0:
        return x, 0, 0.0, False
    p = z.copy()
    its, rel = 0, 1.0
    while its < maxit:
        q = A @ p
        pq = p @ q
        if not (pq > 0.0) or not np.isfinite(rz):
            if its == 0 and np.isfinite(rz):
                x = x + z
            return x, its, rel, True
        a = rz / pq
        x += a * p
        r_new = r - a * q
        its += 1
        z = prec(r_new)
        rz_new = r_new @ z
        rel = (np.sqrt(abs(rz_new)) if norm == "natural" else np.linalg.norm(r_new)) / r0
        if rel <= rtol:
            break
        beta = (z @ (r_new - r)) / rz
        rz = rz_new
        p = z + beta * p
        r = r_new
    return x, its, rel, False


def line_search_cp(resid, u, du):
    """Critical-point line search: one secant step on ``g(a) = F(u + a du)^T du``."""
    g0 = resid(u).reshape(-1) @ du.reshape(-1)
    g1 = resid(u + du).reshape(-1) @ du.reshape(-1)
    if not (g1 - g0 > 0.0):  # secant slope not positive: no critical point ahead
        return 1.0
    return float(np.clip(g0 / (g0 - g1), 0.1, 1.5))


def newton_load_steps(disc, mu, lam, mask, lift, n_steps, linear_solve, rtol=1e-8,
                      max_newton=20, u0=None, line_search=True, f_ext=None):
    """Displacement-driven load stepping, with an optional external load ``f_ext``
    ramped by the same fraction (``F(u) = r(u) - (k / n_steps) f_ext`` in step ``k``).
    ``lift`` holds the full imposed displacement on constrained components and an
    extension of it elsewhere; step ``k`` starts from
    the previous solution plus ``lift / n_steps`` and runs Newton with homogeneous
    corrections on constrained components.  ``linear_solve(K_bc, rhs)`` returns the
    Newton correction.  Returns ``u`` and per-step Newton iteration counts."""
    N = disc.n_nodes
    u = np.zeros((N, 3)) if u0 is None else np.asarray(u0, np.float64).copy()
    lift = np.asarray(lift, np.float64).reshape(N, 3)
    history = []

    fe = None if f_ext is None else np.asarray(f_ext, np.float64).reshape(N, 3) * (
        1.0 if mask is None else 1.0 - np.asarray(mask, np.float64).reshape(N, 3))
    load = [0.0]

    def resid(v):
        r = fem.residual(disc, v, mu, lam, mask)
        return r if fe is None else r - load[0] * fe

    for k in range(n_steps):
        load[0] = (k + 1) / n_steps
        u = u + lift / n_steps
        F = resid(u)
        f0 = np.linalg.norm(F)
        its = 0
        while its < max_newton and np.linalg.norm(F) > rtol * f0 and f0 > 0.0:
            K = fem.apply_bc(fem.tangent_matrix(disc, u, mu, lam), mask)
            du = linear_solve(K, -F.reshape(-1)).reshape(N, 3)
            a = line_search_cp(resid, u, du) if line_search else 1.0
            u = u + a * du
            F = resid(u)
            its += 1
        history.append(its)
    return u, history


def line_search_cp_dir(grad, u, d, clip=(0.1, 1.5)):
    """Critical-point step length along a direction ``d``: one secant step on
    ``phi(a) = grad(u + a d)^T d`` between ``a = 0`` and ``a = 1`` (Section III-A).
    ``clip=None`` returns the unclipped secant root (exact for a quadratic energy)."""
    g0 = grad(u) @ d
    g1 = grad(u + d) @ d
    if not (g1 - g0 > 0.0):  # secant slope not positive: no critical point ahead
        return 1.0
    a = g0 / (g0 - g1)
    return a if clip is None else float(np.clip(a, clip[0], clip[1]))


def lbfgs(grad, u0, h0, memory=5, rtol=1e-8, max_its=500, clip=(0.1, 1.5)):
    """Limited-memory BFGS for ``grad(u) = 0`` with initial inverse Hessian ``h0``
    (a function of a vector).  Search direction by the two-loop recursion: with
    ``rho_i = 1 / (y_i^T s_i)``, first ``a_i = rho_i s_i^T q; q -= a_i y_i`` from the
    newest pair to the oldest, then ``r = h0(q)``, then ``b = rho_i y_i^T r;
    r += (a_i - b) s_i`` from the oldest to the newest; ``d = -r``.  Stops when
    ``||grad(u)||_2 <= rtol ||grad(u0)||_2``.  Returns ``u, its, final_rel``."""
    u = np.array(u0, dtype=np.float64, copy=True)
    g = grad(u)
    gn0 = np.linalg.norm(g)
    pairs = []
    its, rel = 0, 0.0 if gn0 == 0.0 else 1.0
    while gn0 > 0.0 and rel > rtol and its < max_its:
        q = g.copy()
        alph = []
        for s_i, y_i, rho in reversed(pairs):
            a = rho * (s_i @ q)
            q -= a * y_i
            alph.append(a)
        r = h0(q)
        for (s_i, y_i, rho), a in zip(pairs, reversed(alph)):
            b = rho * (y_i @ r)
            r += (a - b) * s_i
        d = -r
        if not (g @ d < 0.0):  # not a descent direction: restart from h0
            pairs = []
            d = -h0(g)
        a = line_search_cp_dir(grad, u, d, clip)
        s_new = a * d
        u = u + s_new
        g_new = grad(u)
        y_new = g_new - g
        ys = y_new @ s_new
        if ys > 0.0:
            pairs.append((s_new, y_new, 1.0 / ys))
            if len(pairs) > memory:
                pairs.pop(0)
        g = g_new
        its += 1
        rel = np.linalg.norm(g) / gn0
    return u, its, rel


def lbfgs_load_steps(disc, mu, lam, mask, lift, n_steps, make_h0, memory=5, rtol=1e-8,
                     max_its=500, u0=None):
    """Displacement-driven load stepping with L-BFGS at every load level.  Step ``k``
    starts from the previous solution plus ``lift / n_steps``; ``make_h0(u)`` returns
    the initial inverse Hessian built at that starting point (the V-cycle on the
    tangent there).  Returns ``u`` and per-step iteration counts."""
    N = disc.n_nodes
    u = np.zeros((N, 3)) if u0 is None else np.asarray(u0, np.float64).copy()
    lift = np.asarray(lift, np.float64).reshape(N, 3)

    def grad(v):
        return fem.residual(disc, v.reshape(N, 3), mu, lam, mask).reshape(-1)

    history = []
    for _ in range(n_steps):
        u = u + lift / n_steps
        h0 = make_h0(u)
        x, its, _ = lbfgs(grad, u.reshape(-1), h0, memory=memory, rtol=rtol, max_its=max_its)
        u = x.reshape(N, 3)
        history.append(its)
    return u, history
