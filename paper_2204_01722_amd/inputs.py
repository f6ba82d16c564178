"""Seeded synthetic inputs: hexahedral box meshes, displacement fields, probe vectors,
materials and inclusion layouts.

This module is the only thing the HIP path and the CPU oracle share.  It describes the
*problem* (geometry, topology, fields, random draws), never the method: it holds no
basis tabulation, quadrature, constitutive law or solver arithmetic.

Mesh conventions
----------------
* A box ``[0,Lx]x[0,Ly]x[0,Lz]`` is split into ``nx*ny*nz`` hexahedra of order ``p``
  (``P = p + 1`` nodes per direction).
* Global nodes form the grid ``(p*nx+1) x (p*ny+1) x (p*nz+1)``; node ``(I, J, K)``
  has id ``I + NX*(J + NY*K)``.
* Element ``(ex, ey, ez)`` has id ``ex + nx*(ey + ny*ez)``; its local node
  ``(a1, a2, a3)`` (``a1`` fastest) is global node ``(p*ex+a1, p*ey+a2, p*ez+a3)``.
  ``elem_nodes`` is ``int32 [E][P^3]`` in that lexicographic order.
* Interior *vertices* (element corners off the boundary) may be jittered; the
  high-order nodes are then placed by each element's trilinear map at the
  Gauss-Lobatto reference positions ("linear geometry").  The boundary stays flat,
  so the box volume is unchanged by jitter.
* L-vectors are ``float64 [N][3]`` with components interleaved.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "BoxMesh", "box_mesh", "box_topology", "face_mask", "sinusoid", "sinusoid_grad",
    "config1_u", "calibrated_amplitude", "stretch_field", "random_vector", "rough_seed",
    "lame", "loguniform_materials", "inclusion_materials", "affine_lifting",
]


def _lobatto_positions(P: int) -> np.ndarray:
    """Reference positions in [-1, 1] at which high-order nodes are placed: the end
    points and the roots of the derivative of the Legendre polynomial of degree P-1."""
    p = P - 1
    if p < 1:
        raise ValueError("order must be >= 1")
    inner = np.polynomial.legendre.Legendre.basis(p).deriv().roots() if p > 1 else np.zeros(0)
    return np.concatenate(([-1.0], np.sort(np.real(inner)), [1.0]))


@dataclass
class BoxMesh:
    n: tuple            # elements per direction (nx, ny, nz)
    p: int              # polynomial order
    L: tuple            # box extents
    coords: np.ndarray  # float64 [N][3]
    elem_nodes: np.ndarray  # int32 [E][P^3]
    vertices: np.ndarray = field(repr=False)  # float64 [(nx+1)(ny+1)(nz+1)][3]

    @property
    def P(self) -> int:
        return self.p + 1

    @property
    def n_elem(self) -> int:
        return int(self.elem_nodes.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def grid(self) -> tuple:
        nx, ny, nz = self.n
        return (self.p * nx + 1, self.p * ny + 1, self.p * nz + 1)

    @property
    def n_dof(self) -> int:
        return 3 * self.n_nodes


def box_topology(n, p: int) -> np.ndarray:
    """``int32 [E][P^3]`` element-to-node map of an ``n``-element box of order ``p``."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    P = p + 1
    NX, NY = p * nx + 1, p * ny + 1
    ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ex, ey, ez = (a.transpose(2, 1, 0).reshape(-1) for a in (ex, ey, ez))  # ex fastest
    a1, a2, a3 = np.meshgrid(np.arange(P), np.arange(P), np.arange(P), indexing="ij")
    a1, a2, a3 = (a.transpose(2, 1, 0).reshape(-1) for a in (a1, a2, a3))  # a1 fastest
    I = p * ex[:, None] + a1[None, :]
    J = p * ey[:, None] + a2[None, :]
    K = p * ez[:, None] + a3[None, :]
    return (I + NX * (J + NY * K)).astype(np.int32)


def box_mesh(n, p: int, L=(1.0, 1.0, 1.0), jitter: float = 0.0, seed: int = 2204) -> BoxMesh:
    """Box mesh with interior vertices jittered by ``U(-jitter*h, jitter*h)`` per
    coordinate (``h`` = element size in that direction), seeded."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    L = tuple(float(v) for v in L)
    P = p + 1
    h = np.array([L[0] / nx, L[1] / ny, L[2] / nz])
    vx, vy, vz = (np.linspace(0.0, L[d], m + 1) for d, m in enumerate((nx, ny, nz)))
    VX, VY, VZ = np.meshgrid(vx, vy, vz, indexing="ij")
    vert = np.stack([VX, VY, VZ], axis=-1)  # [nx+1][ny+1][nz+1][3]
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter, jitter, size=vert.shape) * h
        interior = np.zeros(vert.shape[:3], dtype=bool)
        interior[1:-1, 1:-1, 1:-1] = True
        vert = vert + np.where(interior[..., None], d, 0.0)

    r = _lobatto_positions(P)
    NX, NY, NZ = p * nx + 1, p * ny + 1, p * nz + 1
    I, J, K = np.meshgrid(np.arange(NX), np.arange(NY), np.arange(NZ), indexing="ij")
    I, J, K = (a.transpose(2, 1, 0).reshape(-1) for a in (I, J, K))  # node id order
    ex = np.minimum(I // p, nx - 1)
    ey = np.minimum(J // p, ny - 1)
    ez = np.minimum(K // p, nz - 1)
    s = r[I - p * ex]
    t = r[J - p * ey]
    u = r[K - p * ez]
    coords = np.zeros((I.size, 3))
    for cx in (0, 1):
        wx = 0.5 * (1 - s) if cx == 0 else 0.5 * (1 + s)
        for cy in (0, 1):
            wy = 0.5 * (1 - t) if cy == 0 else 0.5 * (1 + t)
            for cz in (0, 1):
                wz = 0.5 * (1 - u) if cz == 0 else 0.5 * (1 + u)
                coords += (wx * wy * wz)[:, None] * vert[ex + cx, ey + cy, ez + cz]
    # Nodes on the outer faces sit exactly on the faces.
    for d, m, Ld in ((0, I, L[0]), (1, J, L[1]), (2, K, L[2])):
        last = (NX, NY, NZ)[d] - 1
        coords[m == 0, d] = 0.0
        coords[m == last, d] = Ld
    elem_nodes = box_topology((nx, ny, nz), p)
    return BoxMesh(n=(nx, ny, nz), p=p, L=L, coords=coords, elem_nodes=elem_nodes,
                   vertices=vert.transpose(2, 1, 0, 3).reshape(-1, 3).copy())


def face_mask(mesh_or_grid, faces: dict, n_nodes: int | None = None, p: int | None = None,
              n=None) -> np.ndarray:
    """``uint8 [N][3]`` Dirichlet mask.  ``faces`` maps a face name (``x0, x1, y0, y1,
    z0, z1``) to a 3-tuple of component flags.  Works for a :class:`BoxMesh` or for
    the node grid of a coarser order on the same elements (pass ``p`` and ``n``)."""
    if isinstance(mesh_or_grid, BoxMesh):
        NX, NY, NZ = mesh_or_grid.grid
    else:
        nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
        NX, NY, NZ = p * nx + 1, p * ny + 1, p * nz + 1
    N = NX * NY * NZ
    idx = np.arange(N)
    I, J, K = idx % NX, (idx // NX) % NY, idx // (NX * NY)
    sel = {"x0": I == 0, "x1": I == NX - 1, "y0": J == 0, "y1": J == NY - 1,
           "z0": K == 0, "z1": K == NZ - 1}
    mask = np.zeros((N, 3), dtype=np.uint8)
    for name, comps in faces.items():
        for c in range(3):
            if comps[c]:
                mask[sel[name], c] = 1
    return mask


def sinusoid(X: np.ndarray, L=(1.0, 1.0, 1.0)) -> np.ndarray:
    """The smooth displacement shape used by the operator workloads (unit amplitude)."""
    x, y, z = (np.pi * X[:, d] / L[d] for d in range(3))
    return np.stack([np.sin(x) * np.sin(y) * np.sin(z),
                     np.cos(x) * np.sin(2 * y) * np.sin(z),
                     np.sin(x) * np.cos(y) * np.sin(2 * z)], axis=1)


def sinusoid_grad(X: np.ndarray, L=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Analytic gradient ``[N][3][3]`` (``[i][J] = d s_i / d X_J``) of :func:`sinusoid`."""
    x, y, z = (np.pi * X[:, d] / L[d] for d in range(3))
    kx, ky, kz = (np.pi / L[d] for d in range(3))
    s, c = np.sin, np.cos
    g = np.zeros((X.shape[0], 3, 3))
    g[:, 0, 0] = kx * c(x) * s(y) * s(z)
    g[:, 0, 1] = ky * s(x) * c(y) * s(z)
    g[:, 0, 2] = kz * s(x) * s(y) * c(z)
    g[:, 1, 0] = -kx * s(x) * s(2 * y) * s(z)
    g[:, 1, 1] = 2 * ky * c(x) * c(2 * y) * s(z)
    g[:, 1, 2] = kz * c(x) * s(2 * y) * c(z)
    g[:, 2, 0] = kx * c(x) * c(y) * s(2 * z)
    g[:, 2, 1] = -ky * s(x) * s(y) * s(2 * z)
    g[:, 2, 2] = 2 * kz * s(x) * c(y) * c(2 * z)
    return g


def config1_u(mesh: BoxMesh, amplitude: float = 0.01, noise_std: float = 1e-4,
              seed: int = 1) -> np.ndarray:
    """Smooth sinusoid of the given amplitude plus seeded Gaussian noise."""
    rng = np.random.default_rng(seed)
    return amplitude * sinusoid(mesh.coords, mesh.L) + rng.normal(0.0, noise_std, (mesh.n_nodes, 3))


def calibrated_amplitude(mesh: BoxMesh, target_stretch: float = 1.3, samples: int = 33) -> float:
    """Amplitude ``A`` such that the largest singular value of ``I + A grad(s)`` over a
    uniform ``samples^3`` grid of the box equals ``target_stretch`` (bisection on the
    analytic field; independent of the mesh resolution)."""
    axes = [np.linspace(0.0, mesh.L[d], samples) for d in range(3)]
    X = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    g = sinusoid_grad(X, mesh.L)
    eye = np.eye(3)[None]

    def stretch(a):
        F = eye + a * g
        return np.sqrt(np.linalg.eigvalsh(np.einsum("nki,nkj->nij", F, F))[:, -1].max())

    lo, hi = 0.0, 1.0
    while stretch(hi) < target_stretch:
        hi *= 2.0
    while hi - lo > 1e-10 * hi:
        mid = 0.5 * (lo + hi)
        if stretch(mid) < target_stretch:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def stretch_field(mesh: BoxMesh, target_stretch: float = 1.3) -> np.ndarray:
    """Smooth displacement with a maximum nodal stretch of ``target_stretch``."""
    return calibrated_amplitude(mesh, target_stretch) * sinusoid(mesh.coords, mesh.L)


def random_vector(n_nodes: int, seed: int, dist: str = "normal") -> np.ndarray:
    rng = np.random.default_rng(seed)
    if dist == "normal":
        return rng.normal(0.0, 1.0, (n_nodes, 3))
    return rng.uniform(-1.0, 1.0, (n_nodes, 3))


def rough_seed(n_nodes: int, mask: np.ndarray | None, seed: int = 7) -> np.ndarray:
    """The "rough" start vector for the eigenvalue estimate: uniform(-1, 1) on the free
    degrees of freedom, zero on constrained ones."""
    v = random_vector(n_nodes, seed, "uniform")
    if mask is not None:
        v[np.asarray(mask, dtype=bool)] = 0.0
    return v


def lame(E: float, nu: float) -> tuple:
    """Lame parameters ``(mu, lambda)`` of Young's modulus ``E`` and Poisson ratio ``nu``."""
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


def loguniform_materials(n_elem: int, lo: float = 0.5, hi: float = 2.0, seed: int = 4) -> tuple:
    """Per-element ``(mu_e, lambda_e)`` drawn i.i.d. log-uniform on ``[lo, hi]``."""
    rng = np.random.default_rng(seed)
    mu = np.exp(rng.uniform(np.log(lo), np.log(hi), n_elem))
    lam = np.exp(rng.uniform(np.log(lo), np.log(hi), n_elem))
    return mu, lam


def inclusion_materials(mesh: BoxMesh, fraction: float = 0.2, r_elems=(2.0, 4.0),
                        E_in: float = 100.0, E_out: float = 1.0, nu: float = 0.3,
                        seed: int = 6) -> tuple:
    """Stiff spherical inclusions: sphere centres uniform in the box, radii uniform in
    ``r_elems`` element sizes, added until ``fraction`` of the element centroids lie
    inside a sphere.  Returns per-element ``(mu_e, lambda_e, inside)``."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = mesh.n
    h = min(mesh.L[0] / nx, mesh.L[1] / ny, mesh.L[2] / nz)
    corners = mesh.coords[mesh.elem_nodes]
    cent = corners.mean(axis=1)
    inside = np.zeros(mesh.n_elem, dtype=bool)
    while inside.mean() < fraction:
        c = rng.uniform(0.0, 1.0, 3) * np.asarray(mesh.L)
        r = rng.uniform(r_elems[0], r_elems[1]) * h
        inside |= np.sum((cent - c) ** 2, axis=1) <= r * r
    mu_i, lam_i = lame(E_in, nu)
    mu_o, lam_o = lame(E_out, nu)
    mu = np.where(inside, mu_i, mu_o)
    lam = np.where(inside, lam_i, lam_o)
    return mu, lam, inside


def affine_lifting(mesh: BoxMesh, face_value=(0.5, 0.0, 0.0), axis: int = 0) -> np.ndarray:
    """Extension of a displacement imposed on the far face ``X_axis = L`` (with the
    near face clamped) into the interior, linear in ``X_axis``.  Load steps add a
    fraction of this vector so the imposed increment is spread over the body."""
    s = mesh.coords[:, axis] / mesh.L[axis]
    return s[:, None] * np.asarray(face_value, dtype=np.float64)[None, :]
