"""Pins of the oracle's multigrid pieces and solver drivers (CPU only): interpolation of
affine fields, the exact-Galerkin identity of coarse operators built on the fine
quadrature, the closed-form Chebyshev error polynomial, Ritz bounds of the eigenvalue
estimate and its exact pins (the tridiagonal read from the CG coefficients has the whole
known spectrum after a full-dimension run, and equals plain Lanczos on the Jacobi-scaled
matrix entry by entry), flexible CG against a direct solve, symmetry of the V-cycle, the homogeneous
uniaxial-stretch solution of the Newton driver, and L-BFGS (its iterates equal those of
CG on a quadratic with exact line search, one step with the exact inverse Hessian, the
Newton answer on a Neo-Hookean problem)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import basis, fem, mg
from paper_2204_01722_amd import inputs

MU, LAM = inputs.lame(1.0, 0.3)


def _levels(n=2, pf=2, pc=1, jitter=0.05):
    mf = inputs.box_mesh(n, pf, jitter=jitter)
    mc = inputs.box_mesh(n, pc, jitter=jitter)
    Pm = mg.prolongation(mf.elem_nodes, mf.P, mf.n_nodes, mc.elem_nodes, mc.P, mc.n_nodes)
    return mf, mc, Pm


@pytest.mark.parametrize("pf,pc", [(2, 1), (4, 2), (3, 1), (4, 1)])
def test_prolongation_exact_for_affine(pf, pc):
    mf, mc, Pm = _levels(2, pf, pc, jitter=0.08)
    G = np.array([[0.3, -0.1, 0.2], [0.05, 0.4, -0.2], [0.1, 0.0, -0.3]])
    b = np.array([0.1, -0.2, 0.3])
    fc = mc.coords @ G.T + b
    ff = mf.coords @ G.T + b
    np.testing.assert_allclose((Pm @ fc.reshape(-1)).reshape(-1, 3), ff, atol=1e-14)


def test_prolongation_preserves_face_zero():
    mf, mc, Pm = _levels(2, 2, 1)
    maskc = inputs.face_mask(mc, {"x0": (1, 1, 1)}).astype(bool)
    maskf = inputs.face_mask(mf, {"x0": (1, 1, 1)}).astype(bool)
    v = inputs.random_vector(mc.n_nodes, 3)
    v[maskc] = 0.0
    assert np.all((Pm @ v.reshape(-1)).reshape(-1, 3)[maskf] == 0.0)


@pytest.mark.parametrize("pf,pc", [(2, 1), (3, 1), (4, 2)])
def test_galerkin_identity(pf, pc):
    """A coarse operator rediscretised with the coarse basis on the fine quadrature and
    the fine linearisation equals P^T K_f P (Section III-B: exact Galerkin)."""
    mf, mc, Pm = _levels(2, pf, pc, jitter=0.06)
    df = fem.make_disc(mf.coords, mf.elem_nodes, mf.P)
    u = inputs.config1_u(mf, amplitude=0.05)
    Kf = fem.tangent_matrix(df, u, MU, LAM)
    _, dxidX, _ = fem.geometry(df)
    Tc = basis.tensor_3d(mc.P, mf.P)
    gpc = np.einsum("dqa,eqdJ->eqJa", Tc["dPhi"], dxidX)
    Ke_c = fem.element_matrices(df, u, MU, LAM, grad_override=gpc)
    Kc = fem.assemble(mc.elem_nodes, Ke_c, mc.n_nodes)
    G = mg.galerkin(Kf, Pm)
    assert abs(G - Kc).max() <= 1e-13 * abs(Kc).max()


def test_chebyshev_closed_form():
    mf = inputs.box_mesh(2, 2, jitter=0.05)
    d = fem.make_disc(mf.coords, mf.elem_nodes, 3)
    mask = inputs.face_mask(mf, {"x0": (1, 1, 1)})
    A = fem.apply_bc(fem.tangent_matrix(d, inputs.config1_u(mf), MU, LAM), mask).toarray()
    Dg = np.diag(A)
    dinv = 1.0 / Dg
    lam_max = 1.7
    rng = np.random.default_rng(3)
    b = rng.normal(size=A.shape[0])
    x0 = rng.normal(size=A.shape[0])
    xs = np.linalg.solve(A, b)
    for m in (1, 2, 3, 5):
        x = mg.chebyshev(A, dinv, b, x0, lam_max, m)
        a, bb = 0.1 * lam_max, 1.1 * lam_max
        th, de = 0.5 * (a + bb), 0.5 * (bb - a)
        S = np.diag(np.sqrt(dinv)) @ A @ np.diag(np.sqrt(dinv))
        ev, V = np.linalg.eigh(S)
        Tm = np.polynomial.chebyshev.Chebyshev.basis(m)
        pol = Tm((th - ev) / de) / Tm(th / de)
        e0 = np.sqrt(Dg) * (xs - x0)
        em = (V @ (pol * (V.T @ e0))) / np.sqrt(Dg)
        np.testing.assert_allclose(xs - x, em, atol=1e-11 * np.abs(xs).max())


def test_lambda_max_estimate_bounds():
    mf = inputs.box_mesh(3, 2, jitter=0.05)
    d = fem.make_disc(mf.coords, mf.elem_nodes, 3)
    mask = inputs.face_mask(mf, {"x0": (1, 1, 1)})
    A = fem.apply_bc(fem.tangent_matrix(d, inputs.config1_u(mf), MU, LAM), mask)
    dinv = 1.0 / A.diagonal()
    seed = inputs.rough_seed(mf.n_nodes, mask, 7).reshape(-1)
    est = mg.estimate_lambda_max(A, dinv, seed, 10)
    Ad = A.toarray()
    S = np.diag(np.sqrt(dinv)) @ Ad @ np.diag(np.sqrt(dinv))
    true = np.linalg.eigvalsh(S).max()
    assert est <= true * (1 + 1e-12)
    assert est >= 0.8 * true


def _spd_with_spectrum(lams, seed):
    """A = D^{1/2} S D^{1/2} with S = V diag(lams) V^T (V a seeded random orthogonal
    matrix) and a seeded positive diagonal D: D^{-1} A is similar to S, so the spectrum
    of the Jacobi-preconditioned operator is exactly ``lams``."""
    rng = np.random.default_rng(seed)
    n = len(lams)
    V, _ = np.linalg.qr(rng.normal(size=(n, n)))
    S = V @ np.diag(lams) @ V.T
    d = rng.uniform(0.5, 3.0, size=n)
    A = np.sqrt(d)[:, None] * S * np.sqrt(d)[None, :]
    return 0.5 * (A + A.T), d, rng.normal(size=n)


def _plain_lanczos(S, w, k):
    """Textbook symmetric Lanczos on S from w / ||w||, with full reorthogonalisation;
    returns the k x k tridiagonal (diagonal a_j = v_j^T S v_j, off-diagonal b_j =
    ||u_j||).  Independent of the CG recurrence."""
    n = len(w)
    Vs = np.zeros((n, k + 1))
    Vs[:, 0] = w / np.linalg.norm(w)
    a, b = np.zeros(k), np.zeros(k)
    for j in range(k):
        u = S @ Vs[:, j]
        a[j] = Vs[:, j] @ u
        u -= Vs[:, : j + 1] @ (Vs[:, : j + 1].T @ u)
        u -= Vs[:, : j + 1] @ (Vs[:, : j + 1].T @ u)
        b[j] = np.linalg.norm(u)
        if j + 1 < k:
            Vs[:, j + 1] = u / b[j]
    return np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)


def test_lanczos_tridiagonal_full_dimension_spectrum():
    """Section III-A: the eigenvalue estimate reads the Lanczos tridiagonal from the CG
    coefficients.  Run for the full dimension, its eigenvalues are the whole spectrum of
    D^{-1} A (known here by construction) up to rounding."""
    lams = np.array([0.3, 0.7, 1.1, 1.9, 2.6, 3.4, 5.0])
    A, d, b = _spd_with_spectrum(lams, 11)
    _, its, al, be = mg.pcg_jacobi(A, 1.0 / d, b, fixed_its=len(lams))
    assert its == len(lams)
    T = mg.lanczos_tridiagonal(al, be[: len(al) - 1])
    np.testing.assert_allclose(np.linalg.eigvalsh(T), lams, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("k", [3, 5])
def test_lanczos_tridiagonal_equals_plain_lanczos(k):
    """Entry by entry, the tridiagonal built from k Jacobi-PCG coefficients equals plain
    Lanczos on D^{-1/2} A D^{-1/2} started from D^{-1/2} b (off-diagonal signs are
    immaterial: compared in absolute value)."""
    lams = np.linspace(0.5, 4.0, 9) ** 1.3
    A, d, b = _spd_with_spectrum(lams, 5)
    _, _, al, be = mg.pcg_jacobi(A, 1.0 / d, b, fixed_its=k)
    T = mg.lanczos_tridiagonal(al, be[: k - 1])
    S = A / np.sqrt(d)[:, None] / np.sqrt(d)[None, :]
    T_ref = _plain_lanczos(S, b / np.sqrt(d), k)
    np.testing.assert_allclose(np.abs(T), np.abs(T_ref), rtol=1e-11, atol=1e-12)


def _two_level(n=2, pf=2, pc=1, coarse_fixed=None, coarse_rtol=1e-3, degree=3, amplitude=0.05):
    mf, mc, Pm = _levels(n, pf, pc)
    d = fem.make_disc(mf.coords, mf.elem_nodes, mf.P)
    maskf = inputs.face_mask(mf, {"x0": (1, 1, 1)})
    maskc = inputs.face_mask(mc, {"x0": (1, 1, 1)})
    u = inputs.config1_u(mf, amplitude=amplitude)
    K = fem.tangent_matrix(d, u, MU, LAM)
    seeds = [inputs.rough_seed(mf.n_nodes, maskf, 7)]
    V = mg.VCycle(K, [Pm], [maskf, maskc], seeds, degree=degree, coarse_rtol=coarse_rtol,
                  coarse_fixed=coarse_fixed)
    return mf, maskf, V


def test_vcycle_symmetric_with_exact_coarse_solve():
    mf, maskf, V = _two_level(coarse_rtol=1e-15, coarse_fixed=None)
    rng = np.random.default_rng(1)
    fr = 1.0 - maskf.reshape(-1)
    v = rng.normal(size=3 * mf.n_nodes) * fr
    w = rng.normal(size=3 * mf.n_nodes) * fr
    a, b = v @ V(w), w @ V(v)
    assert abs(a - b) <= 1e-10 * abs(a)


def test_fcg_matches_direct_solve():
    mf, maskf, V = _two_level()
    A = V.ops[0]
    rng = np.random.default_rng(2)
    b = rng.normal(size=A.shape[0]) * (1.0 - maskf.reshape(-1))
    x, its, rel = mg.fcg(A, V, b, rtol=1e-10, maxit=200)
    xs = spla.spsolve(A.tocsc(), b)
    assert rel <= 1e-10
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert its < 100


@pytest.mark.parametrize("solver", ["fcg", "fcg_truncated"])
def test_fcg_natural_norm_is_the_preconditioned_residual_norm(solver):
    """The natural-norm stop (Section III-A): the reported relative residual is
    sqrt(r^T M^-1 r) / sqrt(b^T M^-1 b) of the returned iterate, with r recomputed from
    x (here M^-1 is a Jacobi preconditioner, so the norm is a weighted 2-norm that can be
    formed without the solver), and the solve stops at the first iteration that meets
    the tolerance."""
    mf, maskf, V = _two_level(amplitude=0.0)
    A = V.ops[0]
    fr = 1.0 - maskf.reshape(-1)
    dinv = 1.0 / A.diagonal()
    M = lambda v: dinv * v  # noqa: E731
    rng = np.random.default_rng(3)
    b = rng.normal(size=A.shape[0]) * fr
    nat = lambda v: np.sqrt(np.sum(dinv * v * v))  # noqa: E731
    run = getattr(mg, solver)
    x, its, rel = run(A, M, b, rtol=1e-4, maxit=500, norm="natural")[:3]
    assert its > 3
    assert rel <= 1e-4
    assert abs(rel - nat(b - A @ x) / nat(b)) <= 1e-9 * rel
    x1, its1, rel1 = run(A, M, b, rtol=1e-4, maxit=its - 1, norm="natural")[:3]
    assert its1 == its - 1 and rel1 > 1e-4
    assert abs(rel1 - nat(b - A @ x1) / nat(b)) <= 1e-9 * rel1
    # the 2-norm stop measures something else: its reported value is ||r||_2 / ||b||_2
    x2, its2, rel2 = run(A, M, b, rtol=1e-4, maxit=500)[:3]
    assert abs(rel2 - np.linalg.norm(b - A @ x2) / np.linalg.norm(b)) <= 1e-9 * rel2


def test_fcg_truncated_solves_spd_systems_like_a_direct_solve():
    # the tangent at the reference configuration (linear elasticity) is positive definite
    mf, maskf, V = _two_level(amplitude=0.0)
    A = V.ops[0]
    assert np.linalg.eigvalsh(A.toarray()).min() > 0.0
    rng = np.random.default_rng(2)
    b = rng.normal(size=A.shape[0]) * (1.0 - maskf.reshape(-1))
    x, its, rel, broke = mg.fcg_truncated(A, V, b, rtol=1e-10, maxit=200)
    xs = spla.spsolve(A.tocsc(), b)
    assert not broke and rel <= 1e-10
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_fcg_truncated_stops_at_negative_curvature():
    """Closed forms with the identity preconditioner.  A = diag(1, -3), b = (1, 1):
    p0^T A p0 = -2 before any step, so the preconditioned residual b comes back.
    A = diag(2, 1, -3), b = (1, 1, 1/2): the first step is the CG step
    x1 = (b.b / b^T A b) b = b (b.b = b^T A b = 9/4), the second direction has
    p1^T A p1 < 0, so x1 comes back after one iteration."""
    ident = lambda r: r.copy()
    x, its, _, broke = mg.fcg_truncated(np.diag([1.0, -3.0]), ident, np.array([1.0, 1.0]))
    assert broke and its == 0
    np.testing.assert_array_equal(x, [1.0, 1.0])
    x, its, _, broke = mg.fcg_truncated(np.diag([2.0, 1.0, -3.0]), ident, np.array([1.0, 1.0, 0.5]))
    assert broke and its == 1
    np.testing.assert_allclose(x, [1.0, 1.0, 0.5], rtol=0, atol=1e-15)


def _uniaxial_stretch(lx, mu, lam):
    """Lateral stretch t with mu (t^2 - 1) + lambda log(lx t^2) = 0 (scalar Newton)."""
    t = 1.0
    for _ in range(50):
        f = mu * (t * t - 1) + lam * np.log(lx * t * t)
        df = 2 * mu * t + 2 * lam / t
        t -= f / df
    return t


@pytest.mark.parametrize("p", [1, 2])
def test_newton_uniaxial_closed_form(p):
    m = inputs.box_mesh(2, p, jitter=0.1)
    d = fem.make_disc(m.coords, m.elem_nodes, m.P)
    mask = inputs.face_mask(m, {"x0": (1, 0, 0), "y0": (0, 1, 0), "z0": (0, 0, 1), "x1": (1, 0, 0)})
    delta = 0.3
    lift = inputs.affine_lifting(m, (delta, 0.0, 0.0))

    def solve(K, rhs):
        return spla.spsolve(K.tocsc(), rhs)

    u, hist = mg.newton_load_steps(d, MU, LAM, mask, lift, 3, solve, rtol=1e-10)
    lx = 1.0 + delta
    lt = _uniaxial_stretch(lx, MU, LAM)
    exact = m.coords * np.array([lx - 1.0, lt - 1.0, lt - 1.0])
    np.testing.assert_allclose(u, exact, atol=1e-10)
    assert max(hist) <= 8


def test_newton_with_pmg_fcg():
    """Newton-FCG with the p-MG V-cycle (Q2 -> Q1) reaches the direct-solve answer."""
    mf, mc, Pm = _levels(2, 2, 1)
    d = fem.make_disc(mf.coords, mf.elem_nodes, 3)
    maskf = inputs.face_mask(mf, {"x0": (1, 1, 1), "x1": (1, 1, 1)})
    maskc = inputs.face_mask(mc, {"x0": (1, 1, 1), "x1": (1, 1, 1)})
    lift = inputs.affine_lifting(mf, (0.1, 0.0, 0.0))
    ctx = {}

    def solve_pmg(K, rhs):
        Kraw = fem.tangent_matrix(d, ctx["u"], MU, LAM)
        V = mg.VCycle(Kraw, [Pm], [maskf, maskc], [inputs.rough_seed(mf.n_nodes, maskf)])
        x, _, _ = mg.fcg(K, V, rhs, rtol=1e-10)
        return x

    def solve_direct(K, rhs):
        return spla.spsolve(K.tocsc(), rhs)

    # the driver calls linear_solve with the tangent at the current u; record u
    orig = fem.tangent_matrix

    def tracking(disc, u, mu, lam):
        ctx["u"] = u
        return orig(disc, u, mu, lam)

    fem.tangent_matrix = tracking
    try:
        u1, h1 = mg.newton_load_steps(d, MU, LAM, maskf, lift, 2, solve_pmg, rtol=1e-9)
    finally:
        fem.tangent_matrix = orig
    u2, h2 = mg.newton_load_steps(d, MU, LAM, maskf, lift, 2, solve_direct, rtol=1e-9)
    np.testing.assert_allclose(u1, u2, atol=1e-9)


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n) * 0.1
    b = rng.standard_normal(n)
    return A, b


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_lbfgs_iterates_are_cg_iterates_on_a_quadratic(k):
    """On a strictly convex quadratic with H0 = I, exact line searches and enough
    memory, (L-)BFGS generates the conjugate-gradient iterates (the BFGS-CG
    equivalence, Nocedal & Wright, Numerical Optimization, Section 6.4); CG is written out independently here."""
    A, b = _spd(12, 3)
    grad = lambda x: A @ x - b
    x_bfgs, its, _ = mg.lbfgs(grad, np.zeros(12), lambda v: v.copy(), memory=12, rtol=0.0, max_its=k,
                              clip=None)
    assert its == k
    x = np.zeros(12)
    r = b.copy()
    p = r.copy()
    for _ in range(k):
        Ap = A @ p
        a = (r @ r) / (p @ Ap)
        x = x + a * p
        r_new = r - a * Ap
        p = r_new + (r_new @ r_new) / (r @ r) * p
        r = r_new
    np.testing.assert_allclose(x_bfgs, x, rtol=1e-9, atol=1e-12)


def test_lbfgs_converges_in_one_step_with_the_exact_inverse_hessian():
    A, b = _spd(10, 4)
    Ainv = np.linalg.inv(A)
    x, its, rel = mg.lbfgs(lambda v: A @ v - b, np.zeros(10), lambda v: Ainv @ v, rtol=1e-12, clip=None)
    assert its == 1
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-12)


def test_lbfgs_load_steps_reach_the_newton_answer():
    """Neo-Hookean, Q2 on 2^3 elements, x = 0 clamped, x = 1 face pulled by 0.2 in two
    load steps: L-BFGS with the tangent inverse at each step's start as H0 converges to
    the equilibrium the Newton driver finds."""
    m = inputs.box_mesh(2, 2, jitter=0.05)
    d = fem.make_disc(m.coords, m.elem_nodes, 3)
    mask = inputs.face_mask(m, {"x0": (1, 1, 1), "x1": (1, 1, 1)})
    lift = inputs.affine_lifting(m, (0.2, 0.0, 0.0))

    def make_h0(u):
        K = fem.apply_bc(fem.tangent_matrix(d, u, MU, LAM), mask).tocsc()
        lu = spla.splu(K)
        return lambda v: lu.solve(v)

    u1, h1 = mg.lbfgs_load_steps(d, MU, LAM, mask, lift, 2, make_h0, rtol=1e-11)
    u2, h2 = mg.newton_load_steps(d, MU, LAM, mask, lift, 2,
                                  lambda K, rhs: spla.spsolve(K.tocsc(), rhs), rtol=1e-11)
    np.testing.assert_allclose(u1, u2, atol=1e-9)
    assert max(h1) <= 30


@pytest.mark.parametrize("scale,expect", [(2.0, 0.5), (0.8, 1.25), (1.0, 1.0)])
def test_line_search_cp_is_exact_on_a_quadratic(scale, expect):
    """For a linear residual F(u) = A u - b the secant on F(u + a du)^T du is exact: a
    direction `scale` times the Newton step gets the step length 1 / scale."""
    A, b = _spd(9, 5)
    du = scale * np.linalg.solve(A, b)
    a = mg.line_search_cp(lambda v: A @ v - b, np.zeros(9), du)
    assert abs(a - expect) < 1e-12
    a2 = mg.line_search_cp_dir(lambda v: A @ v - b, np.zeros(9), du)
    assert abs(a2 - expect) < 1e-12


@pytest.mark.parametrize("pf,pc", [(2, 1), (4, 2), (4, 1)])
def test_rediscretised_coarse_operator_equals_galerkin_for_linear_elasticity(pf, pc):
    """On affine elements at u = 0 the integrand of the coarse stiffness is a polynomial
    that both the fine and the coarse Gauss rules integrate exactly, so the
    rediscretised coarse operator (own order, own (p_c + 1)^3 points) equals the
    Galerkin product P^T K P."""
    mf, mc, Pm = _levels(2, pf, pc, jitter=0.0)
    df = fem.make_disc(mf.coords, mf.elem_nodes, pf + 1)
    dc = fem.make_disc(mc.coords, mc.elem_nodes, pc + 1)
    Kf = fem.tangent_matrix(df, np.zeros((mf.n_nodes, 3)), MU, LAM)
    Kc = fem.tangent_matrix(dc, np.zeros((mc.n_nodes, 3)), MU, LAM)
    G = mg.galerkin(Kf, Pm)
    assert abs(Kc - G).max() < 1e-12 * abs(G).max()


@pytest.mark.parametrize("pf,pc", [(2, 1), (4, 2), (3, 1)])
def test_injection_is_exact_for_affine_fields_and_picks_coinciding_nodes(pf, pc):
    mf, mc, _ = _levels(2, pf, pc, jitter=0.07)
    A = np.array([[0.3, -0.1, 0.2], [0.05, 0.4, -0.2], [0.1, 0.0, -0.3]])
    u_f = mf.coords @ A.T + np.array([0.1, -0.2, 0.3])
    u_c = mg.inject(u_f, mf.elem_nodes, mf.P, mc.elem_nodes, mc.P, mc.n_nodes)
    np.testing.assert_allclose(u_c, mc.coords @ A.T + np.array([0.1, -0.2, 0.3]), atol=1e-13)
    # a non-affine field: coarse vertices coincide with fine vertices
    rng = np.random.default_rng(1)
    w = rng.standard_normal((mf.n_nodes, 3))
    wc = mg.inject(w, mf.elem_nodes, mf.P, mc.elem_nodes, mc.P, mc.n_nodes)
    s = (pf + 1 - 1) // (pc + 1 - 1)
    for e in range(mf.n_elem):
        for a3 in range(pc + 1):
            for a2 in range(pc + 1):
                for a1 in range(pc + 1):
                    ic = mc.elem_nodes[e][a1 + (pc + 1) * (a2 + (pc + 1) * a3)]
                    f_idx = s * a1 + (pf + 1) * (s * a2 + (pf + 1) * s * a3)
                    if pc == 1 or pf % 2 == 0:
                        np.testing.assert_allclose(wc[ic], w[mf.elem_nodes[e][f_idx]], atol=1e-12)
