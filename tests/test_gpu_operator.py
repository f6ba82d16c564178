"""GPU parity of the fused operator kernels against the FP64 oracle (same seeded inputs).

FP64 results must match to 1e-12 relative (2-norm), FP32 applies to 1e-5."""
import numpy as np
import pytest

from _support import LAM, MU, ensure_built, gpu_available, incident_elements, print_case, rel, report, t2n
from oracle import fem, mg as omg
from paper_2204_01722_amd import inputs

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not gpu_available():
        pytest.skip("no GPU")
    ensure_built()


def _setup(n, p, jitter=0.05, faces=None, orders=None, q=None, mu_e=None, lam_e=None, L=(1.0, 1.0, 1.0)):
    from paper_2204_01722_amd.problem import Hierarchy
    m = inputs.box_mesh(n, p, L=L, jitter=jitter)
    H = Hierarchy(m, orders or [p], faces=faces, q=q, mu_e=mu_e, lam_e=lam_e)
    return m, H


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t if dtype is None else t.to(dtype)


@pytest.mark.parametrize("n,p,q", [(3, 1, 2), (3, 2, 3), (2, 3, 4), (2, 4, 5), (2, 2, 4), ((3, 2, 1), 2, 3)])
def test_qdata(n, p, q):
    print_case("qdata", n=n, p=p, q=q)
    m, H = _setup(n, p, jitter=0.08, q=q)
    d = fem.make_disc(m.coords, m.elem_nodes, m.P, q)
    W, dxidX = fem.qdata(d)
    g = t2n(H.fine.qdata_export())
    assert rel(g[:, 0, :], W) < TOL64
    assert rel(g[:, 1:, :].reshape(m.n_elem, 3, 3, -1).transpose(0, 3, 1, 2), dxidX) < TOL64
    assert abs(g[:, 0, :].sum() - 1.0) < 1e-13
    assert H.fine.query_flags() == 0


CASES = [  # (n, p, q, faces)
    (4, 2, 3, None),                                   # the 2,187-DoF parity case
    (4, 2, 3, {"x0": (1, 1, 1), "x1": (1, 0, 0)}),
    ((3, 2, 2), 1, 2, {"y0": (0, 1, 0)}),
    ((2, 3, 2), 3, 4, {"z1": (1, 1, 1)}),
    (2, 4, 5, {"x0": (1, 1, 1)}),
    (3, 2, 4, None),                                   # Q = P + 1
    ((3, 2, 1), 2, 3, None),                           # ragged last tile
    (1, 2, 3, None),                                   # a single element
    (2, 4, 6, {"x1": (1, 1, 1)}),                      # over-integrated order 4 (Q = P + 1)
    (3, 1, 3, {"y0": (1, 1, 1)}),                      # over-integrated order 1
    ((2, 2, 3), 3, 5, {"z0": (0, 0, 1)}),              # over-integrated order 3, a roller face
]


def _oracle_problem(m, q, faces, amplitude=0.05):
    d = fem.make_disc(m.coords, m.elem_nodes, m.P, q)
    mask = inputs.face_mask(m, faces) if faces else None
    u = inputs.config1_u(m, amplitude=amplitude)
    du = inputs.random_vector(m.n_nodes, 2)
    return d, mask, u, du


@pytest.mark.parametrize("n,p,q,faces", CASES)
def test_residual_and_jacobian(n, p, q, faces):
    import torch
    print_case("residual_jacobian", n=n, p=p, q=q, faces=faces)
    m, H = _setup(n, p, faces=faces, q=q)
    d, mask, u, du = _oracle_problem(m, q, faces)
    op = H.fine
    ut, dut = _dev(u), _dev(du)
    r = op.residual(ut, store_state=True)
    r_ref = fem.residual(d, u, MU, LAM, mask)
    assert report("residual", t2n(r), r_ref) < TOL64
    y_ref = fem.jacobian_apply(d, u, du, MU, LAM, mask)
    y = op.jacobian(dut, "f64", "stored")
    assert report("J du FP64 stored", t2n(y), y_ref) < TOL64
    y = op.jacobian(dut, "f64", "recompute", u=ut)
    assert report("J du FP64 recompute", t2n(y), y_ref) < TOL64
    op.state_cast_f32()
    y32 = op.jacobian(dut.float(), "f32", "stored")
    assert y32.dtype == torch.float32
    assert report("J du FP32 stored", t2n(y32), y_ref) < TOL32
    y32 = op.jacobian(dut.float(), "f32", "recompute", u=ut)
    assert report("J du FP32 recompute", t2n(y32), y_ref) < TOL32
    if mask is not None:
        mb = mask.astype(bool)
        assert np.all(t2n(y)[mb] == du[mb])
        assert np.all(t2n(r)[mb] == 0.0)
    assert op.query_flags() == 0


@pytest.mark.parametrize("n,p,q,faces", CASES + [(2, 4, 5, "materials")])
def test_initial_configuration_jacobian(n, p, q, faces):
    """The S(E) (initial-configuration) forms of the same Jacobian, with 19 and 26
    stored scalars, and the 20-scalar current-configuration form, against the oracle's
    first-Piola tangent."""
    print_case("initial_configuration", n=n, p=p, q=q, faces=faces)
    mu_e = lam_e = None
    if faces == "materials":
        m0 = inputs.box_mesh(n, p, jitter=0.05)
        mu_e, lam_e = inputs.loguniform_materials(m0.n_elem, seed=4)
        faces = {"x0": (1, 1, 1)}
    m, H = _setup(n, p, faces=faces, q=q, mu_e=mu_e, lam_e=lam_e)
    d, mask, u, du = _oracle_problem(m, q, faces)
    mu = MU if mu_e is None else mu_e
    lam = LAM if lam_e is None else lam_e
    op = H.fine
    ut, dut = _dev(u), _dev(du)
    op.state_initial(ut)
    y_ref = fem.jacobian_apply(d, u, du, mu, lam, mask)
    for mode in ("initial_native", "initial_tuned", "current_20"):
        y = op.jacobian(dut, "f64", mode)
        assert rel(t2n(y), y_ref) < TOL64, (mode, rel(t2n(y), y_ref))
        if mask is not None:
            mb = mask.astype(bool)
            assert np.all(t2n(y)[mb] == du[mb])
    assert op.query_flags() == 0


@pytest.mark.parametrize("n,p,q,faces", CASES[:5] + CASES[-2:])
def test_diagonal(n, p, q, faces):
    print_case("diagonal", n=n, p=p, q=q, faces=faces)
    m, H = _setup(n, p, faces=faces, q=q)
    d, mask, u, _ = _oracle_problem(m, q, faces)
    op = H.fine
    op.residual(_dev(u), store_state=True)
    ref = fem.diagonal(d, u, MU, LAM, mask)
    assert rel(t2n(op.diagonal("f64")), ref) < TOL64
    op.state_cast_f32()
    assert rel(t2n(op.diagonal("f32")), ref) < TOL32


def _levels_oracle(m, H, u, faces):
    """Oracle prolongations and Galerkin level operators for H's orders."""
    d = fem.make_disc(m.coords, m.elem_nodes, m.P, H.fine.Q)
    K = fem.tangent_matrix(d, u, MU, LAM)
    Ps, Ks = [], [K]
    for l in range(1, len(H.orders)):
        Pf, Pc = H.orders[l - 1] + 1, H.orders[l] + 1
        Pm = omg.prolongation(H.topos[l - 1], Pf, H.ops[l - 1].n_nodes, H.topos[l], Pc, H.ops[l].n_nodes)
        Ps.append(Pm)
        Ks.append(omg.galerkin(Ks[-1], Pm))
    return Ps, Ks


@pytest.mark.parametrize("n,orders,faces", [
    (2, [2, 1], {"x0": (1, 1, 1)}),
    (2, [4, 2, 1], {"x0": (1, 1, 1), "x1": (1, 0, 0)}),
    ((2, 3, 1), [3, 1], None),
    (2, [4, 3], {"y1": (0, 1, 1)}),
])
def test_coarse_levels_and_transfer(n, orders, faces):
    """Coarse operators on the fine quadrature equal the Galerkin products P^T K P;
    prolongation/restriction equal the oracle's interpolation matrix and its transpose."""
    print_case("coarse_levels", n=n, orders=orders, faces=faces)
    m, H = _setup(n, orders[0], faces=faces, orders=orders)
    u = inputs.config1_u(m, amplitude=0.05)
    H.fine.residual(_dev(u), store_state=True)
    H.fine.state_cast_f32()
    Ps, Ks = _levels_oracle(m, H, u, faces)
    from paper_2204_01722_amd.binding import hpmg_prolong_add, hpmg_restrict
    for l in range(1, len(orders)):
        opc, opf = H.ops[l], H.ops[l - 1]
        mc = None if H.masks[l] is None else H.masks[l].reshape(-1).astype(float)
        mf = None if H.masks[l - 1] is None else H.masks[l - 1].reshape(-1).astype(float)
        frc = 1.0 if mc is None else 1.0 - mc
        frf = 1.0 if mf is None else 1.0 - mf
        x = inputs.random_vector(opc.n_nodes, 10 + l)
        Kc = fem.apply_bc(Ks[l], H.masks[l])
        assert rel(t2n(opc.jacobian(_dev(x), "f64")), Kc @ x.reshape(-1)) < TOL64
        assert rel(t2n(opc.jacobian(_dev(x).float(), "f32")), Kc @ x.reshape(-1)) < TOL32
        assert rel(t2n(opc.diagonal("f64")), Kc.diagonal()) < TOL64
        if orders[l] == 1:
            # order-1 coarse level from dense element matrices
            opc.assemble_elements("f64")
            assert rel(t2n(opc.jacobian(_dev(x), "f64")), Kc @ x.reshape(-1)) < TOL64
            opc.assemble_elements("f32")
            assert rel(t2n(opc.jacobian(_dev(x).float(), "f32")), Kc @ x.reshape(-1)) < TOL32
        # prolong_add: y += M_f P M_c x
        y0 = inputs.random_vector(opf.n_nodes, 20 + l)
        yt = _dev(y0.copy())
        hpmg_prolong_add(opc, opf, _dev(x), yt)
        ref = y0.reshape(-1) + frf * (Ps[l - 1] @ (frc * x.reshape(-1)))
        assert rel(t2n(yt), ref) < TOL64
        yt32 = _dev(y0.copy()).float()
        hpmg_prolong_add(opc, opf, _dev(x).float(), yt32, "f32")
        assert rel(t2n(yt32), ref) < TOL32
        # restrict: r_c = M_c P^T M_f r_f
        rf = inputs.random_vector(opf.n_nodes, 30 + l)
        rc = hpmg_restrict(opf, opc, _dev(rf))
        ref = frc * (Ps[l - 1].T @ (frf * rf.reshape(-1)))
        assert rel(t2n(rc), ref) < TOL64


def test_energy_and_flags():
    import torch
    print_case("energy")
    m, H = _setup(3, 2, jitter=0.05)
    d = fem.make_disc(m.coords, m.elem_nodes, 3)
    u = inputs.config1_u(m, amplitude=0.05)
    psi = float(H.fine.energy(_dev(u)))
    ref = fem.energy(d, u, MU, LAM)
    assert abs(psi - ref) <= 1e-12 * abs(ref)
    # a displacement that inverts elements sets the flag (reported, not raised)
    bad = -3.0 * m.coords
    H.fine.residual(_dev(bad), store_state=False)
    torch.cuda.synchronize()
    assert H.fine.query_flags() & 1


def test_inverted_geometry_flag():
    print_case("inverted_geometry")
    from paper_2204_01722_amd.problem import Hierarchy
    m = inputs.box_mesh(2, 2, jitter=0.0)
    c = m.coords.copy()
    c[m.elem_nodes[0, 13]] += np.array([2.0, 0.0, 0.0])
    m.coords = c
    H = Hierarchy(m, [2])
    assert H.fine.query_flags() & 1


@pytest.mark.parametrize("p", [2, 4])
def test_nonfinite_displacement_flag(p):
    """A NaN in the displacement makes J non-finite at the quadrature points of the
    elements around it: the residual raises the non-finite bit, not the inverted one, and
    a finite displacement afterwards leaves the (read-and-cleared) word at zero."""
    import torch
    print_case("nonfinite_u", p=p)
    m, H = _setup(2, p, jitter=0.05)
    u = inputs.config1_u(m, amplitude=0.05)
    assert H.fine.query_flags() == 0
    bad = u.copy()
    bad[m.elem_nodes[0, 0], 1] = np.nan
    H.fine.residual(_dev(bad), store_state=False)
    torch.cuda.synchronize()
    f = H.fine.query_flags()
    assert f & 2 and not f & 1, f
    H.fine.residual(_dev(u), store_state=False)
    torch.cuda.synchronize()
    assert H.fine.query_flags() == 0


def test_nonfinite_geometry_flag():
    print_case("nonfinite_geometry")
    from paper_2204_01722_amd.problem import Hierarchy
    m = inputs.box_mesh(2, 2, jitter=0.0)
    c = m.coords.copy()
    c[m.elem_nodes[0, 13], 2] = np.nan
    m.coords = c
    H = Hierarchy(m, [2])
    assert H.fine.query_flags() & 2


@pytest.mark.parametrize("mode", ["stored", "recompute"])
def test_vjp(mode):
    print_case("vjp", mode=mode)
    m = inputs.box_mesh(3, 2, jitter=0.05)
    mu_e, lam_e = inputs.loguniform_materials(m.n_elem, seed=4)
    faces = {"x0": (1, 1, 1)}
    m, H = _setup(3, 2, faces=faces, mu_e=mu_e, lam_e=lam_e)
    d = fem.make_disc(m.coords, m.elem_nodes, 3)
    mask = inputs.face_mask(m, faces)
    u = inputs.config1_u(m, amplitude=0.05)
    w = inputs.random_vector(m.n_nodes, 5)
    H.fine.residual(_dev(u), store_state=True)
    ub, mub, lamb = H.fine.residual_vjp(_dev(u), _dev(w), mode=mode)
    ub_ref, mub_ref, lamb_ref = fem.residual_vjp(d, u, w, mu_e, lam_e, mask)
    assert rel(t2n(ub), ub_ref) < TOL64
    assert rel(t2n(mub), mub_ref) < TOL64
    assert rel(t2n(lamb), lamb_ref) < TOL64
    # FP32 arithmetic (FP32 state in stored mode)
    H.fine.state_cast_f32()
    import torch
    ub, mub, lamb = H.fine.residual_vjp(_dev(u), _dev(w).float(), mode=mode, precision="f32")
    assert ub.dtype == torch.float32
    assert rel(t2n(ub), ub_ref) < TOL32
    assert rel(t2n(mub), mub_ref) < TOL32
    assert rel(t2n(lamb), lamb_ref) < TOL32


@pytest.mark.parametrize("n,p", [(43, 2), (34, 4)])
def test_full_size_sampled(n, p):
    """The benchmark workloads (Q2 on 43^3 and Q4 on 34^3 jittered boxes, maximum
    stretch 1.3) checked on sampled nodes, each against an oracle run over exactly the
    elements that touch it; plus stored == recompute and FP32 on the whole vector."""
    import torch
    print_case("full_size", n=n, p=p)
    m, H = _setup(n, p, jitter=0.05)
    op = H.fine
    u = inputs.stretch_field(m, 1.3)
    du = inputs.random_vector(m.n_nodes, 3)
    ut, dut = _dev(u), _dev(du)
    r = t2n(op.residual(ut, store_state=True))
    y = t2n(op.jacobian(dut, "f64", "stored"))
    y2 = t2n(op.jacobian(dut, "f64", "recompute", u=ut))
    assert rel(y2, y) < 1e-13
    op.state_cast_f32()
    y32 = t2n(op.jacobian(dut.float(), "f32", "stored"))
    assert rel(y32, y) < TOL32
    assert op.query_flags() == 0
    rng = np.random.default_rng(99)
    nodes = rng.choice(m.n_nodes, 48, replace=False)
    # nodes of the elements where each XCD's contiguous tile range starts (the tiles are
    # split in 8 ranges) and of the last element (the last, possibly ragged, tile)
    info = op.info()
    ET, tiles = info["elems_per_tile"], info["tiles"]
    starts = [min(m.n_elem - 1, ((x * (tiles // 8) + min(x, tiles % 8)) * ET)) for x in range(8)]
    edge = np.unique(np.concatenate([m.elem_nodes[e][[0, m.P ** 3 // 2, m.P ** 3 - 1]]
                                     for e in starts + [m.n_elem - 1]]))
    both = np.concatenate([nodes, edge])
    els = incident_elements(m.elem_nodes, both)
    d = fem.make_disc(m.coords, m.elem_nodes[els], m.P)
    r_all = fem.residual(d, u, MU, LAM)
    y_all = fem.jacobian_apply(d, u, du, MU, LAM)
    assert report(f"residual at {len(nodes)} random nodes", r[nodes], r_all[nodes]) < TOL64
    assert report(f"J du at {len(nodes)} random nodes", y[nodes], y_all[nodes]) < TOL64
    # the tile-boundary nodes sit where the field is small (box corners): their error is
    # measured against the scale of the whole vector
    er = np.abs(r[edge] - r_all[edge]).max() / np.abs(r).max()
    ey = np.abs(y[edge] - y_all[edge]).max() / np.abs(y).max()
    print(f"  {len(edge)} tile-boundary nodes: max error / max|r| {er:.2e}, / max|J du| {ey:.2e}", flush=True)
    assert er < TOL64 and ey < TOL64
    torch.cuda.synchronize()


def test_element_matrices_go_stale_with_the_state():
    """Element matrices built from one linearisation are not used after the fine
    operator stores a new one: the coarse apply follows the new state."""
    print_case("elmat_stale")
    faces = {"x0": (1, 1, 1)}
    m, H = _setup(2, 2, faces=faces, orders=[2, 1])
    u1 = inputs.config1_u(m, amplitude=0.05)
    u2 = inputs.config1_u(m, amplitude=0.02, seed=9)
    H.fine.residual(_dev(u1), store_state=True)
    H.ops[1].assemble_elements("f64")
    H.fine.residual(_dev(u2), store_state=True)
    _, Ks = _levels_oracle(m, H, u2, faces)
    Kc = fem.apply_bc(Ks[1], H.masks[1])
    x = inputs.random_vector(H.ops[1].n_nodes, 41)
    assert rel(t2n(H.ops[1].jacobian(_dev(x), "f64")), Kc @ x.reshape(-1)) < TOL64


@pytest.mark.parametrize("q", [2, 3])
def test_element_matrices_of_a_standalone_order1_operator(q):
    """Element matrices of an order-1 operator from its own linearisation (a rediscretised
    coarse level): the apply from them equals the oracle's Jacobian on the same
    quadrature, in FP64 and FP32."""
    print_case("elmat_standalone", q=q)
    faces = {"x0": (1, 1, 1), "y1": (0, 1, 0)}
    m, H = _setup((3, 2, 2), 1, faces=faces, q=q)
    d, mask, u, du = _oracle_problem(m, q, faces)
    op = H.fine
    op.residual(_dev(u), store_state=True)
    y_ref = fem.jacobian_apply(d, u, du, MU, LAM, mask)
    op.assemble_elements("f64")
    assert rel(t2n(op.jacobian(_dev(du), "f64")), y_ref) < TOL64
    op.state_cast_f32()
    op.assemble_elements("f32")
    assert rel(t2n(op.jacobian(_dev(du).float(), "f32")), y_ref) < TOL32


@pytest.mark.parametrize("p", [2, 4])
def test_external_load_matches_oracle(p):
    """Body force and traction dead loads (Q2, Q4 on a 2 x 1 x 0.5 box, jittered,
    constrained x = 0 face) against the oracle's quadrature of their definitions."""
    print_case("external_load", p=p)
    L = (2.0, 1.0, 0.5)
    faces_bc = {"x0": (1, 1, 1)}
    m = inputs.box_mesh(2, p, L=L, jitter=0.08)
    from paper_2204_01722_amd.problem import Hierarchy
    H = Hierarchy(m, [p], faces=faces_bc)
    d = fem.make_disc(m.coords, m.elem_nodes, m.P)
    g = np.array([0.3, -1.2, 0.7])
    t = np.array([0.25, 0.5, -1.0])
    loaded = [(1 + 2 * (ey + 2 * ez), 1) for ez in range(2) for ey in range(2)]
    mask = inputs.face_mask(m, faces_bc).astype(bool)
    ref = fem.body_force_load(d, g) + fem.traction_load(m.coords, m.elem_nodes, m.P, m.P, loaded, t)
    ref[mask] = 0.0
    f = H.fine.external_load(g, H.coords, loaded, t)
    assert rel(t2n(f), ref) < TOL64
    fb = H.fine.external_load(g)
    refb = fem.body_force_load(d, g)
    refb[mask] = 0.0
    assert rel(t2n(fb), refb) < TOL64
