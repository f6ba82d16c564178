"""The Python binding checks every vector before a pointer reaches the library (a wrong
dtype, size or device raises ValueError and launches nothing), and the autograd
residual's "stored" backward notices a linearisation replaced after its forward."""
import numpy as np
import pytest

from _support import ensure_built, gpu_available, print_case, rel, t2n
from oracle import fem
from paper_2204_01722_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not gpu_available():
        pytest.skip("no GPU")
    ensure_built()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_bad_vectors_raise_before_any_launch():
    import torch
    from paper_2204_01722_amd.binding import PMG, hpmg_prolong_add, hpmg_restrict, hpmg_vec_axpby, hpmg_vec_dot
    from paper_2204_01722_amd.problem import Hierarchy
    print_case("binding_checks")
    faces = {"x0": (1, 1, 1)}
    m = inputs.box_mesh(2, 2, jitter=0.05)
    H = Hierarchy(m, [2, 1], faces=faces)
    fine, coarse = H.ops[0], H.ops[1]
    u = _dev(inputs.config1_u(m, amplitude=0.02))
    fine.residual(u, store_state=True)
    mg = PMG(H.ops, precision="f64")
    mg.setup(H.seeds())
    good = torch.zeros(fine.n_nodes, 3, dtype=torch.float64, device="cuda")
    bad_dtype = good.float()
    bad_size = torch.zeros(fine.n_nodes + 1, 3, dtype=torch.float64, device="cuda")
    host = torch.zeros(fine.n_nodes, 3, dtype=torch.float64)
    stride = torch.zeros(3, fine.n_nodes, dtype=torch.float64, device="cuda").t()
    torch.cuda.synchronize()
    for bad in (bad_dtype, bad_size, host):
        with pytest.raises(ValueError):
            mg.vcycle(bad)
        with pytest.raises(ValueError):
            mg.fcg(bad)
        with pytest.raises(ValueError):
            mg.fcg(good, x=bad)
        with pytest.raises(ValueError):
            mg.set_state(bad)
        with pytest.raises(ValueError):
            mg.newton(bad, good, 1, H.seeds())
        with pytest.raises(ValueError):
            mg.newton(good.clone(), bad, 1, H.seeds())
        with pytest.raises(ValueError):
            mg.lbfgs(good.clone(), bad, 1, H.seeds())
        with pytest.raises(ValueError):
            mg.setup([bad])
        with pytest.raises(ValueError):
            fine.jacobian(bad)
        with pytest.raises(ValueError):
            fine.jacobian(good, out=bad)
        with pytest.raises(ValueError):
            fine.residual(bad)
        with pytest.raises(ValueError):
            hpmg_restrict(fine, coarse, bad)
        with pytest.raises(ValueError):
            hpmg_prolong_add(coarse, fine, torch.zeros(coarse.n_nodes, 3, dtype=torch.float64, device="cuda"), bad)
        with pytest.raises(ValueError):
            hpmg_vec_dot(good, bad)
        with pytest.raises(ValueError):
            hpmg_vec_axpby(1.0, good, 1.0, bad)
    with pytest.raises(ValueError):
        mg.fcg(good, x=stride)  # an output updated in place must be contiguous
    with pytest.raises(ValueError):
        hpmg_prolong_add(coarse, fine, good, good)  # a fine vector where a coarse one belongs
    # nothing was launched on bad input, and the good path still works
    z = mg.vcycle(_dev(inputs.random_vector(fine.n_nodes, 3)))
    torch.cuda.synchronize()
    assert torch.isfinite(z).all()
    assert fine.query_flags() == 0


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_stored_backward_after_a_second_forward(precision):
    """Two forwards with different u on one operator, then the first one's backward: the
    stored linearisation belongs to the second forward, so the backward must not use it
    (it recomputes from the first forward's saved u) and matches the oracle VJP at the
    first u."""
    import torch
    from paper_2204_01722_amd.autograd import NeoHookeanResidual
    from paper_2204_01722_amd.problem import Hierarchy
    print_case("autograd_two_forwards", precision=precision)
    faces = {"x0": (1, 1, 1)}
    m = inputs.box_mesh(3, 2, jitter=0.05)
    mu_e, lam_e = inputs.loguniform_materials(m.n_elem, seed=4)
    H = Hierarchy(m, [2], faces=faces, mu_e=mu_e, lam_e=lam_e)
    op = H.fine
    u1 = inputs.config1_u(m, amplitude=0.05)
    u2 = inputs.config1_u(m, amplitude=0.03, seed=9)
    w = inputs.random_vector(m.n_nodes, 5)
    mu_t = _dev(mu_e).requires_grad_(True)
    lam_t = _dev(lam_e).requires_grad_(True)
    ut1 = _dev(u1).requires_grad_(True)
    ut2 = _dev(u2).requires_grad_(True)
    v0 = op.state_version()
    r1 = NeoHookeanResidual.apply(ut1, mu_t, lam_t, op, "stored", precision)
    v1 = op.state_version()
    r2 = NeoHookeanResidual.apply(ut2, mu_t, lam_t, op, "stored", precision)
    assert op.state_version() > v1 > v0
    (r1 * _dev(w)).sum().backward()
    d = fem.make_disc(m.coords, m.elem_nodes, m.P)
    mask = inputs.face_mask(m, faces)
    ub_ref, mub_ref, lamb_ref = fem.residual_vjp(d, u1, w, mu_e, lam_e, mask)
    tol = 1e-12 if precision == "f64" else 1e-5
    assert rel(t2n(ut1.grad), ub_ref) < tol
    assert rel(t2n(mu_t.grad), mub_ref) < tol
    assert rel(t2n(lam_t.grad), lamb_ref) < tol
    # the second forward's backward still reads its own (current) stored linearisation
    mu_t.grad = None
    lam_t.grad = None
    (r2 * _dev(w)).sum().backward()
    ub_ref2, _, _ = fem.residual_vjp(d, u2, w, mu_e, lam_e, mask)
    assert rel(t2n(ut2.grad), ub_ref2) < tol
    torch.cuda.synchronize()
