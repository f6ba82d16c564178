"""C-ABI checks that need no GPU: the library loads, exports every declared symbol,
tabulates the reference tables correctly, and rejects bad arguments on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from _support import ROOT, ensure_built
from oracle import basis as obasis


@pytest.fixture(scope="module")
def L():
    ensure_built()
    from paper_2204_01722_amd import binding
    return binding.lib()


def _declared():
    src = open(os.path.join(ROOT, "include", "hpmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hpmg_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) > 30
    for n in names:
        assert hasattr(L, n), n
    from paper_2204_01722_amd import binding
    assert set(binding.EXPORTED) == set(names)


# every (P, Q) pair the kernels are instantiated for
@pytest.mark.parametrize("P,Q", [(2, 2), (2, 3), (2, 4), (2, 5), (3, 3), (3, 4), (3, 5), (4, 4), (4, 5),
                                 (5, 5), (5, 6)])
def test_tabulation_matches_oracle(L, P, Q):
    from paper_2204_01722_amd.binding import hpmg_basis_tabulate
    t = hpmg_basis_tabulate(P, Q)
    o = obasis.tables_1d(P, Q)
    np.testing.assert_allclose(t["interp"], o["B"], atol=2e-15)
    np.testing.assert_allclose(t["grad"], o["D"], atol=5e-14)
    np.testing.assert_allclose(t["qref"], o["xq"], atol=1e-15)
    np.testing.assert_allclose(t["qweight"], o["wq"], atol=1e-15)
    np.testing.assert_allclose(t["gll"], o["nodes"], atol=1e-15)
    # collocated derivative reproduces the derivative table (full column rank, Q >= P)
    np.testing.assert_allclose(t["colloc"] @ t["interp"], t["grad"], atol=5e-13)


@pytest.mark.parametrize("Pf,Pc", [(3, 2), (4, 2), (5, 2), (4, 3), (5, 3), (5, 4)])  # every instantiated pair
def test_ctof_matches_oracle(L, Pf, Pc):
    from paper_2204_01722_amd.binding import hpmg_basis_ctof
    M = hpmg_basis_ctof(Pf, Pc)
    nodes_c = obasis.gll_nodes(Pc)
    ref, _ = obasis.lagrange(nodes_c, obasis.gll_nodes(Pf))
    np.testing.assert_allclose(M, ref, atol=1e-14)


def test_host_argument_validation(L):
    h = C.c_void_p()
    fake = C.c_void_p(0x1000)  # never dereferenced by create/workspace queries
    assert L.hpmg_basis_tabulate(1, 3, None, None, None, None, None, None) == 1
    assert L.hpmg_basis_tabulate(4, 3, None, None, None, None, None, None) == 1
    assert L.hpmg_op_create(3, 3, 10, 100, None, None, C.byref(h)) == 1
    assert L.hpmg_op_create(6, 6, 10, 100, fake, None, C.byref(h)) == 3
    assert L.hpmg_op_create(3, 3, 0, 100, fake, None, C.byref(h)) == 2
    assert L.hpmg_op_create(3, 3, 10, 1 << 28, fake, None, C.byref(h)) == 2
    assert L.hpmg_op_create(3, 3, 10, 100, fake, None, C.byref(h)) == 0
    nb = C.c_size_t()
    assert L.hpmg_op_workspace_bytes(h, C.byref(nb)) == 0
    # workspace: tables + map + records + incidence + scratch + 10 + 16 + 16/2 doubles per point
    assert nb.value > 10 * 27 * (10 + 16) * 8
    assert L.hpmg_residual(h, fake, fake, 1, None) == 4  # workspace not bound
    assert b"workspace" in L.hpmg_last_error()
    assert L.hpmg_op_set_material(h, 1.0, 1.0, fake, None) == 1
    hc = C.c_void_p()
    assert L.hpmg_op_create_coarse(h, 3, 50, fake, None, C.byref(hc)) == 1  # not lower order
    assert L.hpmg_op_create_coarse(h, 2, 50, fake, None, C.byref(hc)) == 0
    assert L.hpmg_op_create_coarse(hc, 2, 50, fake, None, C.byref(C.c_void_p())) == 1
    L.hpmg_op_destroy(hc)
    L.hpmg_op_destroy(h)
    assert L.hpmg_status_string(6) == b"non-positive Jacobian determinant"


def test_package_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2204_01722_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        binding.lib()


def test_newton_parameters_rejected_before_any_handle_is_used(L):
    """The Newton driver checks its parameters before it looks behind the operator or
    multigrid handles, so bad values are reported without a GPU."""
    from paper_2204_01722_amd import binding
    fake = C.c_void_p(0x1000)  # never dereferenced
    stats = (C.c_double * 64)()
    seeds = (C.c_void_p * 4)()

    def call(mg=fake, **kw):
        prm = binding.NewtonParams()
        L.hpmg_newton_default_params(C.byref(prm))
        for k, v in kw.items():
            setattr(prm, k, v)
        return L.hpmg_newton_solve(fake, mg, fake, fake, None, 1, C.byref(prm), seeds, stats, None)

    bad = [{"lin_norm": 2}, {"lin_norm": -1}, {"rtol": 0.0}, {"lin_rtol": float("nan")},
           {"max_newton": 0}, {"lin_maxit": 0}, {"max_total_newton": 0}, {"max_total_krylov": 0}]
    for kw in bad:
        assert call(**kw) == 1, kw
        assert L.hpmg_last_error().startswith(b"newton_solve:"), kw
    # both norms pass the parameter checks and stop at the (null) multigrid handle
    for norm in (0, 1):
        assert call(mg=None, lin_norm=norm) == 1
        assert b"null multigrid handle" in L.hpmg_last_error()


def test_lbfgs_parameters_rejected_before_any_handle_is_used(L):
    from paper_2204_01722_amd import binding
    fake = C.c_void_p(0x1000)  # never dereferenced
    stats = (C.c_double * 64)()
    seeds = (C.c_void_p * 4)()

    def call(mg=fake, **kw):
        prm = binding.LbfgsParams()
        L.hpmg_lbfgs_default_params(C.byref(prm))
        for k, v in kw.items():
            setattr(prm, k, v)
        return L.hpmg_lbfgs_solve(fake, mg, fake, fake, None, 1, C.byref(prm), seeds, fake, 1 << 20, stats, None)

    for kw in ({"memory": 0}, {"memory": 33}, {"rtol": 0.0}, {"rtol": float("nan")}, {"max_its": 0}):
        assert call(**kw) == 1, kw
        assert L.hpmg_last_error().startswith(b"lbfgs_solve:"), kw
    assert call(mg=None) == 1
    assert b"null multigrid handle" in L.hpmg_last_error()


def test_mg_parameters_rejected_before_any_level_is_used(L):
    from paper_2204_01722_amd import binding
    levels = (C.c_void_p * 3)(0x1000, 0x2000, 0x3000)  # never dereferenced
    out = C.c_void_p()

    def call(n_levels=3, **kw):
        prm = binding.MGParams()
        L.hpmg_mg_default_params(C.byref(prm))
        for k, v in kw.items():
            setattr(prm, k, v)
        return L.hpmg_mg_create(levels, n_levels, C.byref(prm), C.byref(out))

    bad = [{"n_levels": 1}, {"precision": 7}, {"cheb_degree": 0}, {"cheb_lo": 0.0}, {"cheb_hi": 0.05},
           {"lanczos_its": 0}, {"coarse_maxit": 0}, {"coarse_block_layout": 2}, {"coarse_block_layout": -2}]
    for kw in bad:
        assert call(**kw) == 1, kw
        assert L.hpmg_last_error().startswith(b"mg_create:"), kw
        assert out.value is None
