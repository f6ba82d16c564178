"""Thin ctypes binding of ``libhpmg.so`` (the C ABI declared in ``include/hpmg.h``).

Argument marshalling only: every computation runs in the library's HIP kernels.  Device
buffers are PyTorch tensors on the current CUDA (HIP) device; work is enqueued on
``torch.cuda.current_stream()``.  The module-level ``hpmg_*`` functions mirror the C
entry points one to one; :class:`Operator` and :class:`PMG` own the handles, the
workspaces and references to every borrowed tensor.

If the library has not been built, loading fails loudly (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhpmg.so")

F64, F32 = 0, 1
STORED, RECOMPUTE, INITIAL_NATIVE, INITIAL_TUNED, CURRENT_20 = 0, 1, 2, 3, 4
FLAG_NONPOSITIVE_J, FLAG_NONFINITE, FLAG_BAD_INDEX = 1, 2, 4
REDUCE_SCRATCH = 2048

_lib = None


class HpmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hpmg status {status}: {msg}")
        self.status = status


class MGParams(C.Structure):
    _fields_ = [("cheb_degree", C.c_int), ("cheb_lo", C.c_double), ("cheb_hi", C.c_double),
                ("lanczos_its", C.c_int), ("coarse_rtol", C.c_double), ("coarse_maxit", C.c_int),
                ("coarse_fixed_its", C.c_int), ("precision", C.c_int),
                ("coarse_element_matrices", C.c_int), ("coarse_block_layout", C.c_int)]


class NewtonParams(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_newton", C.c_int), ("lin_rtol", C.c_double),
                ("lin_maxit", C.c_int), ("line_search", C.c_int), ("monitor", C.c_int),
                ("max_total_newton", C.c_int), ("max_total_krylov", C.c_int), ("predictor", C.c_int),
                ("lin_norm", C.c_int)]


class LbfgsParams(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_its", C.c_int), ("memory", C.c_int),
                ("line_search", C.c_int), ("monitor", C.c_int)]


_VP, _I64, _D, _I = C.c_void_p, C.c_int64, C.c_double, C.c_int
_SIGS = {
    "hpmg_status_string": ([_I], C.c_char_p),
    "hpmg_last_error": ([], C.c_char_p),
    "hpmg_version": ([], C.c_char_p),
    "hpmg_basis_tabulate": ([_I, _I, _VP, _VP, _VP, _VP, _VP, _VP], _I),
    "hpmg_basis_ctof": ([_I, _I, _VP], _I),
    "hpmg_op_create": ([_I, _I, _I64, _I64, _VP, _VP, C.POINTER(_VP)], _I),
    "hpmg_op_create_coarse": ([_VP, _I, _I64, _VP, _VP, C.POINTER(_VP)], _I),
    "hpmg_op_destroy": ([_VP], None),
    "hpmg_op_set_material": ([_VP, _D, _D, _VP, _VP], _I),
    "hpmg_op_workspace_bytes": ([_VP, C.POINTER(C.c_size_t)], _I),
    "hpmg_op_bind_workspace": ([_VP, _VP, C.c_size_t, _VP], _I),
    "hpmg_op_info": ([_VP, _VP], _I),
    "hpmg_op_query_flags": ([_VP, _VP, C.POINTER(C.c_uint)], _I),
    "hpmg_op_state_version": ([_VP, C.POINTER(C.c_uint64)], _I),
    "hpmg_qdata_setup": ([_VP, _VP, _VP], _I),
    "hpmg_qdata_export": ([_VP, _VP, _VP], _I),
    "hpmg_residual": ([_VP, _VP, _VP, _I, _VP], _I),
    "hpmg_jacobian_apply": ([_VP, _I, _I, _VP, _VP, _VP, _VP], _I),
    "hpmg_state_cast_f32": ([_VP, _VP], _I),
    "hpmg_op_assemble_elements": ([_VP, _I, _VP], _I),
    "hpmg_diagonal": ([_VP, _I, _VP, _VP], _I),
    "hpmg_prolong_add": ([_VP, _VP, _I, _VP, _VP, _VP], _I),
    "hpmg_restrict": ([_VP, _VP, _I, _VP, _VP, _VP], _I),
    "hpmg_energy": ([_VP, _VP, _VP, _VP], _I),
    "hpmg_residual_vjp": ([_VP, _I, _I, _VP, _VP, _VP, _VP, _VP, _VP], _I),
    "hpmg_vec_dot": ([_I, _I64, _VP, _VP, _VP, _VP, _VP], _I),
    "hpmg_vec_dot_noalloc": ([_I, _I64, _VP, _VP, _VP, _VP], _I),
    "hpmg_vec_axpby": ([_I, _I64, _D, _VP, _D, _VP, _VP], _I),
    "hpmg_vec_cast": ([_I64, _I, _VP, _VP, _VP], _I),
    "hpmg_mg_default_params": ([C.POINTER(MGParams)], None),
    "hpmg_mg_create": ([_VP, _I, C.POINTER(MGParams), C.POINTER(_VP)], _I),
    "hpmg_mg_destroy": ([_VP], None),
    "hpmg_mg_workspace_bytes": ([_VP, C.POINTER(C.c_size_t)], _I),
    "hpmg_mg_bind_workspace": ([_VP, _VP, C.c_size_t], _I),
    "hpmg_mg_setup": ([_VP, _VP, _VP], _I),
    "hpmg_mg_vcycle": ([_VP, _VP, _VP, _VP], _I),
    "hpmg_mg_info": ([_VP, _I, C.POINTER(_D), C.POINTER(_I)], _I),
    "hpmg_mg_stats": ([_VP, _VP], _I),
    "hpmg_fcg_solve": ([_VP, _VP, _VP, _VP, _D, _I, C.POINTER(_I), C.POINTER(_D), _VP], _I),
    "hpmg_newton_default_params": ([C.POINTER(NewtonParams)], None),
    "hpmg_state_initial_bytes": ([_VP, C.POINTER(C.c_size_t)], _I),
    "hpmg_state_initial": ([_VP, _VP, _VP, C.c_size_t, _VP], _I),
    "hpmg_mg_set_state": ([_VP, _VP, _VP], _I),
    "hpmg_newton_solve": ([_VP, _VP, _VP, _VP, _VP, _I, C.POINTER(NewtonParams), _VP, _VP, _VP], _I),
    "hpmg_external_load_workspace_bytes": ([_VP, _I64, C.POINTER(C.c_size_t)], _I),
    "hpmg_external_load": ([_VP, _VP, _VP, _I64, _VP, _VP, _VP, _VP, C.c_size_t, _VP, _VP], _I),
    "hpmg_lbfgs_default_params": ([C.POINTER(LbfgsParams)], None),
    "hpmg_lbfgs_workspace_bytes": ([_VP, _I, C.POINTER(C.c_size_t)], _I),
    "hpmg_lbfgs_solve": ([_VP, _VP, _VP, _VP, _VP, _I, C.POINTER(LbfgsParams), _VP, _VP, C.c_size_t, _VP, _VP],
                         _I),
}
EXPORTED = tuple(_SIGS)


def lib():
    """Loads ``libhpmg.so`` once.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2204_01722_amd.build` (no fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        L = lib()
        raise HpmgError(st, f"{L.hpmg_status_string(st).decode()}: {L.hpmg_last_error().decode()}")


def _p(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_cuda:
            raise ValueError("device tensor expected")
        if not t.is_contiguous():
            raise ValueError("contiguous tensor expected")
        return C.c_void_p(t.data_ptr())
    return t


def _vec(v, n_nodes, dtype, device, what):
    """Checks an L-vector before its pointer reaches the library, which reads and writes
    exactly ``3 * n_nodes`` entries of ``dtype``: a wrong dtype, size, device or layout
    raises here instead of touching memory outside the tensor."""
    if not isinstance(v, torch.Tensor):
        raise ValueError(f"{what}: tensor expected")
    if v.dtype != dtype:
        raise ValueError(f"{what}: {dtype} expected, got {v.dtype}")
    if v.numel() != 3 * n_nodes:
        raise ValueError(f"{what}: {3 * n_nodes} entries expected, got {v.numel()}")
    if not v.is_cuda or v.device != torch.device(device):
        raise ValueError(f"{what}: tensor on {device} expected, got {v.device}")
    if not v.is_contiguous():
        raise ValueError(f"{what}: contiguous tensor expected")
    return v


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _prec(p):
    if p in (F64, "f64", "fp64", torch.float64):
        return F64
    if p in (F32, "f32", "fp32", torch.float32):
        return F32
    raise ValueError(f"bad precision {p!r}")


def _mode(m):
    if m in (STORED, "stored"):
        return STORED
    if m in (RECOMPUTE, "recompute"):
        return RECOMPUTE
    if m in (INITIAL_NATIVE, "initial_native"):
        return INITIAL_NATIVE
    if m in (INITIAL_TUNED, "initial_tuned"):
        return INITIAL_TUNED
    if m in (CURRENT_20, "current_20"):
        return CURRENT_20
    raise ValueError(f"bad mode {m!r}")


def _dtype(prec):
    return torch.float64 if prec == F64 else torch.float32


# ---- host-only entry points --------------------------------------------------------
def hpmg_basis_tabulate(P: int, Q: int):
    """Returns dict of numpy arrays: interp [Q][P], grad [Q][P], colloc [Q][Q], qref,
    qweight [Q], gll [P] (computed by the library on the host)."""
    import numpy as np
    out = {k: np.zeros(s) for k, s in (("interp", (Q, P)), ("grad", (Q, P)), ("colloc", (Q, Q)),
                                        ("qref", (Q,)), ("qweight", (Q,)), ("gll", (P,)))}
    ptr = {k: v.ctypes.data_as(C.c_void_p) for k, v in out.items()}
    _check(lib().hpmg_basis_tabulate(P, Q, ptr["interp"], ptr["grad"], ptr["colloc"], ptr["qref"],
                                     ptr["qweight"], ptr["gll"]))
    return out


def hpmg_basis_ctof(Pf: int, Pc: int):
    import numpy as np
    M = np.zeros((Pf, Pc))
    _check(lib().hpmg_basis_ctof(Pf, Pc, M.ctypes.data_as(C.c_void_p)))
    return M


def hpmg_version() -> str:
    return lib().hpmg_version().decode()


# ---- operator --------------------------------------------------------------------
class Operator:
    """One multigrid level: ``E^T B^T D B E`` on one device (handle + workspace)."""

    def __init__(self, P: int, Q: int, elem_nodes: torch.Tensor, n_nodes: int,
                 mask: torch.Tensor | None = None, fine: "Operator | None" = None):
        if elem_nodes.dtype != torch.int32:
            raise ValueError("elem_nodes must be int32")
        if elem_nodes.dim() != 2 or elem_nodes.shape[1] != P ** 3:
            raise ValueError("elem_nodes must be [n_elem][P^3]")
        if mask is not None and (mask.dtype != torch.uint8 or mask.numel() != 3 * n_nodes):
            raise ValueError("mask must be uint8 [n_nodes][3]")
        self.P, self.Q, self.n_nodes = P, Q, int(n_nodes)
        self.n_elem = int(elem_nodes.shape[0])
        self.device = elem_nodes.device
        self._keep = [elem_nodes, mask]
        self.elem_nodes, self.mask, self.fine = elem_nodes, mask, fine
        h = C.c_void_p()
        if fine is None:
            _check(lib().hpmg_op_create(P, Q, self.n_elem, self.n_nodes, _p(elem_nodes), _p(mask),
                                        C.byref(h)))
        else:
            if Q != fine.Q or self.n_elem != fine.n_elem:
                raise ValueError("a coarse operator shares the fine elements and quadrature")
            _check(lib().hpmg_op_create_coarse(fine.h, P, self.n_nodes, _p(elem_nodes), _p(mask),
                                               C.byref(h)))
        self.h = h
        nb = C.c_size_t()
        _check(lib().hpmg_op_workspace_bytes(self.h, C.byref(nb)))
        self.workspace = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=self.device)
        _check(lib().hpmg_op_bind_workspace(self.h, _p(self.workspace), int(nb.value), _stream()))
        self._mat = []

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.hpmg_op_destroy(h)
            self.h = None

    @property
    def n_dof(self):
        return 3 * self.n_nodes

    def info(self):
        arr = (C.c_int64 * 8)()
        _check(lib().hpmg_op_info(self.h, C.cast(arr, C.c_void_p)))
        keys = ("P", "Q", "n_elem", "n_nodes", "elems_per_tile", "tiles", "threads", "tile_stride")
        return dict(zip(keys, list(arr)))

    def set_material(self, mu, lam, mu_e: torch.Tensor | None = None, lam_e: torch.Tensor | None = None):
        for t in (mu_e, lam_e):
            if t is not None and (t.dtype != torch.float64 or t.numel() != self.n_elem):
                raise ValueError("per-element materials must be float64 [n_elem]")
        self._mat = [mu_e, lam_e]
        _check(lib().hpmg_op_set_material(self.h, float(mu), float(lam), _p(mu_e), _p(lam_e)))

    def query_flags(self) -> int:
        f = C.c_uint()
        _check(lib().hpmg_op_query_flags(self.h, _stream(), C.byref(f)))
        return int(f.value)

    def _vec(self, dtype=torch.float64):
        return torch.empty(self.n_nodes, 3, dtype=dtype, device=self.device)

    def _in(self, v, dtype=torch.float64, what="vector"):
        if isinstance(v, torch.Tensor) and v.dtype == dtype and v.numel() == self.n_dof:
            v = v.contiguous()
        return _vec(v, self.n_nodes, dtype, self.device, what)

    def _out(self, out, dtype):
        return self._vec(dtype) if out is None else _vec(out, self.n_nodes, dtype, self.device, "out")

    def state_version(self) -> int:
        """Counter of the stored linearisation this operator applies (bumped whenever
        it is overwritten)."""
        v = C.c_uint64()
        _check(lib().hpmg_op_state_version(self.h, C.byref(v)))
        return int(v.value)

    def qdata_setup(self, coords: torch.Tensor):
        c = self._in(coords, what="coords")
        self._keep.append(c)
        _check(lib().hpmg_qdata_setup(self.h, _p(c), _stream()))

    def qdata_export(self) -> torch.Tensor:
        out = torch.empty(self.n_elem, 10, self.Q ** 3, dtype=torch.float64, device=self.device)
        _check(lib().hpmg_qdata_export(self.h, _p(out), _stream()))
        return out

    def external_load(self, rho_g=None, coords=None, faces=None, traction=None):
        """External dead load ``f_ext`` ([N][3] FP64): body force ``rho_g`` per unit
        reference volume plus a constant ``traction`` on ``faces`` (pairs (element,
        local face 0..5)); constrained components 0."""
        import numpy as np
        nf = 0 if faces is None else len(faces)
        if nf and (coords is None or traction is None):
            raise ValueError("faces need coords and a traction")
        coords = None if coords is None else self._in(coords, torch.float64, "coords")
        f = self._vec(torch.float64)
        fe = fi = ws = None
        nb = C.c_size_t(0)
        if nf:
            fa = np.asarray(faces, np.int32).reshape(nf, 2)
            fe = torch.from_numpy(np.ascontiguousarray(fa[:, 0])).to(self.device)
            fi = torch.from_numpy(np.ascontiguousarray(fa[:, 1])).to(self.device)
            _check(lib().hpmg_external_load_workspace_bytes(self.h, nf, C.byref(nb)))
            ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=self.device)
        g = None if rho_g is None else (C.c_double * 3)(*[float(v) for v in rho_g])
        t = None if traction is None else (C.c_double * 3)(*[float(v) for v in traction])
        _check(lib().hpmg_external_load(self.h, None if g is None else C.cast(g, C.c_void_p),
                                        None if coords is None else _p(coords), nf,
                                        None if fe is None else _p(fe), None if fi is None else _p(fi),
                                        None if t is None else C.cast(t, C.c_void_p),
                                        None if ws is None else _p(ws), int(nb.value), _p(f), _stream()))
        return f

    def state_initial(self, u):
        """Stores the alternative linearisations at ``u`` (grad_X u, C^-1, lambda log J,
        dxi/dx, J - 1) for the ``initial_native``, ``initial_tuned`` and ``current_20``
        Jacobian modes."""
        nb = C.c_size_t()
        _check(lib().hpmg_state_initial_bytes(self.h, C.byref(nb)))
        self.sinit = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=self.device)
        _check(lib().hpmg_state_initial(self.h, _p(self._in(u, what="u")), _p(self.sinit), int(nb.value),
                                        _stream()))

    def residual(self, u, store_state: bool = True, out=None):
        u = self._in(u, what="u")
        r = self._out(out, torch.float64)
        _check(lib().hpmg_residual(self.h, _p(u), _p(r), int(bool(store_state)), _stream()))
        return r

    def jacobian(self, du, precision="f64", mode="stored", u=None, out=None):
        prec, md = _prec(precision), _mode(mode)
        du = self._in(du, _dtype(prec), "du")
        uu = None if u is None else self._in(u, what="u")
        y = self._out(out, _dtype(prec))
        _check(lib().hpmg_jacobian_apply(self.h, prec, md, _p(uu), _p(du), _p(y), _stream()))
        return y

    def state_cast_f32(self):
        _check(lib().hpmg_state_cast_f32(self.h, _stream()))

    def assemble_elements(self, precision="f64"):
        _check(lib().hpmg_op_assemble_elements(self.h, _prec(precision), _stream()))

    def diagonal(self, precision="f64"):
        prec = _prec(precision)
        d = self._vec(_dtype(prec))
        _check(lib().hpmg_diagonal(self.h, prec, _p(d), _stream()))
        return d

    def energy(self, u) -> torch.Tensor:
        u = self._in(u, what="u")
        psi = torch.empty((), dtype=torch.float64, device=self.device)
        _check(lib().hpmg_energy(self.h, _p(u), _p(psi), _stream()))
        return psi

    def residual_vjp(self, u, w, mode="recompute", want_params=True, precision="f64"):
        prec = _prec(precision)
        u = self._in(u, what="u")
        w = self._in(w, _dtype(prec), "w")
        ub = self._vec(_dtype(prec))
        mub = lamb = None
        if want_params:
            mub = torch.empty(self.n_elem, dtype=torch.float64, device=self.device)
            lamb = torch.empty(self.n_elem, dtype=torch.float64, device=self.device)
        _check(lib().hpmg_residual_vjp(self.h, prec, _mode(mode), _p(u), _p(w), _p(ub), _p(mub), _p(lamb),
                                       _stream()))
        return ub, mub, lamb


def hpmg_prolong_add(coarse: Operator, fine: Operator, xc, yf, precision="f64"):
    prec = _prec(precision)
    xc = coarse._in(xc, _dtype(prec), "xc")
    _vec(yf, fine.n_nodes, _dtype(prec), fine.device, "yf")
    _check(lib().hpmg_prolong_add(coarse.h, fine.h, prec, _p(xc), _p(yf), _stream()))
    return yf


def hpmg_restrict(fine: Operator, coarse: Operator, rf, precision="f64", out=None):
    prec = _prec(precision)
    rf = fine._in(rf, _dtype(prec), "rf")
    rc = coarse._out(out, _dtype(prec))
    _check(lib().hpmg_restrict(fine.h, coarse.h, prec, _p(rf), _p(rc), _stream()))
    return rc


def _same_vectors(*vs):
    v0 = vs[0]
    for v in vs:
        if not isinstance(v, torch.Tensor) or not v.is_cuda or not v.is_contiguous():
            raise ValueError("contiguous device tensors expected")
        if v.dtype != v0.dtype or v.numel() != v0.numel() or v.device != v0.device:
            raise ValueError("vectors of one dtype, size and device expected")
    if v0.dtype not in (torch.float64, torch.float32):
        raise ValueError("float64 or float32 vectors expected")


def hpmg_vec_dot(x, y, scratch=None):
    _same_vectors(x, y)
    prec = _prec(x.dtype)
    if scratch is None:
        scratch = torch.empty(REDUCE_SCRATCH, dtype=torch.float64, device=x.device)
    elif scratch.dtype != torch.float64 or scratch.numel() < REDUCE_SCRATCH or scratch.device != x.device:
        raise ValueError(f"scratch must be float64 with at least {REDUCE_SCRATCH} entries on {x.device}")
    out = torch.empty((), dtype=torch.float64, device=x.device)
    _check(lib().hpmg_vec_dot(prec, x.numel(), _p(x), _p(y), _p(out), _p(scratch), _stream()))
    return out


def hpmg_vec_dot_noalloc(x, y, out=None):
    """``x . y`` into a device FP64 scalar without a scratch buffer (the library keeps
    the partial sums in a static device array; calls overlapping on one GPU race)."""
    _same_vectors(x, y)
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=x.device)
    elif out.dtype != torch.float64 or out.numel() < 1 or out.device != x.device:
        raise ValueError(f"out must be a float64 tensor on {x.device}")
    _check(lib().hpmg_vec_dot_noalloc(_prec(x.dtype), x.numel(), _p(x), _p(y), _p(out), _stream()))
    return out


def hpmg_vec_axpby(alpha, x, beta, y):
    _same_vectors(x, y)
    _check(lib().hpmg_vec_axpby(_prec(x.dtype), x.numel(), float(alpha), _p(x), float(beta), _p(y), _stream()))
    return y


def hpmg_vec_cast(x, dtype):
    if not isinstance(x, torch.Tensor) or x.dtype not in (torch.float64, torch.float32) or not x.is_cuda:
        raise ValueError("float64 or float32 device tensor expected")
    y = torch.empty(x.shape, dtype=dtype, device=x.device)
    _check(lib().hpmg_vec_cast(x.numel(), _prec(dtype), _p(x.contiguous()), _p(y), _stream()))
    return y


# ---- multigrid -------------------------------------------------------------------
class PMG:
    """p-multigrid V-cycle over ``levels`` (fine first), with FCG and Newton drivers."""

    def __init__(self, levels, precision="f64", cheb_degree=3, cheb_lo=0.1, cheb_hi=1.1,
                 lanczos_its=10, coarse_rtol=1e-3, coarse_maxit=10000, coarse_fixed_its=0,
                 coarse_element_matrices=True, coarse_block_layout="auto"):
        self.levels = list(levels)
        prm = MGParams()
        lib().hpmg_mg_default_params(C.byref(prm))
        prm.cheb_degree, prm.cheb_lo, prm.cheb_hi = cheb_degree, cheb_lo, cheb_hi
        prm.lanczos_its, prm.coarse_rtol, prm.coarse_maxit = lanczos_its, coarse_rtol, coarse_maxit
        prm.coarse_fixed_its, prm.precision = coarse_fixed_its, _prec(precision)
        prm.coarse_element_matrices = int(bool(coarse_element_matrices))
        layouts = {"auto": -1, "rows": 0, "nodes": 1}
        if coarse_block_layout not in layouts:
            raise ValueError(f"coarse_block_layout must be one of {sorted(layouts)}")
        prm.coarse_block_layout = layouts[coarse_block_layout]
        self.params = prm
        arr = (C.c_void_p * len(self.levels))(*[op.h.value for op in self.levels])
        h = C.c_void_p()
        _check(lib().hpmg_mg_create(C.cast(arr, C.c_void_p), len(self.levels), C.byref(prm), C.byref(h)))
        self.h = h
        nb = C.c_size_t()
        _check(lib().hpmg_mg_workspace_bytes(self.h, C.byref(nb)))
        dev = self.levels[0].device
        self.workspace = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=dev)
        _check(lib().hpmg_mg_bind_workspace(self.h, _p(self.workspace), int(nb.value)))
        self._seeds = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.hpmg_mg_destroy(h)
            self.h = None

    def _fine_vec(self, v, what):
        """FP64 vector of the fine level (the drivers' and the V-cycle's interface)."""
        return self.levels[0]._in(v, torch.float64, what)

    def _seed_array(self, seeds):
        seeds = list(seeds)
        if len(seeds) < len(self.levels) - 1:
            raise ValueError("one rough seed vector per smoothed level")
        seeds = [self.levels[l]._in(s, torch.float64, f"seed {l}") if l < len(self.levels) - 1 else s
                 for l, s in enumerate(seeds)]
        self._seeds = seeds
        arr = (C.c_void_p * len(seeds))(*[s.data_ptr() for s in seeds])
        self._seed_c = arr
        return C.cast(arr, C.c_void_p)

    def setup(self, seeds):
        _check(lib().hpmg_mg_setup(self.h, self._seed_array(seeds), _stream()))

    def vcycle(self, r):
        r = self._fine_vec(r, "r")
        z = torch.empty_like(r)
        _check(lib().hpmg_mg_vcycle(self.h, _p(r), _p(z), _stream()))
        return z

    def info(self, level):
        lam, its = C.c_double(), C.c_int()
        _check(lib().hpmg_mg_info(self.h, level, C.byref(lam), C.byref(its)))
        return float(lam.value), int(its.value)

    def stats(self):
        arr = (C.c_int64 * 11)()
        _check(lib().hpmg_mg_stats(self.h, C.cast(arr, C.c_void_p)))
        v = list(arr)
        return {"vcycles": v[0], "coarse_its": v[1], "setups": v[2],
                "applies_per_level": v[3:3 + len(self.levels)]}

    def fcg(self, b, x=None, rtol=1e-8, maxit=500):
        b = self._fine_vec(b, "b")
        x = torch.zeros_like(b) if x is None else _vec(x, self.levels[0].n_nodes, torch.float64,
                                                        self.levels[0].device, "x")
        its, rel = C.c_int(), C.c_double()
        _check(lib().hpmg_fcg_solve(self.levels[0].h, self.h, _p(b), _p(x), float(rtol),
                                    int(maxit), C.byref(its), C.byref(rel), _stream()))
        return x, int(its.value), float(rel.value)

    def newton(self, u, lift, n_steps, seeds, rtol=1e-8, max_newton=20, lin_rtol=1e-3, lin_maxit=500,
               line_search=True, monitor=False, f_ext=None, max_total_newton=None, max_total_krylov=None,
               predictor=None, lin_norm="2"):
        """Newton load stepping (``u`` FP64 [N][3], updated in place).  ``lin_norm``: the
        FCG stopping norm, "2" for the residual 2-norm, "natural" for sqrt(r^T M^-1 r)
        with M^-1 the V-cycle.  Returns ``u`` and a statistics dict."""
        if lin_norm not in ("2", "natural"):
            raise ValueError(f"lin_norm must be '2' or 'natural', got {lin_norm!r}")
        _vec(u, self.levels[0].n_nodes, torch.float64, self.levels[0].device, "u")
        lift = self._fine_vec(lift, "lift")
        f_ext = None if f_ext is None else self._fine_vec(f_ext, "f_ext")
        prm = NewtonParams()
        lib().hpmg_newton_default_params(C.byref(prm))
        prm.rtol, prm.max_newton, prm.lin_rtol = rtol, max_newton, lin_rtol
        prm.lin_maxit, prm.line_search = lin_maxit, int(bool(line_search))
        prm.monitor = int(bool(monitor))
        if max_total_newton is not None:
            prm.max_total_newton = int(max_total_newton)
        if max_total_krylov is not None:
            prm.max_total_krylov = int(max_total_krylov)
        if predictor is not None:
            prm.predictor = int(bool(predictor))
        prm.lin_norm = 1 if lin_norm == "natural" else 0
        stats = (C.c_double * (4 + n_steps))()
        st = lib().hpmg_newton_solve(self.levels[0].h, self.h, _p(u), _p(lift),
                                     None if f_ext is None else _p(f_ext), int(n_steps),
                                     C.byref(prm), self._seed_array(seeds), C.cast(stats, C.c_void_p),
                                     _stream())
        s = list(stats)
        res = {"newton_its": int(s[0]), "krylov_its": int(s[1]), "final_rel": s[2], "step_halvings": int(s[3]),
               "per_step": [int(v) for v in s[4:]]}
        if st != 0:
            try:
                _check(st)
            except HpmgError as err:
                raise HpmgError(st, f"{err} (statistics so far: {res})") from None
        return u, res

    def newton_checkpointed(self, u, lift, n_steps, seeds, path, f_ext=None, stop_after=None, **newton_kw):
        """Newton load stepping one load level per driver call, with the state saved to
        ``path`` (``.npz``) after every converged level and a run resumed after the last
        saved level (see :mod:`.checkpoint`).  Level k adds ``lift / n_steps`` to ``u``
        and balances ``(k / n_steps) f_ext``: the same levels as :meth:`newton` with
        ``n_steps``, each starting from the previous level's state with the Euler
        predictor; the iteration budgets of ``newton_kw`` apply per level.  ``stop_after``
        ends the run at that level.  Returns ``u``, the first level run, the level
        reached and the per-level statistics of :meth:`newton`."""
        from . import checkpoint
        _vec(u, self.levels[0].n_nodes, torch.float64, self.levels[0].device, "u")
        lift = self._fine_vec(lift, "lift")
        f_ext = None if f_ext is None else self._fine_vec(f_ext, "f_ext")
        tag = checkpoint.fingerprint(lift, f_ext, extra=f"newton/{self.levels[0].n_nodes}/{n_steps}")
        step_lift = lift / n_steps

        def step(k, v):
            fk = None if f_ext is None else f_ext * (k / n_steps)
            return self.newton(v, step_lift, 1, seeds, f_ext=fk, **newton_kw)[1]

        return checkpoint.run_load_steps(step, u, n_steps, path, tag, stop_after)

    def set_state(self, u):
        """Stores the linearisations of rediscretised coarse levels at the injection of
        ``u`` (no-op for Galerkin levels)."""
        _check(lib().hpmg_mg_set_state(self.h, _p(self._fine_vec(u, "u")), _stream()))

    def lbfgs(self, u, lift, n_steps, seeds, rtol=1e-8, max_its=200, memory=5, line_search=True,
              monitor=False, f_ext=None):
        """L-BFGS load stepping with this V-cycle as the initial inverse Hessian; ``u``
        (FP64 [N][3]) is updated in place.  Returns ``u`` and a statistics dict."""
        _vec(u, self.levels[0].n_nodes, torch.float64, self.levels[0].device, "u")
        lift = self._fine_vec(lift, "lift")
        f_ext = None if f_ext is None else self._fine_vec(f_ext, "f_ext")
        prm = LbfgsParams()
        lib().hpmg_lbfgs_default_params(C.byref(prm))
        prm.rtol, prm.max_its, prm.memory = rtol, max_its, memory
        prm.line_search, prm.monitor = int(bool(line_search)), int(bool(monitor))
        nb = C.c_size_t()
        _check(lib().hpmg_lbfgs_workspace_bytes(self.h, int(memory), C.byref(nb)))
        ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=u.device)
        stats = (C.c_double * (4 + n_steps))()
        st = lib().hpmg_lbfgs_solve(self.levels[0].h, self.h, _p(u), _p(lift),
                                    None if f_ext is None else _p(f_ext), int(n_steps),
                                    C.byref(prm), self._seed_array(seeds), _p(ws), int(nb.value),
                                    C.cast(stats, C.c_void_p), _stream())
        s = list(stats)
        res = {"iterations": int(s[0]), "vcycles": int(s[1]), "final_rel": s[2], "restarts": int(s[3]),
               "per_step": [int(v) for v in s[4:]]}
        if st != 0:
            try:
                _check(st)
            except HpmgError as err:
                raise HpmgError(st, f"{err} (statistics so far: {res})") from None
        return u, res
