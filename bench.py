#!/usr/bin/env python3
"""Benchmark: matrix-free Neo-Hookean Jacobian apply on one MI355X.

Workload (the operator-at-scale configuration): jittered unit-cube box meshes with a
smooth displacement of maximum stretch 1.3, E = 1, nu = 0.3,
  * Q4 (P = 5 nodes, 5^3 Gauss points) on 34^3 elements: 7,714,059 DoF  (headline)
  * Q2 (P = 3, 3^3 points) on 43^3 elements: 1,975,509 DoF.
A timed "step" is one FP64 Jacobian apply y = J(u) du from the stored 16-scalar
linearisation (gather, sum-factorised gradient, pointwise tangent, transpose, scatter),
inputs resident in HBM.  The JSON line also carries Q2 / FP32 / recompute variants,
the residual, the roofline of the apply kernel, an FP64-vs-mixed p-multigrid solve,
and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 50] [--warmup 10] [--no-cpu] [--no-solve] [--only-headline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def algorithmic_bytes(E, P, Q, N, word, nstate=16, nvec=2):
    """Bytes each apply must move once: the per-point linearisation, the input and
    output L-vectors, and the int32 element-to-node map."""
    return E * Q ** 3 * nstate * word + nvec * 3 * N * word + 4 * E * P ** 3


def measured_traffic():
    """HBM bytes per apply from the committed counter summary, if it was taken on the
    current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_jacobian_q4_fp64_34cubed.json")
    src = os.path.join(ROOT, "paper_2204_01722_amd", "csrc", "op_kernels.hip")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return rec.get("bytes_per_apply")


def prime(fn, seconds):
    """Runs ``fn`` untimed for about ``seconds`` of wall time, so the GPU reaches its
    steady clock before a measurement (as a solver loop keeps it)."""
    import torch
    if seconds <= 0:
        return
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()


def time_op(fn, steps, warmup, stream, prime_s=0.0):
    import torch
    prime(fn, prime_s)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        fn()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps  # ms


def time_median(fn, steps, warmup, stream, reps=3, prime_s=0.2):
    """Median over ``reps`` timed loops of ``steps`` calls (after priming and one warm-up
    loop)."""
    return float(np.median([time_op(fn, steps, warmup if r == 0 else 1, stream, prime_s if r == 0 else 0.0)
                            for r in range(reps)]))


def copy_bandwidth(nbytes=2 << 30):
    """Plain streaming kernel of known size (read 2 GiB, write 2 GiB): the achievable
    bandwidth, and the reference that scales the byte counters of a profiled run."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    s = torch.cuda.current_stream()
    ms = time_op(lambda: torch.mul(a, 1.0, out=b), 10, 3, s)
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


class Workload:
    def __init__(self, n, p, device="cuda"):
        import torch
        from paper_2204_01722_amd import inputs
        from paper_2204_01722_amd.problem import Hierarchy
        self.n, self.p = n, p
        self.mesh = inputs.box_mesh(n, p, jitter=0.05, seed=2204)
        self.H = Hierarchy(self.mesh, [p])
        self.op = self.H.fine
        self.u_np = inputs.stretch_field(self.mesh, 1.3)
        self.du_np = inputs.random_vector(self.mesh.n_nodes, 3)
        self.u = torch.from_numpy(self.u_np).to(device)
        self.du = torch.from_numpy(self.du_np).to(device)
        self.du32 = self.du.float()
        self.r = self.op.residual(self.u, store_state=True)
        self.op.state_cast_f32()
        self.y = torch.empty_like(self.du)
        self.y32 = torch.empty_like(self.du32)
        self.E, self.P, self.Q, self.N = self.mesh.n_elem, p + 1, p + 1, self.mesh.n_nodes
        self.dof = 3 * self.N
        if self.op.query_flags():
            raise RuntimeError("device flags set during setup")

    def apply(self, prec="f64", mode="stored"):
        if prec == "f64":
            return lambda: self.op.jacobian(self.du, "f64", mode, u=self.u, out=self.y)
        return lambda: self.op.jacobian(self.du32, "f32", mode, u=self.u, out=self.y32)

    def residual(self):
        return lambda: self.op.residual(self.u, store_state=True, out=self.r)


def coarse_iteration(sizes, stream, k0=10, k1=210, reps=5):
    """Time of one iteration of the assembled order-1 coarse Jacobi-PCG inside the
    V-cycle, per precision, on the n^3 jittered box (Q4 -> Q2 -> Q1, (n+1)^3 coarse
    nodes, x = 0 and x = 1 faces clamped, linearised at a 10 % stretch): the difference
    of median V-cycle times with k1 and k0 fixed coarse iterations, over k1 - k0, for
    both block layouts (a thread per row, a thread per node) and the default's choice."""
    import torch
    from paper_2204_01722_amd import inputs
    from paper_2204_01722_amd.binding import PMG
    from paper_2204_01722_amd.problem import Hierarchy
    out = {}
    for n in sizes:
        m = inputs.box_mesh(n, 4, jitter=0.05, seed=2204)
        H = Hierarchy(m, [4, 2, 1], faces={"x0": (1, 1, 1), "x1": (1, 1, 1)})
        u = torch.from_numpy(inputs.stretch_field(m, 1.1)).cuda()
        H.fine.residual(u, store_state=True)
        r = torch.from_numpy(inputs.random_vector(m.n_nodes, 5) * (1.0 - H.masks[0])).cuda()
        rec = {"coarse_nodes": (n + 1) ** 3,
               "default_layout": "nodes" if (n + 1) ** 3 >= 65536 else "rows"}
        for prec in ("f64", "f32"):
            for layout in ("rows", "nodes"):
                ms = {}
                for k in (k0, k1):
                    mg = PMG(H.ops, precision=prec, cheb_degree=3, coarse_fixed_its=k, coarse_block_layout=layout)
                    mg.setup(H.seeds(7))
                    ms[k] = time_median(lambda: mg.vcycle(r), 10, 3, stream, reps=reps, prime_s=0.0)
                    del mg
                key = f"{prec}_{layout}_us_per_iteration"
                rec[key] = (ms[k1] - ms[k0]) / (k1 - k0) * 1e3
                print(f"[coarse] {(n + 1) ** 3} coarse nodes, {prec}, a thread per {layout[:-1]}: {rec[key]:.1f} us "
                      f"per iteration", file=sys.stderr, flush=True)
        out[f"{n}^3"] = rec
        del H, u, r
    return out


def adjoint_bench(steps, warmup, stream):
    """The differentiation workload: Q3 on a 23^3 jittered box (1,029,000 DoF), per-element
    Lame parameters log-uniform on [0.5, 2]; times of the adjoint (VJP) kernel giving
    u_bar, mu_bar and lambda_bar, FP64 and FP32, stored and recomputed linearisation."""
    import torch
    from paper_2204_01722_amd import inputs
    from paper_2204_01722_amd.problem import Hierarchy
    m = inputs.box_mesh(23, 3, jitter=0.05, seed=2204)
    mu_e, lam_e = inputs.loguniform_materials(m.n_elem, seed=4)
    H = Hierarchy(m, [3], faces={"x0": (1, 1, 1)}, mu_e=mu_e, lam_e=lam_e)
    op = H.fine
    u = torch.from_numpy(inputs.config1_u(m, amplitude=0.05)).cuda()
    w = torch.from_numpy(inputs.random_vector(m.n_nodes, 5)).cuda()
    w32 = w.float()
    op.residual(u, store_state=True)
    op.state_cast_f32()
    out = {"workload": "Q3 on a 23^3 jittered box, 1,029,000 DoF, per-element Lame parameters log-uniform "
                       "on [0.5, 2]; one VJP = u_bar, mu_bar, lambda_bar", "dof": 3 * m.n_nodes}
    for prec, ww in (("f64", w), ("f32", w32)):
        for mode in ("stored", "recompute"):
            t = time_median(lambda: op.residual_vjp(u, ww, mode=mode, precision=prec), steps, warmup, stream)
            out[f"{prec}_{mode}"] = {"ms": t, "GDoF/s": 3 * m.n_nodes / (t * 1e-3) / 1e9}
    return out


def _host_description():
    import platform
    info = {"cpu_count": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "processor": platform.processor() or platform.machine()}
    try:
        from threadpoolctl import threadpool_info
        info["blas"] = [{"api": t.get("internal_api"), "threads": t.get("num_threads")} for t in threadpool_info()]
    except Exception:  # pragma: no cover
        info["blas"] = None
    return info


def _submesh(mesh, els, *fields):
    """The elements ``els`` of ``mesh`` with their own node numbering and the given nodal
    fields restricted to those nodes (what one CPU worker needs)."""
    en = mesh.elem_nodes[els]
    nodes, local = np.unique(en, return_inverse=True)
    return (mesh.coords[nodes], local.reshape(en.shape)) + tuple(f[nodes] for f in fields)


def _oracle_apply_worker(args):
    """One process of the oracle CPU runs: ``reps`` oracle applies (FP64 numpy, one BLAS
    thread) on a sub-mesh; returns the seconds it took."""
    kind, coords, elem_nodes, P, u, du, mu, lam, reps = args
    from threadpoolctl import threadpool_limits
    from oracle import fem
    with threadpool_limits(limits=1):
        d = fem.make_disc(coords, elem_nodes, P)
        if kind == "elmat":
            Ke = fem.element_matrices(d, u, mu, lam)
            dof = (3 * elem_nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(len(elem_nodes), -1)
            t0 = time.perf_counter()
            for _ in range(reps):
                ye = np.einsum("eij,ej->ei", Ke, du.reshape(-1)[dof])
                y = np.zeros(du.size)
                np.add.at(y, dof.reshape(-1), ye.reshape(-1))
            return time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(reps):
            if kind == "jacobian":
                fem.jacobian_apply(d, u, du, mu, lam, chunk=512)
            else:
                fem.residual(d, u, mu, lam, chunk=512)
        return time.perf_counter() - t0


def _oracle_rate(mesh, u, du, kind, seconds, workers=1, reps=2, max_elements=None):
    """Oracle apply rate (GDoF/s of the full mesh) from a sample of elements sized to take
    about ``seconds`` per worker (at most ``max_elements`` per worker, the apply then
    repeated to fill the time); ``workers`` > 1 runs that many spawned processes, each on
    its own slice of the sample (wall time = the slowest worker)."""
    import multiprocessing as mp
    mu, lam = 0.38461538461538464, 0.5769230769230769  # E = 1, nu = 0.3
    probe = min(mesh.n_elem, 16)
    c, en, us, dus = _submesh(mesh, np.arange(probe), u, du)
    per_el = _oracle_apply_worker((kind, c, en, mesh.P, us, dus, mu, lam, 3)) / (3 * probe)
    k = int(min(mesh.n_elem // workers, max(16, seconds / reps / per_el)))
    if max_elements is not None and k > max_elements:
        k = max_elements
        reps = max(reps, int(seconds / (per_el * k)))
    slices = [np.arange(w * k, (w + 1) * k) for w in range(workers)]
    jobs = [(kind,) + _submesh(mesh, sl, u, du)[:2] + (mesh.P,) + _submesh(mesh, sl, u, du)[2:] +
            (mu, lam, reps) for sl in slices]
    if workers == 1:
        dt = _oracle_apply_worker(jobs[0])
    else:
        with mp.get_context("spawn").Pool(workers) as pool:
            dt = max(pool.map(_oracle_apply_worker, jobs))
    frac = workers * k / mesh.n_elem
    return {"GDoF/s": 3 * mesh.n_nodes * frac / (dt / reps) / 1e9, "elements": workers * k, "workers": workers,
            "seconds": dt}


def _oracle_tiny_solve():
    """The first load step of the configuration's p-MG Newton solve on a tiny replica
    (Q4 -> Q2 -> Q1 on 2^3 elements, x = 0 clamped, x = 1 face displaced by 0.1 = one of
    five steps of 0.5, FCG with the oracle's V-cycle to 1e-3, Newton to 1e-8), timed on
    one thread."""
    from threadpoolctl import threadpool_limits
    from oracle import fem, mg as omg
    from paper_2204_01722_amd import inputs
    mu, lam = inputs.lame(1.0, 0.3)
    faces = {"x0": (1, 1, 1), "x1": (1, 1, 1)}
    m = inputs.box_mesh(2, 4, jitter=0.05, seed=2204)
    d = fem.make_disc(m.coords, m.elem_nodes, m.P)
    orders = [4, 2, 1]
    topos = [m.elem_nodes] + [inputs.box_topology(m.n, p) for p in orders[1:]]
    nn = [int(np.prod([p * n + 1 for n in m.n])) for p in orders]
    masks = [inputs.face_mask(m, faces)] + [inputs.face_mask(None, faces, p=p, n=m.n) for p in orders[1:]]
    Ps = [omg.prolongation(topos[l - 1], orders[l - 1] + 1, nn[l - 1], topos[l], orders[l] + 1, nn[l])
          for l in range(1, 3)]
    seeds = [inputs.rough_seed(nn[l], masks[l], 7 + l) for l in range(2)]
    lift = inputs.affine_lifting(m, (0.1, 0.0, 0.0))
    its = []

    def solve(K, rhs):
        V = omg.VCycle(K, Ps, masks, seeds, degree=3)
        x, k, _ = omg.fcg(K, lambda v: V(v), rhs, rtol=1e-3)[:3]
        its.append(k)
        return x

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        u, hist = omg.newton_load_steps(d, mu, lam, masks[0], lift, 1, solve, rtol=1e-8)
        dt = time.perf_counter() - t0
    return {"seconds": dt, "dof": 3 * m.n_nodes, "newton_its": int(sum(hist)), "fcg_its": int(sum(its)),
            "workload": "first load step of the configuration's solve on a Q4->Q2->Q1 2^3 jittered box: x=0 "
                        "clamped, x=1 face displaced by 0.1, FCG + oracle V-cycle to 1e-3, Newton to 1e-8"}


def cpu_baseline(wl, seconds=6.0):
    """The FP64 oracle (dense element tables, numpy) timed on this host: the Jacobian
    apply on bounded samples of the Q4 34^3 and Q2 43^3 workloads on one thread and on
    all allowed cores (at most 16 processes, one BLAS thread each), the residual, the Q2
    apply from assembled element matrices, and the p-MG Newton solve on a tiny replica."""
    from paper_2204_01722_amd import inputs
    host = _host_description()
    cores = max(1, min(16, host["affinity"]))
    legs = {}
    print("[bench] CPU oracle: Q4 Jacobian", file=sys.stderr, flush=True)
    legs["q4_jacobian_1thread"] = _oracle_rate(wl.mesh, wl.u_np, wl.du_np, "jacobian", seconds)
    legs["q4_jacobian_all_cores"] = _oracle_rate(wl.mesh, wl.u_np, wl.du_np, "jacobian", seconds, workers=cores)
    legs["q4_residual_1thread"] = _oracle_rate(wl.mesh, wl.u_np, wl.du_np, "residual", seconds / 2)
    print("[bench] CPU oracle: Q2", file=sys.stderr, flush=True)
    m2 = inputs.box_mesh(43, 2, jitter=0.05, seed=2204)
    u2, du2 = inputs.stretch_field(m2, 1.3), inputs.random_vector(m2.n_nodes, 3)
    legs["q2_jacobian_1thread"] = _oracle_rate(m2, u2, du2, "jacobian", seconds / 2)
    legs["q2_jacobian_all_cores"] = _oracle_rate(m2, u2, du2, "jacobian", seconds / 2, workers=cores)
    legs["q2_element_matrix_apply_1thread"] = _oracle_rate(m2, u2, du2, "elmat", seconds / 2, reps=4,
                                                           max_elements=2000)
    legs["q4_element_matrix_apply"] = "skipped: 375 x 375 element matrices of 39,304 elements need 44 GB"
    print("[bench] CPU oracle: tiny p-MG solve", file=sys.stderr, flush=True)
    legs["pmg_newton_tiny_replica_1thread"] = _oracle_tiny_solve()
    main = legs["q4_jacobian_all_cores"]
    return {"value": main["GDoF/s"], "unit": "GDoF/s", "cores": main["workers"], "kind": "oracle",
            "sample": f"{main['elements']} of {wl.mesh.n_elem} elements of the Q{wl.p} {wl.n}^3 mesh, FP64 "
                      f"Jacobian apply (dense element tables, numpy), {main['workers']} processes with one "
                      f"BLAS thread each; rate = DoF x sampled fraction / wall time",
            "host": host, "legs": legs}


def pmg_solve(n=16, p=4, steps=5, total_disp=0.5, inclusions=False, monitor=False, lbfgs=True,
              rediscretize=True, exact=True, prime_s=0.3, natural=True):
    """FP64 vs mixed-precision p-MG Newton solve (Q4 -> Q2 -> Q1, Chebyshev degree 3,
    order-1 coarse level solved by Jacobi-PCG to 1e-3, Newton to 1e-8).  Default: x = 0
    clamped, x = 1 face displaced by `total_disp` along x in `steps` load steps.  With
    `inclusions`: stiff spherical inclusions (E ratio 100, 20 % of the elements, radii
    2-4 elements) in a soft matrix, compressed by `total_disp` (negative) along x between
    frictionless (roller) faces: u_x = 0 on x = 0, u_x = total_disp on x = 1, u_y = 0 on
    y = 0, u_z = 0 on z = 0.

    Forms: `fp64` / `mixed` solve every Newton step's linear system by FCG to 1e-8 (the
    configuration as stated); `inexact_fp64` / `inexact_mixed` stop FCG at 1e-3 (the
    paper's inexact Newton) in the residual 2-norm, `natural_fp64` / `natural_mixed` at
    1e-3 in the natural norm; rediscretised coarse levels and L-BFGS are further variants
    on the inexact form."""
    import torch
    from paper_2204_01722_amd import inputs
    from paper_2204_01722_amd.binding import PMG
    from paper_2204_01722_amd.problem import Hierarchy
    faces = {"x0": (1, 1, 1), "x1": (1, 1, 1)}
    m = inputs.box_mesh(n, p, jitter=0.05, seed=2204)
    mu_e = lam_e = None
    desc = f"x=0 clamped, x=1 face displaced by {total_disp} along x in {steps} load steps"
    if inclusions:
        faces = {"x0": (1, 0, 0), "x1": (1, 0, 0), "y0": (0, 1, 0), "z0": (0, 0, 1)}
        desc = (f"roller faces x=0, y=0, z=0, x=1 face displaced by {total_disp} along x in {steps} "
                f"load steps")
        mu_e, lam_e, inside = inputs.inclusion_materials(m, fraction=0.2, r_elems=(2.0, 4.0), E_in=100.0,
                                                          E_out=1.0, nu=0.3, seed=6)
        desc += f"; stiff inclusions (E 100:1) in {inside.mean():.1%} of the elements"
    lift = torch.from_numpy(inputs.affine_lifting(m, (total_disp, 0.0, 0.0))).cuda()
    out = {"workload": f"Q4->Q2->Q1 on {n}^3 jittered box, {3 * m.n_nodes} DoF, {desc}; Newton rtol 1e-8, "
                       f"Chebyshev degree 3, coarse Jacobi-PCG rtol 1e-3", "dof": 3 * m.n_nodes}

    def run(prec, lin_rtol, redisc=False, quasi_newton=False, lin_norm="2"):
        H = Hierarchy(m, [p, 2, 1], faces=faces, mu_e=mu_e, lam_e=lam_e, rediscretize=redisc)
        mg = PMG(H.ops, precision=prec, cheb_degree=3, coarse_rtol=1e-3)
        u = torch.zeros(m.n_nodes, 3, dtype=torch.float64, device="cuda")
        seeds = H.seeds(7)
        prime(lambda: H.fine.residual(u, store_state=False), prime_s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if quasi_newton:
            u, st = mg.lbfgs(u, lift, steps, seeds, rtol=1e-8, max_its=500, monitor=monitor)
        else:
            u, st = mg.newton(u, lift, steps, seeds, rtol=1e-8, lin_rtol=lin_rtol, lin_maxit=1000,
                              monitor=monitor, lin_norm=lin_norm)
        torch.cuda.synchronize()
        rec = {"seconds": time.perf_counter() - t0, "fcg_rtol": None if quasi_newton else lin_rtol,
               "fcg_norm": None if quasi_newton else lin_norm, **st,
               **mg.stats()}
        del mg, H
        return rec, u

    def diff(a, b):
        return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))

    us = {}
    # the inexact forms stop FCG at 1e-3 in the residual 2-norm and, as the paper states
    # it, in the natural norm of the preconditioned system
    forms = [("inexact_fp64", "f64", 1e-3, "2"), ("inexact_mixed", "f32", 1e-3, "2")]
    if natural:
        forms += [("natural_fp64", "f64", 1e-3, "natural"), ("natural_mixed", "f32", 1e-3, "natural")]
    if exact:
        forms = [("fp64", "f64", 1e-8, "2"), ("mixed", "f32", 1e-8, "2")] + forms
    for key, prec, rt, norm in forms:
        out[key], us[key] = run(prec, rt, lin_norm=norm)
        print(f"[bench] p-MG {key}: {out[key]['seconds']:.3f} s, {out[key]['newton_its']} Newton, "
              f"{out[key]['krylov_its']} FCG", file=sys.stderr, flush=True)
    base = "fp64" if exact else "inexact_fp64"
    if exact:
        out["rel_diff_mixed_vs_fp64"] = diff(us["mixed"], us["fp64"])
        out["speedup_mixed"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
        out["fcg_its_change_mixed_vs_fp64"] = out["mixed"]["krylov_its"] - out["fp64"]["krylov_its"]
    out["inexact_rel_diff_mixed_vs_fp64"] = diff(us["inexact_mixed"], us["inexact_fp64"])
    out["inexact_speedup_mixed"] = out["inexact_fp64"]["seconds"] / out["inexact_mixed"]["seconds"]
    for key in ("natural_fp64", "natural_mixed") if natural else ():
        out[key]["rel_diff_vs_inexact_fp64"] = diff(us[key], us["inexact_fp64"])
        out[key]["fcg_its_change_vs_2norm"] = (out[key]["krylov_its"]
                                               - out[key.replace("natural", "inexact")]["krylov_its"])
    if exact:
        out["inexact_rel_diff_vs_exact_fp64"] = diff(us["inexact_fp64"], us["fp64"])
    if rediscretize:
        # the inexact Newton solve with rediscretised coarse levels (own order and Gauss
        # points, linearised at the injected field) instead of Galerkin levels
        for key, prec in (("rediscretised_fp64", "f64"), ("rediscretised_mixed", "f32")):
            out[key], u = run(prec, 1e-3, redisc=True)
            out[key]["rel_diff_vs_" + base] = diff(u, us[base])
    if lbfgs:
        # the same load path with L-BFGS (V-cycle as initial inverse Hessian, built once
        # per load step)
        for key, prec in (("lbfgs_fp64", "f64"), ("lbfgs_mixed", "f32")):
            out[key], u = run(prec, None, quasi_newton=True)
            out[key]["rel_diff_vs_" + base] = diff(u, us[base])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--prime", type=float, default=0.5,
                    help="seconds of untimed applies before the warm-up steps of the headline (steady GPU clock)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--only-headline", action="store_true")
    ap.add_argument("--pmg-n", type=int, default=40, help="elements per direction of the p-MG solve")
    ap.add_argument("--pmg-only", action="store_true", help="run only the FP64-vs-mixed p-MG solve")
    ap.add_argument("--pmg-monitor", action="store_true", help="print one line per Newton iteration")
    ap.add_argument("--pmg-inclusions", action="store_true",
                    help="p-MG solve of the multiscale block: stiff inclusions, compression between roller faces "
                         "in 10 load steps")
    ap.add_argument("--pmg-inexact-only", action="store_true",
                    help="only the inexact-Newton forms (FCG to 1e-3), not the FCG-to-1e-8 ones")
    ap.add_argument("--pmg-no-natural", action="store_true",
                    help="skip the forms whose FCG stops in the natural norm")
    ap.add_argument("--pmg-newton-only", action="store_true",
                    help="only the Galerkin Newton solves (FP64 and mixed): no rediscretised or L-BFGS legs")
    ap.add_argument("--profile-applies", action="store_true",
                    help="only run the stored Jacobian applies (Q4 34^3 and Q2 43^3, FP64 and FP32) --steps "
                         "times each, for a profiler")
    ap.add_argument("--coarse-iteration", type=str, default=None, metavar="N1,N2,...",
                    help="only time one coarse PCG iteration on the N^3 boxes (Q1 level of (N+1)^3 nodes)")
    ap.add_argument("--jsonl", type=str, default=None, metavar="PATH",
                    help="also append the record, with the run's arguments and time, to a JSON-lines log")
    ap.add_argument("--pmg-strain", type=float, default=0.10,
                    help="compressive strain of the multiscale block (0.10: solved on every mesh up to 80^3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.coarse_iteration:
        sizes = [int(v) for v in args.coarse_iteration.split(",")]
        print(json.dumps({"coarse_pcg_iteration": coarse_iteration(sizes, stream)}))
        return
    if args.profile_applies:
        for n, p in ((34, 4), (43, 2)):
            wl = Workload(n, p)
            for prec in ("f64", "f32"):
                ms = time_op(wl.apply(prec, "stored"), args.steps, args.warmup, stream, prime_s=args.prime)
                print(f"[profile] Q{p} {n}^3 {prec} stored: {args.steps} applies, {ms * 1000:.1f} us each",
                      file=sys.stderr, flush=True)
            del wl
            torch.cuda.empty_cache()
        # a plain copy of known size (2 GiB read, 2 GiB written): the reference that
        # scales the HBM byte counters
        print(f"[profile] copy: {copy_bandwidth():.1f} GB/s", file=sys.stderr, flush=True)
        return
    if args.pmg_only:
        if args.pmg_inclusions:
            res = pmg_solve(n=args.pmg_n, steps=10, total_disp=-args.pmg_strain, inclusions=True,
                            monitor=args.pmg_monitor, lbfgs=not args.pmg_newton_only,
                            rediscretize=not args.pmg_newton_only, exact=not args.pmg_inexact_only,
                            prime_s=min(0.3, args.prime), natural=not args.pmg_no_natural)
        else:
            res = pmg_solve(n=args.pmg_n, monitor=args.pmg_monitor, lbfgs=not args.pmg_newton_only,
                            rediscretize=not args.pmg_newton_only, exact=not args.pmg_inexact_only,
                            prime_s=min(0.3, args.prime), natural=not args.pmg_no_natural)
        print(json.dumps({"pmg_solve": res}))
        return

    print("[bench] building Q4 34^3 workload", file=sys.stderr, flush=True)
    q4 = Workload(34, 4)
    ms = time_op(q4.apply("f64", "stored"), args.steps, args.warmup, stream, prime_s=args.prime)
    value = q4.dof / (ms * 1e-3) / 1e9
    nbytes = algorithmic_bytes(q4.E, q4.P, q4.Q, q4.N, 8)
    achieved = nbytes / (ms * 1e-3) / 1e9
    print(f"[bench] Q4 f64 stored: {ms:.4f} ms, {value:.2f} GDoF/s", file=sys.stderr, flush=True)

    # the same loop repeated: the spread of the headline on this machine
    variants = {"headline_repeats_ms": [time_op(q4.apply("f64", "stored"), args.steps, 1, stream) for _ in range(4)]}
    if not args.only_headline:
        for prec, mode in (("f32", "stored"), ("f64", "recompute"), ("f32", "recompute")):
            t = time_median(q4.apply(prec, mode), args.steps, args.warmup, stream)
            variants[f"q4_{prec}_{mode}"] = {"ms": t, "GDoF/s": q4.dof / (t * 1e-3) / 1e9}
        t = time_median(q4.residual(), max(5, args.steps // 5), 2, stream)
        variants["q4_residual_f64"] = {"ms": t, "GDoF/s": q4.dof / (t * 1e-3) / 1e9}
        variants["q4_f32_stored"]["hbm_frac"] = (algorithmic_bytes(q4.E, q4.P, q4.Q, q4.N, 4) /
                                                 (variants["q4_f32_stored"]["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS)
        # the initial-configuration (S(E)) forms of the same operator: 19 and 26 scalars
        q4.op.state_initial(q4.u)
        for mode, ns in (("initial_native", 19), ("initial_tuned", 26), ("current_20", 20)):
            t = time_median(q4.apply("f64", mode), args.steps, args.warmup, stream)
            variants[f"q4_f64_{mode}"] = {
                "ms": t, "GDoF/s": q4.dof / (t * 1e-3) / 1e9, "scalars_per_point": ns,
                "hbm_frac": algorithmic_bytes(q4.E, q4.P, q4.Q, q4.N, 8, nstate=ns) / (t * 1e-3) / 1e9 /
                HBM_PEAK_GBPS}
        print("[bench] building Q2 43^3 workload", file=sys.stderr, flush=True)
        q2 = Workload(43, 2)
        for prec, mode in (("f64", "stored"), ("f32", "stored"), ("f64", "recompute")):
            t = time_median(q2.apply(prec, mode), args.steps, args.warmup, stream)
            v = {"ms": t, "GDoF/s": q2.dof / (t * 1e-3) / 1e9}
            if mode == "stored":
                v["hbm_frac"] = (algorithmic_bytes(q2.E, q2.P, q2.Q, q2.N, 8 if prec == "f64" else 4) /
                                 (t * 1e-3) / 1e9 / HBM_PEAK_GBPS)
            variants[f"q2_{prec}_{mode}"] = v
        del q2
        # working sets well beyond the 256 MB Infinity Cache
        for n, p in ((68, 4), (86, 2)):
            print(f"[bench] building Q{p} {n}^3 workload (cache-busting)", file=sys.stderr, flush=True)
            wl = Workload(n, p)
            for prec in ("f64", "f32"):
                t = time_median(wl.apply(prec, "stored"), max(10, args.steps // 2), 3, stream)
                variants[f"q{p}_{n}cubed_{prec}_stored"] = {
                    "ms": t, "dof": wl.dof, "GDoF/s": wl.dof / (t * 1e-3) / 1e9,
                    "hbm_frac": algorithmic_bytes(wl.E, wl.P, wl.Q, wl.N, 8 if prec == "f64" else 4) /
                    (t * 1e-3) / 1e9 / HBM_PEAK_GBPS}
            del wl
            torch.cuda.empty_cache()
        print("[bench] adjoint (Q3 23^3)", file=sys.stderr, flush=True)
        variants["adjoint_q3_23cubed"] = adjoint_bench(max(5, args.steps // 5), 2, stream)
        print(f"[bench] variants done", file=sys.stderr, flush=True)
    # a plain device copy of known size: achievable bandwidth, and the reference kernel
    # that scales the HBM byte counters of a profiled run
    variants["hbm_copy_GBps"] = copy_bandwidth()

    solve = None
    if not args.no_solve and not args.only_headline:
        print("[bench] p-MG solve FP64 vs mixed", file=sys.stderr, flush=True)
        solve = pmg_solve(n=args.pmg_n, prime_s=min(0.3, args.prime))

    cpu = None
    if not args.no_cpu:
        print("[bench] CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(q4)

    out = {
        "metric": "GDoF/s Neo-Hookean Jacobian apply (Q2/Q4, fp64 vs fp32) + p-MG solve time",
        "value": value,
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Q4 (P=5 GLL nodes, 5^3 Gauss points) on a 34^3 jittered unit box, "
                               "7,714,059 DoF, stored 16-scalar FP64 Jacobian apply, max stretch 1.3, "
                               "E=1, nu=0.3", "global_batch": 1, "seq_len": 0, "parallelism": "none"},
        "roofline": {"bound": "hbm", "kernel": "k_jacobian_lines<double,5,5> + k_assemble<double> (one apply)",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": measured_traffic(),
                     "algorithmic_bytes_per_launch": nbytes},
        "variants": variants,
        "pmg_solve": solve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    if args.jsonl:
        append_jsonl(args.jsonl, out, vars(args))


def append_jsonl(path, record, run_args):
    """Appends ``record`` with the run's arguments, wall-clock time and host CPU count as
    one line of a JSON-lines log (one record per run)."""
    import datetime
    line = dict(record, run={"args": run_args, "host_cpus": os.cpu_count(),
                             "time": datetime.datetime.now(datetime.timezone.utc).isoformat()})
    with open(path, "a") as f:
        f.write(json.dumps(line) + "\n")


if __name__ == "__main__":
    main()
