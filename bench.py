#!/usr/bin/env python3
"""Benchmark of the matrix-free hot path on one MI355X.

Step = one matrix-free application y = A x of the variable-coefficient Q4 Laplacian on the
curved 64^3-cell mesh (257^3 = 16,974,593 DoFs; deformation amplitude 0.1, coefficient
a = 1 + 0.5 sin sin sin), FP64, with the input resident in HBM.  Prints one JSON line:
DoFs/s of the step, the roofline of the dominant kernel (the cell loop, timed with HIP events
on its stream), an FP32 figure of the same operator, the same operator assembled as a sparse
matrix and applied by the library's CSR product, the DG-SIPG Q4 operator of the paper's
multigrid experiment and its V-cycle and solve, time to 1e-10 of the Q3 128^3 multigrid and CG
solvers, the 2,000-request serving stream (solves/s, p50/p99 latency), and the CPU oracle on a
bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-solves] [--serve N] [--no-csr]
                    [--no-dg-mg] [--csr-sweep] [--vcycle] [--copy-probe]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DoFs/s matrix-free vmult FP64 vs FP32; solves/s + p99 latency at 1e-10"
HBM_PEAK_GBS = 8000.0
# sources that define the cell-loop kernel; HBM counter figures are used only while they match
KERNEL_SOURCES = ["paper_1910_13247_amd/csrc/kernels_cell.hip", "paper_1910_13247_amd/csrc/kernels_common.hpp",
                  "paper_1910_13247_amd/csrc/mfq_internal.hpp", "paper_1910_13247_amd/csrc/tables_ct.hpp"]
TRAFFIC_PROFILE = "profiles/vmult_q4_64_fp64_hbm_counters.md"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per cell-loop launch from the committed counter summary (FETCH_SIZE + WRITE_SIZE,
    each scaled by a copy kernel's reading), or None when the kernel changed since it was taken."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel source sha256/16") != kernel_source_hash():
        return None
    try:
        return float(fields["hbm bytes per launch"])
    except (KeyError, ValueError):
        return None


def algorithmic_bytes(p, n, real_bytes):
    """src read + dst write once, 6 G values per quadrature point, one int32 index per cell DoF."""
    N = (p * n + 1) ** 3
    C = n ** 3
    Q = C * (p + 1) ** 3
    return 2 * real_bytes * N + 6 * real_bytes * Q + 4 * (p + 1) ** 3 * C


def algorithmic_flops(p, n):
    C = n ** 3
    return C * (24 * (p + 1) ** 4 + 15 * (p + 1) ** 3)


# ---------------------------------------------------------------- algorithmic bytes of solves
# Byte counts of the solvers' algorithmic traffic, from the operators' algorithmic bytes (above)
# and the vector streams each step reads or writes once (b bytes per value):
#   FP64 CG iteration: p.Ap (2 streams), x += a p, r -= a Ap (6), r.z (2), p = z + beta p (3);
#     unpreconditioned: z = r, no r.z pass (11);
#   V-cycle level l >= 1 (Chebyshev degree k, V(1,1)): pre-smoothing from zero = first step (read
#     b, dinv; write r, d, x: 5) + (k-1) x (operator + step: read Ad, dinv, x, r, d; write r, d, x:
#     8); residual = operator + (read b, t; write r: 3); restriction (read the fine residual, write
#     the coarse right-hand side: N_l + N_{l-1}); prolongation (read coarse, write fine: N_{l-1} +
#     N_l); x += t (3); post-smoothing = operator + first step (read b, t, dinv, x; write r, d, x:
#     7) + (k-1) x (operator + 8): 2k operator applications and 5 + 8(k-1) + 3 + 3 + 7 + 8(k-1)
#     vector streams, plus the two transfers;
#   coarsest level: dense inverse (nf^2 FP64 values read, b and x) or Chebyshev of the coarse
#     degree from zero (5 + (deg-1) x (operator + 8));
#   FP32 V-cycle under FP64 CG: casts of r in and z out (8 + 4 bytes per DoF each way);
#   each correction pass: the FP64 residual check (operator + read b, t, write r: 3 x 8 N).
def hierarchy(p, n, limit=4096):
    """(p, n) per multigrid level, coarsest first: halve n while even and > limit free DoFs, then p ->
    ceil(p/2) (the library's rule)."""
    free = lambda p_, n_: max(p_ * n_ - 1, 0) ** 3
    lv = [(p, n)]
    while n % 2 == 0 and free(p, n) > limit:
        n //= 2
        lv.append((p, n))
    while p > 1 and free(p, n) > limit:
        p = (p + 1) // 2
        lv.append((p, n))
    return lv[::-1]


def geo_saving(p, n, b, cart=False, coef=False):
    """G bytes an operator application does not read: all 6 values per point on undeformed cells
    with coefficient 1 (formed in registers), 5 of them with a variable coefficient (only the
    diagonal a(x_q) h w_q is read)."""
    return (6 if cart else 5 if coef else 0) * b * n ** 3 * (p + 1) ** 3


def vcycle_bytes(levels, b, smoother_degree=3, coarse_mode=0, coarse_degree=16, cart=False, coef=False):
    """Algorithmic bytes of one V-cycle over `levels` (coarsest first) in value size b."""
    N = [(p_ * n_ + 1) ** 3 for p_, n_ in levels]
    k = smoother_degree
    op = lambda l: algorithmic_bytes(levels[l][0], levels[l][1], b) - geo_saving(levels[l][0], levels[l][1], b,
                                                                                  cart, coef)
    tot = 0
    for l in range(1, len(levels)):
        streams = 5 + 8 * (k - 1) + 3 + 3 + 7 + 8 * (k - 1)
        tot += 2 * k * op(l) + streams * b * N[l] + 2 * b * (N[l] + N[l - 1])
    p0, n0 = levels[0]
    if coarse_mode == 1:
        tot += (coarse_degree - 1) * op(0) + (5 + 8 * (coarse_degree - 1)) * b * N[0]
    else:
        nf = max(p0 * n0 - 1, 0) ** 3
        tot += 8 * nf * nf + 2 * b * N[0]
    return tot


def solve_bytes(kind, p, n, iterations, passes, smoother_degree=3, coarse_mode=0, coarse_degree=16, cart=False,
                coef=False):
    """Algorithmic bytes of a whole solve (iterations summed over passes, `passes` residual checks)."""
    N = (p * n + 1) ** 3
    op64 = algorithmic_bytes(p, n, 8) - geo_saving(p, n, 8, cart, coef)
    check = op64 + 3 * 8 * N
    if kind == "cg_fp64":
        return iterations * (op64 + 11 * 8 * N) + passes * check
    lv = hierarchy(p, n)
    if kind == "gmg_fp64":
        vc = vcycle_bytes(lv, 8, smoother_degree, coarse_mode, coarse_degree, cart, coef)
        return iterations * (op64 + 13 * 8 * N + vc) + passes * check
    vc = vcycle_bytes(lv, 4, smoother_degree, coarse_mode, coarse_degree, cart, coef) + 24 * N
    if kind == "gmg_mixed":
        return iterations * (op64 + 13 * 8 * N + vc) + passes * check
    # gmg_mixed_ir: inner CG on the FP32 operator (casts p in and Ap out: 24 B per DoF) with FP64
    # vectors; each pass also adds its correction into x (3 x 8 N)
    op32 = algorithmic_bytes(p, n, 4) - geo_saving(p, n, 4, cart, coef)
    return iterations * (op32 + 24 * N + 13 * 8 * N + vc) + passes * (check + 3 * 8 * N)


def setup_bytes(p, n, smoother_degree=3, coarse_mode=1, lanczos=12, coef=False):
    """Algorithmic bytes of a solver's set-up on the device: index maps and geometry written for the
    FP64 operator and every FP32 level (with a variable coefficient on undeformed cells also the
    diagonal of G, one value per point), each level's diagonal (operator data read, diagonal
    written), and the Lanczos steps (operator + about 10 vector streams each)."""
    lv = hierarchy(p, n)
    tot = 0
    for l, (pl, nl) in enumerate(lv):
        Nl = (pl * nl + 1) ** 3
        Ql = nl ** 3 * (pl + 1) ** 3
        geo4 = algorithmic_bytes(pl, nl, 4) - 8 * Nl           # idx + G in FP32
        tot += geo4 + geo4 + 4 * Nl                             # written, read back by the diagonal
        if coef:
            tot += 6 * 4 * Ql + 4 * Ql                          # G read again, its diagonal written
        if l > 0 or coarse_mode == 1:
            tot += lanczos * (algorithmic_bytes(pl, nl, 4) - geo_saving(pl, nl, 4, coef=coef) + 10 * 4 * Nl)
    N = (p * n + 1) ** 3
    tot += algorithmic_bytes(p, n, 8) - 16 * N                 # FP64 operator's idx + G written
    if coef:
        tot += 7 * 8 * n ** 3 * (p + 1) ** 3                    # its G read again, the diagonal written
    return tot


def copy_bandwidth(gib=1, reps=5):
    """HBM bandwidth of a plain device copy (torch, 1 GiB): bytes read + written per second."""
    import torch
    a = torch.empty(gib << 27, dtype=torch.float64, device="cuda").uniform_()
    b = torch.empty_like(a)
    s = time_events(lambda: b.copy_(a), reps, 2)
    nbytes = 2 * a.numel() * 8
    del a, b
    torch.cuda.synchronize()
    return {"bytes_per_copy": nbytes, "ms": s * 1e3, "GB_per_s": nbytes / s / 1e9,
            "frac_of_peak": nbytes / s / 1e9 / HBM_PEAK_GBS}


def time_vmult(op, x, steps, warmup):
    """(wall s per step, event-timed s of the cell-loop launches of one step)."""
    import torch
    y = op.new_vector()
    for _ in range(warmup):
        op.vmult(x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        op.vmult(x, y)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    # dominant kernel alone: the step's cell-loop launches (an application is nothing else: the
    # first colour stores, so no clearing pass) back to back between two events on the stream they
    # are launched on (torch's current stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        op.vmult(x, y)
    e1.record()
    torch.cuda.synchronize()
    kern = e0.elapsed_time(e1) / 1e3 / steps
    return wall, kern, y


def cpu_baseline(p, n, amp, alpha, x_np, budget_s=12.0, check_rows=None, y64_rows=None, y32_rows=None):
    """Oracle element-by-element application on a bounded sample of cells, scaled to DoFs/s; and
    the FP64 and FP32 benchmark results on `check_rows` against the oracle's rows (the FP32 path
    against the oracle applied to the input rounded to FP32, the input that path sees)."""
    import numpy as np
    from oracle.ebe import ebe_rows, ebe_vmult
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    cores = len(os.sched_getaffinity(0))
    C = n ** 3
    N = (p * n + 1) ** 3
    chunk = 256
    done, elapsed = 0, 0.0
    ctx = threadpool_limits(limits=cores) if threadpool_limits else None
    try:
        while elapsed < budget_s and done < C:
            cells = np.arange(done, min(C, done + chunk))
            t0 = time.perf_counter()
            ebe_vmult(p, n, amp, alpha, x_np, 1, cells=cells, chunk=chunk)
            elapsed += time.perf_counter() - t0
            done += len(cells)
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    dofs_per_s = (done / C) * N / elapsed
    out = {"value": dofs_per_s, "unit": "DoFs/s", "cores": cores, "kind": "oracle",
           "sample": f"{done} of {C} cells (element-by-element, dense cell matrices), {elapsed:.1f} s, "
                     f"scaled by cells/total to a full application"}
    if check_rows is not None:
        yo = ebe_rows(p, n, amp, alpha, x_np, 1, check_rows)
        x32 = x_np.astype(np.float32).astype(np.float64)
        yo32 = ebe_rows(p, n, amp, alpha, x32, 1, check_rows)
        out["oracle_check"] = {
            "rows": int(len(check_rows)),
            "fp64_normwise_rel_err": float(np.abs(y64_rows - yo).max() / np.abs(yo).max()),
            "fp32_normwise_rel_err": float(np.abs(y32_rows - yo32).max() / np.abs(yo32).max()),
            "bars": "FP64 1e-12 normwise; FP32 componentwise 2k u32 (sum of |terms|), k = 8(p+1)+16"}
    return out


def high_degree_comparison(steps, warmup):
    """Q8 on the curved 24^3 mesh (7,189,057 DoFs): the operator in FP64, FP32 (vector ALU) and
    FP32 with the 1D contractions on the matrix cores; per-application times of the cell loop and
    the FP32 forms' normwise error against the FP64 result."""
    import torch
    import paper_1910_13247_amd as mfq
    from synthetic import VARCOEF_Q8_24, uniform_vector
    pr = VARCOEF_Q8_24
    mesh = mfq.Mesh(pr.cells_1d, pr.amplitude)
    space = mfq.Space(mesh, pr.degree, mfq.MFQ_BC_DIRICHLET0)
    x64 = torch.from_numpy(uniform_vector(space.n_dofs, seed=0)).cuda()
    out = {"workload": pr.name, "dofs": space.n_dofs}
    ref = None
    for name, prec in [("fp64", mfq.MFQ_FP64), ("fp32", mfq.MFQ_FP32), ("fp32_mfma", mfq.MFQ_FP32_MFMA)]:
        op = mfq.Operator(space, pr.alpha, prec)
        x = x64 if prec == mfq.MFQ_FP64 else x64.float()
        wall, kern, y = time_vmult(op, x, steps, warmup)
        rb = algorithmic_bytes(pr.degree, pr.cells_1d, 8 if prec == mfq.MFQ_FP64 else 4)
        rec = {"ms": kern * 1e3, "GB_per_s": rb / kern / 1e9, "frac": rb / kern / 1e9 / HBM_PEAK_GBS,
               "DoFs_per_s": space.n_dofs / kern}
        if ref is None:
            ref = y.clone()
        else:
            rec["normwise_rel_err_vs_fp64"] = ((y.double() - ref).abs().max() / ref.abs().max()).item()
        out[name] = rec
        del op, y
        torch.cuda.synchronize()
    # the workload's solve: FP64 iterative refinement around the FP32 inner CG and V-cycle
    # (levels 3^3 .. 24^3), manufactured right-hand side, to 1e-10; timed on its second solve
    op = mfq.Operator(space, pr.alpha, mfq.MFQ_FP64)
    b = op.rhs_manufactured()
    sv = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED_IR)
    sv.solve(b, rtol=1e-10, max_iter=300, check=False)
    torch.cuda.synchronize()
    x, info, st = sv.solve(b, rtol=1e-10, max_iter=300, check=False)
    torch.cuda.synchronize()
    lb = solve_bytes("gmg_mixed_ir", pr.degree, pr.cells_1d, info.iterations, info.outer_iterations)
    out["solve_gmg_mixed_ir"] = {"seconds": info.seconds, "iterations": info.iterations,
                                 "outer": info.outer_iterations, "rel_residual": info.rel_residual,
                                 "status": st, "levels": info.n_levels, "algorithmic_bytes": lb,
                                 "roofline_lower_bound_s": lb / (HBM_PEAK_GBS * 1e9),
                                 "roofline_frac": lb / (HBM_PEAK_GBS * 1e9) / info.seconds}
    out["_solution"] = (b.cpu().numpy(), x.cpu().numpy())
    del sv, op, b, x
    torch.cuda.synchronize()
    return out


def time_events(fn, steps, warmup):
    """Average seconds per call of fn() between two events on torch's current stream."""
    import torch
    for _ in range(warmup):
        fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def csr_bytes(n_rows, nnz, value_bytes=8):
    """Algorithmic bytes of one CSR product: values (8 or 4 B) and columns (4 B) per entry, row
    pointers (8 B per row + 1), the source and destination vectors (one value per row each)."""
    return (value_bytes + 4) * nnz + 8 * (n_rows + 1) + 2 * value_bytes * n_rows


def assembled_comparison(op, x, y_mf, mf_s, steps, warmup, precision=None):
    """The same operator assembled as a CSR matrix on the device and applied by the library's
    sparse product: assembly time, product time, its HBM roofline fraction, and the matrix-free
    application's speed-up over it (matrix-free time = the cell loop of one application in the
    same precision; `y_mf` the FP64 matrix-free result)."""
    import torch
    import paper_1910_13247_amd as mfq
    precision = mfq.MFQ_FP64 if precision is None else precision
    vb = 8 if precision == mfq.MFQ_FP64 else 4
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A = mfq.SparseMatrix(op, precision)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    x = x.to(A.dtype)
    y = torch.empty_like(x)
    s = time_events(lambda: A.spmv(x, y), steps, warmup)
    rb = csr_bytes(A.n_rows, A.nnz, vb)
    out = {"nnz": A.nnz, "device_bytes": A.device_bytes, "assemble_s": t_asm, "ms": s * 1e3,
           "algorithmic_bytes": rb, "achieved_GBs": rb / s / 1e9, "frac": rb / s / 1e9 / HBM_PEAK_GBS,
           "kernel": "csr_spmv_rows_kernel" if A.nnz / A.n_rows >= 384 else "csr_spmv_kernel (row blocks)",
           "matrix_free_ms": mf_s * 1e3, "speedup_matrix_free": s / mf_s,
           "bytes_ratio": rb / algorithmic_bytes(op.space.degree, op.space.mesh.n, vb),
           "normwise_rel_diff_vs_matrix_free_fp64": ((y.double() - y_mf).abs().max() / y_mf.abs().max()).item()}
    del A, y
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


# degree sweep of the assembled-matrix comparison: (p, n) with about 16M DoFs (7.5M at p = 7, 8,
# whose matrices would otherwise exceed 100 GB)
CSR_SWEEP = [(1, 256), (2, 128), (3, 85), (4, 64), (5, 50), (6, 42), (7, 28), (8, 24)]


def csr_sweep(steps, warmup):
    import torch
    import paper_1910_13247_amd as mfq
    from synthetic import uniform_vector
    out = []
    for p, n in CSR_SWEEP:
        print(f"# csr sweep p={p} n={n}", file=sys.stderr, flush=True)
        op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.1), p, mfq.MFQ_BC_DIRICHLET0), 0.5, mfq.MFQ_FP64)
        x = torch.from_numpy(uniform_vector(op.n_dofs, seed=0)).cuda()
        y = op.new_vector()
        mf = time_events(lambda: op.vmult(x, y), steps, warmup)
        rec = assembled_comparison(op, x, y, mf, steps, warmup)
        rec.update({"degree": p, "cells_1d": n, "dofs": op.n_dofs,
                    "csr_bytes_per_dof": rec["algorithmic_bytes"] / op.n_dofs,
                    "matrix_free_bytes_per_dof": algorithmic_bytes(p, n, 8) / op.n_dofs,
                    "matrix_free_GBs": algorithmic_bytes(p, n, 8) / mf / 1e9})
        out.append(rec)
        del op, x, y
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


SOLVE_KINDS = ["gmg_mixed", "gmg_mixed_ir", "gmg_fp64", "cg_fp64"]


def solve_benchmarks(steps, kinds=None):
    """Time-to-1e-10 of the multigrid and CG solvers on the Q3 128^3 curved problem (multigrid
    forms timed on their second solve, after one solve that loads every kernel; plain CG on its
    first, which takes seconds)."""
    import torch
    import paper_1910_13247_amd as mfq
    out = {}
    mesh = mfq.Mesh(128, 0.1)
    space = mfq.Space(mesh, 3, mfq.MFQ_BC_DIRICHLET0)
    op = mfq.Operator(space, 0.5, mfq.MFQ_FP64)
    b = op.rhs_manufactured()
    table = {"gmg_mixed": mfq.MFQ_SOLVER_GMG_MIXED, "gmg_mixed_ir": mfq.MFQ_SOLVER_GMG_MIXED_IR,
             "gmg_fp64": mfq.MFQ_SOLVER_GMG_FP64, "cg_fp64": mfq.MFQ_SOLVER_CG}
    for name in kinds or SOLVE_KINDS:
        kind = table[name]
        s = mfq.Solver(op, kind)
        if kind != mfq.MFQ_SOLVER_CG:
            s.solve(b, rtol=1e-10, max_iter=20000, check=False)
            torch.cuda.synchronize()
        x, info, st = s.solve(b, rtol=1e-10, max_iter=20000, check=False)
        lb = solve_bytes(name, 3, 128, info.iterations, info.outer_iterations)
        out[name] = {"seconds": info.seconds, "iterations": info.iterations, "outer": info.outer_iterations,
                     "rel_residual": info.rel_residual, "status": st, "levels": info.n_levels,
                     "algorithmic_bytes": lb, "roofline_lower_bound_s": lb / (HBM_PEAK_GBS * 1e9),
                     "roofline_frac": lb / (HBM_PEAK_GBS * 1e9) / info.seconds}
        del s
        torch.cuda.synchronize()
    return out


def small_poisson(steps, warmup):
    """The small Poisson workload (Q2, affine 8^3 cells, 4,913 DoFs, Dirichlet, b = masked seeded
    uniform f): operator application time (cache and launch bound, reported in microseconds) and
    unpreconditioned FP64 CG to relative residual 1e-10."""
    import torch
    import paper_1910_13247_amd as mfq
    from synthetic import POISSON_Q2_8, uniform_vector
    pr = POISSON_Q2_8
    space = mfq.Space(mfq.Mesh(pr.cells_1d, pr.amplitude), pr.degree, mfq.MFQ_BC_DIRICHLET0)
    op = mfq.Operator(space, pr.alpha, mfq.MFQ_FP64)
    f = torch.from_numpy(uniform_vector(space.n_dofs, seed=0)).cuda()
    y = op.new_vector()
    us = time_events(lambda: op.vmult(f, y), steps, warmup) * 1e6
    b = space.apply_mask(f.clone())
    sv = mfq.Solver(op, mfq.MFQ_SOLVER_CG)
    sv.solve(b, rtol=1e-10, max_iter=10000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info, st = sv.solve(b, rtol=1e-10, max_iter=10000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"workload": pr.name, "dofs": space.n_dofs, "vmult_us": us, "cg_s": wall, "cg_iterations": info.iterations,
            "cg_rel_residual": info.rel_residual, "status": st}


def dg_benchmark(steps, warmup, degree=4, cells_1d=64):
    """The symmetric interior penalty DG Laplacian of the paper's multigrid experiment (degree 4,
    undeformed 64^3 mesh, 32,768,000 DoFs), one matrix-free application: one launch, each cell's
    volume term and six faces.  Algorithmic bytes: read the source and write the result once (16 B
    per DoF; the affine cells store no geometry); the neighbours' normal lines that miss in the
    caches are fetched again on top."""
    import torch
    import paper_1910_13247_amd as mfq
    from synthetic import uniform_vector
    op = mfq.DGOperator(mfq.Mesh(cells_1d, 0.0), degree)
    x = torch.from_numpy(uniform_vector(op.n_dofs, seed=0)).cuda()
    y = torch.empty_like(x)
    s = time_events(lambda: op.vmult(x, y), steps, warmup)
    rb = 16 * op.n_dofs
    out = {"workload": f"dg_sipg_q{degree}_{cells_1d}^3_affine", "dofs": op.n_dofs, "ms": s * 1e3,
           "DoFs_per_s": op.n_dofs / s, "algorithmic_bytes": rb, "achieved_GBs": rb / s / 1e9,
           "frac": rb / s / 1e9 / HBM_PEAK_GBS}
    del op, x, y
    torch.cuda.synchronize()
    return out


def hanging_benchmark(steps, warmup, degree=4, n_coarse=32):
    """The operator on the two-block mesh with hanging nodes (Q4, the unit cube in 32^3 cells
    joined at X1 = 1 to 64^3 cells of half the size, curved, variable coefficient, FP64;
    19,121,282 DoFs): one application, both blocks' cell loops and the interface kernels.
    Algorithmic bytes: each block's (vectors, index maps, G) plus the interface arrays (the
    interpolated trace and the fine face's results, written and read once)."""
    import torch
    import paper_1910_13247_amd as mfq
    from synthetic import uniform_vector
    p, n = degree, n_coarse
    op = mfq.HangingOperator(n, p, 0.1, 0.5, mfq.MFQ_FP64)
    x = torch.from_numpy(uniform_vector(op.n_dofs, seed=0)).cuda()
    y = torch.empty_like(x)
    s = time_events(lambda: op.vmult(x, y), steps, warmup)
    face = (2 * p * n + 1) ** 2
    rb = algorithmic_bytes(p, n, 8) + algorithmic_bytes(p, 2 * n, 8) + 4 * 8 * face
    out = {"workload": f"hanging_q{p}_{n}^3+{2 * n}^3_curved", "dofs": op.n_dofs, "ms": s * 1e3,
           "DoFs_per_s": op.n_dofs / s, "algorithmic_bytes": rb, "achieved_GBs": rb / s / 1e9,
           "frac": rb / s / 1e9 / HBM_PEAK_GBS}
    del op, x, y
    torch.cuda.synchronize()
    return out


def cpu_small_poisson():
    """Oracle side of the small Poisson workload: SciPy CSR product of the assembled matrix on one
    thread, and the oracle's CG to 1e-10 on it."""
    import numpy as np
    from oracle import assemble, mesh, solve
    from synthetic import POISSON_Q2_8, uniform_vector
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    pr = POISSON_Q2_8
    A = assemble.operator_csr(pr.degree, pr.cells_1d, pr.amplitude, pr.alpha, 1)
    f = uniform_vector(A.shape[0], seed=0)
    b = f * mesh.boundary_mask(pr.degree, pr.cells_1d)
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        reps = 200
        t0 = time.perf_counter()
        for _ in range(reps):
            A @ f
        spmv = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        x, it, rr = solve.cg(lambda v: A @ v, b, rtol=1e-10)
        cg = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    return {"workload": pr.name, "cores": 1, "csr_spmv_us": spmv * 1e6, "cg_s": cg, "cg_iterations": it,
            "cg_rel_residual": rr}


def q8_solve_check(b, x, n_rows=24):
    """The Q8 24^3 solve's residual b - A x on sampled rows, the load vector and the operator rows
    recomputed by the oracle from each row's cells, relative to ||b||_2 (every row of a solution
    certified to 1e-10 lies within 1e-10)."""
    import numpy as np
    from oracle import ebe, rhs
    from synthetic import VARCOEF_Q8_24 as pr
    p, n = pr.degree, pr.cells_1d
    N1 = p * n + 1
    rng = np.random.default_rng(17)
    rows = np.concatenate([rng.integers(0, len(b), n_rows - 2), [N1 ** 3 // 2, 24 + 7 * N1 + 9 * N1 * N1]])
    t0 = time.perf_counter()
    bo = rhs.rhs_rows(p, n, pr.amplitude, pr.alpha, lambda xx: rhs.manufactured_f(xx, pr.alpha), rows, 1)
    r = bo - ebe.ebe_rows(p, n, pr.amplitude, pr.alpha, x, 1, rows)
    nb = float(np.linalg.norm(b))
    return {"rows": int(len(rows)), "max_abs_residual_over_norm_b": float(np.abs(r).max() / nb),
            "load_vector_max_rel_diff": float(np.abs(b[rows] - bo).max() / np.abs(b).max()),
            "bar": "each |r_i| <= 1e-10 ||b||_2", "seconds": time.perf_counter() - t0}


# Q4 V-cycles beside the paper's only measurements (an FP32 V-cycle of DG Q4, Chebyshev degree 6,
# matrix-free, on one 48-core node: 31.7 ms for 65,536 cells, 264 ms for 524,288 cells)
VCYCLE_MESHES = [40, 80]


def vcycle_benchmark(steps, warmup):
    """One FP32 V-cycle (the GMG_MIXED preconditioner: Chebyshev degree 6 on every level, coarse
    Chebyshev) of the constant-coefficient Q4 Laplacian on the undeformed cube, timed with HIP
    events; undeformed cells with coefficient 1 run the Cartesian cell loop (G_q = h w I formed in
    registers)."""
    import torch
    import paper_1910_13247_amd as mfq
    from synthetic import uniform_vector
    out = []
    for n in VCYCLE_MESHES:
        print(f"# V-cycle Q4 {n}^3", file=sys.stderr, flush=True)
        space = mfq.Space(mfq.Mesh(n, 0.0), 4, mfq.MFQ_BC_DIRICHLET0)
        op = mfq.Operator(space, 0.0, mfq.MFQ_FP64)
        sv = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED, smoother_degree=6, coarse_mode=1)
        r = torch.from_numpy(uniform_vector(space.n_dofs, seed=3)).cuda()
        z = torch.empty_like(r)
        sec = time_events(lambda: sv.precondition(r, z), steps, warmup)
        out.append({"degree": 4, "cells": space.n_cells, "dofs": space.n_dofs,
                    "ms": sec * 1e3, "DoFs_per_s": space.n_dofs / sec, "cells_per_s": space.n_cells / sec})
        del sv, op, r, z
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def dg_multigrid_benchmark(steps, warmup, solve_rtol=1e-10):
    """The paper's multigrid experiment on one GPU: the DG-SIPG Q4 operator on the undeformed n^3
    mesh, one FP32 V-cycle (Chebyshev degree 6 on the DG level, switch to the continuous Q4 space
    on the same mesh, its h- and p-hierarchy, dense coarse inverse) timed with HIP events, and a
    full FP64 CG solve to `solve_rtol` from a seeded right-hand side, with the mean residual
    reduction per iteration."""
    import torch
    import paper_1910_13247_amd as mfq
    from synthetic import uniform_vector
    out = []
    for n in VCYCLE_MESHES:
        print(f"# DG V-cycle Q4 {n}^3", file=sys.stderr, flush=True)
        op = mfq.DGOperator(mfq.Mesh(n, 0.0), 4)
        t0 = time.perf_counter()
        sv = mfq.DGSolver(op)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        r = torch.from_numpy(uniform_vector(op.n_dofs, seed=3)).cuda()
        z = torch.empty_like(r)
        side = torch.cuda.Stream()          # a non-default stream: the V-cycle replays as a graph
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            sec = time_events(lambda: sv.precondition(r, z, stream=side), steps, warmup)
        rec = {"degree": 4, "cells": n ** 3, "dofs": op.n_dofs, "vcycle_ms": sec * 1e3,
               "DoFs_per_s": op.n_dofs / sec, "setup_s": setup}
        with torch.cuda.stream(side):
            x, info, st = sv.solve(r, rtol=solve_rtol, max_iter=200, stream=side)
            x, info, st = sv.solve(r, rtol=solve_rtol, max_iter=200, stream=side)     # warm
        rec.update({"solve_s": info.seconds, "iterations": info.iterations, "passes": info.outer_iterations,
                    "rel_residual": info.rel_residual, "levels": info.n_levels,
                    "rate_per_iteration": info.rel_residual ** (1.0 / max(info.iterations, 1)),
                    "status": int(st)})
        del x
        out.append(rec)
        del sv, op, r, z
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def serve_benchmark(n_requests, rate=200.0, seed=0, iters_per_step=2, n_streams=4, mode="async", setup_threads=1,
                    solver_params=None):
    """The serving stream: Poisson arrivals at `rate`/s, degree U{1..6}, n U{4..48}, alpha
    U[0,0.9], right-hand side from the request's seed; each solved to relative residual 1e-10."""
    import torch
    from synthetic import serving_stream
    from paper_1910_13247_amd.serve import DeviceExecutor, Request, Server, run_stream
    stream = serving_stream(n_requests, rate, seed)
    reqs = [Request(degree=d["degree"], n=d["cells_1d"], alpha=d["alpha"], seed=d["rhs_seed"]) for d in stream]
    arrivals = [d["arrival"] for d in stream]
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(0.75 * free, 160e9))
    batched = mode == "batched"
    srv = Server(DeviceExecutor(n_streams=n_streams, batched=batched, **(solver_params or {})), budget,
                 iters_per_step=iters_per_step, mode="sync" if batched else mode, setup_threads=setup_threads)
    t0 = time.perf_counter()
    st = run_stream(srv, reqs, arrivals)
    srv.close()
    torch.cuda.synchronize()
    st["wall_s"] = time.perf_counter() - t0
    st["budget_bytes"] = budget
    st["iters_per_step"] = iters_per_step
    st["streams"] = n_streams
    st["mode"] = mode
    st["setup_threads"] = setup_threads
    st["solver_params"] = solver_params or {}
    st["rate_per_s"] = rate
    st["dofs_total"] = sum((r.degree * r.n + 1) ** 3 for r in reqs)
    st["iterations_mean"] = sum(r.iterations for r in srv.done) / max(len(srv.done), 1)
    st["not_converged"] = sum(1 for r in srv.done if r.status != 0)
    # aggregate algorithmic traffic: every request's set-up and solve (the requests' meshes are
    # undeformed: with a variable coefficient the cell loops read only the diagonal of G, with
    # coefficient 1 none of it)
    prm = solver_params or {}
    kw = dict(smoother_degree=prm.get("smoother_degree", 3), coarse_mode=prm.get("coarse_mode", 1),
              coarse_degree=prm.get("coarse_degree", 16))
    lz = prm.get("lanczos_iters", srv.ex.params.get("lanczos_iters", 12))
    tot = sum(solve_bytes("gmg_mixed", r.degree, r.n, r.iterations, 1, cart=r.alpha == 0, coef=r.alpha != 0, **kw) +
              setup_bytes(r.degree, r.n, kw["smoother_degree"], kw["coarse_mode"], lz, coef=r.alpha != 0)
              for r in srv.done)
    st["algorithmic_bytes"] = tot
    st["aggregate_algorithmic_GBs"] = tot / st["wall_s"] / 1e9
    st["aggregate_frac_of_peak"] = tot / st["wall_s"] / 1e9 / HBM_PEAK_GBS
    return st


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solves", action="store_true",
                    help="skip the time-to-1e-10 of the Q3 128^3 solvers (multigrid forms and plain FP64 CG)")
    ap.add_argument("--solve-kinds", default=",".join(SOLVE_KINDS),
                    help="which Q3 128^3 solvers to time (comma-separated subset of the default)")
    ap.add_argument("--serve", type=int, default=2000, metavar="N",
                    help="replay N requests of the serving stream (200 requests/s) and report solves/s, p50/p99 "
                         "(default 2000, the full stream; 0 skips)")
    ap.add_argument("--serve-mode", choices=["batched", "sync", "async"], default="batched",
                    help="serving steps: batched launches over all running solves (batched), each solve's own "
                         "launches, all waited for together (sync), or each at its own pace (async)")
    ap.add_argument("--serve-streams", type=int, default=8)
    ap.add_argument("--serve-iters", type=int, default=2, help="CG iterations per serving step")
    ap.add_argument("--serve-params", default="",
                    help="solver parameters of the served requests, e.g. coarse_degree=8,smoother_degree=3")
    ap.add_argument("--serve-setup-threads", type=int, default=1,
                    help="worker threads that set up admitted requests (0: on the scheduler thread)")
    ap.add_argument("--no-csr", action="store_true", help="skip the assembled-matrix (CSR) comparison")
    ap.add_argument("--vcycle", action="store_true",
                    help="add FP32 V-cycle times of the Q4 Laplacian (40^3 and 80^3 cells)")
    ap.add_argument("--no-dg-mg", action="store_true",
                    help="skip the DG-SIPG Q4 multigrid (V-cycle at 40^3 and 80^3 cells, solve at 40^3)")
    ap.add_argument("--csr-sweep", action="store_true",
                    help="add the assembled-matrix comparison for degrees 1..8 at about 16M DoFs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run 3 plain device copies of 1 GiB (reference reading for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the operator, CG and "
              "multigrid run on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1910_13247_amd as mfq
    from synthetic import VARCOEF_Q4_64, uniform_vector

    pr = VARCOEF_Q4_64
    p, n = pr.degree, pr.cells_1d
    torch.cuda.set_device(0)
    mesh = mfq.Mesh(n, pr.amplitude)
    space = mfq.Space(mesh, p, mfq.MFQ_BC_DIRICHLET0)
    op64 = mfq.Operator(space, pr.alpha, mfq.MFQ_FP64)
    x_np = uniform_vector(space.n_dofs, seed=0)
    x64 = torch.from_numpy(x_np).cuda()
    print(f"# workload {pr.name}: {space.n_dofs} DoFs, {space.n_cells} cells", file=sys.stderr, flush=True)
    wall64, kern64, y64 = time_vmult(op64, x64, args.steps, args.warmup)
    print(f"# fp64: {wall64 * 1e3:.3f} ms/step, cell kernel {kern64 * 1e3:.3f} ms", file=sys.stderr, flush=True)

    op32 = mfq.Operator(space, pr.alpha, mfq.MFQ_FP32)
    x32 = x64.float()
    wall32, kern32, y32 = time_vmult(op32, x32, args.steps, args.warmup)
    rel32 = ((y32.double() - y64).abs().max() / y64.abs().max()).item()
    N1 = p * n + 1
    rng = np.random.default_rng(1)
    check_rows = np.unique(np.concatenate([rng.integers(0, space.n_dofs, 200),
                                           [0, N1 ** 3 - 1, 1 + N1 + N1 * N1, N1 ** 3 // 2]]))
    rows_t = torch.from_numpy(check_rows).cuda()
    y64_rows = y64[rows_t].cpu().numpy()
    y32_rows = y32[rows_t].double().cpu().numpy()
    print(f"# fp32: {wall32 * 1e3:.3f} ms/step, cell kernel {kern32 * 1e3:.3f} ms", file=sys.stderr, flush=True)
    del op32, x32, y32
    torch.cuda.synchronize()

    N = space.n_dofs
    lay = op64.layout()
    launches = lay["launches"]
    bytes64 = algorithmic_bytes(p, n, 8)
    bytes32 = algorithmic_bytes(p, n, 4)
    # per launch: the colours split the cells evenly on this mesh (64 rows of bricks per direction)
    per_launch64 = bytes64 / launches
    launch_s = kern64 / launches
    achieved = per_launch64 / launch_s / 1e9
    rec = {
        "metric": METRIC,
        "value": N / wall64,
        "unit": "DoFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Q4 variable-coefficient Laplacian, curved 64^3 hex mesh, FP64 matrix-free vmult",
                   "degree": p, "cells": space.n_cells, "dofs": N, "amplitude": pr.amplitude, "alpha": pr.alpha,
                   "input": "uniform[-1,1) seed 0, resident in HBM"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "vmult_kernel<4, double, false, false, false> (cell loop)", "launches_per_step": launches,
                     "launch_ms": launch_s * 1e3, "algorithmic_bytes_per_launch": per_launch64,
                     "layout": lay, "kernel_source": kernel_source_hash(),
                     "algorithmic_tflops": algorithmic_flops(p, n) / kern64 / 1e12},
        "fp32": {"value": N / wall32, "unit": "DoFs/s", "ms_per_step": wall32 * 1e3, "cell_loop_ms": kern32 * 1e3,
                 "achieved_GBs": bytes32 / kern32 / 1e9, "frac": bytes32 / kern32 / 1e9 / HBM_PEAK_GBS,
                 "normwise_rel_err_vs_fp64": rel32},
    }
    rec["copy_kernel"] = copy_bandwidth()
    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").uniform_()
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        rec["copy_probe_bytes"] = {"read": a.numel() * 8, "write": b.numel() * 8}
        del a, b
    if not args.no_csr:
        print("# assembled matrix (CSR) of the same operator", file=sys.stderr, flush=True)
        rec["assembled_csr"] = assembled_comparison(op64, x64, y64, kern64, min(args.steps, 20), args.warmup)
        rec["assembled_csr_fp32"] = assembled_comparison(op64, x64, y64, kern32, min(args.steps, 20), args.warmup,
                                                         precision=mfq.MFQ_FP32)
    if args.csr_sweep:
        rec["csr_sweep"] = csr_sweep(min(args.steps, 20), args.warmup)
    rec["small_poisson"] = small_poisson(min(args.steps, 50), args.warmup)
    rec["dg_sipg_q4_64"] = dg_benchmark(min(args.steps, 20), args.warmup)
    rec["hanging_q4_32_64"] = hanging_benchmark(min(args.steps, 20), args.warmup)
    print("# Q8 24^3: FP64 / FP32 / FP32 matrix cores", file=sys.stderr, flush=True)
    rec["high_degree_q8_24"] = high_degree_comparison(min(args.steps, 20), args.warmup)
    q8_solution = rec["high_degree_q8_24"].pop("_solution")
    if not args.no_solves:
        print("# Q3 128^3 solves to 1e-10", file=sys.stderr, flush=True)
        rec["solves_q3_128"] = solve_benchmarks(args.steps, [k for k in args.solve_kinds.split(",") if k])
    if args.vcycle:
        rec["vcycle_q4"] = vcycle_benchmark(min(args.steps, 20), args.warmup)
    if not args.no_dg_mg:
        rec["dg_multigrid_q4"] = dg_multigrid_benchmark(min(args.steps, 20), args.warmup)
    if args.serve:
        print(f"# serving {args.serve} requests", file=sys.stderr, flush=True)
        prm = {}
        for kv in filter(None, args.serve_params.split(",")):
            k, v = kv.split("=")
            prm[k.strip()] = float(v) if "." in v else int(v)
        rec["serving"] = serve_benchmark(args.serve, mode=args.serve_mode, n_streams=args.serve_streams,
                                         iters_per_step=args.serve_iters,
                                         setup_threads=args.serve_setup_threads, solver_params=prm)
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle, bounded sample)", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(p, n, pr.amplitude, pr.alpha, x_np, check_rows=check_rows,
                                           y64_rows=y64_rows, y32_rows=y32_rows)
        rec["cpu_baseline"]["small_poisson"] = cpu_small_poisson()
        rec["cpu_baseline"]["q8_24_solve_check"] = q8_solve_check(*q8_solution)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
