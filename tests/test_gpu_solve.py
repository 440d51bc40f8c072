"""GPU solvers against the oracle: residual certificates, iteration counts, V-cycle parity."""
import numpy as np
import pytest

from oracle import assemble, ebe, gmg, mesh, rhs, solve
from synthetic import uniform_vector

pytestmark = pytest.mark.gpu


def _mfq():
    import paper_1910_13247_amd as mfq
    return mfq


def _torch():
    import torch
    return torch


def _setup(p, n, amp, alpha):
    mfq = _mfq()
    m = mfq.Mesh(n, amp)
    s = mfq.Space(m, p, mfq.MFQ_BC_DIRICHLET0)
    return m, s, mfq.Operator(s, alpha, mfq.MFQ_FP64)


def test_poisson_q2_8_cg_to_1e10():
    # unpreconditioned FP64 CG on the small Poisson workload, b = m * f (seeded nodal f)
    mfq = _mfq()
    torch = _torch()
    print("cg poisson q2 8^3", flush=True)
    _, s, op = _setup(2, 8, 0.0, 0.0)
    f = uniform_vector(op.n_dofs, 0)
    b_np = rhs.rhs_nodal(2, 8, f)
    solver = mfq.Solver(op, mfq.MFQ_SOLVER_CG, check_every=1)
    x, info, _ = solver.solve(torch.from_numpy(b_np).cuda(), rtol=1e-10)
    At = assemble.operator_csr(2, 8, 0.0, 0.0, 1)
    xo, it_o, _ = solve.cg(lambda v: At @ v, b_np, rtol=1e-10)
    cert = solve.rel_residual(lambda v: At @ v, b_np, x.cpu().numpy())
    assert cert <= 1e-10
    assert abs(info.rel_residual - cert) <= 1e-12
    assert abs(info.iterations - it_o) <= 2, (info.iterations, it_o)
    np.testing.assert_allclose(x.cpu().numpy(), solve.direct_solve(At, b_np), atol=1e-8)


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_gmg_solvers_certified(kind):
    # curved, variable coefficient, Q3 on 8^3 (two levels: 4^3 coarse solved densely)
    mfq = _mfq()
    torch = _torch()
    print(f"gmg kind={kind}", flush=True)
    p, n = 3, 8
    _, s, op = _setup(p, n, 0.1, 0.5)
    b = op.rhs_manufactured()
    solver = mfq.Solver(op, kind)
    x, info, _ = solver.solve(b, rtol=1e-10, max_iter=200)
    At = assemble.operator_csr(p, n, 0.1, 0.5, 1)
    b_np = b.cpu().numpy()
    cert = solve.rel_residual(lambda v: At @ v, b_np, x.cpu().numpy())
    assert cert <= 1e-10
    assert info.iterations <= 40
    assert info.n_levels == 2
    # the discrete solution: L2 error equals the oracle's direct solution's
    xo = solve.direct_solve(At, rhs.rhs_manufactured(p, n, 0.1, 0.5))
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-8


def test_gmg_beats_cg_iterations():
    mfq = _mfq()
    p, n = 2, 16
    _, s, op = _setup(p, n, 0.1, 0.5)
    b = op.rhs_manufactured()
    _, i_cg, _ = mfq.Solver(op, mfq.MFQ_SOLVER_CG).solve(b, rtol=1e-10, max_iter=5000)
    _, i_mg, _ = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED).solve(b, rtol=1e-10, max_iter=200)
    assert i_mg.iterations * 5 < i_cg.iterations
    assert i_mg.rel_residual <= 1e-10 and i_cg.rel_residual <= 1e-10


def test_vcycle_matches_oracle_fp64():
    # one FP64 V-cycle application with the oracle's Chebyshev interval: same hierarchy, smoother,
    # transfers and exact coarse solve => same result up to rounding
    mfq = _mfq()
    torch = _torch()
    p, n = 3, 8          # (3,8): 23^3 free > 4096 -> coarse (3,4): 11^3 = 1331
    levels, prolong = gmg.build_hierarchy(p, n, 0.1, 0.5, bc=1)
    assert [(L.p, L.n) for L in levels] == [(3, 4), (3, 8)]
    lhats = [L.estimate() for L in levels[1:]]
    _, s, op = _setup(p, n, 0.1, 0.5)
    solver = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_FP64, lambda_override=[1.2 * l for l in lhats])
    lam_gpu = solver.lambdas(2)
    assert abs(lam_gpu[0] - lhats[0]) <= 1e-8 * lhats[0]
    r = mesh.boundary_mask(p, n) * uniform_vector(op.n_dofs, 21)
    z = solver.precondition(torch.from_numpy(r).cuda()).cpu().numpy()
    zo = gmg.vcycle(levels, prolong, 1, r)
    assert np.abs(z - zo).max() <= 1e-11 * np.abs(zo).max()


@pytest.mark.parametrize("p,n,limit", [(4, 2, 8), (3, 4, 30), (6, 2, 30)])
def test_vcycle_fp32_within_derived_bound(p, n, limit):
    """One FP32 V-cycle against the oracle's FP64 V-cycle, within the first-order componentwise
    bound that propagates each FP32 kernel's rounding model through the cycle (tests/fp32_bound.py):
    3 levels with h- then p-coarsening (4,2) -> (4,1) -> (2,1) and (6,2) -> (6,1) -> (3,1), and
    3 h-levels (3,4) -> (3,2) -> (3,1) (small coarse limits keep the meshes small enough for the
    dense analysis)."""
    from fp32_bound import vcycle_fp32_bound
    from oracle.ebe import magnitude_csr
    mfq = _mfq()
    torch = _torch()
    print(f"fp32 V-cycle p={p} n={n} coarse_dofs={limit}", flush=True)
    levels, prolong = gmg.build_hierarchy(p, n, 0.1, 0.5, bc=1, coarse_dofs=limit)
    lhats = [L.estimate() for L in levels[1:]]
    _, s, op = _setup(p, n, 0.1, 0.5)
    solver = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED, lambda_override=[1.2 * l for l in lhats],
                        coarse_dofs=limit)
    assert len(solver.lambdas(len(levels))) == len(levels) - 1
    r = mesh.boundary_mask(p, n) * uniform_vector(op.n_dofs, 22)
    z = solver.precondition(torch.from_numpy(r).cuda()).cpu().numpy()
    zo = gmg.vcycle(levels, prolong, len(levels) - 1, r)
    mags = [magnitude_csr(L.p, L.n, 0.1, 0.5, 1) for L in levels]
    zt, bound = vcycle_fp32_bound(levels, prolong, mags, r)
    assert np.abs(zt - zo).max() <= 1e-12 * np.abs(zo).max()
    err = np.abs(z - zo)
    print(f"  max err / bound {np.max(err / (bound + 1e-300)):.2e}, rel err {err.max() / np.abs(zo).max():.2e}")
    assert np.all(err <= 1.01 * bound + 1e-12 * np.abs(zo).max())


def test_vcycle_three_levels_h_and_p_fp64():
    """FP64 V-cycle on the hierarchy (2,5) -> (4,5) -> (4,10): an h-transfer and a p-transfer,
    dense coarse solve; equal to the oracle's V-cycle up to FP64 rounding."""
    mfq = _mfq()
    torch = _torch()
    p, n = 4, 10
    print("fp64 V-cycle 3 levels", flush=True)
    levels, prolong = gmg.build_hierarchy(p, n, 0.1, 0.5, bc=1)
    assert [(L.p, L.n) for L in levels] == [(2, 5), (4, 5), (4, 10)]
    lhats = [L.estimate() for L in levels[1:]]
    _, s, op = _setup(p, n, 0.1, 0.5)
    solver = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_FP64, lambda_override=[1.2 * l for l in lhats])
    r = mesh.boundary_mask(p, n) * uniform_vector(op.n_dofs, 24)
    z = solver.precondition(torch.from_numpy(r).cuda()).cpu().numpy()
    zo = gmg.vcycle(levels, prolong, 2, r)
    assert np.abs(z - zo).max() <= 1e-11 * np.abs(zo).max()
    # without the override the device's own eigenvalue estimates match the oracle's
    lam = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_FP64).lambdas(3)
    np.testing.assert_allclose(lam, lhats, rtol=1e-8)


@pytest.mark.parametrize("p,n,levels_expected", [(1, 38, [(1, 19), (1, 38)]), (2, 19, [(1, 19), (2, 19)])])
@pytest.mark.parametrize("kind", [1, 2])
def test_jacobi_cg_coarse_solve(p, n, levels_expected, kind):
    """Coarsest levels above the dense limit (5,832 free DoFs) are solved by Jacobi-CG to 1e-12 on
    the host-polled path: an h-hierarchy and a p-hierarchy (odd n), FP64 and mixed V-cycles;
    solutions certified by the oracle's assembled operator."""
    mfq = _mfq()
    print(f"jacobi-cg coarse p={p} n={n} kind={kind}", flush=True)
    assert gmg.hierarchy(p, n) == levels_expected
    _, s, op = _setup(p, n, 0.1, 0.5)
    b = op.rhs_manufactured()
    x, info, st = mfq.Solver(op, kind).solve(b, rtol=1e-10, max_iter=200)
    assert st == mfq.MFQ_OK and info.n_levels == 2 and info.rel_residual <= 1e-10
    At = assemble.operator_csr(p, n, 0.1, 0.5, 1)
    assert solve.rel_residual(lambda v: At @ v, b.cpu().numpy(), x.cpu().numpy()) <= 1e-10


def test_q3_128_gmg_mixed_certified_on_oracle_rows():
    """The benchmark's Q3 128^3 solve (57,066,625 DoFs, 6 levels, GMG_MIXED to 1e-10): the load
    vector on 300 rows against the oracle's cell sums, and the residual b - A x on the same rows,
    each recomputed by the oracle from the row's cells, within 1e-10 ||b||_2."""
    mfq = _mfq()
    torch = _torch()
    p, n = 3, 128
    print("Q3 128^3 GMG_MIXED certified rows", flush=True)
    _, s, op = _setup(p, n, 0.1, 0.5)
    b = op.rhs_manufactured()
    x, info, st = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED).solve(b, rtol=1e-10, max_iter=200)
    torch.cuda.synchronize()
    assert st == mfq.MFQ_OK and info.rel_residual <= 1e-10 and info.n_levels == 6
    b_np = b.cpu().numpy()
    x_np = x.cpu().numpy()
    del x
    N1 = p * n + 1
    rng = np.random.default_rng(6)
    # random rows plus nodes on x-brick faces (bricks of 16 cells: I = 48, 96), cell faces, corners
    rows = np.concatenate([rng.integers(0, op.n_dofs, 288),
                           [48 + 10 * N1 + 20 * N1 * N1, 96 + 96 * N1 + 96 * N1 * N1, 1 + N1 + N1 * N1,
                            N1 ** 3 // 2, 3 + 3 * N1 + 3 * N1 * N1, 192 + 191 * N1 + 190 * N1 * N1,
                            (N1 - 2) * (1 + N1 + N1 * N1), 49 + 47 * N1 + 300 * N1 * N1, 0, N1 ** 3 - 1,
                            144 + 3 * N1 + 381 * N1 * N1, 4 + 380 * N1 + 7 * N1 * N1]])
    f = lambda xx: rhs.manufactured_f(xx, 0.5)
    bo = rhs.rhs_rows(p, n, 0.1, 0.5, f, rows, 1)
    assert np.abs(b_np[rows] - bo).max() <= 1e-12 * np.abs(b_np).max()
    r = bo - ebe.ebe_rows(p, n, 0.1, 0.5, x_np, 1, rows)
    nb = np.linalg.norm(b_np)
    print(f"  max sampled |r_i| / ||b|| = {np.abs(r).max() / nb:.2e}")
    assert np.abs(r).max() <= 1e-10 * nb


def test_q8_mixed_ir_certified_in_full():
    """The high-degree solve reduced to Q8 on the curved 4^3 mesh (35,937 DoFs, levels (8,2) and
    (8,4)): GMG_MIXED_IR (FP32 inner CG and V-cycle, FP64 refinement) to 1e-10, certified by the
    oracle's assembled operator and manufactured load vector."""
    mfq = _mfq()
    p, n = 8, 4
    print("Q8 4^3 mixed IR", flush=True)
    _, s, op = _setup(p, n, 0.1, 0.5)
    b = op.rhs_manufactured()
    bo = rhs.rhs_manufactured(p, n, 0.1, 0.5)
    assert np.abs(b.cpu().numpy() - bo).max() <= 1e-12 * np.abs(bo).max()
    x, info, st = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED_IR).solve(b, rtol=1e-10, max_iter=300)
    assert st == mfq.MFQ_OK and info.rel_residual <= 1e-10 and info.n_levels == 2
    At = assemble.operator_csr(p, n, 0.1, 0.5, 1)
    assert solve.rel_residual(lambda v: At @ v, bo, x.cpu().numpy()) <= 1e-10


def test_q8_24_mixed_ir_certified_on_oracle_rows():
    """The high-degree workload's solve (Q8, curved 24^3, 7,189,057 DoFs, levels 3^3..24^3):
    GMG_MIXED_IR to 1e-10, residual rows recomputed by the oracle within 1e-10 ||b||_2."""
    mfq = _mfq()
    torch = _torch()
    p, n = 8, 24
    print("Q8 24^3 mixed IR certified rows", flush=True)
    _, s, op = _setup(p, n, 0.1, 0.5)
    b = op.rhs_manufactured()
    x, info, st = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED_IR).solve(b, rtol=1e-10, max_iter=300)
    torch.cuda.synchronize()
    assert st == mfq.MFQ_OK and info.rel_residual <= 1e-10
    b_np, x_np = b.cpu().numpy(), x.cpu().numpy()
    N1 = p * n + 1
    rng = np.random.default_rng(9)
    rows = np.concatenate([rng.integers(0, op.n_dofs, 22), [24 + 7 * N1 + 9 * N1 * N1, N1 ** 3 // 2,
                                                             1 + N1 + N1 * N1, 72 + 72 * N1 + 72 * N1 * N1]])
    f = lambda xx: rhs.manufactured_f(xx, 0.5)
    bo = rhs.rhs_rows(p, n, 0.1, 0.5, f, rows, 1)
    assert np.abs(b_np[rows] - bo).max() <= 1e-12 * np.abs(b_np).max()
    r = bo - ebe.ebe_rows(p, n, 0.1, 0.5, x_np, 1, rows)
    assert np.abs(r).max() <= 1e-10 * np.linalg.norm(b_np)


def test_nonconvergence_reports_enoconv():
    mfq = _mfq()
    _, s, op = _setup(2, 4, 0.1, 0.5)
    b = op.rhs_manufactured()
    st, info = None, None
    _, info, st = mfq.Solver(op, mfq.MFQ_SOLVER_CG).solve(b, rtol=1e-10, max_iter=3, check=False)
    assert st == mfq._lib.MFQ_ENOCONV
    assert info.iterations == 3 and info.rel_residual > 1e-10


def test_zero_rhs_gives_zero_solution():
    mfq = _mfq()
    torch = _torch()
    _, s, op = _setup(2, 4, 0.1, 0.5)
    b = torch.zeros(op.n_dofs, dtype=torch.float64, device="cuda")
    for kind in (0, 2, 3):
        x, info, _ = mfq.Solver(op, kind).solve(b, rtol=1e-10)
        assert x.abs().max().item() == 0.0


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_solvers_need_no_initialised_memory(kind):
    """Operator, solver and solution buffers filled with NaN bit patterns before binding: every
    value the solve reads must have been written by the library first (regression: the first CG
    direction once read the previous contents of p)."""
    mfq = _mfq()
    torch = _torch()
    _lib = mfq._lib
    print(f"nan-filled buffers kind={kind}", flush=True)
    p, n = 3, 8
    m = _lib.mfq_mesh_create(n, 0.1)
    s = _lib.mfq_space_create(m, p, mfq.MFQ_BC_DIRICHLET0)
    op = _lib.mfq_op_create(s, 0.5, mfq.MFQ_FP64)
    ob = _lib.mfq_op_device_bytes(op)
    obuf = torch.full((ob,), 0xFF, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    _lib.mfq_op_bind(op, obuf.data_ptr(), ob, st)
    prm = _lib.mfq_solver_default_params()
    sv = _lib.mfq_solver_create(op, kind, prm)
    sb = _lib.mfq_solver_device_bytes(sv)
    sbuf = torch.full((sb,), 0xFF, dtype=torch.uint8, device="cuda")
    _lib.mfq_solver_bind(sv, sbuf.data_ptr(), sb, st)
    N = _lib.mfq_space_n_dofs(s)
    b = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
    x = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
    _lib.mfq_rhs_manufactured(op, b.data_ptr(), st)
    status, info = _lib.mfq_solve(sv, b.data_ptr(), x.data_ptr(), 1e-10, 5000, st)
    torch.cuda.synchronize()
    assert status == mfq.MFQ_OK and info.rel_residual <= 1e-10
    assert bool(torch.isfinite(x).all())
    _lib.mfq_solver_destroy(sv)
    _lib.mfq_op_destroy(op)
    _lib.mfq_space_destroy(s)
    _lib.mfq_mesh_destroy(m)
