"""GPU solvers against the oracle: residual certificates, iteration counts, V-cycle parity."""
import numpy as np
import pytest

from oracle import assemble, gmg, mesh, rhs, solve
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


def test_vcycle_fp32_close_to_oracle():
    mfq = _mfq()
    torch = _torch()
    p, n = 3, 8
    levels, prolong = gmg.build_hierarchy(p, n, 0.1, 0.5, bc=1)
    lhats = [L.estimate() for L in levels[1:]]
    _, s, op = _setup(p, n, 0.1, 0.5)
    solver = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED, lambda_override=[1.2 * l for l in lhats])
    lam_gpu = solver.lambdas(2)
    assert abs(lam_gpu[0] - lhats[0]) <= 1e-4 * lhats[0]
    r = mesh.boundary_mask(p, n) * uniform_vector(op.n_dofs, 22)
    z = solver.precondition(torch.from_numpy(r).cuda()).cpu().numpy()
    zo = gmg.vcycle(levels, prolong, 1, r)
    assert np.abs(z - zo).max() <= 1e-4 * np.abs(zo).max()


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
