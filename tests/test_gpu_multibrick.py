"""Operator parity on meshes more than one brick wide in every direction, for every degree.

The cell loop cuts the mesh into bricks of (32,2,1), (14,2,1), (16,1,1), (5,2,1), (7,1,1),
(4,1,1), (4,1,1), (3,1,1) cells for p = 1..8 and writes nodes shared between bricks by colour
(the first colour to touch a node stores, later ones add).  These sizes put at least two bricks
along x (both x parities, the x-face store/add rule, a ragged last brick) and several along y and
z.  FP64 bar: ||y - y_o||_inf <= 1e-12 ||y_o||_inf against the oracle's assembled matrix; FP32:
|y32 - y_o| <= 2 k u32 (|A| |x32|) componentwise, k = 8(p+1) + 16.  At full size the Q8 24^3
workload is checked on oracle rows for the vector-ALU FP64 and FP32 kernels.
"""
import functools

import numpy as np
import pytest

from oracle import assemble, ebe
from synthetic import uniform_vector

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
BRICK_X = {1: 32, 2: 14, 3: 16, 4: 5, 5: 7, 6: 4, 7: 4, 8: 3}
WIDE = {1: 33, 2: 15, 3: 17, 4: 11, 5: 8, 6: 5, 7: 5, 8: 4}


@functools.lru_cache(maxsize=2)
def _oracle(p, n):
    return assemble.operator_csr(p, n, 0.1, 0.5, 1)


def _run(p, n, prec, x_np):
    import torch
    import paper_1910_13247_amd as mfq
    op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.1), p, mfq.MFQ_BC_DIRICHLET0), 0.5, prec)
    lay = op.layout()
    assert lay["brick"][0] == BRICK_X[p]
    assert n > BRICK_X[p], "the mesh must be wider than one brick in x"
    y = op.vmult(torch.from_numpy(x_np).to(op.dtype).cuda())
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


@pytest.mark.parametrize("p", range(1, 9))
def test_multibrick_fp64(p):
    n = WIDE[p]
    print(f"multi-brick fp64 p={p} n={n}", flush=True)
    import paper_1910_13247_amd as mfq
    x = uniform_vector((p * n + 1) ** 3, seed=80 + p)
    y = _run(p, n, mfq.MFQ_FP64, x)
    yo = _oracle(p, n) @ x
    err = np.abs(y - yo).max() / np.abs(yo).max()
    print(f"  normwise rel err {err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("p", range(1, 9))
def test_multibrick_fp32(p):
    n = WIDE[p]
    print(f"multi-brick fp32 p={p} n={n}", flush=True)
    import paper_1910_13247_amd as mfq
    x = uniform_vector((p * n + 1) ** 3, seed=90 + p)
    x32 = x.astype(np.float32).astype(np.float64)
    y = _run(p, n, mfq.MFQ_FP32, x)
    yo = _oracle(p, n) @ x32
    mag = ebe.magnitude_bound(p, n, 0.1, 0.5, x32, 1)
    k = 8 * (p + 1) + 16
    assert np.all(np.abs(y - yo) <= 2 * k * U32 * mag + 1e-30)


@pytest.mark.parametrize("prec", [0, 1])
def test_sampled_parity_full_size_q8_24_vector_alu(prec):
    """Q8 on the curved 24^3 mesh (7,189,057 DoFs, eight bricks of 3 cells along x) with the
    vector-ALU kernels, FP64 and FP32: 28 rows recomputed by the oracle cell by cell."""
    import torch
    import paper_1910_13247_amd as mfq
    p, n = 8, 24
    print(f"full-size Q8 24^3 vector ALU prec={prec}", flush=True)
    op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.1), p, mfq.MFQ_BC_DIRICHLET0), 0.5, prec)
    x_np = uniform_vector(op.n_dofs, seed=12)
    xin = x_np if prec == 0 else x_np.astype(np.float32).astype(np.float64)
    y = op.vmult(torch.from_numpy(xin).to(op.dtype).cuda())
    torch.cuda.synchronize()
    N1 = p * n + 1
    rng = np.random.default_rng(13)
    # random rows plus nodes on brick faces (I = 24 between x bricks 0 and 1), edges and a corner
    rows = np.concatenate([rng.integers(0, op.n_dofs, 20),
                           [24 + 7 * N1 + 9 * N1 * N1, 24 + 8 * N1 + 8 * N1 * N1, 48 + 16 * N1 + 17 * N1 * N1,
                            72 + 5 * N1 + 3 * N1 * N1, 1 + N1 + N1 * N1, N1 ** 3 // 2, 25 + 30 * N1 + 40 * N1 * N1,
                            96 + 96 * N1 + 96 * N1 * N1]])
    yo = ebe.ebe_rows(p, n, 0.1, 0.5, xin, 1, rows)
    yg = y[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    if prec == 0:
        assert np.abs(yg - yo).max() <= 1e-12 * np.abs(yo).max()
    else:
        mag = ebe.ebe_rows(p, n, 0.1, 0.5, np.abs(xin), 1, rows, magnitude=True)
        k = 8 * (p + 1) + 16
        assert np.all(np.abs(yg - yo) <= 2 * k * U32 * mag + 1e-30)


def _cheb_inputs(p, n):
    import torch
    A = _oracle(p, n)
    dinv = 1.0 / A.diagonal()
    N = A.shape[0]
    b = uniform_vector(N, seed=110 + p)
    x0 = uniform_vector(N, seed=120 + p)
    return A, dinv, b, x0, torch


@pytest.mark.parametrize("p", range(1, 9))
def test_fused_chebyshev_multibrick_fp64(p):
    """Chebyshev steps with the update fused into the cell loop (the brick completing a node
    applies it) on meshes several bricks wide, from a non-zero start that is also non-zero on the
    Dirichlet rows (identity rows): the oracle's Chebyshev to 1e-12, and bitwise the result of
    the separate operator application and vector kernel."""
    from oracle import gmg
    import paper_1910_13247_amd as mfq
    n = WIDE[p]
    print(f"fused chebyshev fp64 p={p} n={n}", flush=True)
    A, dinv, b, x0, torch = _cheb_inputs(p, n)
    lmax, lmin = 2.0, 2.0 / 15
    ref = gmg.chebyshev(lambda v: A @ v, dinv, b, x0, 4, lmin, lmax)
    op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.1), p, mfq.MFQ_BC_DIRICHLET0), 0.5, mfq.MFQ_FP64)
    out = []
    for fused in (True, False):
        op.set_fused_updates(fused)
        x = torch.from_numpy(x0.copy()).cuda()
        op.chebyshev(torch.from_numpy(dinv).cuda(), torch.from_numpy(b).cuda(), x, False, 4, lmin, lmax)
        torch.cuda.synchronize()
        out.append(x.cpu().numpy())
    err = np.abs(out[0] - ref).max() / np.abs(ref).max()
    print(f"  normwise rel err {err:.2e}")
    assert err <= 1e-12
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("x_is_zero", [True, False])
def test_fused_chebyshev_multibrick_fp32_bitwise(p, x_is_zero):
    """FP32: the fused and the separate form round alike (same expressions per entry), so the
    results are bitwise equal; and they stay within 1e-5 of the oracle's FP64 Chebyshev."""
    from oracle import gmg
    import paper_1910_13247_amd as mfq
    n = WIDE[p]
    print(f"fused chebyshev fp32 p={p} n={n} x_is_zero={x_is_zero}", flush=True)
    A, dinv, b, x0, torch = _cheb_inputs(p, n)
    lmax, lmin = 2.0, 2.0 / 15
    op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.1), p, mfq.MFQ_BC_DIRICHLET0), 0.5, mfq.MFQ_FP32)
    d32 = torch.from_numpy(dinv).float().cuda()
    b32 = torch.from_numpy(b).float().cuda()
    out = []
    for fused in (True, False):
        op.set_fused_updates(fused)
        x = torch.from_numpy(x0.copy()).float().cuda()
        op.chebyshev(d32, b32, x, x_is_zero, 5, lmin, lmax)
        torch.cuda.synchronize()
        out.append(x.cpu().numpy())
    assert np.array_equal(out[0], out[1])
    x32 = x0.astype(np.float32).astype(np.float64)
    ref = gmg.chebyshev(lambda v: A @ v, dinv.astype(np.float32).astype(np.float64),
                        b.astype(np.float32).astype(np.float64), None if x_is_zero else x32, 5, lmin, lmax)
    err = np.abs(out[0] - ref).max() / np.abs(ref).max()
    print(f"  normwise rel err vs FP64 oracle {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("p,n", [(2, 15), (4, 11), (3, 17)])
def test_fused_residual_vcycle_bitwise(p, n):
    """The solvers' V-cycle with the residual and smoother updates fused and separate: bitwise
    equal preconditioned vectors (FP32 levels, several bricks per level)."""
    import torch
    import paper_1910_13247_amd as mfq
    print(f"fused V-cycle p={p} n={n}", flush=True)
    out = []
    for fused in (True, False):
        op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.1), p, mfq.MFQ_BC_DIRICHLET0), 0.5, mfq.MFQ_FP64)
        op.set_fused_updates(fused)
        sv = mfq.Solver(op, mfq.MFQ_SOLVER_GMG_MIXED, coarse_mode=1, coarse_dofs=200)
        r = op.space.random(31)
        out.append(sv.precondition(r).cpu().numpy())
    torch.cuda.synchronize()
    assert np.all(np.isfinite(out[0]))
    assert np.array_equal(out[0], out[1])


@functools.lru_cache(maxsize=2)
def _oracle_undeformed(p, n):
    return assemble.operator_csr(p, n, 0.0, 0.5, 1)


@pytest.mark.parametrize("p", range(1, 9))
def test_undeformed_variable_coefficient_fp64(p):
    """Undeformed mesh with the variable coefficient: the cell loop reads only the diagonal of
    G_q = a(x_q) h w_q I (one value per quadrature point); vmult and vmult_add against the
    oracle's assembled matrix to 1e-12 on meshes several bricks wide."""
    import torch
    import paper_1910_13247_amd as mfq
    n = WIDE[p]
    print(f"undeformed variable coefficient fp64 p={p} n={n}", flush=True)
    op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.0), p, mfq.MFQ_BC_DIRICHLET0), 0.5, mfq.MFQ_FP64)
    x = uniform_vector(op.n_dofs, seed=130 + p)
    y0 = uniform_vector(op.n_dofs, seed=140 + p)
    xt = torch.from_numpy(x).cuda()
    y = op.vmult(xt)
    ya = op.vmult_add(xt, torch.from_numpy(y0).cuda())
    torch.cuda.synchronize()
    yo = _oracle_undeformed(p, n) @ x
    err = np.abs(y.cpu().numpy() - yo).max() / np.abs(yo).max()
    erra = np.abs(ya.cpu().numpy() - (yo + y0)).max() / np.abs(yo + y0).max()
    print(f"  normwise rel err {err:.2e}, accumulate {erra:.2e}")
    assert err <= 1e-12 and erra <= 1e-12


@pytest.mark.parametrize("p", [1, 3, 4, 6, 8])
def test_undeformed_variable_coefficient_fp32(p):
    import torch
    import paper_1910_13247_amd as mfq
    n = WIDE[p]
    print(f"undeformed variable coefficient fp32 p={p} n={n}", flush=True)
    op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.0), p, mfq.MFQ_BC_DIRICHLET0), 0.5, mfq.MFQ_FP32)
    x32 = uniform_vector(op.n_dofs, seed=150 + p).astype(np.float32).astype(np.float64)
    y = op.vmult(torch.from_numpy(x32).float().cuda())
    torch.cuda.synchronize()
    yo = _oracle_undeformed(p, n) @ x32
    mag = ebe.magnitude_bound(p, n, 0.0, 0.5, x32, 1)
    k = 8 * (p + 1) + 16
    assert np.all(np.abs(y.double().cpu().numpy() - yo) <= 2 * k * U32 * mag + 1e-30)


@functools.lru_cache(maxsize=2)
def _oracle_cartesian(p, n, bc):
    return assemble.operator_csr(p, n, 0.0, 0.0, bc)


@pytest.mark.parametrize("p", range(1, 9))
def test_cartesian_fp64(p):
    """Undeformed mesh, coefficient 1: the cell loop applies the cell matrix in its tensor-product
    form and computes its index lattice; vmult and vmult_add against the oracle's assembled matrix
    to 1e-12 on meshes several bricks wide (Dirichlet faces)."""
    import torch
    import paper_1910_13247_amd as mfq
    n = WIDE[p]
    print(f"cartesian fp64 p={p} n={n}", flush=True)
    op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.0), p, mfq.MFQ_BC_DIRICHLET0), 0.0, mfq.MFQ_FP64)
    assert op.layout()["brick"][0] == BRICK_X[p] and n > BRICK_X[p]
    x = uniform_vector(op.n_dofs, seed=160 + p)
    y0 = uniform_vector(op.n_dofs, seed=170 + p)
    xt = torch.from_numpy(x).cuda()
    y = op.vmult(xt)
    ya = op.vmult_add(xt, torch.from_numpy(y0).cuda())
    torch.cuda.synchronize()
    yo = _oracle_cartesian(p, n, 1) @ x
    err = np.abs(y.cpu().numpy() - yo).max() / np.abs(yo).max()
    erra = np.abs(ya.cpu().numpy() - (yo + y0)).max() / np.abs(yo + y0).max()
    print(f"  normwise rel err {err:.2e}, accumulate {erra:.2e}")
    assert err <= 1e-12 and erra <= 1e-12


@pytest.mark.parametrize("p", [1, 2, 4, 5, 8])
def test_cartesian_fp32(p):
    import torch
    import paper_1910_13247_amd as mfq
    n = WIDE[p]
    print(f"cartesian fp32 p={p} n={n}", flush=True)
    op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.0), p, mfq.MFQ_BC_DIRICHLET0), 0.0, mfq.MFQ_FP32)
    x32 = uniform_vector(op.n_dofs, seed=180 + p).astype(np.float32).astype(np.float64)
    y = op.vmult(torch.from_numpy(x32).float().cuda())
    torch.cuda.synchronize()
    yo = _oracle_cartesian(p, n, 1) @ x32
    mag = ebe.magnitude_bound(p, n, 0.0, 0.0, x32, 1)
    k = 8 * (p + 1) + 16
    assert np.all(np.abs(y.double().cpu().numpy() - yo) <= 2 * k * U32 * mag + 1e-30)


@pytest.mark.parametrize("p", [2, 4, 7])
def test_cartesian_natural_boundary(p):
    """The same without Dirichlet faces (every node free, the computed index lattice marks none)."""
    import torch
    import paper_1910_13247_amd as mfq
    n = WIDE[p]
    print(f"cartesian natural bc p={p} n={n}", flush=True)
    op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.0), p, 0), 0.0, mfq.MFQ_FP64)
    x = uniform_vector(op.n_dofs, seed=190 + p)
    y = op.vmult(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    yo = _oracle_cartesian(p, n, 0) @ x
    assert np.abs(y.cpu().numpy() - yo).max() <= 1e-12 * np.abs(yo).max()
