"""GPU parity of the HIP path (through the C ABI) against the CPU oracle, element by element.

Sizes span several workgroups (256 // (p+1)^2 cells each) with a ragged last one.  FP64 bar:
||y - y_oracle||_inf <= 1e-12 ||y_oracle||_inf.  FP32 bar: |y32 - y_oracle| <= 2 k u32 m
componentwise, with m = (sum_q |B_q|^T |G_q| |B_q|) |x| the magnitude of the summed terms and
k = 8(p+1) + 16 the longest chain of roundings (eight 1D contractions forward and back, the
3x3 product, the stored G and input roundings, up to 8 cell contributions per node).
"""
import numpy as np
import pytest

from oracle import assemble, ebe, geometry, gmg, mesh, rhs
from synthetic import uniform_vector

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
# (p, n): n chosen so that n^3 cells fill more than one workgroup with a partial last one
SIZES = {1: 5, 2: 4, 3: 3, 4: 3, 5: 2, 6: 2, 7: 3, 8: 2}


def _mfq():
    import paper_1910_13247_amd as mfq
    return mfq


def _torch():
    import torch
    return torch


def _op(p, n, amp, alpha, bc, prec):
    mfq = _mfq()
    m = mfq.Mesh(n, amp)
    s = mfq.Space(m, p, bc)
    return mfq.Operator(s, alpha, prec)


def _run(op, x_np):
    torch = _torch()
    x = torch.from_numpy(x_np).to(op.dtype).cuda()
    y = op.vmult(x)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("amp,alpha,bc", [(0.0, 0.0, 1), (0.1, 0.5, 1), (0.1, 0.5, 0)])
def test_vmult_fp64_matches_assembled_matrix(p, amp, alpha, bc):
    n = SIZES[p]
    print(f"vmult fp64 p={p} n={n} amp={amp} alpha={alpha} bc={bc}", flush=True)
    mfq = _mfq()
    op = _op(p, n, amp, alpha, bc, mfq.MFQ_FP64)
    x = uniform_vector(op.n_dofs, seed=p)
    y = _run(op, x)
    yo = assemble.operator_csr(p, n, amp, alpha, bc) @ x
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()


@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("amp,alpha", [(0.1, 0.5), (0.0, 0.0)])
def test_vmult_fp32_within_rounding_bound(p, amp, alpha):
    """(0, 0): undeformed cells, coefficient 1, the path that forms G_q = h w I in registers."""
    n = SIZES[p]
    mfq = _mfq()
    op = _op(p, n, amp, alpha, 1, mfq.MFQ_FP32)
    x = uniform_vector(op.n_dofs, seed=10 + p)
    x32 = x.astype(np.float32).astype(np.float64)     # the input the FP32 path sees
    y = _run(op, x)
    yo = assemble.operator_csr(p, n, amp, alpha, 1) @ x32
    mag = ebe.magnitude_bound(p, n, amp, alpha, x32, 1)
    k = 8 * (p + 1) + 16
    assert np.all(np.abs(y - yo) <= 2 * k * U32 * mag + 1e-30)
    print(f"p={p} fp32 normwise rel err {np.abs(y - yo).max() / np.abs(yo).max():.2e}")


@pytest.mark.parametrize("p", range(1, 9))
def test_vmult_fp32_mfma_within_rounding_bound(p):
    """The matrix-core form of the FP32 operator: the same componentwise bound as the VALU FP32
    path (each MFMA dot product sums at most p+1 terms in FP32, the padding adds exact zeros), and
    both FP32 forms within twice that bound of each other."""
    n = SIZES[p]
    mfq = _mfq()
    print(f"vmult fp32 mfma p={p} n={n}", flush=True)
    opm = _op(p, n, 0.1, 0.5, 1, mfq.MFQ_FP32_MFMA)
    opv = _op(p, n, 0.1, 0.5, 1, mfq.MFQ_FP32)
    x = uniform_vector(opm.n_dofs, seed=20 + p)
    x32 = x.astype(np.float32).astype(np.float64)
    ym = _run(opm, x)
    yv = _run(opv, x)
    yo = assemble.operator_csr(p, n, 0.1, 0.5, 1) @ x32
    mag = ebe.magnitude_bound(p, n, 0.1, 0.5, x32, 1)
    k = 8 * (p + 1) + 16
    assert np.all(np.abs(ym - yo) <= 2 * k * U32 * mag + 1e-30)
    assert np.all(np.abs(ym - yv) <= 4 * k * U32 * mag + 1e-30)
    print(f"p={p} fp32-mfma normwise rel err {np.abs(ym - yo).max() / np.abs(yo).max():.2e}")


@pytest.mark.parametrize("p,n", [(8, 5), (6, 4), (3, 9)])
def test_vmult_fp32_mfma_accumulate_and_dirichlet(p, n):
    """dst += A src on the matrix-core path equals dst + A src of the VALU path (same bound)."""
    mfq = _mfq()
    torch = _torch()
    opm = _op(p, n, 0.1, 0.5, 1, mfq.MFQ_FP32_MFMA)
    x = torch.from_numpy(uniform_vector(opm.n_dofs, seed=3)).float().cuda()
    d0 = torch.from_numpy(uniform_vector(opm.n_dofs, seed=4)).float().cuda()
    d = d0.clone()
    opm.vmult_add(x, d)
    y = opm.vmult(x)
    torch.cuda.synchronize()
    ref = (d0.double() + y.double()).cpu().numpy()
    got = d.double().cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    # Dirichlet rows: identity on the input
    bmask = mesh.boundary_mask(p, n) == 0
    np.testing.assert_array_equal(y.cpu().numpy()[bmask], x.cpu().numpy()[bmask])


def test_sampled_parity_full_size_q8_24_mfma():
    """The high-degree workload at full size (Q8 on the curved 24^3 mesh, 7,189,057 DoFs) on the
    matrix cores: sampled rows recomputed by the oracle cell by cell, within the FP32 bound."""
    mfq = _mfq()
    torch = _torch()
    p, n = 8, 24
    print("full-size sampled parity Q8 24^3 fp32-mfma", flush=True)
    op = _op(p, n, 0.1, 0.5, 1, mfq.MFQ_FP32_MFMA)
    x_np = uniform_vector(op.n_dofs, seed=5)
    x32 = x_np.astype(np.float32).astype(np.float64)
    y = op.vmult(torch.from_numpy(x32).float().cuda())
    torch.cuda.synchronize()
    N1 = p * n + 1
    rng = np.random.default_rng(2)
    rows = np.concatenate([rng.integers(0, op.n_dofs, 8), [1 + N1 + N1 * N1, N1 * N1 * N1 // 2,
                                                            8 + 8 * N1 + 8 * N1 * N1, 9 + 17 * N1 + 100 * N1 * N1]])
    yo = ebe.ebe_rows(p, n, 0.1, 0.5, x32, 1, rows)
    mag = ebe.ebe_rows(p, n, 0.1, 0.5, np.abs(x32), 1, rows, magnitude=True)
    yg = y[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    k = 8 * (p + 1) + 16
    assert np.all(np.abs(yg - yo) <= 2 * k * U32 * mag + 1e-30)


def test_poisson_q2_8_vmult():
    # the small Poisson workload: Q2 on 8^3 affine cells (4,913 DoFs), applied to the seeded f
    mfq = _mfq()
    op = _op(2, 8, 0.0, 0.0, 1, mfq.MFQ_FP64)
    assert op.n_dofs == 4913
    f = uniform_vector(4913, seed=0)
    y = _run(op, f)
    yo = assemble.operator_csr(2, 8, 0.0, 0.0, 1) @ f
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()


@pytest.mark.parametrize("p,n", [(1, 1), (2, 1), (8, 1)])
@pytest.mark.parametrize("amp,alpha", [(0.1, 0.5), (0.0, 0.0)])
def test_single_cell_degenerate(p, n, amp, alpha):
    # one cell: with Dirichlet rows every node but the interior ones is the identity (curved, and
    # the Cartesian instance with its tensor-product cell term and computed index lattice)
    mfq = _mfq()
    op = _op(p, n, amp, alpha, 1, mfq.MFQ_FP64)
    x = uniform_vector(op.n_dofs, seed=3)
    y = _run(op, x)
    yo = assemble.operator_csr(p, n, amp, alpha, 1) @ x
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()
    if p == 1:
        np.testing.assert_array_equal(y, x)


def test_vmult_repeatable_and_linear():
    mfq = _mfq()
    torch = _torch()
    op = _op(3, 4, 0.1, 0.5, 1, mfq.MFQ_FP64)
    x = torch.from_numpy(uniform_vector(op.n_dofs, 5)).cuda()
    z = torch.from_numpy(uniform_vector(op.n_dofs, 6)).cuda()
    y1 = op.vmult(x)
    y2 = op.vmult(x)
    lin = op.vmult(2.0 * x + z) - (2.0 * y1 + op.vmult(z))
    torch.cuda.synchronize()
    assert (y1 - y2).abs().max().item() <= 1e-14 * y1.abs().max().item()
    assert lin.abs().max().item() <= 1e-13 * y1.abs().max().item()


@pytest.mark.parametrize("p,n", [(2, 3), (4, 2), (8, 1)])
@pytest.mark.parametrize("prec", [0, 1])
def test_geometry_matches_oracle(p, n, prec):
    op = _op(p, n, 0.1, 0.5, 1, prec)
    g = op.geometry().cpu().numpy()                 # [cells][q][6]
    G = geometry.qpoint_data(p, n, 0.1, 0.5)["G"]    # [cells][q][3][3]
    ref = np.stack([G[..., 0, 0], G[..., 0, 1], G[..., 0, 2], G[..., 1, 1], G[..., 1, 2], G[..., 2, 2]], -1)
    tol = 1e-14 if prec == 0 else 2 * U32
    assert np.abs(g - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("amp,alpha,bc", [(0.1, 0.5, 1), (0.0, 0.0, 1), (0.1, 0.5, 0)])
def test_diagonal_matches_assembled(p, amp, alpha, bc):
    """The operator's diagonal (sum-factorised per cell, colour-ordered node sums) against the
    diagonal of the oracle's assembled matrix, FP64, all degrees, ragged bricks."""
    mfq = _mfq()
    n = SIZES[p]
    op = _op(p, n, amp, alpha, bc, mfq.MFQ_FP64)
    d = op.diagonal().cpu().numpy()
    do = assemble.operator_csr(p, n, amp, alpha, bc).diagonal()
    assert np.abs(d - do).max() <= 1e-13 * np.abs(do).max()


@pytest.mark.parametrize("p", range(1, 9))
def test_diagonal_fp32_within_rounding_bound(p):
    """FP32 diagonal within k u32 of the summed magnitudes: the regrouped 1D contractions mix
    signs, so the bound is taken on sum_q |B_q|^T |G_q| |B_q| (its row sums bound each diagonal
    entry's terms); k = 4(p+1) + 16 (stored G, three contractions of p+1 terms, up to 8 cell
    contributions).  Dirichlet rows are exactly 1."""
    mfq = _mfq()
    n = SIZES[p]
    op = _op(p, n, 0.1, 0.5, 1, mfq.MFQ_FP32)
    d = op.diagonal().double().cpu().numpy()
    do = assemble.operator_csr(p, n, 0.1, 0.5, 1).diagonal()
    mag = ebe.magnitude_bound(p, n, 0.1, 0.5, np.ones(op.n_dofs), 1)
    k = 4 * (p + 1) + 16
    assert np.all(np.abs(d - do) <= k * U32 * mag + 1e-30)
    m = mesh.boundary_mask(p, n) == 0
    assert np.all(d[m] == 1.0)


@pytest.mark.parametrize("p,n", [(1, 4), (3, 3), (4, 2)])
def test_rhs_manufactured_matches_oracle(p, n):
    mfq = _mfq()
    op = _op(p, n, 0.1, 0.5, 1, mfq.MFQ_FP64)
    b = op.rhs_manufactured().cpu().numpy()
    bo = rhs.rhs_manufactured(p, n, 0.1, 0.5, 1)
    assert np.abs(b - bo).max() <= 1e-12 * np.abs(bo).max()


@pytest.mark.parametrize("pc,nc,pf,nf", [(1, 2, 1, 4), (2, 2, 2, 4), (3, 1, 3, 2), (2, 3, 3, 3), (4, 2, 8, 2)])
@pytest.mark.parametrize("prec", [0, 1])
def test_transfer_matches_interpolation_matrix(pc, nc, pf, nf, prec):
    mfq = _mfq()
    torch = _torch()
    mc, mf = mfq.Mesh(nc, 0.1), mfq.Mesh(nf, 0.1)
    sc, sf = mfq.Space(mc, pc, 1), mfq.Space(mf, pf, 1)
    tr = mfq.Transfer(sc, sf)
    P = gmg.prolongation(pc, nc, pf, nf, bc=1)
    dt = torch.float64 if prec == 0 else torch.float32
    u = uniform_vector(sc.n_dofs, 7)
    v = uniform_vector(sf.n_dofs, 8)
    fine = torch.empty(sf.n_dofs, dtype=dt, device="cuda")
    coarse = torch.empty(sc.n_dofs, dtype=dt, device="cuda")
    tr.prolongate(torch.from_numpy(u).to(dt).cuda(), fine, prec)
    tr.restrict(torch.from_numpy(v).to(dt).cuda(), coarse, prec)
    torch.cuda.synchronize()
    u_in = u if prec == 0 else u.astype(np.float32).astype(np.float64)
    v_in = v if prec == 0 else v.astype(np.float32).astype(np.float64)
    tol = 1e-14 if prec == 0 else 64 * U32
    pf_ref = P @ u_in
    rc_ref = P.T @ v_in
    assert np.abs(fine.double().cpu().numpy() - pf_ref).max() <= tol * max(1, np.abs(pf_ref).max())
    assert np.abs(coarse.double().cpu().numpy() - rc_ref).max() <= tol * max(1, np.abs(rc_ref).max()) * (pf + 1)


@pytest.mark.parametrize("x_is_zero", [True, False])
def test_chebyshev_matches_oracle(x_is_zero):
    mfq = _mfq()
    torch = _torch()
    p, n = 3, 3
    op = _op(p, n, 0.1, 0.5, 1, mfq.MFQ_FP64)
    At = assemble.operator_csr(p, n, 0.1, 0.5, 1)
    dinv = 1.0 / At.diagonal()
    lmax, lmin = 2.1, 2.1 / 15
    b = mesh.boundary_mask(p, n) * uniform_vector(op.n_dofs, 11)
    x0 = mesh.boundary_mask(p, n) * uniform_vector(op.n_dofs, 12)
    ref = gmg.chebyshev(lambda v: At @ v, dinv, b, None if x_is_zero else x0, 3, lmin, lmax)
    x = torch.from_numpy(x0.copy()).cuda()
    op.chebyshev(torch.from_numpy(dinv).cuda(), torch.from_numpy(b).cuda(), x, x_is_zero, 3, lmin, lmax)
    torch.cuda.synchronize()
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_sampled_parity_full_size_q4_64_curved():
    # the 64^3-cell Q4 curved variable-coefficient operator at full size (16,974,593 DoFs), in the
    # launch configuration the benchmark times; 600 sampled rows recomputed by the oracle cell by cell
    mfq = _mfq()
    torch = _torch()
    p, n = 4, 64
    print("full-size sampled parity Q4 64^3", flush=True)
    op = _op(p, n, 0.1, 0.5, 1, mfq.MFQ_FP64)
    x_np = uniform_vector(op.n_dofs, seed=0)
    x = torch.from_numpy(x_np).cuda()
    y = op.vmult(x)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    N1 = p * n + 1
    rows = np.concatenate([rng.integers(0, op.n_dofs, 560),
                           [0, N1 * N1 * N1 - 1, 1 + N1 + N1 * N1, N1 * N1 * N1 // 2, 4 + 4 * N1 + 4 * N1 * N1]])
    yo = ebe.ebe_rows(p, n, 0.1, 0.5, x_np, 1, rows)
    yg = y[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert np.abs(yg - yo).max() <= 1e-12 * np.abs(yo).max()


def test_sampled_parity_full_size_q4_64_fp32():
    """The FP32 operator at the benchmark's full size (Q4 curved 64^3): 400 sampled rows against
    the oracle applied to the FP32-rounded input, to the componentwise FP32 bound."""
    mfq = _mfq()
    torch = _torch()
    p, n = 4, 64
    print("full-size sampled parity Q4 64^3 FP32", flush=True)
    op = _op(p, n, 0.1, 0.5, 1, mfq.MFQ_FP32)
    x_np = uniform_vector(op.n_dofs, seed=0)
    x32 = x_np.astype(np.float32).astype(np.float64)
    y = op.vmult(torch.from_numpy(x_np).float().cuda())
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    N1 = p * n + 1
    rows = np.concatenate([rng.integers(0, op.n_dofs, 400), [1 + N1 + N1 * N1, N1 ** 3 // 2]])
    yo = ebe.ebe_rows(p, n, 0.1, 0.5, x32, 1, rows)
    mag = ebe.ebe_rows(p, n, 0.1, 0.5, np.abs(x32), 1, rows, magnitude=True)
    yg = y[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    k = 8 * (p + 1) + 16
    assert np.all(np.abs(yg - yo) <= 2 * k * U32 * mag + 1e-30)
