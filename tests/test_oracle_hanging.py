"""Pins of the hanging-node oracle (two-block mesh, 2:1 interface; Sec. 3.3 of the paper):
exactness of the interface interpolation on polynomials, agreement of each block with the pinned
single-block operator where they coincide, symmetry, the Neumann kernel, definiteness, and exact
reproduction of a degree-2 solution across the interface (affine) or of its analytic bilinear form
(curved, variable coefficient), which a wrong constraint row, offset or mask fails."""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg as spla

from oracle import assemble, geometry, hanging
from oracle.tables import gll_nodes


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_interface_interpolation_exact_on_polynomials(p, n):
    Pi = hanging.interface_interpolation(p, n)
    xc = hanging.lattice_1d(p, n)
    xf = hanging.lattice_1d(p, 2 * n)
    assert Pi.shape == (2 * p * n + 1, p * n + 1)
    np.testing.assert_allclose(Pi.sum(1), 1.0, atol=1e-13)
    for deg in range(p + 1):
        np.testing.assert_allclose(Pi @ xc ** deg, xf ** deg, atol=1e-12)
    # not exact beyond degree p on a single coarse cell (the constraint is not an identity)
    if n == 1:
        assert np.abs(Pi @ xc ** (p + 1) - xf ** (p + 1)).max() > 1e-6
    # fine nodes at coarse cell vertices copy the coarse vertex value
    for c in range(n + 1):
        row = Pi[2 * p * c]
        assert row[p * c] == pytest.approx(1.0, abs=1e-14) and np.abs(row).sum() == pytest.approx(1.0, abs=1e-13)


def test_interface_interpolation_p2_closed_form():
    # p = 2 on one coarse cell: GLL nodes 0, 1/2, 1; fine nodes 0, 1/4, 1/2, 3/4, 1; quadratic
    # Lagrange weights at 1/4: (3/8, 3/4, -1/8)
    Pi = hanging.interface_interpolation(2, 1)
    np.testing.assert_allclose(Pi[1], [3 / 8, 3 / 4, -1 / 8], atol=1e-15)
    np.testing.assert_allclose(Pi[3], [-1 / 8, 3 / 4, 3 / 8], atol=1e-15)
    np.testing.assert_allclose(Pi[2], [0, 1, 0], atol=1e-15)


@pytest.mark.parametrize("p,n,A,alpha", [(2, 2, 0.1, 0.5), (3, 1, 0.0, 0.0), (1, 3, 0.1, 0.3)])
def test_block0_is_the_single_block_operator(p, n, A, alpha):
    B0 = hanging.block_matrix(p, n, 0.0, A, alpha)
    ref = assemble.assemble_csr(p, n, A, alpha)
    assert abs(B0 - ref).max() <= 1e-15 * abs(ref).max()


@pytest.mark.parametrize("p,n", [(2, 1), (3, 2)])
def test_block1_affine_is_a_translated_single_block(p, n):
    # undeformed, coefficient 1: the fine block is the (2n)^3 unit-cube operator translated by X1 = 1
    B1 = hanging.block_matrix(p, 2 * n, 1.0, 0.0, 0.0)
    ref = assemble.assemble_csr(p, 2 * n, 0.0, 0.0)
    assert abs(B1 - ref).max() <= 1e-13 * abs(ref).max()


def test_block1_uses_the_shifted_map():
    # with a deformation the fine block is not a translated copy: sin(pi X1) changes sign at X1 = 1
    B1 = hanging.block_matrix(2, 2, 1.0, 0.1, 0.5)
    ref = assemble.assemble_csr(2, 2, 0.1, 0.5)
    assert abs(B1 - ref).max() > 1e-4 * abs(ref).max()


@pytest.mark.parametrize("p,n,A,alpha", [(1, 2, 0.0, 0.0), (2, 1, 0.1, 0.5), (3, 1, 0.1, 0.5), (2, 2, 0.1, 0.9)])
def test_symmetry_kernel_definiteness(p, n, A, alpha):
    hang = hanging.hanging_mask(p, n)
    An = hanging.operator_csr(p, n, A, alpha, bc=0)
    assert abs(An - An.T).max() <= 1e-14 * abs(An).max()
    y = An @ np.ones(An.shape[0])
    assert np.abs(y[~hang]).max() <= 1e-12 * abs(An).max()
    np.testing.assert_array_equal(y[hang], 1.0)
    Ad = hanging.operator_csr(p, n, A, alpha, bc=1)
    assert abs(Ad - Ad.T).max() <= 1e-14 * abs(Ad).max()
    scipy.linalg.cholesky(Ad.toarray())          # SPD


def _ustar(X):
    return X[..., 0] * (2 - X[..., 0]) * X[..., 1] * (1 - X[..., 1]) * X[..., 2] * (1 - X[..., 2])


def _minus_lap_ustar(X):
    x, y, z = X[..., 0], X[..., 1], X[..., 2]
    return 2 * (y * (1 - y) * z * (1 - z) + x * (2 - x) * z * (1 - z) + x * (2 - x) * y * (1 - y))


@pytest.mark.parametrize("p,n", [(2, 1), (2, 2), (3, 1), (4, 1)])
def test_galerkin_exact_across_the_interface(p, n):
    """u* = X1 (2 - X1) X2 (1 - X2) X3 (1 - X3) is in the conforming Q_p space for p >= 2 and vanishes
    on the boundary: the discrete solution with the load of -Laplace u* equals u* at every node,
    hanging nodes included once distributed."""
    At = hanging.operator_csr(p, n, 0.0, 0.0, bc=1)
    b = hanging.load_vector(p, n, 0.0, 0.0, _minus_lap_ustar)
    x = spla.spsolve(At.tocsc(), b)
    X = hanging.node_coords(p, n)
    hang = hanging.hanging_mask(p, n)
    ref = _ustar(X)
    np.testing.assert_allclose(x[~hang], ref[~hang], atol=1e-12)
    np.testing.assert_allclose(hanging.distribute(p, n, x), ref, atol=1e-12)


@pytest.mark.parametrize("p,n", [(2, 1), (3, 1)])
def test_curved_bilinear_form_of_a_conforming_polynomial(p, n):
    """Curved map, variable coefficient: u(X) = X1^2 X2 + X3 (degree 2 in X, so in the pulled-back
    Q_p space on both sides of the interface).  (C^T A C u)_i must equal the cell loop's
    sum_q a grad_x u . grad_x phi_i JxW with grad_x u from the analytic chain rule
    J_F^{-T} grad_X u (no nodal interpolation of u); with bc = 0 on every independent row."""
    A, alpha = 0.1, 0.5
    hang = hanging.hanging_mask(p, n)
    X = hanging.node_coords(p, n)
    u = X[:, 0] ** 2 * X[:, 1] + X[:, 2]
    y = hanging.operator_csr(p, n, A, alpha, bc=0) @ np.where(hang, 0.0, u)

    from oracle.element import reference_tabulation
    _, B = reference_tabulation(p)
    zhat, wq = geometry.reference_qpoints(p)
    Cx = hanging.expansion(p, n)
    N0, _, N = hanging.sizes(p, n)
    full = np.zeros(N)
    for nb, x0, off in ((n, 0.0, 0), (2 * n, 1.0, N0)):
        hb = 1.0 / nb
        org, dofs = hanging._block_cells(p, nb, x0, hb)
        Xq = org[:, None, :] + hb * zhat[None, :, :]
        xq = geometry.deformation(Xq, A)
        JF = geometry.deformation_jacobian(Xq, A)                       # dx/dX
        gX = np.stack([2 * Xq[..., 0] * Xq[..., 1], Xq[..., 0] ** 2, np.ones(Xq.shape[:-1])], -1)
        gx = np.linalg.solve(np.swapaxes(JF, -1, -2), gX[..., None])[..., 0]   # J_F^{-T} grad_X u
        J = hb * JF                                                      # dx/dxhat
        Jinv = np.linalg.inv(J)
        coef = geometry.coefficient(xq, alpha) * np.linalg.det(J) * wq[None, :]
        # grad_x phi_i = J^{-T} grad_xhat phi_i;  term_i = sum_q coef (gx . J^{-T} B_i)
        v = np.einsum("cqdk,cqk->cqd", Jinv, gx * coef[..., None])      # J^{-1} (coef gx), contracted with B
        cell = np.einsum("cqd,qdi->ci", v, B)
        np.add.at(full, off + dofs.reshape(-1), cell.reshape(-1))
    ref = Cx.T @ full
    scale = np.abs(ref).max()
    assert np.abs(y[~hang] - ref[~hang]).max() <= 1e-12 * scale


def test_dirichlet_and_hanging_masks():
    p, n = 2, 1
    N0, N1, N = hanging.sizes(p, n)
    assert (N0, N1) == (27, 125)
    hang = hanging.hanging_mask(p, n)
    assert hang.sum() == 25 and not hang[:N0].any()
    m = hanging.dirichlet_mask(p, n)
    # block 0: the 3x3 interface face minus its boundary ring is free; interior node (1,1,1) too
    L0 = 3
    assert m[1 + L0 * 1 + L0 * L0 * 1] == 1 and m[2 + L0 * 1 + L0 * L0 * 1] == 1
    assert m[0 + L0 * 1 + L0 * L0 * 1] == 0 and m[2 + L0 * 0 + L0 * L0 * 1] == 0
    # block 1: its X1 = 2 face is boundary, X1 = 1 face hanging (mask 1 there)
    L1 = 5
    assert m[N0 + 4 + L1 * 2 + L1 * L1 * 2] == 0 and m[N0 + 2 + L1 * 2 + L1 * L1 * 2] == 1
    assert m[N0 + 0 + L1 * 2 + L1 * L1 * 2] == 1
    # GLL nodes used on both lattices
    np.testing.assert_allclose(hanging.lattice_1d(3, 1), gll_nodes(3), atol=1e-15)


def test_block_matrix_chunking_is_exact():
    a = hanging.block_matrix(2, 2, 1.0, 0.1, 0.5, chunk=3)
    b = hanging.block_matrix(2, 2, 1.0, 0.1, 0.5, chunk=64)
    assert abs(a - b).max() <= 1e-15 * abs(b).max()


def test_magnitude_bounds_the_operator_entrywise():
    p, n = 2, 1
    At = hanging.operator_csr(p, n, 0.1, 0.5)
    M = hanging.magnitude_csr(p, n, 0.1, 0.5)
    assert (abs(At) - M).max() <= 1e-15 * M.max()
    # and is not the operator's own absolute value where the constraint combines couplings
    assert abs(M - abs(At)).max() > 1e-6 * M.max()
