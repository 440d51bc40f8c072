"""Pins of the DG-SIPG oracle (oracle/dg.py) against properties fixed by the mathematics:
symmetry, positive definiteness on small meshes, and consistency: for p >= 2 the function
u = x(1-x) y(1-y) z(1-z) lies in the space and vanishes on the boundary, so the discrete operator
applied to it must reproduce the load vector of f = -lap u exactly (the face terms of integration
by parts cancel against the consistency terms only with the right signs, normals and factors)."""
import numpy as np
import pytest

from oracle import assemble, dg, mesh


def _u(x, y, z):
    return x * (1 - x) * y * (1 - y) * z * (1 - z)


def _f(x, y, z):
    return 2 * (y * (1 - y) * z * (1 - z) + x * (1 - x) * z * (1 - z) + x * (1 - x) * y * (1 - y))


@pytest.mark.parametrize("p,n", [(1, 2), (2, 2), (3, 3), (4, 2)])
def test_symmetric(p, n):
    A = dg.assemble(p, n)
    assert A.shape == (dg.n_dofs(p, n),) * 2
    assert abs(A - A.T).max() <= 1e-13 * abs(A).max()


@pytest.mark.parametrize("p,n", [(1, 1), (1, 2), (2, 2), (3, 1)])
def test_positive_definite(p, n):
    w = np.linalg.eigvalsh(dg.assemble(p, n).toarray())
    assert w.min() > 0


@pytest.mark.parametrize("p,n", [(2, 1), (2, 3), (3, 2), (4, 2), (5, 1)])
def test_consistency_with_a_polynomial_solution(p, n):
    A = dg.assemble(p, n)
    u = dg.nodal_interpolant(p, n, _u)
    F = dg.load_vector(p, n, _f)
    assert np.abs(A @ u - F).max() <= 1e-11 * np.abs(F).max()


def test_wrong_penalty_sign_breaks_definiteness():
    # the penalty keeps the form coercive: without it (sigma = 0) the matrix is indefinite
    p, n = 2, 2
    tr, dn, W = dg._face_tables(p, n)
    M0 = dg.face_matrix(np.hstack([tr[0][1], -tr[0][0]]), 0.5 * np.hstack([dn[0][1], dn[0][0]]), W, 0.0)
    assert np.linalg.eigvalsh(M0).min() < 0


def test_sampled_rows_match_assembly():
    p, n = 3, 3
    A = dg.assemble(p, n)
    x = np.random.default_rng(0).uniform(-1, 1, dg.n_dofs(p, n))
    rows = np.random.default_rng(1).integers(0, dg.n_dofs(p, n), 60)
    y = A @ x
    assert np.abs(dg.dg_rows(p, n, x, rows) - y[rows]).max() <= 1e-12 * np.abs(y).max()


def _v(x, y, z):
    # vanishes on the boundary, different along each axis (a transposed index changes it)
    return x * (1 - x) * (1 + 2 * x) * y * (1 - y) * z * (1 - z) * (2 - z) ** 2


@pytest.mark.parametrize("p,n", [(1, 3), (2, 2), (3, 2), (4, 2)])
def test_embedding_maps_nodal_values(p, n):
    """E applied to the continuous nodal interpolant is the DG nodal interpolant of the same
    function (both spaces interpolate at the GLL nodes of every cell)."""
    E = dg.cg_embedding(p, n)
    X = mesh.node_coords(p, n)
    c = _v(X[:, 0], X[:, 1], X[:, 2])
    assert np.abs(E @ c - dg.nodal_interpolant(p, n, _v)).max() <= 1e-15
    # every DG DoF on an interior lattice node gets exactly one value; boundary rows are empty
    assert set(np.unique(E.sum(axis=1).A.ravel())) <= {0.0, 1.0}


@pytest.mark.parametrize("p,n", [(1, 3), (2, 2), (3, 2), (4, 1), (4, 2)])
def test_galerkin_product_is_the_continuous_operator(p, n):
    """For continuous functions vanishing on the boundary every jump is zero, so all face terms
    of the SIPG form vanish and E^T A_DG E is the continuous stiffness matrix on the free nodes
    (a face term that survives on continuous functions, such as a jump with the wrong sign or a
    trace taken at the wrong end, or a wrong index in E breaks this)."""
    E = dg.cg_embedding(p, n)
    G = (E.T @ dg.assemble(p, n) @ E).toarray()
    m = mesh.boundary_mask(p, n)
    Acg = assemble.assemble_csr(p, n, 0.0, 0.0).toarray() * np.outer(m, m)
    assert np.abs(G - Acg).max() <= 1e-11 * np.abs(Acg).max()


@pytest.mark.parametrize("p,n", [(1, 2), (3, 2), (4, 1)])
def test_magnitude_bounds_the_matrix(p, n):
    """The magnitude matrix bounds |A| entrywise, and its cell part has the cell matrix's
    diagonal (a sum of squares has no cancellation)."""
    A = dg.assemble(p, n).toarray()
    M = dg.assemble(p, n, magnitude=True).toarray()
    assert np.all(np.abs(A) <= M * (1 + 1e-13) + 1e-15)
    # diagonal of the cell term: a sum of squares, so no cancellation
    Ac = dg.element_matrices(p, n, 0.0, 0.0, np.array([0]))[0]
    assert np.allclose(np.diag(dg.cell_magnitude(p, n)), np.diag(Ac), rtol=1e-13)


def _dg_multigrid(p, n):
    from oracle import gmg
    A = dg.assemble(p, n)
    dinv = 1.0 / A.diagonal()
    E = dg.cg_embedding(p, n)
    levels, prolong = gmg.build_hierarchy(p, n, 0.0, 0.0, bc=1)
    for L in levels[1:]:
        L.estimate()
    v0 = gmg.splitmix64_uniform(A.shape[0], 0)
    lmax = 1.2 * gmg.lanczos_lambda_max(lambda v: A @ v, dinv, v0, 12)
    return A, dinv, E, levels, prolong, lmax


@pytest.mark.parametrize("p,n", [(1, 2), (2, 2)])
def test_dg_vcycle_is_a_convergent_symmetric_preconditioner(p, n):
    """The V-cycle as a matrix M (columns from unit vectors): symmetric (the same smoother before
    and after, E^T and E, an exact symmetric coarse solve), positive definite, and I - M A
    contracts (spectral radius well below 1)."""
    A, dinv, E, levels, prolong, lmax = _dg_multigrid(p, n)
    N = A.shape[0]
    M = np.column_stack([dg.vcycle(A, dinv, E, np.eye(N)[:, j], lmax / 15, lmax, levels, prolong)
                         for j in range(N)])
    assert np.abs(M - M.T).max() <= 1e-10 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    rho = np.abs(np.linalg.eigvals(np.eye(N) - M @ A.toarray())).max()
    assert rho < 0.3, rho


def test_sampled_magnitude_rows_match_assembly():
    p, n = 2, 3
    M = dg.assemble(p, n, magnitude=True)
    x = np.abs(np.random.default_rng(2).uniform(-1, 1, dg.n_dofs(p, n)))
    rows = np.random.default_rng(3).integers(0, dg.n_dofs(p, n), 40)
    y = M @ x
    assert np.abs(dg.dg_rows(p, n, x, rows, magnitude=True) - y[rows]).max() <= 1e-12 * np.abs(y).max()
