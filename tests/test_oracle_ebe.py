"""Pins of the oracle's cell-by-cell forms: ``ebe_rows`` (sampled rows of A x and of the magnitude
bound) and ``magnitude_bound`` (the scale of every FP32 tolerance).

* ``ebe_rows`` over every row equals the assembled operator applied to x (both geometries, both
  boundary treatments): its own cell/local-index arithmetic against the assembled matrix;
* ``ebe_rows(magnitude=True)`` over every row equals ``magnitude_bound``;
* on the affine mesh with coefficient 1 (G_q = h w_q I) the magnitude matrix separates like the
  operator does, into a Kronecker sum of 1D matrices built from |l_a| and |l_a'| at the Gauss
  points, evaluated here from numpy's Legendre series and Gauss rule (independent of the oracle's
  tables, tabulation and assembly);
* the magnitude matrix bounds the operator entrywise, |A| <= M (triangle inequality), and its
  diagonal equals A's wherever G_q is diagonal and positive (affine mesh).
"""
import numpy as np
import numpy.polynomial.legendre as npleg
import pytest
import scipy.sparse as sp

from oracle import assemble, mesh
from oracle.ebe import ebe_rows, magnitude_bound
from oracle.tables import gll_nodes
from synthetic import uniform_vector

CASES = [(1, 3), (2, 3), (3, 2), (4, 2)]
GEOMS = [(0.0, 0.0), (0.1, 0.5)]


@pytest.mark.parametrize("p,n", CASES)
@pytest.mark.parametrize("amp,alpha", GEOMS)
@pytest.mark.parametrize("bc", [0, 1])
def test_ebe_rows_all_rows_equal_assembled_operator(p, n, amp, alpha, bc):
    At = assemble.operator_csr(p, n, amp, alpha, bc)
    x = uniform_vector(At.shape[0], seed=40 + p)
    rows = np.arange(At.shape[0])
    y = ebe_rows(p, n, amp, alpha, x, bc, rows)
    yo = At @ x
    assert np.abs(y - yo).max() <= 1e-13 * np.abs(yo).max()


@pytest.mark.parametrize("p,n", CASES)
@pytest.mark.parametrize("amp,alpha", GEOMS)
@pytest.mark.parametrize("bc", [0, 1])
def test_ebe_rows_magnitude_equals_magnitude_bound(p, n, amp, alpha, bc):
    N = mesh.n_dofs(p, n)
    x = uniform_vector(N, seed=50 + p)
    m_rows = ebe_rows(p, n, amp, alpha, np.abs(x), bc, np.arange(N), magnitude=True)
    m_full = magnitude_bound(p, n, amp, alpha, x, bc)
    assert np.all(m_full >= 0)
    assert np.abs(m_rows - m_full).max() <= 1e-13 * m_full.max()


def _abs_1d(p, n):
    """1D assembled K'_ab = (1/h) sum_q w_q |l_a'(t_q)| |l_b'(t_q)| and M'_ab = h sum_q w_q |l_a(t_q)| |l_b(t_q)|
    on n cells, (p+1)-point Gauss on [0,1]; Lagrange basis on the GLL nodes as Legendre series."""
    xi = gll_nodes(p)
    V = npleg.legvander(2 * xi - 1, p)
    basis = [np.linalg.solve(V, np.eye(p + 1)[a]) for a in range(p + 1)]
    s, w = npleg.leggauss(p + 1)
    w = w / 2
    val = np.array([np.abs(npleg.legval(s, c)) for c in basis])                    # [a][q]
    der = np.array([np.abs(2.0 * npleg.legval(s, npleg.legder(c))) for c in basis])
    h = 1.0 / n
    N1 = p * n + 1
    K = np.zeros((N1, N1))
    M = np.zeros((N1, N1))
    Kc = (der * w) @ der.T / h
    Mc = (val * w) @ val.T * h
    for c in range(n):
        K[p * c:p * c + p + 1, p * c:p * c + p + 1] += Kc
        M[p * c:p * c + p + 1, p * c:p * c + p + 1] += Mc
    return K, M


@pytest.mark.parametrize("p,n", [(1, 3), (2, 2), (3, 2), (4, 1), (5, 1)])
@pytest.mark.parametrize("bc", [0, 1])
def test_magnitude_bound_affine_is_kronecker_sum_of_absolute_1d(p, n, bc):
    K, M = _abs_1d(p, n)
    Mag = np.kron(K, np.kron(M, M)) + np.kron(M, np.kron(K, M)) + np.kron(M, np.kron(M, K))
    x = uniform_vector(mesh.n_dofs(p, n), seed=60 + p)
    m = mesh.boundary_mask(p, n) if bc else np.ones(len(x))
    expect = m * (Mag @ (m * np.abs(x))) + (1 - m) * np.abs(x)
    got = magnitude_bound(p, n, 0.0, 0.0, x, bc)
    assert np.abs(got - expect).max() <= 1e-13 * expect.max()


@pytest.mark.parametrize("p,n,amp,alpha", [(2, 2, 0.1, 0.5), (3, 1, 0.1, 0.9), (2, 2, 0.0, 0.0), (1, 3, 0.0, 0.5)])
def test_magnitude_matrix_bounds_operator_entrywise(p, n, amp, alpha):
    At = assemble.operator_csr(p, n, amp, alpha, 0).toarray()
    N = At.shape[0]
    Mag = np.stack([magnitude_bound(p, n, amp, alpha, np.eye(N)[j], 0) for j in range(N)], axis=1)
    assert np.all(np.abs(At) <= Mag * (1 + 1e-13) + 1e-300)
    np.testing.assert_allclose(Mag, Mag.T, rtol=1e-13, atol=1e-15 * Mag.max())
    x = uniform_vector(N, seed=7)
    assert np.all(np.abs(At @ x) <= Mag @ np.abs(x) * (1 + 1e-13))
    if amp == 0.0:
        # G_q = a(x_q) h w_q I: each diagonal term is a square times a positive weight
        np.testing.assert_allclose(np.diag(Mag), np.diag(At), rtol=1e-13)
    else:
        assert np.all(np.diag(Mag) >= np.diag(At) * (1 - 1e-13))


def test_ebe_rows_sampled_subset_matches_full_rows():
    """A scattered subset (boundary, vertex, edge and interior nodes) in arbitrary order gives the
    same entries as the full evaluation: rows are independent of which other rows are asked."""
    p, n, amp, alpha = 3, 3, 0.1, 0.5
    N1 = p * n + 1
    x = uniform_vector(N1 ** 3, seed=8)
    full = ebe_rows(p, n, amp, alpha, x, 1, np.arange(N1 ** 3))
    rows = np.array([N1 ** 3 - 1, 0, 3 + 3 * N1 + 3 * N1 * N1, 4 + 5 * N1 + 6 * N1 * N1, 1 + N1 + N1 * N1,
                     3 + 3 * N1 + 3 * N1 * N1])
    np.testing.assert_array_equal(ebe_rows(p, n, amp, alpha, x, 1, rows), full[rows])


def test_magnitude_bound_with_dirichlet_uses_identity_rows():
    p, n = 2, 2
    x = uniform_vector(mesh.n_dofs(p, n), seed=9)
    m = mesh.boundary_mask(p, n)
    got = magnitude_bound(p, n, 0.1, 0.5, x, 1)
    np.testing.assert_array_equal(got[m == 0], np.abs(x)[m == 0])
    # interior rows see only interior columns
    free = magnitude_bound(p, n, 0.1, 0.5, m * x, 0)
    np.testing.assert_allclose(got[m == 1], free[m == 1], rtol=1e-15)
    assert sp.issparse(assemble.operator_csr(p, n, 0.1, 0.5, 1))


@pytest.mark.parametrize("p,n", [(1, 3), (3, 2)])
@pytest.mark.parametrize("amp,alpha", GEOMS)
@pytest.mark.parametrize("bc", [0, 1])
def test_magnitude_csr_applies_magnitude_bound(p, n, amp, alpha, bc):
    from oracle.ebe import magnitude_csr
    x = uniform_vector(mesh.n_dofs(p, n), seed=70 + p)
    M = magnitude_csr(p, n, amp, alpha, bc)
    got = M @ np.abs(x)
    ref = magnitude_bound(p, n, amp, alpha, x, bc)
    assert np.abs(got - ref).max() <= 1e-13 * ref.max()
    # entrywise bound of the operator's own matrix (Dirichlet rows: both identity)
    At = assemble.operator_csr(p, n, amp, alpha, bc)
    assert np.all(np.abs(At.toarray()) <= M.toarray() * (1 + 1e-13) + 1e-300)
