"""Pins of the DG-SIPG oracle (oracle/dg.py) against properties fixed by the mathematics:
symmetry, positive definiteness on small meshes, and consistency: for p >= 2 the function
u = x(1-x) y(1-y) z(1-z) lies in the space and vanishes on the boundary, so the discrete operator
applied to it must reproduce the load vector of f = -lap u exactly (the face terms of integration
by parts cancel against the consistency terms only with the right signs, normals and factors)."""
import numpy as np
import pytest

from oracle import dg


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
