"""Pins of the oracle's right-hand sides and solves: exact discrete solutions and convergence orders."""
import numpy as np
import pytest

from oracle import assemble, mesh, rhs, solve


@pytest.mark.parametrize("p,n", [(2, 3), (3, 2), (4, 2)])
def test_q2_polynomial_solution_is_exact(p, n):
    # u* = x(1-x)y(1-y)z(1-z) is in Q_2 subset Q_p and vanishes on the boundary; with
    # b_i = int f phi_i integrated exactly by (p+1)-point Gauss, the discrete solution equals
    # the nodal interpolant of u* (Galerkin orthogonality with u* in the space).
    def f(x):
        q = x * (1 - x)
        return 2 * (q[..., 1] * q[..., 2] + q[..., 0] * q[..., 2] + q[..., 0] * q[..., 1])
    At = assemble.operator_csr(p, n, 0.0, 0.0, 1)
    b = rhs.rhs_from_function(p, n, 0.0, 0.0, f, bc=1)
    x = solve.direct_solve(At, b)
    X = mesh.node_coords(p, n)
    ustar = np.prod(X * (1 - X), axis=1)
    np.testing.assert_allclose(x, ustar, atol=1e-14)


def test_cg_matches_direct():
    At = assemble.operator_csr(2, 4, 0.1, 0.5, 1)
    b = rhs.rhs_manufactured(2, 4, 0.1, 0.5)
    xd = solve.direct_solve(At, b)
    xc, it, res = solve.cg(lambda v: At @ v, b, rtol=1e-12)
    assert res <= 1e-12 and it < 200
    np.testing.assert_allclose(xc, xd, atol=1e-10 * np.abs(xd).max())


@pytest.mark.slow
@pytest.mark.parametrize("p", [1, 2, 3])
def test_manufactured_convergence_curved_variable(p):
    # L2 error of the curved, variable-coefficient problem decays like h^(p+1): a dropped term,
    # sign error or wrong index in geometry, coefficient, operator or right-hand side breaks this.
    errs = []
    ns = [2, 4, 8]
    for n in ns:
        At = assemble.operator_csr(p, n, 0.1, 0.5, 1)
        b = rhs.rhs_manufactured(p, n, 0.1, 0.5)
        x = solve.direct_solve(At, b)
        errs.append(rhs.l2_error(p, n, 0.1, x, rhs.manufactured_u))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p + 1 - 0.35, (errs, rates)


def test_nodal_rhs_mask():
    f = np.arange(mesh.n_dofs(1, 2), dtype=float)
    b = rhs.rhs_nodal(1, 2, f)
    assert b[13] == 13 and b[0] == 0 and np.count_nonzero(b) == 1


@pytest.mark.parametrize("p,n,amp,alpha,bc", [(2, 3, 0.1, 0.5, 1), (3, 2, 0.1, 0.9, 0), (1, 4, 0.0, 0.3, 1)])
def test_rhs_rows_equal_assembled_load_vector(p, n, amp, alpha, bc):
    """The sampled load-vector rows summed over each node's cells equal the assembled vector at every row."""
    from oracle import mesh
    f = lambda x: rhs.manufactured_f(x, alpha)
    full = rhs.rhs_from_function(p, n, amp, alpha, f, bc)
    rows = np.arange(mesh.n_dofs(p, n))
    got = rhs.rhs_rows(p, n, amp, alpha, f, rows, bc)
    assert np.abs(got - full).max() <= 1e-13 * np.abs(full).max()
