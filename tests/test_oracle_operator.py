"""Pins of the oracle operator: closed forms, independent Kronecker constructions, invariants, brute force."""
import mpmath
import numpy as np
import numpy.polynomial.legendre as npleg
import pytest
import scipy.linalg
import scipy.sparse as sp

from oracle import assemble, element, geometry, mesh
from oracle.ebe import ebe_vmult
from oracle.tables import gll_nodes
from golden_fixtures import read_table
from synthetic import uniform_vector

EL = read_table("element_closed_forms.txt")


def _ndiff(i, j, p):
    ai, bi, ci = i % (p + 1), (i // (p + 1)) % (p + 1), i // (p + 1) ** 2
    aj, bj, cj = j % (p + 1), (j // (p + 1)) % (p + 1), j // (p + 1) ** 2
    return int(ai != aj) + int(bi != bj) + int(ci != cj)


@pytest.mark.parametrize("n,cell", [(1, 0), (3, 13), (4, 37)])
def test_q1_element_closed_form(n, cell):
    h = 1.0 / n
    Ak = element.element_matrices(1, n, 0.0, 0.0, [cell])[0]
    for i in range(8):
        for j in range(8):
            assert abs(Ak[i, j] - h * EL[("q1", _ndiff(i, j, 1))][0]) < 1e-15


def test_q2_element_is_kronecker_sum_of_closed_forms():
    n, h = 2, 0.5
    K1 = np.array([EL[("q2k", r)] for r in range(3)]) / (3 * h)
    M1 = np.array([EL[("q2m", r)] for r in range(3)]) * h / 30
    expect = np.kron(K1, np.kron(M1, M1)) + np.kron(M1, np.kron(K1, M1)) + np.kron(M1, np.kron(M1, K1))
    Ak = element.element_matrices(2, n, 0.0, 0.0, [5])[0]
    np.testing.assert_allclose(Ak, expect, atol=1e-14)


def _legendre_basis(p):
    """Lagrange basis on the GLL nodes as Legendre series in s = 2t-1, by solving the
    Legendre-Vandermonde system (independent of the oracle's product-formula tables)."""
    xi = gll_nodes(p)   # nodes are pinned separately (closed forms / 40-digit roots)
    V = npleg.legvander(2 * xi - 1, p)
    return [np.linalg.solve(V, np.eye(p + 1)[a]) for a in range(p + 1)]


def _global_1d(p, n, weight=None, nq=None):
    """1D global stiffness and mass on n cells: exact polynomial integrals (weight None) or
    nq-point Gauss with a weight function (numpy's leggauss, independent of the oracle's rule)."""
    basis = _legendre_basis(p)
    dbasis = [2.0 * npleg.legder(c) for c in basis]          # d/dt = 2 d/ds
    h = 1.0 / n
    N1 = p * n + 1

    def integral01(c):                                        # int_0^1 f dt = 1/2 int_-1^1 f ds
        ci = npleg.legint(c)
        return 0.5 * (npleg.legval(1.0, ci) - npleg.legval(-1.0, ci))

    K = np.zeros((N1, N1))
    M = np.zeros((N1, N1))
    for cell in range(n):
        for a in range(p + 1):
            for b in range(p + 1):
                if weight is None:
                    kab = integral01(npleg.legmul(dbasis[a], dbasis[b])) / h
                    mab = integral01(npleg.legmul(basis[a], basis[b])) * h
                else:
                    s, w = npleg.leggauss(nq)
                    wt = weight((cell + (s + 1) / 2) * h) * w / 2
                    kab = np.sum(wt * npleg.legval(s, dbasis[a]) * npleg.legval(s, dbasis[b])) / h
                    mab = np.sum(wt * npleg.legval(s, basis[a]) * npleg.legval(s, basis[b])) * h
                K[p * cell + a, p * cell + b] += kab
                M[p * cell + a, p * cell + b] += mab
    return K, M


def _kron_sum(K, M):
    return np.kron(K, np.kron(M, M)) + np.kron(M, np.kron(K, M)) + np.kron(M, np.kron(M, K))


@pytest.mark.parametrize("p,n", [(1, 3), (2, 2), (3, 2), (4, 2), (5, 1), (6, 1)])
def test_affine_unit_coefficient_is_kronecker_sum(p, n):
    # (p+1)-point Gauss integrates the affine a=1 integrands exactly, so the assembled matrix
    # equals the Kronecker sum of exactly integrated 1D matrices.
    K, M = _global_1d(p, n)
    A = assemble.assemble_csr(p, n, 0.0, 0.0).toarray()
    np.testing.assert_allclose(A, _kron_sum(K, M), atol=2e-13 * np.abs(A).max())


@pytest.mark.parametrize("p,n,alpha", [(2, 2, 0.5), (3, 2, 0.9), (4, 1, 0.3)])
def test_affine_separable_coefficient_kronecker(p, n, alpha):
    # a = 1 + alpha*s(x)s(y)s(z), s = sin(2 pi .): with a tensor quadrature the matrix splits into
    # Kronecker sums of 1D matrices with and without the weight s.
    K, M = _global_1d(p, n)
    s = lambda x: np.sin(2 * np.pi * x)
    Ks, Ms = _global_1d(p, n, weight=s, nq=p + 1)
    expect = _kron_sum(K, M) + alpha * _kron_sum(Ks, Ms)
    A = assemble.assemble_csr(p, n, 0.0, alpha).toarray()
    np.testing.assert_allclose(A, expect, atol=2e-13 * np.abs(A).max())


def test_q1_interior_stencil():
    n, h = 4, 0.25
    A = assemble.assemble_csr(1, n, 0.0, 0.0)
    N1 = n + 1
    centre = 2 + N1 * 2 + N1 * N1 * 2
    row = A.getrow(centre).toarray()[0]
    for I in range(N1):
        for J in range(N1):
            for K in range(N1):
                g = I + N1 * J + N1 * N1 * K
                d = (abs(I - 2), abs(J - 2), abs(K - 2))
                if max(d) > 1:
                    assert row[g] == 0
                else:
                    assert abs(row[g] - h * EL[("q1stencil", sum(d))][0]) < 1e-15


def test_q1_dirichlet_spectrum():
    n = 5
    h = 1.0 / n
    At = assemble.operator_csr(1, n, 0.0, 0.0, 1).toarray()
    m = mesh.boundary_mask(1, n).astype(bool)
    ev = np.sort(np.linalg.eigvalsh(At[np.ix_(m, m)]))
    th = np.arange(1, n) * np.pi / n
    kap = (2 / h) * (1 - np.cos(th))
    mu = (h / 3) * (2 + np.cos(th))
    expect = np.sort((kap[:, None, None] * mu[None, :, None] * mu[None, None, :]
                      + mu[:, None, None] * kap[None, :, None] * mu[None, None, :]
                      + mu[:, None, None] * mu[None, :, None] * kap[None, None, :]).reshape(-1))
    np.testing.assert_allclose(ev, expect, rtol=1e-12)
    # identity rows of the constrained nodes add the eigenvalue 1
    assert np.allclose(At[np.ix_(~m, ~m)], np.eye((~m).sum()))


@pytest.mark.parametrize("p,n,A,alpha", [(1, 3, 0.1, 0.5), (2, 2, 0.1, 0.5), (3, 2, 0.1, 0.9), (4, 1, 0.1, 0.5)])
def test_invariants_curved_variable(p, n, A, alpha):
    Ar = assemble.assemble_csr(p, n, A, alpha)
    ones = np.ones(Ar.shape[0])
    assert np.abs(Ar @ ones).max() < 1e-13 * abs(Ar).max()          # partition of unity: A 1 = 0
    assert abs(Ar - Ar.T).max() < 1e-15 * abs(Ar).max() * 10         # symmetry
    At = assemble.operator_csr(p, n, A, alpha, 1).toarray()
    scipy.linalg.cholesky(At)                                        # SPD with Dirichlet rows


def test_nnz_certificate():
    A = assemble.operator_csr(2, 8, 0.0, 0.0, 0)
    assert A.nnz == (8 * 9 - 8 + 1) ** 3 == 274625


def test_jacobian_by_complex_step():
    # J from the analytic derivative vs complex-step differentiation of the deformation itself
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, (20, 3))
    Jan = geometry.deformation_jacobian(X, 0.1)
    eps = 1e-30
    for c in range(3):
        Xc = X.astype(complex)
        Xc[:, c] += 1j * eps
        col = geometry.deformation(Xc, 0.1).imag / eps
        np.testing.assert_allclose(Jan[:, :, c], col, atol=1e-15)


def test_G_formula_alternative():
    # G = w a detJ (J^T J)^{-1}, the same tensor through a different formula
    qd = geometry.qpoint_data(3, 2, 0.1, 0.5, [0, 5, 7])
    J = qd["J"]
    alt = (qd["w"][None, :] * qd["a"] * np.linalg.det(J))[..., None, None] * np.linalg.inv(np.swapaxes(J, -1, -2) @ J)
    np.testing.assert_allclose(qd["G"], alt, rtol=1e-13, atol=1e-16)


def _mp_element_matrix(p, n, cell, A, alpha):
    """Brute force at 30 digits: GLL/Gauss from mpmath roots, Lagrange products, J by mpmath.diff,
    G by mpmath matrix inverse, sum over all quadrature points of grad phi_i^T G grad phi_j."""
    mpmath.mp.dps = 30
    N1 = p + 1
    dP = lambda s: mpmath.diff(lambda u: mpmath.legendre(p, u), s)
    inner = [mpmath.findroot(dP, mpmath.cos(mpmath.pi * k / p)) for k in range(1, p)]
    xi = sorted([mpmath.mpf(0), mpmath.mpf(1)] + [(r + 1) / 2 for r in inner])
    gp = [mpmath.findroot(lambda u: mpmath.legendre(N1, u), mpmath.cos(mpmath.pi * (k + 0.75) / (N1 + 0.5)))
          for k in range(N1)]
    gp = sorted(gp)
    gw = [2 / ((1 - s ** 2) * mpmath.diff(lambda u: mpmath.legendre(N1, u), s) ** 2) for s in gp]
    z = [(s + 1) / 2 for s in gp]
    w = [v / 2 for v in gw]
    ell = lambda a, t: mpmath.fprod([(t - xi[b]) / (xi[a] - xi[b]) for b in range(N1) if b != a])
    dell = lambda a, t: mpmath.diff(lambda u: ell(a, u), t)
    S = [[ell(a, z[r]) for a in range(N1)] for r in range(N1)]
    D = [[dell(a, z[r]) for a in range(N1)] for r in range(N1)]
    h = mpmath.mpf(1) / n
    org = [cell % n, (cell // n) % n, cell // (n * n)]
    F = lambda X: [X[d] + A * mpmath.sin(mpmath.pi * X[0]) * mpmath.sin(mpmath.pi * X[1]) * mpmath.sin(mpmath.pi * X[2])
                   for d in range(3)]
    nd = N1 ** 3
    Ak = mpmath.zeros(nd, nd)
    for t in range(N1):
        for s in range(N1):
            for r in range(N1):
                xh = [z[r], z[s], z[t]]
                X = [h * (org[d] + xh[d]) for d in range(3)]
                J = mpmath.matrix(3, 3)
                for c in range(3):
                    for rr in range(3):
                        J[rr, c] = h * mpmath.diff(lambda u: F([u if d == c else X[d] for d in range(3)])[rr], X[c])
                x = F(X)
                a = 1 + alpha * mpmath.sin(2 * mpmath.pi * x[0]) * mpmath.sin(2 * mpmath.pi * x[1]) * mpmath.sin(2 * mpmath.pi * x[2])
                Ji = J ** -1
                G = (w[r] * w[s] * w[t] * a * mpmath.det(J)) * (Ji * Ji.T)
                grads = []
                for c in range(N1):
                    for b in range(N1):
                        for aa in range(N1):
                            grads.append(mpmath.matrix([D[r][aa] * S[s][b] * S[t][c],
                                                        S[r][aa] * D[s][b] * S[t][c],
                                                        S[r][aa] * S[s][b] * D[t][c]]))
                Gg = [G * g for g in grads]
                for i in range(nd):
                    for j in range(nd):
                        Ak[i, j] += (grads[i].T * Gg[j])[0]
    return np.array(Ak.tolist(), dtype=np.float64)


@pytest.mark.slow
@pytest.mark.parametrize("p,n,cell", [(1, 2, 5), (2, 2, 6)])
def test_bruteforce_mpmath_curved_variable(p, n, cell):
    ref = _mp_element_matrix(p, n, cell, mpmath.mpf("0.1"), mpmath.mpf("0.5"))
    Ak = element.element_matrices(p, n, 0.1, 0.5, [cell])[0]
    np.testing.assert_allclose(Ak, ref, atol=1e-14 * np.abs(ref).max())


@pytest.mark.parametrize("p,n", [(2, 3), (3, 2)])
def test_polynomial_reproduction(p, n):
    # u = x^2 is in Q_p; integration by parts with phi_i vanishing on the boundary gives
    # (A u)_i = int (-Delta u) phi_i = -2 int phi_i for every interior node i.
    from oracle.rhs import rhs_from_function
    A = assemble.assemble_csr(p, n, 0.0, 0.0)
    X = mesh.node_coords(p, n)
    u = X[:, 0] ** 2
    b = rhs_from_function(p, n, 0.0, 0.0, lambda x: -2.0 + 0 * x[..., 0], bc=1)
    m = mesh.boundary_mask(p, n).astype(bool)
    np.testing.assert_allclose((A @ u)[m], b[m], atol=1e-13)


@pytest.mark.parametrize("p,n", [(1, 3), (2, 2), (4, 2)])
def test_ebe_equals_csr(p, n):
    x = uniform_vector(mesh.n_dofs(p, n), 1)
    At = assemble.operator_csr(p, n, 0.1, 0.5, 1)
    np.testing.assert_allclose(ebe_vmult(p, n, 0.1, 0.5, x, 1), At @ x, atol=1e-13 * np.abs(At @ x).max())
