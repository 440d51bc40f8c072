"""Pins of the oracle's multigrid pieces: exact transfer, Chebyshev polynomial, symmetry, eigenvalue bounds."""
import numpy as np
import pytest

from oracle import assemble, gmg, mesh


def _interp(p, n, fun):
    X = mesh.node_coords(p, n)
    return fun(X[:, 0], X[:, 1], X[:, 2])


@pytest.mark.parametrize("pc,nc,pf,nf", [(1, 2, 1, 4), (2, 2, 2, 4), (3, 1, 3, 2), (2, 3, 4, 3), (1, 3, 2, 3)])
def test_prolongation_reproduces_coarse_polynomials(pc, nc, pf, nf):
    # P I_H u = I_h u for every u in the coarse space; x^a y^b z^c with a,b,c <= pc are in it
    # (on an h-coarse mesh they are even global polynomials)
    P = gmg.prolongation(pc, nc, pf, nf, bc=0)
    for (a, b, c) in [(0, 0, 0), (pc, 0, 0), (1, pc, 0), (pc, pc, pc)]:
        f = lambda x, y, z: x ** a * y ** b * z ** c
        np.testing.assert_allclose(P @ _interp(pc, nc, f), _interp(pf, nf, f), atol=1e-13)


def test_prolongation_dirichlet_mask():
    P = gmg.prolongation(2, 2, 2, 4, bc=1).toarray()
    mf = mesh.boundary_mask(2, 4).astype(bool)
    mc = mesh.boundary_mask(2, 2).astype(bool)
    assert np.all(P[~mf] == 0) and np.all(P[:, ~mc] == 0)


def test_hierarchy_rule():
    assert gmg.hierarchy(3, 128) == [(3, 4), (3, 8), (3, 16), (3, 32), (3, 64), (3, 128)]
    assert gmg.hierarchy(8, 24) == [(4, 3), (8, 3), (8, 6), (8, 12), (8, 24)]
    assert gmg.hierarchy(5, 47) == [(1, 47), (2, 47), (3, 47), (5, 47)]
    assert gmg.hierarchy(1, 4) == [(1, 4)]


@pytest.mark.parametrize("degree", [1, 2, 3, 5])
def test_chebyshev_recurrence_is_the_chebyshev_polynomial(degree):
    p, n = 2, 3
    At = assemble.operator_csr(p, n, 0.1, 0.5, 1)
    dinv = 1.0 / At.diagonal()
    Z = dinv[:, None] * At.toarray()
    lmax = 1.2 * np.linalg.eigvals(Z).real.max()
    lmin = lmax / 15
    E = gmg.chebyshev_error_matrix(Z, degree, lmin, lmax)
    rng = np.random.default_rng(0)
    xs = rng.standard_normal(At.shape[0])
    b = At @ xs
    x0 = rng.standard_normal(At.shape[0])
    # error after smoothing from x0 is E (x0 - x*); from zero it is E (0 - x*)
    x1 = gmg.chebyshev(lambda v: At @ v, dinv, b, x0, degree, lmin, lmax)
    np.testing.assert_allclose(x1 - xs, E @ (x0 - xs), atol=1e-10 * np.abs(xs).max())
    x2 = gmg.chebyshev(lambda v: At @ v, dinv, b, None, degree, lmin, lmax)
    np.testing.assert_allclose(x2 - xs, E @ (-xs), atol=1e-10 * np.abs(xs).max())
    # the polynomial is bounded by 1/T_k(theta/delta) on [lmin, lmax]
    theta, delta = (lmax + lmin) / 2, (lmax - lmin) / 2
    bound = 1.0 / np.cosh(degree * np.arccosh(theta / delta))
    lam = np.linspace(lmin, lmax, 101)
    vals = np.cos(degree * np.arccos((theta - lam) / delta)) * bound
    assert np.abs(vals).max() <= bound * (1 + 1e-12)


def test_lanczos_estimate_q1():
    # interior diagonal of the Q1 Laplacian is 8h/3, so the spectrum of D^{-1}A on the free block is
    # the closed-form Q1 spectrum divided by 8h/3; identity rows add eigenvalue 1
    n = 6
    h = 1.0 / n
    lv = gmg.Level(1, n, assemble.operator_csr(1, n, 0.0, 0.0, 1))
    th = np.arange(1, n) * np.pi / n
    kap = (2 / h) * (1 - np.cos(th))
    mu = (h / 3) * (2 + np.cos(th))
    top = (3 * kap.max() * mu.max() ** 2) / (8 * h / 3)
    top_exact = max(kap[i] * mu[j] * mu[k] + mu[i] * kap[j] * mu[k] + mu[i] * mu[j] * kap[k]
                    for i in range(n - 1) for j in range(n - 1) for k in range(n - 1)) / (8 * h / 3)
    lhat = lv.estimate(iters=30)
    assert abs(lhat - top_exact) < 1e-8 * top_exact
    lhat12 = lv.estimate(iters=12)
    assert 0.9 * top_exact < lhat12 <= top_exact * (1 + 1e-12)
    assert top >= top_exact


@pytest.mark.parametrize("p,n", [(1, 4), (2, 4)])
def test_vcycle_symmetric_and_two_grid_matrix(p, n):
    levels, prolong = gmg.build_hierarchy(p, n, 0.1, 0.5, bc=1)
    if len(levels) < 2:
        from oracle.gmg import Level, prolongation
        At_c = assemble.operator_csr(p, n // 2, 0.1, 0.5, 1)
        At_f = assemble.operator_csr(p, n, 0.1, 0.5, 1)
        levels = [Level(p, n // 2, At_c), Level(p, n, At_f)]
        prolong = [None, prolongation(p, n // 2, p, n, 1)]
    for L in levels[1:]:
        L.estimate()
    Nf = levels[-1].A.shape[0]
    l = len(levels) - 1
    B = np.column_stack([gmg.vcycle(levels, prolong, l, e) for e in np.eye(Nf)])
    np.testing.assert_allclose(B, B.T, atol=1e-12 * np.abs(B).max())
    if l == 1:
        # explicit two-grid preconditioner: B = S^T-post ... built from dense matrices
        L = levels[1]
        Af = L.A.toarray()
        Z = L.dinv[:, None] * Af
        E = gmg.chebyshev_error_matrix(Z, 3, L.lmin, L.lmax)
        P = prolong[1].toarray()
        Ac = levels[0].A.toarray()
        CGC = np.eye(Nf) - P @ np.linalg.solve(Ac, P.T @ Af)
        Etg = E @ CGC @ E
        np.testing.assert_allclose(np.eye(Nf) - B @ Af, Etg, atol=1e-10)
        rho = np.abs(np.linalg.eigvals(Etg)).max()
        assert rho < 0.5


def test_splitmix_known_values():
    # first outputs of SplitMix64 with state 0 (counter form: z = (i+1)*golden before mixing)
    v = gmg.splitmix64_uniform(3, 0)
    raw = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    expect = [2.0 * ((r >> 11) * 2.0 ** -53) - 1.0 for r in raw]
    np.testing.assert_allclose(v, expect, rtol=0, atol=0)


@pytest.mark.parametrize("p,n,limit,expect", [
    (4, 2, 8, [(2, 1), (4, 1), (4, 2)]),      # 343 free -> n/2: 27 -> p/2: 1
    (3, 4, 30, [(3, 1), (3, 2), (3, 4)]),     # 1331 -> 125 -> 8
    (6, 2, 30, [(3, 1), (6, 1), (6, 2)]),     # 1331 -> 125 -> p 3: 8
    (2, 38, 4096, [(1, 19), (2, 19), (2, 38)]),
    (1, 38, 4096, [(1, 19), (1, 38)]),        # 5832 free on the coarsest level: above the dense limit
    (1, 33, 4096, [(1, 33)]),
])
def test_hierarchy_rule_with_coarse_limit(p, n, limit, expect):
    from oracle.gmg import hierarchy
    assert hierarchy(p, n, limit) == expect
