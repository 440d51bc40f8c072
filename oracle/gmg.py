"""Geometric multigrid pieces (oracle; test infrastructure only).

The paper's Sec. 3.5 describes a geometric multigrid built from matrix-free
smoothers and transfer operators on a hierarchy of nested hexahedral meshes
(isotropic refinement, Sec. 3.1), and Sec. 6.1 runs it with Chebyshev
smoothing, a switch between discretisations inside the hierarchy and a
single-precision V-cycle under a double-precision correction.  Readings of
what it leaves open (binding for the GPU path too):

* Hierarchy: from the finest (p, n), halve n while n is even and the level
  has more than 4096 free DoFs; then, on the same mesh, lower p to
  ceil(p/2) while the level has more than 4096 free DoFs and p > 1.
* Level operators are rediscretised (same geometry and coefficient, exact
  mapping, so every level space is the pull-back of a Q_p space on the
  undeformed lattice and the spaces are nested).
* Prolongation P: interpolation of the coarse function at the fine nodes
  (exact embedding of nested spaces).  Restriction R = P^T.  With Dirichlet
  rows, P_tilde = diag(m_f) P diag(m_c) and R_tilde = P_tilde^T.
* Smoother: Chebyshev iteration on D^{-1} A_l with D = diag(A_l) (1 on
  constrained rows), of degree k = number of updates of x; the error after
  smoothing is T_k((theta - D^{-1}A)/delta) / T_k(theta/delta) times the
  initial error, theta = (lmax+lmin)/2, delta = (lmax-lmin)/2.  The
  recurrence is the Chebyshev semi-iteration (Saad, Iterative Methods for
  Sparse Linear Systems, 2nd ed., Alg. 12.1, with the preconditioner D).
* Eigenvalue bound: lhat = largest eigenvalue of the Lanczos matrix built
  from `iters` steps of Jacobi-preconditioned CG on A_l x = v0;
  interval [lmax/15, lmax] with lmax = 1.2*lhat.
* Cycle: V(1,1): pre-smooth from zero, residual, restrict, coarse
  correction (recursively; exact solve on the coarsest level), prolongate
  and add, post-smooth from the current iterate.
"""
import numpy as np
import scipy.sparse as sp

from .tables import gll_nodes, lagrange_values
from .mesh import node_coords_1d, n_dofs, boundary_mask

FREE_DOF_COARSE_LIMIT = 4096


def n_free(p, n):
    return (p * n - 1) ** 3


def hierarchy(p, n, coarse_dofs=FREE_DOF_COARSE_LIMIT):
    """List of (p, n) from coarsest to finest, by the rule in the module docstring (with the free-DoF
    limit `coarse_dofs` in place of 4096 when given)."""
    levels = [(p, n)]
    while n % 2 == 0 and n_free(p, n) > coarse_dofs:
        n //= 2
        levels.append((p, n))
    while p > 1 and n_free(p, n) > coarse_dofs:
        p = (p + 1) // 2
        levels.append((p, n))
    return levels[::-1]


def prolongation_1d(pc, nc, pf, nf):
    """1D global interpolation matrix [pf*nf+1, pc*nc+1]: coarse 1D basis evaluated at fine nodes."""
    Xf = node_coords_1d(pf, nf)
    xi_c = gll_nodes(pc)
    P = np.zeros((len(Xf), pc * nc + 1))
    for I, X in enumerate(Xf):
        cell = min(int(np.floor(X * nc)), nc - 1)
        xhat = X * nc - cell
        vals = lagrange_values(xi_c, np.array([xhat]))[0]
        for a in range(pc + 1):
            P[I, pc * cell + a] += vals[a]
    return P


def prolongation(pc, nc, pf, nf, bc=1):
    """3D P (scipy CSR) = P1 (x) P1 (x) P1 (x fastest), masked on constrained rows/columns when bc=1."""
    P1 = sp.csr_matrix(prolongation_1d(pc, nc, pf, nf))
    P1.eliminate_zeros()
    P = sp.kron(P1, sp.kron(P1, P1)).tocsr()
    if bc:
        P = (sp.diags(boundary_mask(pf, nf)) @ P @ sp.diags(boundary_mask(pc, nc))).tocsr()
    return P


def jacobi_diagonal(Acsr):
    return Acsr.diagonal().copy()


def chebyshev(apply, dinv, b, x0, degree, lmin, lmax):
    """`degree` Chebyshev updates of x for A x = b, preconditioned by D^{-1} (x0=None means zero)."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = x0.copy()
        r = b - apply(x)
    d = dinv * r / theta
    x = x + d
    for _ in range(degree - 1):
        r = r - apply(d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * r)
        rho = rho_new
        x = x + d
    return x


def chebyshev_error_matrix(Z_dense, degree, lmin, lmax):
    """Dense T_k((theta I - Z)/delta) / T_k(theta/delta) for Z = D^{-1}A (three-term recurrence of T_k)."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    I = np.eye(Z_dense.shape[0])
    Y = (theta * I - Z_dense) / delta
    T_prev, T_cur = I, Y
    s_prev, s_cur = 1.0, theta / delta
    for _ in range(degree - 1):
        T_prev, T_cur = T_cur, 2.0 * Y @ T_cur - T_prev
        s_prev, s_cur = s_cur, 2.0 * (theta / delta) * s_cur - s_prev
    if degree == 0:
        return I
    return T_cur / s_cur


def lanczos_lambda_max(apply, dinv, v0, iters=12):
    """Largest eigenvalue of the Lanczos tridiagonal from `iters` Jacobi-PCG steps on A x = v0."""
    x = np.zeros_like(v0)
    r = v0.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    alphas, betas = [], []
    for _ in range(iters):
        Ap = apply(p)
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        z = dinv * r
        rz_new = r @ z
        beta = rz_new / rz
        alphas.append(alpha)
        betas.append(beta)
        p = z + beta * p
        rz = rz_new
    k = len(alphas)
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    return np.linalg.eigvalsh(T)[-1]


def splitmix64_uniform(n, seed):
    """Counter-based start vector: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) of counter i, mapped to [-1,1).

    z = seed + (i+1)*0x9E3779B97F4A7C15; z = (z ^ z>>30)*0xBF58476D1CE4E5B9;
    z = (z ^ z>>27)*0x94D049BB133111EB; z ^= z>>31; u = (z >> 11) * 2^-53; v = 2u - 1.
    """
    with np.errstate(over="ignore"):
        i = np.arange(n, dtype=np.uint64)
        z = np.uint64(seed) + (i + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return 2.0 * u - 1.0


class Level:
    """One level: operator (CSR, Dirichlet rows), inverse diagonal, Chebyshev interval."""

    def __init__(self, p, n, Acsr, bc=1):
        self.p, self.n, self.A = p, n, Acsr
        self.m = boundary_mask(p, n) if bc else np.ones(n_dofs(p, n))
        self.dinv = 1.0 / jacobi_diagonal(Acsr)
        self.lmin = self.lmax = None

    def apply(self, x):
        return self.A @ x

    def estimate(self, iters=12, seed=0, factor=1.2, ratio=15.0):
        v0 = self.m * splitmix64_uniform(self.A.shape[0], seed)
        lhat = lanczos_lambda_max(self.apply, self.dinv, v0, iters)
        self.lmax = factor * lhat
        self.lmin = self.lmax / ratio
        return lhat


def build_hierarchy(p, n, A, alpha, bc=1, operator=None, coarse_dofs=FREE_DOF_COARSE_LIMIT):
    """Levels (coarsest first) and prolongations P_l: level l-1 -> level l (index l)."""
    from .assemble import operator_csr
    op = operator or operator_csr
    spec = hierarchy(p, n, coarse_dofs)
    levels = [Level(pl, nl, op(pl, nl, A, alpha, bc), bc) for (pl, nl) in spec]
    prolong = [None] + [prolongation(spec[l - 1][0], spec[l - 1][1], spec[l][0], spec[l][1], bc)
                        for l in range(1, len(spec))]
    return levels, prolong


def vcycle(levels, prolong, l, b, degree=3, coarse_solve=None):
    """V(1,1) cycle applied to b on level l (coarsest level solved exactly)."""
    L = levels[l]
    if l == 0:
        if coarse_solve is not None:
            return coarse_solve(b)
        return np.linalg.solve(L.A.toarray(), b)
    x = chebyshev(L.apply, L.dinv, b, None, degree, L.lmin, L.lmax)
    r = b - L.apply(x)
    rc = prolong[l].T @ r
    ec = vcycle(levels, prolong, l - 1, rc, degree, coarse_solve)
    x = x + prolong[l] @ ec
    return chebyshev(L.apply, L.dinv, b, x, degree, L.lmin, L.lmax)
