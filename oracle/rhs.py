"""Right-hand sides (oracle; test infrastructure only).

* Manufactured solution (curved, variable-coefficient problem): u*(x) =
  sin(pi x1) sin(pi x2) sin(pi x3) in physical coordinates, which vanishes on
  the boundary of the unit cube (the deformation maps the cube onto itself).
  f = -div(a grad u*) = -grad a . grad u* + 3 pi^2 a u*.
* b_i = sum_q f(x_q) phi_i(q) JxW(q): the right-hand-side term of the Sec. 2.4
  cell loop, assembled over cells, then b <- m * b (zero on constrained rows).
* Algebraic right-hand side of the random-vector problems (paper silent;
  reading): b = m * f with f the seeded nodal vector.
"""
import numpy as np

from .element import reference_tabulation
from .geometry import qpoint_data, deformation, deformation_jacobian
from .tables import gauss, lagrange_values, gll_nodes
from .mesh import cell_dofs, n_dofs, boundary_mask


def manufactured_u(x):
    return np.sin(np.pi * x[..., 0]) * np.sin(np.pi * x[..., 1]) * np.sin(np.pi * x[..., 2])


def manufactured_f(x, alpha):
    """-div(a grad u*) for a = 1 + alpha*prod sin(2 pi x_d), u* = prod sin(pi x_d)."""
    s1 = np.sin(np.pi * x)
    c1 = np.cos(np.pi * x)
    s2 = np.sin(2 * np.pi * x)
    c2 = np.cos(2 * np.pi * x)
    u = s1[..., 0] * s1[..., 1] * s1[..., 2]
    gu = np.pi * np.stack([c1[..., 0] * s1[..., 1] * s1[..., 2],
                           s1[..., 0] * c1[..., 1] * s1[..., 2],
                           s1[..., 0] * s1[..., 1] * c1[..., 2]], axis=-1)
    a = 1.0 + alpha * s2[..., 0] * s2[..., 1] * s2[..., 2]
    ga = 2 * np.pi * alpha * np.stack([c2[..., 0] * s2[..., 1] * s2[..., 2],
                                       s2[..., 0] * c2[..., 1] * s2[..., 2],
                                       s2[..., 0] * s2[..., 1] * c2[..., 2]], axis=-1)
    return -(ga * gu).sum(-1) + 3 * np.pi ** 2 * a * u


def rhs_from_function(p, n, A, alpha, f, bc=1, chunk=4096):
    """b_i = sum_K sum_q f(x_q) phi_i(q) JxW(q); masked to zero on constrained rows when bc=1."""
    N = n_dofs(p, n)
    Phi, _ = reference_tabulation(p)
    b = np.zeros(N)
    C = n ** 3
    for c0 in range(0, C, chunk):
        cells = np.arange(c0, min(C, c0 + chunk))
        qd = qpoint_data(p, n, A, alpha, cells)
        fq = f(qd["x"]) * qd["JxW"]                       # [Cc, Q]
        bk = fq @ Phi                                     # [Cc, n_dofs]
        np.add.at(b, cell_dofs(p, n, cells).reshape(-1), bk.reshape(-1))
    if bc:
        b *= boundary_mask(p, n)
    return b


def rhs_rows(p, n, A, alpha, f, rows, bc=1):
    """Entries `rows` of ``rhs_from_function``, each summed over the cells whose closure holds the
    row's node (the sampled form for meshes too large to assemble the whole vector)."""
    N1 = p * n + 1
    rows = np.asarray(rows, dtype=np.int64)
    Phi, _ = reference_tabulation(p)

    def cells_1d(I):
        if I % p == 0:
            return [c for c in (I // p - 1, I // p) if 0 <= c < n]
        return [I // p]

    out = np.zeros(len(rows))
    for r, g in enumerate(rows):
        I, J, K = g % N1, (g // N1) % N1, g // (N1 * N1)
        if bc and (min(I, J, K) == 0 or max(I, J, K) == N1 - 1):
            continue
        for ck in cells_1d(K):
            for cj in cells_1d(J):
                for ci in cells_1d(I):
                    cell = ci + n * cj + n * n * ck
                    qd = qpoint_data(p, n, A, alpha, [cell])
                    fq = f(qd["x"][0]) * qd["JxW"][0]
                    loc = (I - p * ci) + (p + 1) * (J - p * cj) + (p + 1) ** 2 * (K - p * ck)
                    out[r] += fq @ Phi[:, loc]
    return out


def rhs_manufactured(p, n, A, alpha, bc=1):
    return rhs_from_function(p, n, A, alpha, lambda x: manufactured_f(x, alpha), bc)


def rhs_nodal(p, n, f, bc=1):
    """b = m * f for a nodal vector f."""
    f = np.asarray(f, dtype=np.float64)
    return boundary_mask(p, n) * f if bc else f.copy()


def l2_error(p, n, A, u_nodal, u_exact, nq_extra=2):
    """|| u_h - u* ||_L2 over the deformed cube, by a (p+1+nq_extra)-point Gauss rule per direction."""
    nq = p + 1 + nq_extra
    z, w = gauss(nq)
    xi = gll_nodes(p)
    V = lagrange_values(xi, z)                            # [nq, p+1]
    h = 1.0 / n
    err2 = 0.0
    C = n ** 3
    g_all = cell_dofs(p, n)
    N1 = p + 1
    # tensor evaluation matrix [nq^3, (p+1)^3] with q = r + nq s + nq^2 t, i = a + N1 b + N1^2 c
    E = np.einsum("ra,sb,tc->tsrcba", V, V, V).reshape(nq ** 3, N1 ** 3)
    W = np.einsum("r,s,t->tsr", w, w, w).reshape(-1)
    pts = np.empty((nq, nq, nq, 3))
    pts[..., 0] = z[None, None, :]
    pts[..., 1] = z[None, :, None]
    pts[..., 2] = z[:, None, None]
    pts = pts.reshape(-1, 3)
    for c in range(C):
        org = np.array([c % n, (c // n) % n, c // (n * n)], dtype=np.float64)
        X = h * (org[None, :] + pts)
        x = deformation(X, A)
        detJ = np.linalg.det(h * deformation_jacobian(X, A))
        uh = E @ u_nodal[g_all[c]]
        err2 += np.sum(W * detJ * (uh - u_exact(x)) ** 2)
    return np.sqrt(err2)
