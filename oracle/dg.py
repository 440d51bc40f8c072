"""Symmetric interior penalty DG discretisation of the Laplacian (oracle; test infrastructure only).

The paper's only measured experiment (Sec. 6.1) solves the 3D Laplace equation with a symmetric
interior penalty discontinuous Galerkin discretisation of degree p = 4 on a hyper-rectangle.  It
gives no penalty, boundary treatment or basis; the readings used here (and by the GPU path):

* mesh: n^3 affine cubes of side h = 1/n on the unit cube (no deformation), coefficient 1;
* space: discontinuous Q_p, per cell the tensor-product Lagrange basis on the GLL nodes; DoF
  (a, b, c) of cell K = i + n j + n^2 k has index K (p+1)^3 + a + (p+1) b + (p+1)^2 c;
* quadrature: (p+1)^3 Gauss points on cells, (p+1)^2 on faces;
* bilinear form, for every interior face F with unit normal n pointing from the cell of lower
  coordinate (L) to the higher one (R), [u] = u_L - u_R, {w} = (w_L + w_R) / 2:
      a(u, v) = sum_K int_K grad u . grad v
              + sum_F int_F ( -{d_n u}[v] - {d_n v}[u] + sigma [u][v] )
  and on boundary faces the same terms with the outside values zero and the average replaced by
  the inside value (homogeneous Dirichlet data imposed weakly);
* penalty sigma = 2 (p+1)^2 / h on every face.

The face terms are assembled from dense tabulations of the traces and normal derivatives of
both cells' basis functions at the face quadrature points; nothing is sum-factorised.
"""
import numpy as np
import scipy.sparse as sp

from .element import element_matrices, reference_tabulation
from .gmg import chebyshev, vcycle as cg_vcycle
from .mesh import boundary_mask, cell_dofs
from .tables import gauss, gll_nodes, lagrange_derivs, lagrange_values


def penalty(p, n):
    return 2.0 * (p + 1) ** 2 * n


def n_dofs(p, n):
    return n ** 3 * (p + 1) ** 3


def _face_tables(p, n):
    """Per local DoF of a cell, its trace and normal derivative (physical, along +e_d) on the
    cell faces ξ_d = 0 and ξ_d = 1, at the face Gauss points; and the face weights.

    Returns (tr, dn, W): tr[d][end] and dn[d][end] are [(p+1)^2 face points, (p+1)^3 DoFs]; face
    point m = q1 + (p+1) q2 over the two tangential directions in increasing order; W [(p+1)^2]
    holds h^2 w_q1 w_q2."""
    N1 = p + 1
    h = 1.0 / n
    xi = gll_nodes(p)
    zeta, omega = gauss(N1)
    Lz = lagrange_values(xi, zeta)                     # [q, a]
    Lend = lagrange_values(xi, np.array([0.0, 1.0]))    # [end, a]
    Dend = lagrange_derivs(xi, np.array([0.0, 1.0]))    # [end, a]
    tr = [[None, None] for _ in range(3)]
    dn = [[None, None] for _ in range(3)]
    for d in range(3):
        t1, t2 = [e for e in range(3) if e != d]
        for end in range(2):
            T = np.zeros((N1 * N1, N1 ** 3))
            Dn = np.zeros((N1 * N1, N1 ** 3))
            for q2 in range(N1):
                for q1 in range(N1):
                    m = q1 + N1 * q2
                    for c in range(N1):
                        for b in range(N1):
                            for a in range(N1):
                                idx = (a, b, c)
                                i = a + N1 * b + N1 * N1 * c
                                tang = Lz[q1, idx[t1]] * Lz[q2, idx[t2]]
                                T[m, i] = Lend[end, idx[d]] * tang
                                Dn[m, i] = Dend[end, idx[d]] / h * tang
            tr[d][end] = T
            dn[d][end] = Dn
    W = h * h * np.outer(omega, omega).T.reshape(-1)   # m = q1 + N1 q2 -> w_q1 w_q2
    return tr, dn, W


def face_matrix(jump, avg, W, sigma):
    """M[i, j] = sum_m W_m ( -J_m[i] A_m[j] - A_m[i] J_m[j] + sigma J_m[i] J_m[j] ) for the jump
    rows J and normal-derivative average rows A of the face's DoFs (test i, trial j)."""
    JW = jump * W[:, None]
    AW = avg * W[:, None]
    return -JW.T @ avg - AW.T @ jump + sigma * JW.T @ jump


def face_magnitude(jump, avg, W, sigma):
    """Entrywise bound of the terms face_matrix sums: |J|^T W |A| + |A|^T W |J| + sigma |J|^T W |J|."""
    J, A = np.abs(jump), np.abs(avg)
    JW = J * W[:, None]
    return JW.T @ A + (A * W[:, None]).T @ J + sigma * JW.T @ J


def cell_magnitude(p, n):
    """Entrywise bound of the terms of the cell matrix of an affine cube of side h = 1/n:
    h sum_q w_q sum_d |d_d phi_i(q)| |d_d phi_j(q)| over the reference Gauss points."""
    _, B = reference_tabulation(p)
    _, omega = gauss(p + 1)
    w3 = np.einsum('t,s,r->tsr', omega, omega, omega).reshape(-1)
    Bd = np.abs(B)
    return (1.0 / n) * sum(Bd[:, d, :].T @ (w3[:, None] * Bd[:, d, :]) for d in range(3))


def _cell(n, i, j, k):
    return i + n * (j + n * k)


def assemble(p, n, magnitude=False):
    """The DG-SIPG matrix (scipy CSR, float64).  magnitude=True: the same assembly with every cell
    and face matrix replaced by the entrywise bound of its terms (cell_magnitude, face_magnitude),
    the magnitude that rounding errors of an evaluation in lower precision scale with."""
    N1 = p + 1
    nloc = N1 ** 3
    sig = penalty(p, n)
    tr, dn, W = _face_tables(p, n)
    fmat = face_magnitude if magnitude else face_matrix
    rows, cols, vals = [], [], []

    def add(dofs, M):
        rows.append(np.repeat(dofs, len(dofs)))
        cols.append(np.tile(dofs, len(dofs)))
        vals.append(M.reshape(-1))

    C = n ** 3
    if magnitude:
        Am = cell_magnitude(p, n)
        for K in range(C):
            add(K * nloc + np.arange(nloc), Am)
    else:
        Ak = element_matrices(p, n, 0.0, 0.0, np.arange(C))
        for K in range(C):
            add(K * nloc + np.arange(nloc), Ak[K])
    # interior faces: L at its xi_d = 1 end, R at its xi_d = 0 end
    Mint = [fmat(np.hstack([tr[d][1], -tr[d][0]]), 0.5 * np.hstack([dn[d][1], dn[d][0]]), W, sig)
            for d in range(3)]
    # boundary faces: only the inside cell; low boundary: inside cell at its xi_d = 0 end, outside
    # on the L side ([u] = -u_R); high boundary: inside at xi_d = 1 ([u] = u_L)
    Mlo = [fmat(-tr[d][0], dn[d][0], W, sig) for d in range(3)]
    Mhi = [fmat(tr[d][1], dn[d][1], W, sig) for d in range(3)]
    for d in range(3):
        for a in range(n):
            for b in range(n):
                for f in range(n + 1):
                    ijk_R = [0, 0, 0]
                    t1, t2 = [e for e in range(3) if e != d]
                    ijk_R[t1], ijk_R[t2], ijk_R[d] = a, b, f
                    ijk_L = list(ijk_R)
                    ijk_L[d] = f - 1
                    if 0 < f < n:
                        L = _cell(n, *ijk_L)
                        R = _cell(n, *ijk_R)
                        dofs = np.concatenate([L * nloc + np.arange(nloc), R * nloc + np.arange(nloc)])
                        add(dofs, Mint[d])
                    elif f == 0:
                        add(_cell(n, *ijk_R) * nloc + np.arange(nloc), Mlo[d])
                    else:
                        add(_cell(n, *ijk_L) * nloc + np.arange(nloc), Mhi[d])
    N = n_dofs(p, n)
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N)).tocsr()


def nodal_interpolant(p, n, fun):
    """DG nodal vector of fun(x, y, z): its values at every cell's GLL nodes."""
    N1 = p + 1
    xi = gll_nodes(p)
    h = 1.0 / n
    out = np.empty(n_dofs(p, n))
    for k in range(n):
        for j in range(n):
            for i in range(n):
                K = _cell(n, i, j, k)
                X = (i + xi)[None, None, :] * h
                Y = (j + xi)[None, :, None] * h
                Z = (k + xi)[:, None, None] * h
                out[K * N1 ** 3:(K + 1) * N1 ** 3] = np.broadcast_to(fun(X, Y, Z), (N1, N1, N1)).reshape(-1)
    return out


def load_vector(p, n, f):
    """F_i = int_K f phi_i over every cell by the (p+1)^3-point Gauss rule."""
    N1 = p + 1
    xi = gll_nodes(p)
    zeta, omega = gauss(N1)
    S = lagrange_values(xi, zeta)                       # [q, a]
    h = 1.0 / n
    w3 = np.einsum('t,s,r->tsr', omega, omega, omega) * h ** 3
    out = np.empty(n_dofs(p, n))
    for k in range(n):
        for j in range(n):
            for i in range(n):
                K = _cell(n, i, j, k)
                X = (i + zeta)[None, None, :] * h
                Y = (j + zeta)[None, :, None] * h
                Z = (k + zeta)[:, None, None] * h
                fq = np.broadcast_to(f(X, Y, Z), (N1, N1, N1)) * w3            # [t, s, r]
                out[K * N1 ** 3:(K + 1) * N1 ** 3] = np.einsum('tsr,tc,sb,ra->cba', fq, S, S, S).reshape(-1)
    return out


def dg_rows(p, n, x, rows, magnitude=False):
    """Entries `rows` of A x for the DG-SIPG matrix, each from its cell's matrix and that cell's
    six faces: the sampled form of ``assemble`` for meshes too large to assemble.  magnitude=True:
    the same rows of the magnitude matrix of ``assemble(p, n, magnitude=True)``."""
    N1 = p + 1
    nloc = N1 ** 3
    sig = penalty(p, n)
    tr, dn, W = _face_tables(p, n)
    fmat = face_magnitude if magnitude else face_matrix
    Mint = [fmat(np.hstack([tr[d][1], -tr[d][0]]), 0.5 * np.hstack([dn[d][1], dn[d][0]]), W, sig)
            for d in range(3)]
    Mlo = [fmat(-tr[d][0], dn[d][0], W, sig) for d in range(3)]
    Mhi = [fmat(tr[d][1], dn[d][1], W, sig) for d in range(3)]
    # affine cells, coefficient 1: the same cell matrix for every cell
    Acell = cell_magnitude(p, n) if magnitude else element_matrices(p, n, 0.0, 0.0, np.array([0]))[0]
    out = np.empty(len(rows))
    for r, g in enumerate(rows):
        K, il = divmod(int(g), nloc)
        i, j, k = K % n, (K // n) % n, K // (n * n)
        xs = x[K * nloc:(K + 1) * nloc]
        val = Acell[il] @ xs
        ijk = [i, j, k]
        for d in range(3):
            c = ijk[d]
            # face at the low side of K (K is R) and at the high side (K is L)
            if c > 0:
                nb = list(ijk)
                nb[d] = c - 1
                L = _cell(n, *nb)
                u = np.concatenate([x[L * nloc:(L + 1) * nloc], xs])
                val += Mint[d][nloc + il] @ u
            else:
                val += Mlo[d][il] @ xs
            if c < n - 1:
                nb = list(ijk)
                nb[d] = c + 1
                R = _cell(n, *nb)
                u = np.concatenate([xs, x[R * nloc:(R + 1) * nloc]])
                val += Mint[d][il] @ u
            else:
                val += Mhi[d][il] @ xs
        out[r] = val
    return out


def cg_embedding(p, n):
    """E [DG DoFs x lattice nodes] (scipy CSR): row K (p+1)^3 + local has a single 1 in the column
    of the lattice node that local DoF of cell K sits on, and the columns of boundary nodes are
    zero (the continuous space with Dirichlet nodes carries no value there).  E c is the
    continuous function c written in the DG basis (the two spaces share the GLL nodes); E^T moves
    a DG residual to the continuous space.  This is the change of space in the multigrid
    hierarchy of the paper's DG experiment (Sec. 6.1)."""
    nloc = (p + 1) ** 3
    cols = cell_dofs(p, n).reshape(-1)
    vals = boundary_mask(p, n)[cols]
    N = n_dofs(p, n)
    return sp.csr_matrix((vals, (np.arange(N), cols)), shape=(N, (p * n + 1) ** 3))


def vcycle(A, dinv, E, b, lmin, lmax, cg_levels, cg_prolong, degree=6):
    """One V-cycle of the multigrid of the paper's DG experiment (Sec. 6.1) applied to b: Chebyshev
    smoothing of the DG system (Jacobi, interval [lmin, lmax] of D^{-1}A, from zero), the residual
    moved to the continuous space on the same mesh by E^T, one V-cycle of the continuous hierarchy
    (same smoother degree, exact coarse solve), the correction moved back by E, and the same
    smoothing again from the corrected iterate."""
    apply = lambda v: A @ v
    x = chebyshev(apply, dinv, b, None, degree, lmin, lmax)
    r = b - apply(x)
    ec = cg_vcycle(cg_levels, cg_prolong, len(cg_levels) - 1, E.T @ r, degree)
    x = x + E @ ec
    return chebyshev(apply, dinv, b, x, degree, lmin, lmax)
