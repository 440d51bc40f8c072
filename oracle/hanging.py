"""Hanging-node constraints on a two-block mesh with a 2:1 interface (oracle; test infrastructure only).

Sec. 3.3 of the paper: adaptive refinement with hanging nodes, cells of different sizes meeting at
a face (Sec. 3.2, Fig. 3 shows such a mesh).  The smallest mesh with that feature that keeps the
tensor-product structure of each part, and the readings used here and by the GPU path:

* Domain [0,2] x [0,1] x [0,1] in undeformed coordinates X.  Block 0 (coarse): the unit cube
  [0,1]^3 cut into n^3 cells of side h = 1/n.  Block 1 (fine): [1,2] x [0,1]^2 cut into (2n)^3 cells
  of side h/2.  Every coarse cell face on X1 = 1 meets 2 x 2 fine cell faces.
* The deformation x = X + A sin(pi X1) sin(pi X2) sin(pi X3) (1,1,1) and the coefficient
  a(x) = 1 + alpha sin(2 pi x1) sin(2 pi x2) sin(2 pi x3) are those of the single-block meshes,
  evaluated on the whole domain (the same analytic map on both sides of the interface).
* Degrees of freedom: block 0's lattice of (pn+1)^3 GLL nodes, numbered x fastest, then block 1's
  lattice of (2pn+1)^3 nodes, x fastest, offset by (pn+1)^3.  Vector length (pn+1)^3 + (2pn+1)^3.
* Constraints: block 1's nodes on X1 = 1 (lattice I = 0) are hanging: the conforming function
  takes there the value of the coarse side's trace, u_f(J, K) = sum_{J', K'} Pi[J][J'] Pi[K][K']
  u_c(pn, J', K'), where Pi is the 1D interpolation of a function of the coarse lattice (degree p
  on n cells of [0,1]) at the fine lattice's nodes (2n cells).  Their entries in the vector are
  not unknowns: the operator's rows there are identity rows, as for Dirichlet rows.
* Homogeneous Dirichlet data on the boundary of the domain: block 0's faces X1 = 0, X2, X3 in
  {0, 1}; block 1's faces X1 = 2, X2, X3 in {0, 1}.  The interface X1 = 1 is not boundary.
* Operator: with the independent set F (all block-0 nodes, block-1 nodes with I > 0), the
  expansion C from F to both lattices (identity on F, Pi x Pi on the hanging nodes), the
  unconstrained block matrices A_0, A_1 (the same cell loop as the single-block operator) and the
  Dirichlet mask m on F: y_F = m C^T blockdiag(A_0, A_1) C (m x_F) + (1 - m) x_F, and y = x on the
  hanging entries.  This is C^T A C, the form the paper's constraint handling gives.
"""
import numpy as np
import scipy.sparse as sp

from .element import reference_tabulation
from .geometry import deformation, deformation_jacobian, coefficient, reference_qpoints
from .tables import gll_nodes, lagrange_values


def lattice_1d(p, n, x0=0.0, length=1.0):
    """Undeformed 1D coordinates of the p*n+1 GLL lattice nodes on [x0, x0 + length] cut into n cells."""
    xi = gll_nodes(p)
    h = length / n
    x = np.empty(p * n + 1)
    for i in range(n):
        x[p * i: p * i + p + 1] = x0 + (i + xi) * h
    return x


def interface_interpolation(p, n):
    """Pi [2pn+1, pn+1]: values at the fine lattice nodes (2n cells of [0,1]) of the coarse lattice's
    nodal basis (n cells, degree p): row J holds the coarse basis functions of the coarse cell that
    contains fine node J, evaluated there."""
    xc = lattice_1d(p, n)
    xf = lattice_1d(p, 2 * n)
    Pi = np.zeros((len(xf), len(xc)))
    for J, t in enumerate(xf):
        c = min(int(np.floor(t * n)), n - 1)
        nodes = xc[p * c: p * c + p + 1]
        Pi[J, p * c: p * c + p + 1] = lagrange_values(nodes, t)[0]
    return Pi


def sizes(p, n):
    """(N0, N1, N): block 0 lattice size, block 1 lattice size, vector length."""
    N0 = (p * n + 1) ** 3
    N1 = (2 * p * n + 1) ** 3
    return N0, N1, N0 + N1


def _block_cells(p, nb, x0, hb):
    """Global undeformed cell origins [C, 3] of an nb^3 block at X1 offset x0 with side hb, cell
    c = i + nb j + nb^2 k, and its local-to-lattice maps [C, (p+1)^3]."""
    C = nb ** 3
    c = np.arange(C, dtype=np.int64)
    i, j, k = c % nb, (c // nb) % nb, c // (nb * nb)
    L1 = p * nb + 1
    loc = np.arange(p + 1)
    a = loc[None, None, None, :]
    b = loc[None, None, :, None]
    cc = loc[None, :, None, None]
    dofs = (p * i[:, None, None, None] + a) + L1 * (p * j[:, None, None, None] + b) \
        + L1 * L1 * (p * k[:, None, None, None] + cc)
    org = np.stack([x0 + hb * i, hb * j, hb * k], axis=-1).astype(np.float64)
    return org, dofs.reshape(C, -1)


def block_qpoints(p, nb, x0, A, alpha):
    """G [C, Q, 3, 3], x [C, Q, 3], JxW [C, Q] of an nb^3 block of side 1/nb cells at X1 offset x0."""
    hb = 1.0 / nb
    zhat, wq = reference_qpoints(p)
    org, _ = _block_cells(p, nb, x0, hb)
    X = org[:, None, :] + hb * zhat[None, :, :]
    x = deformation(X, A)
    J = hb * deformation_jacobian(X, A)
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    a = coefficient(x, alpha)
    JxW = detJ * wq[None, :]
    G = (a * JxW)[..., None, None] * (Jinv @ np.swapaxes(Jinv, -1, -2))
    return G, x, JxW


def block_matrix(p, nb, x0, A, alpha, chunk=32):
    """Unconstrained stiffness matrix of one block on its own lattice (scipy CSR): sum over cells of
    grad phi_i^T G_q grad phi_j at every quadrature point (the Sec. 2.4 cell loop), cells taken in
    chunks to bound memory."""
    _, B = reference_tabulation(p)
    G, _, _ = block_qpoints(p, nb, x0, A, alpha)
    _, dofs = _block_cells(p, nb, x0, 1.0 / nb)
    Q = B.shape[0]
    Bf = B.reshape(Q * 3, -1)
    L = (p * nb + 1) ** 3
    out = sp.csr_matrix((L, L))
    for c0 in range(0, G.shape[0], chunk):
        Gc, dc = G[c0:c0 + chunk], dofs[c0:c0 + chunk]
        GB = Gc @ B[None]                                      # [Cc, Q, 3, nloc]
        Ak = Bf.T[None] @ GB.reshape(GB.shape[0], Q * 3, -1)   # [Cc, nloc, nloc]
        rows = np.repeat(dc[:, :, None], dc.shape[1], axis=2).reshape(-1)
        cols = np.repeat(dc[:, None, :], dc.shape[1], axis=1).reshape(-1)
        out = out + sp.coo_matrix((Ak.reshape(-1), (rows, cols)), shape=(L, L)).tocsr()
    return out.tocsr()


def block_load(p, nb, x0, A, alpha, f):
    """Load vector of one block on its own lattice: sum over cells and points of f(x_q) phi_i JxW."""
    Phi, _ = reference_tabulation(p)
    _, x, JxW = block_qpoints(p, nb, x0, A, alpha)
    _, dofs = _block_cells(p, nb, x0, 1.0 / nb)
    bk = (f(x) * JxW) @ Phi
    out = np.zeros((p * nb + 1) ** 3)
    np.add.at(out, dofs.reshape(-1), bk.reshape(-1))
    return out


def hanging_mask(p, n):
    """[N] bool: True on block 1's interface nodes (lattice I = 0), the hanging entries."""
    N0, N1, N = sizes(p, n)
    L1 = 2 * p * n + 1
    I = np.arange(N1) % L1
    out = np.zeros(N, dtype=bool)
    out[N0:] = I == 0
    return out


def dirichlet_mask(p, n):
    """[N] float64: 0 on nodes of the domain's boundary, 1 elsewhere (hanging entries: 1)."""
    N0, N1, N = sizes(p, n)
    L0, L1 = p * n + 1, 2 * p * n + 1
    g0 = np.arange(N0)
    I0, J0, K0 = g0 % L0, (g0 // L0) % L0, g0 // (L0 * L0)
    b0 = (I0 == 0) | (J0 == 0) | (J0 == L0 - 1) | (K0 == 0) | (K0 == L0 - 1)
    g1 = np.arange(N1)
    I1, J1, K1 = g1 % L1, (g1 // L1) % L1, g1 // (L1 * L1)
    b1 = (I1 == L1 - 1) | (J1 == 0) | (J1 == L1 - 1) | (K1 == 0) | (K1 == L1 - 1)
    b1 &= I1 > 0
    return np.concatenate([~b0, ~b1]).astype(np.float64)


def expansion(p, n):
    """C [N, N] (scipy CSR): the full vector of both lattices from the independent entries; identity
    on independent entries, Pi x Pi of block 0's X1 = 1 face on the hanging ones (the hanging
    entries of the input are not read)."""
    N0, N1, N = sizes(p, n)
    L0, L1 = p * n + 1, 2 * p * n + 1
    Pi = interface_interpolation(p, n)
    hang = hanging_mask(p, n)
    keep = np.flatnonzero(~hang)
    rows = [keep]
    cols = [keep]
    vals = [np.ones(len(keep))]
    P2 = sp.kron(sp.csr_matrix(Pi), sp.csr_matrix(Pi)).tocoo()    # [(J,K) fine, (J',K') coarse], J fastest
    Jf, Kf = P2.row % L1, P2.row // L1
    Jc, Kc = P2.col % L0, P2.col // L0
    rows.append(N0 + L1 * Jf + L1 * L1 * Kf)
    cols.append((L0 - 1) + L0 * Jc + L0 * L0 * Kc)
    vals.append(P2.data)
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N)).tocsr()


def unconstrained(p, n, A, alpha):
    """blockdiag(A_0, A_1) on the vector layout (scipy CSR)."""
    return sp.block_diag([block_matrix(p, n, 0.0, A, alpha), block_matrix(p, 2 * n, 1.0, A, alpha)]).tocsr()


def operator_csr(p, n, A, alpha, bc=1):
    """The operator on the vector layout: m C^T A C m + (1 - m) on independent rows, identity on the
    hanging rows (bc=0: no Dirichlet rows, m = 1)."""
    hang = hanging_mask(p, n).astype(np.float64)
    free = 1.0 - hang
    m = dirichlet_mask(p, n) if bc else np.ones(len(hang))
    m = m * free
    Cx = expansion(p, n)
    Af = unconstrained(p, n, A, alpha)
    Mm = sp.diags(m)
    return (Mm @ Cx.T @ Af @ Cx @ Mm + sp.diags(1.0 - m)).tocsr()


def load_vector(p, n, A, alpha, f):
    """b = m C^T (b_0, b_1): the load vector of the conforming space, zero on Dirichlet and hanging rows."""
    b = np.concatenate([block_load(p, n, 0.0, A, alpha, f), block_load(p, 2 * n, 1.0, A, alpha, f)])
    m = dirichlet_mask(p, n) * (1.0 - hanging_mask(p, n))
    return m * (expansion(p, n).T @ b)


def distribute(p, n, x):
    """The full nodal vector of the conforming function: hanging entries set from the coarse face."""
    hang = hanging_mask(p, n)
    out = expansion(p, n) @ x
    out[~hang] = x[~hang]
    return out


def node_coords(p, n):
    """[N, 3] undeformed coordinates X of every vector entry (block 0, then block 1)."""
    out = []
    for nb, x0 in ((n, 0.0), (2 * n, 1.0)):
        xs = lattice_1d(p, nb, x0)
        yz = lattice_1d(p, nb)
        L = len(xs)
        X = np.empty((L, L, L, 3))
        X[..., 0] = xs[None, None, :]
        X[..., 1] = yz[None, :, None]
        X[..., 2] = yz[:, None, None]
        out.append(X.reshape(-1, 3))
    return np.concatenate(out)


def magnitude_csr(p, n, A, alpha, bc=1):
    """Entrywise bound of the operator's rounding terms: m |C|^T |blockdiag(A_0, A_1)| |C| m + (1 - m)
    (the absolute values of every product summed by the cell loops and the face interpolation)."""
    hang = hanging_mask(p, n).astype(np.float64)
    m = (dirichlet_mask(p, n) if bc else np.ones(len(hang))) * (1.0 - hang)
    Cx = abs(expansion(p, n))
    Af = abs(unconstrained(p, n, A, alpha))
    Mm = sp.diags(m)
    return (Mm @ Cx.T @ Af @ Cx @ Mm + sp.diags(1.0 - m)).tocsr()
