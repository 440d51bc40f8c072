"""Element-by-element application of the operator (oracle; test infrastructure only).

For meshes whose assembled matrix does not fit in host memory the oracle
applies the same operator cell by cell: y += P_K^T (A^K (P_K x)), where P_K
picks the cell's DoFs and A^K is the dense cell matrix of ``element``.  This is
the same sum as the assembled matrix of ``assemble``, in a different order.
"""
import numpy as np

from .element import element_matrices, reference_tabulation
from .mesh import cell_dofs, n_dofs, boundary_mask


def ebe_vmult(p, n, A, alpha, x, bc, cells=None, chunk=2048):
    """y = A_tilde x (bc=1) or A x (bc=0), optionally restricted to the contribution of `cells`.

    When `cells` is a subset, only those cells' terms are summed (the identity
    rows of constrained DoFs are added only when all cells are included).
    """
    x = np.asarray(x, dtype=np.float64)
    C = n ** 3
    full = cells is None
    if full:
        cells = np.arange(C)
    cells = np.asarray(cells, dtype=np.int64)
    m = boundary_mask(p, n) if bc else np.ones(n_dofs(p, n))
    xm = m * x
    y = np.zeros_like(x)
    tab = reference_tabulation(p)
    for c0 in range(0, len(cells), chunk):
        cc = cells[c0:c0 + chunk]
        Ak = element_matrices(p, n, A, alpha, cc, tab)
        g = cell_dofs(p, n, cc)
        yk = (Ak @ xm[g][:, :, None])[:, :, 0]
        np.add.at(y, g.reshape(-1), yk.reshape(-1))
    y = m * y
    if full and bc:
        y += (1.0 - m) * x
    return y


def _cells_of_index_1d(p, n, I):
    """Cells (1D indices) whose closure contains lattice node I."""
    if I % p == 0:
        k = I // p
        return [c for c in (k - 1, k) if 0 <= c < n]
    return [I // p]


def ebe_rows(p, n, A, alpha, x, bc, rows, magnitude=False):
    """Entries `rows` of A_tilde x (or of the bound (sum_q |B_q|^T |G_q| |B_q|) |x| when magnitude),
    each summed over the cells that contain the row's node: the sampled form of ``ebe_vmult`` for
    meshes too large to apply in full."""
    from .geometry import qpoint_data
    x = np.asarray(x)
    N1 = p * n + 1
    rows = np.asarray(rows, dtype=np.int64)
    per_row = []
    cellset = {}
    for g in rows:
        I, J, K = g % N1, (g // N1) % N1, g // (N1 * N1)
        cs = [ci + n * cj + n * n * ck for ck in _cells_of_index_1d(p, n, K)
              for cj in _cells_of_index_1d(p, n, J) for ci in _cells_of_index_1d(p, n, I)]
        per_row.append((I, J, K, cs))
        for c in cs:
            cellset.setdefault(c, len(cellset))
    cells = np.array(sorted(cellset, key=cellset.get), dtype=np.int64)
    if magnitude:
        _, B = reference_tabulation(p)
        G = np.abs(qpoint_data(p, n, A, alpha, cells)["G"])
        Ba = np.abs(B)
        Q = B.shape[0]
        Ak = Ba.reshape(Q * 3, -1).T[None] @ (G @ Ba[None]).reshape(len(cells), Q * 3, -1)
    else:
        Ak = element_matrices(p, n, A, alpha, cells)
    gl = cell_dofs(p, n, cells)
    out = np.zeros(len(rows))
    for r, (I, J, K, cs) in enumerate(per_row):
        bnd = lambda L: (L == 0) | (L == N1 - 1)
        if bc and (bnd(I) or bnd(J) or bnd(K)):
            out[r] = abs(x[rows[r]]) if magnitude else x[rows[r]]
            continue
        for c in cs:
            k = cellset[c]
            ci, cj, ck = c % n, (c // n) % n, c // (n * n)
            loc = (I - p * ci) + (p + 1) * (J - p * cj) + (p + 1) ** 2 * (K - p * ck)
            gi = gl[k]
            xv = x[gi].astype(np.float64)
            if bc:
                Ig, Jg, Kg = gi % N1, (gi // N1) % N1, gi // (N1 * N1)
                xv = xv * ~(bnd(Ig) | bnd(Jg) | bnd(Kg))
            out[r] += Ak[k, loc] @ (np.abs(xv) if magnitude else xv)
    return out


def magnitude_bound(p, n, A, alpha, x, bc, chunk=2048):
    """m = sum_K P_K^T (sum_q |B_q|^T |G_q| |B_q|) P_K |m x| (+ |x| on constrained rows): the
    magnitude of the terms summed by any evaluation order of the quadrature sums, the scale of
    componentwise rounding-error bounds."""
    from .geometry import qpoint_data
    x = np.abs(np.asarray(x, dtype=np.float64))
    C = n ** 3
    m = boundary_mask(p, n) if bc else np.ones(n_dofs(p, n))
    _, B = reference_tabulation(p)
    Ba = np.abs(B)
    Q = B.shape[0]
    y = np.zeros_like(x)
    for c0 in range(0, C, chunk):
        cc = np.arange(c0, min(C, c0 + chunk))
        G = np.abs(qpoint_data(p, n, A, alpha, cc)["G"])
        Ak = Ba.reshape(Q * 3, -1).T[None] @ (G @ Ba[None]).reshape(len(cc), Q * 3, -1)
        g = cell_dofs(p, n, cc)
        yk = (Ak @ (m * x)[g][:, :, None])[:, :, 0]
        np.add.at(y, g.reshape(-1), yk.reshape(-1))
    y = m * y
    if bc:
        y += (1.0 - m) * x
    return y



def magnitude_csr(p, n, A, alpha, bc, chunk=2048):
    """The magnitude matrix itself (scipy CSR): sum_K P_K^T (sum_q |B_q|^T |G_q| |B_q|) P_K, with
    Dirichlet rows and columns replaced by identity rows when bc=1, so that
    magnitude_csr(...) @ |x| == magnitude_bound(..., x, bc)."""
    import scipy.sparse as sp
    from .geometry import qpoint_data
    N = n_dofs(p, n)
    C = n ** 3
    _, B = reference_tabulation(p)
    Ba = np.abs(B)
    Q = B.shape[0]
    rows, cols, vals = [], [], []
    for c0 in range(0, C, chunk):
        cc = np.arange(c0, min(C, c0 + chunk))
        G = np.abs(qpoint_data(p, n, A, alpha, cc)["G"])
        Ak = Ba.reshape(Q * 3, -1).T[None] @ (G @ Ba[None]).reshape(len(cc), Q * 3, -1)
        g = cell_dofs(p, n, cc)
        rows.append(np.repeat(g[:, :, None], g.shape[1], axis=2).reshape(-1))
        cols.append(np.repeat(g[:, None, :], g.shape[1], axis=1).reshape(-1))
        vals.append(Ak.reshape(-1))
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N)).tocsr()
    if bc:
        m = boundary_mask(p, n)
        M = (sp.diags(m) @ M @ sp.diags(m) + sp.diags(1.0 - m)).tocsr()
    return M
