"""Global sparse matrix and its action (oracle; test infrastructure only).

Sec. 3.6 of the paper defines the matrix-free operator as the action of the
assembled operator on a vector: the global matrix is never built on the
product path, but the result must equal A x for the matrix built here.

* Assembly: A[g_i, g_j] += A^K_ij over all cells (COO with duplicates summed).
* Dirichlet reading (paper silent): constrained rows and columns are removed
  from the coupling and replaced by identity rows, i.e.
  A_tilde x = m * A (m * x) + (1 - m) * x with the boundary mask m of ``mesh``.
  Vectors keep their boundary entries (length (p*n+1)^3).
"""
import numpy as np
import scipy.sparse as sp

from .element import element_matrices, reference_tabulation
from .mesh import cell_dofs, n_dofs, boundary_mask


def assemble_csr(p, n, A, alpha, chunk=4096):
    """Unconstrained global matrix (scipy CSR, float64)."""
    N = n_dofs(p, n)
    C = n ** 3
    tab = reference_tabulation(p)
    rows, cols, vals = [], [], []
    for c0 in range(0, C, chunk):
        cells = np.arange(c0, min(C, c0 + chunk))
        Ak = element_matrices(p, n, A, alpha, cells, tab)
        g = cell_dofs(p, n, cells)
        rows.append(np.repeat(g[:, :, None], g.shape[1], axis=2).reshape(-1))
        cols.append(np.repeat(g[:, None, :], g.shape[1], axis=1).reshape(-1))
        vals.append(Ak.reshape(-1))
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return M.tocsr()


def constrain(Acsr, m):
    """A_tilde = diag(m) A diag(m) + diag(1 - m)."""
    Mm = sp.diags(m)
    return (Mm @ Acsr @ Mm + sp.diags(1.0 - m)).tocsr()


def operator_csr(p, n, A, alpha, bc):
    """The operator the GPU path applies: A (bc=0) or A_tilde (bc=1, homogeneous Dirichlet)."""
    Acsr = assemble_csr(p, n, A, alpha)
    if bc:
        return constrain(Acsr, boundary_mask(p, n))
    return Acsr
