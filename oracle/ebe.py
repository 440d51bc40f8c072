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


def abs_operator_times_abs(p, n, A, alpha, x, bc, chunk=2048):
    """(|A_tilde| |x|): the componentwise magnitude bound used by rounding-error tolerances."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    C = n ** 3
    m = boundary_mask(p, n) if bc else np.ones(n_dofs(p, n))
    y = np.zeros_like(x)
    tab = reference_tabulation(p)
    for c0 in range(0, C, chunk):
        cc = np.arange(c0, min(C, c0 + chunk))
        Ak = np.abs(element_matrices(p, n, A, alpha, cc, tab))
        g = cell_dofs(p, n, cc)
        yk = (Ak @ (m * x)[g][:, :, None])[:, :, 0]
        np.add.at(y, g.reshape(-1), yk.reshape(-1))
    y = m * y
    if bc:
        y += (1.0 - m) * x
    return y
