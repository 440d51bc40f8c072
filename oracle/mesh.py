"""Uniform hexahedral mesh of the unit cube and Q_p degree-of-freedom numbering (oracle).

The paper's meshes are hexahedral and refined isotropically (Sec. 3.1); the
DoF numbering of its DoFHandler is not specified.  Readings used here:

* n^3 cells of side h = 1/n; cell (i, j, k) has index i + n*j + n^2*k.
* Global nodes sit on the lattice of (p*n+1)^3 points whose 1D coordinates
  are (i + xi_a)*h for GLL nodes xi_a; node (I, J, K) has global index
  I + N1*J + N1^2*K with N1 = p*n+1 (x fastest).
* Local DoF (a, b, c) of a cell has local index a + (p+1)*b + (p+1)^2*c and
  is global node (p*i+a, p*j+b, p*k+c).
* Homogeneous Dirichlet data: a node is constrained when any of I, J, K is 0
  or p*n.  The mask m is 1 on free nodes and 0 on constrained ones.
"""
import numpy as np

from .tables import gll_nodes


def n_dofs(p, n):
    return (p * n + 1) ** 3


def cell_dofs(p, n, cells=None):
    """int64 [len(cells), (p+1)^3]: global DoF of each local DoF of each cell."""
    N1 = p * n + 1
    if cells is None:
        cells = np.arange(n ** 3)
    cells = np.asarray(cells, dtype=np.int64)
    ci = cells % n
    cj = (cells // n) % n
    ck = cells // (n * n)
    loc = np.arange(p + 1)
    # local index a + (p+1) b + (p+1)^2 c  ->  reshape order (c, b, a)
    a = loc[None, None, :]
    b = loc[None, :, None]
    c = loc[:, None, None]
    out = np.empty((len(cells), (p + 1) ** 3), dtype=np.int64)
    for r in range(len(cells)):
        I = p * ci[r] + a
        J = p * cj[r] + b
        K = p * ck[r] + c
        out[r] = (I + N1 * J + N1 * N1 * K).reshape(-1)
    return out


def boundary_mask(p, n):
    """float64 [N]: 1 on free nodes, 0 on nodes of the cube's boundary."""
    N1 = p * n + 1
    idx = np.arange(N1)
    inner = ((idx > 0) & (idx < N1 - 1)).astype(np.float64)
    return (inner[None, None, :] * inner[None, :, None] * inner[:, None, None]).reshape(-1)


def node_coords_1d(p, n):
    """Undeformed 1D coordinates of the N1 = p*n+1 lattice nodes."""
    xi = gll_nodes(p)
    h = 1.0 / n
    x = np.empty(p * n + 1)
    for i in range(n):
        x[p * i: p * i + p + 1] = (i + xi) * h
    return x


def node_coords(p, n):
    """float64 [N, 3]: undeformed coordinates X of every global node (x fastest)."""
    x = node_coords_1d(p, n)
    N1 = len(x)
    X = np.empty((N1, N1, N1, 3))
    X[..., 0] = x[None, None, :]
    X[..., 1] = x[None, :, None]
    X[..., 2] = x[:, None, None]
    return X.reshape(-1, 3)
