"""Cell matrices by dense quadrature (oracle; test infrastructure only).

This is the cell loop printed in Sec. 2.4 of the paper (the step-4 assembly):
for every quadrature point q and every pair (i, j) of local DoFs, add
shape_grad(i,q) . shape_grad(j,q) * JxW(q), here with the coefficient and the
inverse-Jacobian transforms merged into G_q (see ``geometry``), and the
right-hand side term shape_value(i,q) * f(x_q) * JxW(q).

The shape functions are tabulated densely at all (p+1)^3 points: no
sum factorisation, so this is an independent route to the numbers the
tensor-product kernels produce.
"""
import numpy as np

from .tables import shape_1d
from .geometry import qpoint_data


def reference_tabulation(p):
    """(Phi [Q, n_dofs], B [Q, 3, n_dofs]): phi_i and grad_xhat phi_i at the reference Gauss points.

    Local DoF i = a + N1*b + N1^2*c has phi_i(xhat) = l_a(x1) l_b(x2) l_c(x3);
    quadrature point q = r + N1*s + N1^2*t sits at (zeta_r, zeta_s, zeta_t).
    """
    _, _, _, S, D = shape_1d(p)
    N1 = p + 1
    Q = N1 ** 3
    Phi = np.empty((Q, Q))
    B = np.empty((Q, 3, Q))
    for t in range(N1):
        for s in range(N1):
            for r in range(N1):
                q = r + N1 * s + N1 * N1 * t
                for c in range(N1):
                    for b in range(N1):
                        for a in range(N1):
                            i = a + N1 * b + N1 * N1 * c
                            Phi[q, i] = S[r, a] * S[s, b] * S[t, c]
                            B[q, 0, i] = D[r, a] * S[s, b] * S[t, c]
                            B[q, 1, i] = S[r, a] * D[s, b] * S[t, c]
                            B[q, 2, i] = S[r, a] * S[s, b] * D[t, c]
    return Phi, B


def element_matrices(p, n, A, alpha, cells=None, tab=None):
    """[Cc, n_dofs, n_dofs]: A^K_ij = sum_q grad phi_i(q)^T G_q grad phi_j(q) for each requested cell."""
    if tab is None:
        tab = reference_tabulation(p)
    _, B = tab
    G = qpoint_data(p, n, A, alpha, cells)["G"]          # [Cc, Q, 3, 3]
    GB = G @ B[None]                                     # [Cc, Q, 3, n_dofs]: G_q grad phi_j
    Q = B.shape[0]
    Bf = B.reshape(Q * 3, -1)                            # rows (q, d)
    return Bf.T[None] @ GB.reshape(GB.shape[0], Q * 3, -1)
