"""Geometry and coefficient at quadrature points (oracle; test infrastructure only).

Reference cell [0,1]^3 mapped to each cell (Sec. 3.4).  The curved meshes use
an "exact" mapping in the sense of Sec. 3.2: the analytic deformation is
evaluated directly at every quadrature point, no polynomial approximation of
the geometry.

* Undeformed point of cell (i,j,k): X = h*((i,j,k) + xhat).
* Deformation with amplitude A: x = F(X) = X + A*s(X)*(1,1,1) with
  s(X) = sin(pi X1) sin(pi X2) sin(pi X3).  F maps the unit cube onto itself.
* Jacobian of the reference-to-real map: J = dx/dxhat = h*(I + A*(1,1,1)^T grad s(X)^T).
* Coefficient a(x) = 1 + alpha * sin(2 pi x1) sin(2 pi x2) sin(2 pi x3) at the
  physical point x = F(X).
* Merged quadrature-point tensor: with grad_x phi = J^{-T} grad_xhat phi and
  JxW = det(J)*w_q (Sec. 2.4 cell loop), the bilinear form a(x) grad u . grad v
  becomes grad_xhat u^T G_q grad_xhat v with
  G_q = w_q * a(x_q) * det(J_q) * J_q^{-1} J_q^{-T}  (symmetric 3x3).

Quadrature point q = r + (p+1)*s + (p+1)^2*t sits at (zeta_r, zeta_s, zeta_t)
with weight omega_r*omega_s*omega_t.
"""
import numpy as np

from .tables import gauss


def deformation(X, A):
    """x = X + A * sin(pi X1) sin(pi X2) sin(pi X3) * (1,1,1).  X: [..., 3]."""
    s = np.sin(np.pi * X[..., 0]) * np.sin(np.pi * X[..., 1]) * np.sin(np.pi * X[..., 2])
    return X + A * s[..., None]


def deformation_jacobian(X, A):
    """dx/dX = I + A * (1,1,1)^T grad s(X)^T, shape [..., 3, 3] (row = component of x)."""
    sx = np.sin(np.pi * X)
    cx = np.cos(np.pi * X)
    grad_s = np.stack([
        np.pi * cx[..., 0] * sx[..., 1] * sx[..., 2],
        np.pi * sx[..., 0] * cx[..., 1] * sx[..., 2],
        np.pi * sx[..., 0] * sx[..., 1] * cx[..., 2],
    ], axis=-1)
    Jm = np.zeros(X.shape[:-1] + (3, 3))
    for r in range(3):
        for c in range(3):
            Jm[..., r, c] = (1.0 if r == c else 0.0) + A * grad_s[..., c]
    return Jm


def coefficient(x, alpha):
    """a(x) = 1 + alpha * sin(2 pi x1) sin(2 pi x2) sin(2 pi x3)."""
    return 1.0 + alpha * np.sin(2 * np.pi * x[..., 0]) * np.sin(2 * np.pi * x[..., 1]) * np.sin(2 * np.pi * x[..., 2])


def reference_qpoints(p):
    """([Q,3] reference points, [Q] weights) of the tensor Gauss rule, q = r + N1 s + N1^2 t."""
    z, w = gauss(p + 1)
    N1 = p + 1
    pts = np.empty((N1, N1, N1, 3))
    pts[..., 0] = z[None, None, :]
    pts[..., 1] = z[None, :, None]
    pts[..., 2] = z[:, None, None]
    wq = w[:, None, None] * w[None, :, None] * w[None, None, :]
    return pts.reshape(-1, 3), wq.reshape(-1)


def cell_origins(n, cells):
    cells = np.asarray(cells, dtype=np.int64)
    return np.stack([cells % n, (cells // n) % n, cells // (n * n)], axis=-1).astype(np.float64)


def qpoint_data(p, n, A, alpha, cells=None):
    """Per cell and quadrature point: dict with X, x, J, detJ, a, JxW, G.

    Shapes: X, x [Cc, Q, 3]; J [Cc, Q, 3, 3]; detJ, a, JxW [Cc, Q]; G [Cc, Q, 3, 3].
    """
    if cells is None:
        cells = np.arange(n ** 3)
    h = 1.0 / n
    zhat, wq = reference_qpoints(p)
    org = cell_origins(n, cells)
    X = h * (org[:, None, :] + zhat[None, :, :])
    x = deformation(X, A)
    J = h * deformation_jacobian(X, A)
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    a = coefficient(x, alpha)
    JxW = detJ * wq[None, :]
    G = (a * JxW)[..., None, None] * (Jinv @ np.swapaxes(Jinv, -1, -2))
    return dict(X=X, x=x, J=J, detJ=detJ, a=a, JxW=JxW, G=G, w=wq)
