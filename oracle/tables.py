"""1D reference data of the tensor-product Q_p element (oracle; test infrastructure only).

The paper's Sec. 3.4 describes elements defined on the reference cell [0,1]^d
and evaluated at quadrature points, and Sec. 3.1 notes that quadrature and
elements on hexahedra are tensor products of 1D objects.  It does not fix the
node family or the quadrature rule; the readings used here (and by the GPU
path) are:

* Lagrange nodes: the p+1 Gauss-Lobatto-Legendre points mapped to [0,1],
  i.e. 0, 1 and the roots of P_p'(2t-1).
* Quadrature: the (p+1)-point Gauss-Legendre rule mapped to [0,1] (weights sum
  to 1), used in every direction.

Functions here use numpy's Legendre module and direct product formulas.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(p):
    """Gauss-Lobatto-Legendre nodes on [0,1], ascending (p+1 values).

    Interior nodes are the roots of the derivative of the Legendre polynomial
    P_p on [-1,1] (numpy companion-matrix roots, then one Newton step on
    P_p' to polish), mapped by t -> (t+1)/2.
    """
    if p < 1:
        raise ValueError("degree must be >= 1")
    if p == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(p + 1)
    c[p] = 1.0
    d1 = npleg.legder(c)
    d2 = npleg.legder(d1)
    r = np.sort(npleg.legroots(d1).real)
    r = r - npleg.legval(r, d1) / npleg.legval(r, d2)
    t = np.concatenate(([-1.0], r, [1.0]))
    return (t + 1.0) / 2.0


def gauss(nq):
    """nq-point Gauss-Legendre rule on [0,1]: (points ascending, weights, sum 1)."""
    x, w = npleg.leggauss(nq)
    return (x + 1.0) / 2.0, w / 2.0


def lagrange_values(nodes, t):
    """V[k, a] = l_a(t_k), l_a the Lagrange polynomial of `nodes` with l_a(nodes[b]) = delta_ab."""
    nodes = np.asarray(nodes, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(t), n))
    for a in range(n):
        for b in range(n):
            if b != a:
                V[:, a] *= (t - nodes[b]) / (nodes[a] - nodes[b])
    return V


def lagrange_derivs(nodes, t):
    """Dv[k, a] = l_a'(t_k) by the product rule: sum over the dropped factor c."""
    nodes = np.asarray(nodes, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = len(nodes)
    Dv = np.zeros((len(t), n))
    for a in range(n):
        for c in range(n):
            if c == a:
                continue
            term = np.full(len(t), 1.0 / (nodes[a] - nodes[c]))
            for b in range(n):
                if b != a and b != c:
                    term *= (t - nodes[b]) / (nodes[a] - nodes[b])
            Dv[:, a] += term
    return Dv


def shape_1d(p):
    """(xi, zeta, omega, S, D): nodes, Gauss points, weights, S[q,a]=l_a(zeta_q), D[q,a]=l_a'(zeta_q)."""
    xi = gll_nodes(p)
    zeta, omega = gauss(p + 1)
    return xi, zeta, omega, lagrange_values(xi, zeta), lagrange_derivs(xi, zeta)
