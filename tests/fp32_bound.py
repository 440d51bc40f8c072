"""First-order componentwise error bound of an FP32 V-cycle against the exact (FP64 oracle) V-cycle.

The V-cycle is linear in its input and in every intermediate vector, so the deviation of a result
computed with rounding is, to first order, the sum over all computing steps of (the linear map
from that step's output to the result) times (the rounding error committed in that step):

    |z_fp32 - z| <= sum_i |L_i| beta_i,

with beta_i a componentwise bound on step i's own rounding error.  The steps are recorded as a
straight-line program (``Tape``) while the oracle's V-cycle is evaluated in FP64 with the same
definition, and the maps L_i are accumulated backwards from the result as dense matrices (small
meshes only).  Each step's beta is the rounding model of the FP32 kernel that performs it
(u = 2^-24):

* operator application y = A x: 2 k u (|A| |x|) on free rows, k = 8(p+1) + 16 (eight 1D
  contractions of p+1 terms, the 3x3 product, the stored G and input roundings, node sums), with
  |A| the magnitude matrix sum_q |B_q|^T |G_q| |B_q|; Dirichlet rows are copied exactly;
* Jacobi scaling by the FP32 diagonal: its relative error eps_d = k_d u (|A| 1)_i / A_ii + u
  (k_d = 4(p+1) + 16; the FP32 diagonal's own bound) plus the cast coefficients and products;
* vector updates: u per rounded sum or product, coefficients cast from FP64 (u each);
* restriction and prolongation: (3 NF1 + 14) u (|P|^T |r|) and (3 (p_c+1) + 4) u (|P| |x|);
* dense coarse solve: FP64 accumulation, one rounding to FP32 (u |x|);
* casts of the input to FP32: u |r|.
"""
import numpy as np
import scipy.sparse as sp

U32 = 2.0 ** -24


class Tape:
    """Straight-line program of linear steps; ``bound(out)`` accumulates |d out / d step| beta."""

    def __init__(self):
        self.vals = []
        self.steps = []

    def input(self, v):
        self.vals.append(np.asarray(v, dtype=np.float64))
        return len(self.vals) - 1

    @staticmethod
    def _apply(M, v):
        kind, m = M
        if kind == "scalar":
            return m * v
        if kind == "diag":
            return m * v
        return m @ v

    def step(self, ins, beta):
        """y = sum_j M_j x_j, M_j = ('scalar', s) | ('diag', vec) | ('mat', matrix); beta = rounding bound of y."""
        y = None
        for i, M in ins:
            t = self._apply(M, self.vals[i])
            y = t if y is None else y + t
        self.vals.append(y)
        out = len(self.vals) - 1
        self.steps.append((out, ins, np.asarray(beta, dtype=np.float64)))
        return out

    def value(self, i):
        return self.vals[i]

    def bound(self, out):
        n_out = len(self.vals[out])
        lam = {out: np.eye(n_out)}
        total = np.zeros(n_out)
        for o, ins, beta in reversed(self.steps):
            L = lam.pop(o, None)
            if L is None:
                continue
            total += np.abs(L) @ beta
            for i, (kind, m) in ins:
                if kind == "scalar":
                    G = m * L
                elif kind == "diag":
                    G = L * m[None, :]
                elif sp.issparse(m):
                    G = (m.T @ L.T).T
                else:
                    G = L @ m
                lam[i] = lam[i] + G if i in lam else G
        return total


class Fp32Level:
    """One level of the oracle hierarchy with what the rounding model needs."""

    def __init__(self, level, mag, prolong=None, prolong_kind=None):
        self.L = level
        self.A = level.A.tocsr()
        self.Mag = mag.tocsr()
        self.m = level.m
        self.dinv = level.dinv
        d = 1.0 / self.dinv
        kd = 4 * (level.p + 1) + 16
        mag1 = self.Mag @ np.ones(self.A.shape[0])
        self.eps_d = np.where(self.m > 0, kd * U32 * mag1 / d + U32, 0.0)
        self.k = 8 * (level.p + 1) + 16
        self.P = prolong              # from the next coarser level to this one (None on the coarsest)
        self.Pabs = abs(prolong) if prolong is not None else None
        self.nf1 = prolong_kind       # fine nodes per coarse cell in 1D for the transfer into this level


def _I():
    return ("scalar", 1.0)


def _vmult(tp, lv, x):
    xv = tp.value(x)
    beta = 2 * lv.k * U32 * (lv.Mag @ np.abs(xv)) * lv.m
    return tp.step([(x, ("mat", lv.A))], beta)


def _chebyshev(tp, lv, b, x, degree):
    """The GPU's Chebyshev smoother (first step, then degree-1 steps), step by step."""
    theta = 0.5 * (lv.L.lmax + lv.L.lmin)
    delta = 0.5 * (lv.L.lmax - lv.L.lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    if x is None:
        r = b
    else:
        t = _vmult(tp, lv, x)
        r = tp.step([(b, _I()), (t, ("scalar", -1.0))], U32 * np.abs(tp.value(b) - tp.value(t)))
    dv = lv.dinv * tp.value(r) / theta
    d = tp.step([(r, ("diag", lv.dinv / theta))], (3 * U32 + lv.eps_d) * np.abs(dv))
    if x is None:
        x = d
    else:
        x = tp.step([(x, _I()), (d, _I())], U32 * np.abs(tp.value(x) + tp.value(d)))
    for _ in range(degree - 1):
        t = _vmult(tp, lv, d)
        r = tp.step([(r, _I()), (t, ("scalar", -1.0))], U32 * np.abs(tp.value(r) - tp.value(t)))
        rho_new = 1.0 / (2.0 * sigma - rho)
        c1, c2 = rho_new * rho, 2.0 * rho_new / delta
        t1 = np.abs(c1 * tp.value(d))
        t2 = np.abs(c2 * lv.dinv * tp.value(r))
        d = tp.step([(d, ("scalar", c1)), (r, ("diag", c2 * lv.dinv))], 4 * U32 * t1 + (4 * U32 + lv.eps_d) * t2)
        x = tp.step([(x, _I()), (d, _I())], U32 * np.abs(tp.value(x) + tp.value(d)))
        rho = rho_new
    return x


def _vcycle(tp, lvs, l, b, degree):
    lv = lvs[l]
    if l == 0:
        Ainv = np.linalg.inv(lv.A.toarray())
        xv = Ainv @ tp.value(b)
        return tp.step([(b, ("mat", Ainv))], U32 * np.abs(xv))
    x = _chebyshev(tp, lv, b, None, degree)
    t = _vmult(tp, lv, x)
    r = tp.step([(b, _I()), (t, ("scalar", -1.0))], U32 * np.abs(tp.value(b) - tp.value(t)))
    PT = lv.P.T.tocsr()
    rv = tp.value(r)
    bc = tp.step([(r, ("mat", PT))], (3 * lv.nf1 + 14) * U32 * (abs(PT) @ np.abs(rv)))
    xc = _vcycle(tp, lvs, l - 1, bc, degree)
    pc = lvs[l - 1].L.p
    xcv = tp.value(xc)
    t = tp.step([(xc, ("mat", lv.P))], (3 * (pc + 1) + 4) * U32 * (lv.Pabs @ np.abs(xcv)))
    x = tp.step([(x, _I()), (t, _I())], U32 * np.abs(tp.value(x) + tp.value(t)))
    return _chebyshev(tp, lv, b, x, degree)


def vcycle_fp32_bound(levels, prolong, mags, r, degree=3):
    """(z, bound): the V-cycle of ``oracle.gmg.vcycle`` applied to r in FP64, and the first-order
    componentwise bound of an FP32 evaluation's deviation from it.  ``mags`` holds each level's
    magnitude matrix (``oracle.ebe.magnitude_csr``); every level's lmin/lmax must be set."""
    lvs = []
    for l, L in enumerate(levels):
        if l == 0:
            lvs.append(Fp32Level(L, mags[l]))
            continue
        C = levels[l - 1]
        nf1 = 2 * C.p + 1 if L.n == 2 * C.n else L.p + 1
        lvs.append(Fp32Level(L, mags[l], prolong[l], nf1))
    tp = Tape()
    r0 = tp.input(r)
    b = tp.step([(r0, _I())], U32 * np.abs(r))
    z = _vcycle(tp, lvs, len(lvs) - 1, b, degree)
    return tp.value(z), tp.bound(z)
