"""Linear solves and residual certificates (oracle; test infrastructure only).

* Conjugate gradients (Hestenes-Stiefel), x0 = 0, stopping on the recurred
  residual and re-checking the true residual at exit.
* Sparse direct solve through scipy's SuperLU.
* Residual certificate (reading of "relative residual 1e-10"): the true
  residual ||b - A x||_2 / ||b||_2 in FP64.  Any x meeting the bound is a
  correct solution, so GPU solutions are compared by certificate, not bitwise.
"""
import numpy as np
import scipy.sparse.linalg as spla


def rel_residual(apply, b, x):
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    r = b - apply(np.asarray(x, dtype=np.float64))
    return np.linalg.norm(r) / (nb if nb > 0 else 1.0)


def cg(apply, b, rtol=1e-10, maxit=10000, precond=None):
    """Preconditioned CG; returns (x, iterations, true relative residual)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    nb = np.linalg.norm(b)
    if nb == 0:
        return x, 0, 0.0
    r = b.copy()
    z = precond(r) if precond else r
    pdir = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        Ap = apply(pdir)
        alpha = rz / (pdir @ Ap)
        x += alpha * pdir
        r -= alpha * Ap
        it += 1
        if np.linalg.norm(r) / nb <= rtol:
            break
        z = precond(r) if precond else r
        rz_new = r @ z
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
    return x, it, rel_residual(apply, b, x)


def direct_solve(Acsr, b):
    return spla.spsolve(Acsr.tocsc(), b)
