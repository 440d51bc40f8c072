"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds problem sizes and random draws only: none of the finite element
arithmetic.  Both the GPU path and the CPU oracle receive these arrays as
arguments; neither generates its own random inputs.

The paper's only experiment (Sec. 6.1) is a synthetic Laplace problem on a
box, so no dataset is being stood in for; the workloads below are the
Poisson / variable-coefficient problems the benchmark and tests run.
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Problem:
    name: str
    degree: int          # p of Q_p
    cells_1d: int        # n, mesh of n^3 cells on the unit cube
    amplitude: float     # A of the sine deformation x + A*s(x)*(1,1,1); 0 = affine
    alpha: float         # a(x) = 1 + alpha*sin(2 pi x)sin(2 pi y)sin(2 pi z)
    bc: int = 1          # 1 = homogeneous Dirichlet on the cube boundary

    @property
    def n_dofs(self):
        return (self.degree * self.cells_1d + 1) ** 3

    @property
    def n_cells(self):
        return self.cells_1d ** 3


# Workloads (sizes, geometry, coefficient)
POISSON_Q2_8 = Problem("poisson_q2_8^3_affine", 2, 8, 0.0, 0.0)              # 4,913 DoFs
VARCOEF_Q4_64 = Problem("varcoef_q4_64^3_curved", 4, 64, 0.1, 0.5)           # 16,974,593 DoFs
VARCOEF_Q3_128 = Problem("varcoef_q3_128^3_curved", 3, 128, 0.1, 0.5)        # 57,066,625 DoFs
VARCOEF_Q8_24 = Problem("varcoef_q8_24^3_curved", 8, 24, 0.1, 0.5)           # 7,189,057 DoFs


def uniform_vector(n, seed=0):
    """Seeded FP64 vector, uniform in [-1, 1): numpy default_rng(seed).uniform(-1, 1, n)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, int(n))


def serving_stream(n_requests=2000, rate=200.0, seed=0):
    """Request stream for the serving loop: Poisson arrivals and per-request problem draws.

    Returns a list of dicts with arrival time (s), degree p ~ U{1..6},
    cells_1d n ~ U{4..48}, alpha ~ U[0, 0.9] and the seed of the request's
    right-hand side (= the request index).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    t = np.cumsum(gaps)
    ps = rng.integers(1, 7, n_requests)
    ns = rng.integers(4, 49, n_requests)
    alphas = rng.uniform(0.0, 0.9, n_requests)
    return [dict(index=i, arrival=float(t[i]), degree=int(ps[i]), cells_1d=int(ns[i]),
                 alpha=float(alphas[i]), rhs_seed=i) for i in range(n_requests)]
