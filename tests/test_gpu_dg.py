"""GPU parity of the matrix-free DG-SIPG operator (mfq_dg_*) against the oracle's assembled DG
matrix: FP64, ||y - y_o||_inf <= 1e-12 ||y_o||_inf, every degree, meshes with boundary and
interior faces of both parities; the full Q4 64^3 size on rows the oracle recomputes one by one."""
import numpy as np
import pytest

from oracle import dg
from synthetic import uniform_vector

pytestmark = pytest.mark.gpu

SIZES = {1: 5, 2: 4, 3: 3, 4: 3, 5: 2, 6: 2, 7: 2, 8: 2}


def _mfq():
    import paper_1910_13247_amd as mfq
    return mfq


def _torch():
    import torch
    return torch


def _apply(p, n, x_np):
    mfq = _mfq()
    torch = _torch()
    op = mfq.DGOperator(mfq.Mesh(n, 0.0), p)
    y = op.vmult(torch.from_numpy(x_np).cuda())
    torch.cuda.synchronize()
    return op, y.cpu().numpy()


@pytest.mark.parametrize("p", range(1, 9))
def test_dg_vmult_matches_assembled(p):
    n = SIZES[p]
    print(f"dg vmult p={p} n={n}", flush=True)
    x = uniform_vector(dg.n_dofs(p, n), seed=70 + p)
    op, y = _apply(p, n, x)
    assert op.n_dofs == dg.n_dofs(p, n)
    yo = dg.assemble(p, n) @ x
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()


@pytest.mark.parametrize("p", [1, 3, 8])
def test_dg_single_cell(p):
    """n = 1: every face is a boundary face."""
    x = uniform_vector(dg.n_dofs(p, 1), seed=5)
    _, y = _apply(p, 1, x)
    yo = dg.assemble(p, 1) @ x
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()


@pytest.mark.parametrize("p,n", [(2, 3), (4, 2)])
def test_dg_consistency_on_the_gpu(p, n):
    """The polynomial solution of the oracle's consistency pin, through the GPU operator."""
    f = lambda x, y, z: 2 * (y * (1 - y) * z * (1 - z) + x * (1 - x) * z * (1 - z) + x * (1 - x) * y * (1 - y))
    u = dg.nodal_interpolant(p, n, lambda x, y, z: x * (1 - x) * y * (1 - y) * z * (1 - z))
    _, y = _apply(p, n, u)
    F = dg.load_vector(p, n, f)
    assert np.abs(y - F).max() <= 1e-11 * np.abs(F).max()


def test_dg_deterministic_and_errors():
    mfq = _mfq()
    torch = _torch()
    op = mfq.DGOperator(mfq.Mesh(4, 0.0), 3)
    x = torch.from_numpy(uniform_vector(op.n_dofs, seed=2)).cuda()
    y1 = op.vmult(x)
    y2 = op.vmult(x)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    with pytest.raises(mfq.MfqError):
        mfq.DGOperator(mfq.Mesh(4, 0.1), 3)


def test_dg_full_size_q4_64_sampled():
    """Q4 on 64^3 cells (32,768,000 DoFs): 300 sampled rows recomputed by the oracle from their
    cell's matrix and its six faces."""
    p, n = 4, 64
    print("dg full-size Q4 64^3", flush=True)
    x = uniform_vector(dg.n_dofs(p, n), seed=0)
    _, y = _apply(p, n, x)
    nloc = (p + 1) ** 3
    rng = np.random.default_rng(3)
    rows = np.concatenate([rng.integers(0, len(x), 290),
                           [0, nloc - 1, len(x) - 1, (n ** 3 // 2) * nloc + 62, 63 * nloc + 124]])
    yo = dg.dg_rows(p, n, x, rows)
    assert np.abs(y[rows] - yo).max() <= 1e-12 * np.abs(yo).max()
