"""The workspace-free Chebyshev smoother (mfq_chebyshev_noalloc) against mfq_chebyshev with a
caller workspace, through the C ABI: same kernels, so the results must be bitwise equal.  Two calls
in a row on one device, the second on a smaller operator (the fixed array keeps the first call's
contents), in FP64 and FP32, from zero and from a given x, and one call at the largest FP64 size
that fits the array."""
import numpy as np
import pytest

from synthetic import uniform_vector

pytestmark = pytest.mark.gpu


def _case(mfq, torch, p, n, prec, seed):
    op = mfq.Operator(mfq.Space(mfq.Mesh(n, 0.1), p, mfq.MFQ_BC_DIRICHLET0), 0.5, prec)
    d = op.diagonal()
    dinv = 1.0 / d
    b = torch.from_numpy(uniform_vector(op.n_dofs, seed)).to(op.dtype).cuda()
    op.space.apply_mask(b, prec)
    x0 = torch.from_numpy(uniform_vector(op.n_dofs, seed + 1)).to(op.dtype).cuda()
    return op, dinv, b, x0


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("x_is_zero", [True, False])
def test_noalloc_matches_workspace_entry_point_twice(prec, x_is_zero):
    import torch
    import paper_1910_13247_amd as mfq
    lmin, lmax = 0.15, 2.2
    for (p, n, seed) in ((4, 12, 5), (3, 6, 7)):  # 117,649 then 6,859 DoFs
        print(f"no-alloc chebyshev p={p} n={n} prec={prec} x_is_zero={x_is_zero}", flush=True)
        op, dinv, b, x0 = _case(mfq, torch, p, n, prec, seed)
        x_ref = x0.clone()
        op.chebyshev(dinv, b, x_ref, x_is_zero, 3, lmin, lmax)
        x_na = x0.clone()
        op.chebyshev_noalloc(dinv, b, x_na, x_is_zero, 3, lmin, lmax)
        torch.cuda.synchronize()
        assert torch.isfinite(x_ref).all()
        assert torch.equal(x_na, x_ref), (p, n, (x_na - x_ref).abs().max().item())
        assert not torch.equal(x_ref, x0)


def test_noalloc_at_the_largest_fp64_size():
    import torch
    import paper_1910_13247_amd as mfq
    from paper_1910_13247_amd import _lib
    p, n = 4, 34                                   # 137^3 = 2,571,353 DoFs: 61.7 MB of work vectors
    op, dinv, b, x0 = _case(mfq, torch, p, n, mfq.MFQ_FP64, 21)
    assert 3 * op.n_dofs * 8 <= _lib.mfq_chebyshev_noalloc_max_bytes()
    print(f"no-alloc chebyshev at {op.n_dofs} DoFs", flush=True)
    x_ref = x0.clone()
    op.chebyshev(dinv, b, x_ref, False, 4, 0.15, 2.2)
    x_na = x0.clone()
    op.chebyshev_noalloc(dinv, b, x_na, False, 4, 0.15, 2.2)
    torch.cuda.synchronize()
    assert torch.equal(x_na, x_ref)
    big = mfq.Operator(mfq.Space(mfq.Mesh(36, 0.1), 4, mfq.MFQ_BC_DIRICHLET0), 0.5, mfq.MFQ_FP64)
    with pytest.raises(_lib.MfqError):
        big.chebyshev_noalloc(big.new_vector(), big.new_vector(), big.new_vector(), True, 3, 0.1, 1.0)
