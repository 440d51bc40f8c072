"""CPU checks of the C ABI: every declared symbol is exported, and host-side validation errors
(no device needed) come back as documented status codes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfq.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mfq_[a-z0-9_]+)\s*\(", src)))


def _lib():
    from paper_1910_13247_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol():
    L = _lib().lib()
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(_lib().EXPORTED)


def test_host_validation_errors():
    lib = _lib()
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_mesh_create(0, 0.0)
    assert e.value.status == lib.MFQ_EINVAL
    with pytest.raises(lib.MfqError):
        lib.mfq_mesh_create(4, 0.2)          # non-invertible deformation
    m = lib.mfq_mesh_create(4, 0.1)
    with pytest.raises(lib.MfqError):
        lib.mfq_space_create(m, 9, 1)
    with pytest.raises(lib.MfqError):
        lib.mfq_space_create(m, 2, 7)
    s = lib.mfq_space_create(m, 4, 1)
    assert lib.mfq_space_n_dofs(s) == 17 ** 3 and lib.mfq_space_n_cells(s) == 64
    with pytest.raises(lib.MfqError):
        lib.mfq_op_create(s, 1.5, 0)
    with pytest.raises(lib.MfqError):
        lib.mfq_op_create(s, 0.5, 5)
    op = lib.mfq_op_create(s, 0.5, 0)
    nbytes = lib.mfq_op_device_bytes(op)
    # 5x2x1-cell bricks at p=4 (one ragged brick spans x of the 4^3 mesh, 2x4 bricks in y and z):
    # a 21x9x5 int32 node lattice per brick plus 6 doubles per quadrature point of its 250 pencils
    nbricks = 1 * 2 * 4
    rnd = lambda b: -(-b // 256) * 256
    assert nbytes == rnd(nbricks * 21 * 9 * 5 * 4) + rnd(nbricks * 5 * 250 * 6 * 8)
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_vmult(op, 256, 512, None)   # unbound operator: rejected before any launch
    assert e.value.status == lib.MFQ_EINVAL
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_op_bind(op, 256, nbytes - 1, None)
    assert e.value.status == lib.MFQ_ENOMEM
    with pytest.raises(lib.MfqError):
        lib.mfq_op_bind(op, 3, nbytes, None)  # misaligned
    # transfer pairs must be nested
    m2 = lib.mfq_mesh_create(8, 0.1)
    s2 = lib.mfq_space_create(m2, 4, 1)
    t = lib.mfq_transfer_create(s, s2)
    lib.mfq_transfer_destroy(t)
    with pytest.raises(lib.MfqError):
        lib.mfq_transfer_create(s2, s)
    s3 = lib.mfq_space_create(m, 2, 1)
    t = lib.mfq_transfer_create(s3, s)       # p-coarsening 4 -> 2 on the same mesh
    lib.mfq_transfer_destroy(t)
    # solver kinds and precision
    with pytest.raises(lib.MfqError):
        lib.mfq_solver_create(op, 9)
    op32 = lib.mfq_op_create(s, 0.5, 1)
    with pytest.raises(lib.MfqError):
        lib.mfq_solver_create(op32, 0)
    sv = lib.mfq_solver_create(op, 2)
    assert lib.mfq_solver_device_bytes(sv) > 0
    with pytest.raises(lib.MfqError):
        lib.mfq_solve(sv, 256, 512, 1e-10, 10, None)   # not bound
    for h, f in [(sv, lib.mfq_solver_destroy), (op32, lib.mfq_op_destroy), (op, lib.mfq_op_destroy),
                 (s3, lib.mfq_space_destroy), (s2, lib.mfq_space_destroy), (s, lib.mfq_space_destroy),
                 (m2, lib.mfq_mesh_destroy), (m, lib.mfq_mesh_destroy)]:
        f(h)


@pytest.mark.parametrize("p", range(1, 9))
def test_library_tables_agree_with_oracle_tables(p):
    # the library's tables (Newton on the Legendre recurrence) and the oracle's (numpy companion
    # roots, leggauss) are independent codes; both feed every parity test
    import numpy as np
    from oracle.tables import shape_1d
    xi, z, w, S, D = _lib().mfq_reference_tables(p)
    xo, zo, wo, So, Do = shape_1d(p)
    np.testing.assert_allclose(xi, xo, atol=2e-16)
    np.testing.assert_allclose(z, zo, atol=2e-16)
    np.testing.assert_allclose(w, wo, atol=2e-16)
    np.testing.assert_allclose(S, So, atol=1e-14)
    np.testing.assert_allclose(D, Do, atol=1e-12 * np.abs(Do).max())


@pytest.mark.parametrize("p,n,brick,launches,groups", [
    (4, 64, (5, 2, 1), 8, 13 * 32 * 64),
    (4, 4, (5, 2, 1), 4, 8),                  # one (ragged) brick along x: the odd-x colours are empty
    (8, 24, (3, 1, 1), 8, 8 * 24 * 24),
    (3, 128, (16, 1, 1), 8, 8 * 128 * 128),
    (1, 1, (32, 2, 1), 1, 1),                 # a single ragged brick
])
def test_operator_layout(p, n, brick, launches, groups):
    """The cell loop's work decomposition: brick shape per degree, one workgroup per brick, one
    launch per non-empty colour of the brick grid."""
    lib = _lib()
    m = lib.mfq_mesh_create(n, 0.1 if n > 1 else 0.0)
    s = lib.mfq_space_create(m, p, 1)
    op = lib.mfq_op_create(s, 0.5, 0)
    lay = lib.mfq_op_get_layout(op)
    assert lay == {"brick": brick, "launches": launches, "workgroups": groups}
    lib.mfq_op_destroy(op)
    lib.mfq_space_destroy(s)
    lib.mfq_mesh_destroy(m)


@pytest.mark.parametrize("p,n", [(1, 1), (1, 4), (2, 3), (3, 2), (4, 3), (8, 1)])
def test_csr_size_matches_assembled_pattern(p, n):
    """Rows, stored entries and buffer size of the assembled matrix, host only: the entry count is
    that of the oracle's assembled matrix, (n(p+1)^2 - n + 1)^3."""
    from oracle import assemble
    lib = _lib()
    m = lib.mfq_mesh_create(n, 0.0)
    s = lib.mfq_space_create(m, p, 1)
    op = lib.mfq_op_create(s, 0.0, lib.MFQ_FP64)
    a = lib.mfq_csr_create(op)
    rows, nnz, nbytes = lib.mfq_csr_size(a)
    Ao = assemble.assemble_csr(p, n, 0.0, 0.0)
    assert rows == Ao.shape[0] == (p * n + 1) ** 3
    assert nnz == Ao.nnz == (n * (p + 1) ** 2 - n + 1) ** 3
    rnd = lambda b: -(-b // 256) * 256
    len1 = 2 * p + 1 if n >= 2 else p + 1
    window = min(2048, (8192 - len1 ** 3) // 256 * 256)
    nblk = -(-nnz // window)
    assert nbytes == rnd((rows + 1) * 8) + rnd(nnz * 4) + rnd(nnz * 8) + rnd((nblk + 1) * 8)
    a32 = lib.mfq_csr_create(op, lib.MFQ_FP32)     # float values: 4 bytes per entry, same pattern
    r32, z32, b32 = lib.mfq_csr_size(a32)
    assert (r32, z32) == (rows, nnz)
    assert b32 == rnd((rows + 1) * 8) + rnd(nnz * 4) + rnd(nnz * 4) + rnd((-(-nnz // 4096) + 1) * 8)
    lib.mfq_csr_destroy(a32)
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_csr_create(op, 7)                  # unknown value precision
    assert e.value.status == lib.MFQ_EINVAL
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_csr_arrays(a)                      # not bound
    assert e.value.status == lib.MFQ_EINVAL
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_csr_bind(a, 256, nbytes, None)     # operator not bound: refused before any launch
    assert e.value.status == lib.MFQ_EINVAL
    lib.mfq_csr_destroy(a)
    op32 = lib.mfq_op_create(s, 0.0, lib.MFQ_FP32)
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_csr_create(op32)
    assert e.value.status == lib.MFQ_EINVAL
    for h, f in ((op32, lib.mfq_op_destroy), (op, lib.mfq_op_destroy), (s, lib.mfq_space_destroy),
                 (m, lib.mfq_mesh_destroy)):
        f(h)


def test_dg_host_validation():
    """DG operator: undeformed meshes only, degree 1..8, n^3 (p+1)^3 DoFs; no device needed."""
    lib = _lib()
    m = lib.mfq_mesh_create(3, 0.0)
    g = lib.mfq_dg_create(m, 4)
    assert lib.mfq_dg_n_dofs(g) == 27 * 125
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_dg_vmult(g, 256, 256, None)          # src and dst overlap
    assert e.value.status == lib.MFQ_EINVAL
    assert lib.mfq_dg_cg_n_dofs(g) == 13 ** 3
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_dg_vmult_prec(g, lib.MFQ_FP32_MFMA, 256, 1 << 20, None)   # precision not offered
    assert e.value.status == lib.MFQ_EINVAL
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_dg_transfer(g, lib.MFQ_FP64, 1, 256, 512, None)           # in and out overlap
    assert e.value.status == lib.MFQ_EINVAL
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_dg_diagonal(g, lib.MFQ_FP64, None, None)
    assert e.value.status == lib.MFQ_EINVAL
    # the multigrid solver: host-side set-up and sizing, the continuous hierarchy under it
    sv = lib.mfq_dg_solver_create(g)
    nbytes = lib.mfq_dg_solver_device_bytes(sv)
    assert nbytes >= 6 * 4 * 27 * 125 + 6 * 8 * 27 * 125
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_dg_solve(sv, 256, 512, 1e-10, 10, None)                   # not bound
    assert e.value.status == lib.MFQ_EINVAL
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_dg_solver_bind(sv, 256, nbytes - 1, None)                 # too small
    assert e.value.status == lib.MFQ_ENOMEM
    lib.mfq_dg_solver_destroy(sv)
    prm = lib.mfq_solver_default_params()
    prm.smoother_degree = 0
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_dg_solver_create(g, prm)
    assert e.value.status == lib.MFQ_EINVAL
    m1 = lib.mfq_mesh_create(1, 0.0)
    g1 = lib.mfq_dg_create(m1, 1)                     # Q1 on one cell: no interior lattice node
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_dg_solver_create(g1)
    assert e.value.status == lib.MFQ_EINVAL
    lib.mfq_dg_destroy(g1)
    lib.mfq_mesh_destroy(m1)
    lib.mfq_dg_destroy(g)
    with pytest.raises(lib.MfqError):
        lib.mfq_dg_create(m, 9)
    md = lib.mfq_mesh_create(3, 0.1)
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_dg_create(md, 2)                     # deformed mesh refused
    assert e.value.status == lib.MFQ_EINVAL
    lib.mfq_mesh_destroy(md)
    lib.mfq_mesh_destroy(m)


def test_chebyshev_noalloc_limits_on_the_host():
    """The workspace-free smoother states its fixed array size and rejects, before any device
    call, operators whose three work vectors would not fit and operators not yet bound."""
    lib = _lib()
    cap = lib.mfq_chebyshev_noalloc_max_bytes()
    assert cap == 64 << 20
    m = lib.mfq_mesh_create(40, 0.1)
    s = lib.mfq_space_create(m, 4, 1)                      # 161^3 = 4,173,281 DoFs
    big = lib.mfq_op_create(s, 0.5, 0)
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_chebyshev_noalloc(big, 256, 256, 256, 1, 3, 0.1, 1.0, None)
    assert e.value.status == lib.MFQ_EINVAL and "fixed device array" in str(e.value)
    m2 = lib.mfq_mesh_create(8, 0.1)
    s2 = lib.mfq_space_create(m2, 4, 1)
    small = lib.mfq_op_create(s2, 0.5, 0)
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_chebyshev_noalloc(small, 256, 256, 256, 1, 3, 0.1, 1.0, None)
    assert e.value.status == lib.MFQ_EINVAL and "not bound" in str(e.value)
    for h, f in ((big, "mfq_op_destroy"), (small, "mfq_op_destroy"), (s, "mfq_space_destroy"),
                 (s2, "mfq_space_destroy"), (m, "mfq_mesh_destroy"), (m2, "mfq_mesh_destroy")):
        getattr(lib.lib(), f)(h)


def test_hanging_operator_host_validation():
    lib = _lib()
    for args in ((0, 0.0, 2, 0.0, 0), (2, 0.2, 2, 0.0, 0), (2, 0.0, 9, 0.0, 0), (2, 0.0, 2, 0.0, 2),
                 (2, 0.0, 2, 1.5, 0)):
        with pytest.raises(lib.MfqError) as e:
            lib.mfq_hang_create(*args)
        assert e.value.status == lib.MFQ_EINVAL
    h = lib.mfq_hang_create(3, 0.1, 4, 0.5, 0)
    assert lib.mfq_hang_n_dofs(h) == 13 ** 3 + 25 ** 3
    nbytes = lib.mfq_hang_device_bytes(h)
    assert nbytes > 0 and nbytes % 256 == 0
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_hang_vmult(h, 256, 512, None)      # unbound: rejected before any launch
    assert e.value.status == lib.MFQ_EINVAL
    with pytest.raises(lib.MfqError) as e:
        lib.mfq_hang_bind(h, 256, nbytes - 1, None)
    assert e.value.status == lib.MFQ_ENOMEM
    assert lib.mfq_hang_cg_work_bytes(h) >= 3 * 8 * lib.mfq_hang_n_dofs(h)
    lib.mfq_hang_destroy(h)
