"""ctypes binding of libmfq.so: one Python function per C entry point, same names.

Argument marshalling only: every computation runs in the library's HIP kernels.  Device
pointers are plain integers (e.g. ``tensor.data_ptr()``) and streams are hipStream_t handles
(e.g. ``torch.cuda.current_stream().cuda_stream``).  A non-zero status raises ``MfqError``.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# MFQ_LIBRARY selects another build of the same library (the host-sanitized one)
LIB_PATH = os.environ.get("MFQ_LIBRARY") or os.path.join(_HERE, "libmfq.so")

MFQ_OK, MFQ_EINVAL, MFQ_ENOMEM, MFQ_EHIP, MFQ_ENOCONV, MFQ_ENONFINITE, MFQ_EBUSY = 0, -1, -2, -3, -4, -5, -6
MFQ_FP64, MFQ_FP32, MFQ_FP32_MFMA = 0, 1, 2
MFQ_BC_NONE, MFQ_BC_DIRICHLET0 = 0, 1
MFQ_SOLVER_CG, MFQ_SOLVER_GMG_FP64, MFQ_SOLVER_GMG_MIXED, MFQ_SOLVER_GMG_MIXED_IR = 0, 1, 2, 3

STATUS_NAMES = {0: "MFQ_OK", -1: "MFQ_EINVAL", -2: "MFQ_ENOMEM", -3: "MFQ_EHIP", -4: "MFQ_ENOCONV",
                -5: "MFQ_ENONFINITE", -6: "MFQ_EBUSY"}


class MfqError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class SolverParams(C.Structure):
    _fields_ = [("smoother_degree", C.c_int), ("lanczos_iters", C.c_int), ("lambda_factor", C.c_double),
                ("lambda_ratio", C.c_double), ("inner_rtol", C.c_double), ("check_every", C.c_int),
                ("n_lambda_override", C.c_int), ("lambda_override", C.POINTER(C.c_double)),
                ("coarse_mode", C.c_int), ("coarse_degree", C.c_int), ("coarse_ratio", C.c_double),
                ("coarse_dofs", C.c_int), ("use_graphs", C.c_int)]


class OpLayout(C.Structure):
    _fields_ = [("brick", C.c_int * 3), ("launches", C.c_int), ("workgroups", C.c_int64)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("outer_iterations", C.c_int), ("rel_residual", C.c_double),
                ("seconds", C.c_double), ("n_levels", C.c_int)]


_lib = None

P = C.c_void_p
PP = C.POINTER(C.c_void_p)
I = C.c_int
D = C.c_double
SZ = C.c_size_t
I64 = C.c_int64

_SIGS = {
    "mfq_version": ([], C.c_char_p),
    "mfq_last_error": ([], C.c_char_p),
    "mfq_reference_tables": ([I, P, P, P, P, P], I),
    "mfq_mesh_create": ([I, D, PP], I),
    "mfq_mesh_destroy": ([P], None),
    "mfq_space_create": ([P, I, I, PP], I),
    "mfq_space_destroy": ([P], None),
    "mfq_space_n_dofs": ([P], I64),
    "mfq_space_n_cells": ([P], I64),
    "mfq_space_apply_mask": ([P, I, P, P], I),
    "mfq_space_random": ([P, I, P, C.c_uint64, P], I),
    "mfq_op_create": ([P, D, I, PP], I),
    "mfq_op_destroy": ([P], None),
    "mfq_op_device_bytes": ([P, C.POINTER(SZ)], I),
    "mfq_op_set_fused_updates": ([P, I], I),
    "mfq_op_bind": ([P, P, SZ, P], I),
    "mfq_vmult": ([P, P, P, P], I),
    "mfq_vmult_add": ([P, P, P, P], I),
    "mfq_op_get_layout": ([P, C.POINTER(OpLayout)], I),
    "mfq_op_diagonal": ([P, P, P], I),
    "mfq_op_geometry": ([P, P, P], I),
    "mfq_rhs_manufactured": ([P, P, P], I),
    "mfq_csr_create": ([P, I, PP], I),
    "mfq_csr_destroy": ([P], None),
    "mfq_csr_size": ([P, C.POINTER(I64), C.POINTER(I64), C.POINTER(SZ)], I),
    "mfq_csr_bind": ([P, P, SZ, P], I),
    "mfq_csr_arrays": ([P, PP, PP, PP], I),
    "mfq_csr_spmv": ([P, P, P, P], I),
    "mfq_dg_create": ([P, I, PP], I),
    "mfq_dg_destroy": ([P], None),
    "mfq_dg_n_dofs": ([P], I64),
    "mfq_dg_vmult": ([P, P, P, P], I),
    "mfq_dg_vmult_prec": ([P, I, P, P, P], I),
    "mfq_dg_diagonal": ([P, I, P, P], I),
    "mfq_dg_cg_n_dofs": ([P], I64),
    "mfq_dg_transfer": ([P, I, I, P, P, P], I),
    "mfq_dg_solver_create": ([P, C.POINTER(SolverParams), PP], I),
    "mfq_dg_solver_destroy": ([P], None),
    "mfq_dg_solver_device_bytes": ([P, C.POINTER(SZ)], I),
    "mfq_dg_solver_bind": ([P, P, SZ, P], I),
    "mfq_dg_precondition": ([P, P, P, P], I),
    "mfq_dg_solve": ([P, P, P, D, I, P, C.POINTER(SolveInfo)], I),
    "mfq_transfer_create": ([P, P, PP], I),
    "mfq_transfer_destroy": ([P], None),
    "mfq_prolongate": ([P, I, P, P, P], I),
    "mfq_restrict": ([P, I, P, P, P], I),
    "mfq_chebyshev": ([P, P, P, P, I, I, D, D, P, P], I),
    "mfq_chebyshev_noalloc": ([P, P, P, P, I, I, D, D, P], I),
    "mfq_chebyshev_noalloc_max_bytes": ([], SZ),
    "mfq_solver_default_params": ([C.POINTER(SolverParams)], None),
    "mfq_solver_create": ([P, I, C.POINTER(SolverParams), PP], I),
    "mfq_solver_destroy": ([P], None),
    "mfq_solver_device_bytes": ([P, C.POINTER(SZ)], I),
    "mfq_solver_bind": ([P, P, SZ, P], I),
    "mfq_solver_bind_lazy": ([P, P, SZ, P], I),
    "mfq_solve": ([P, P, P, D, I, P, C.POINTER(SolveInfo)], I),
    "mfq_solve_begin": ([P, P, P, D, I, P], I),
    "mfq_batch_step": ([C.POINTER(C.c_void_p), I, I, C.POINTER(C.c_int)], I),
    "mfq_solve_end": ([P, C.POINTER(SolveInfo)], I),
    "mfq_solve_step_async": ([P, I], I),
    "mfq_solve_step_poll": ([P, C.POINTER(C.c_int), C.POINTER(C.c_int)], I),
    "mfq_solver_lambdas": ([P, C.POINTER(D), I], I),
    "mfq_solver_precondition": ([P, P, P, P], I),
    "mfq_batch_create": ([I, PP], I),
    "mfq_batch_destroy": ([P], None),
    "mfq_batch_device_bytes": ([P, C.POINTER(SZ)], I),
    "mfq_batch_bind": ([P, P, SZ, P], I),
    "mfq_batch_run": ([P, C.POINTER(C.c_void_p), I, I, P, C.POINTER(C.c_int)], I),
    "mfq_hang_create": ([I, D, I, D, I, PP], I),
    "mfq_hang_destroy": ([P], None),
    "mfq_hang_n_dofs": ([P], I64),
    "mfq_hang_device_bytes": ([P, C.POINTER(SZ)], I),
    "mfq_hang_bind": ([P, P, SZ, P], I),
    "mfq_hang_vmult": ([P, P, P, P], I),
    "mfq_hang_cg_work_bytes": ([P], SZ),
    "mfq_hang_cg": ([P, P, P, D, I, P, SZ, P, C.POINTER(SolveInfo)], I),
}

EXPORTED = tuple(_SIGS)


def lib():
    """The loaded library; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1910_13247_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(status):
    if status != MFQ_OK:
        raise MfqError(status, lib().mfq_last_error().decode())
    return status


def _handle(fn, *args):
    out = C.c_void_p()
    _check(fn(*args, C.byref(out)))
    return out.value


# ---- one wrapper per entry point (same names as the C ABI)
def mfq_version():
    return lib().mfq_version().decode()


def mfq_last_error():
    return lib().mfq_last_error().decode()


def mfq_reference_tables(degree):
    """(xi, zeta, omega, S, D) as numpy arrays (S, D of shape [p+1, p+1])."""
    import numpy as np
    n1 = degree + 1
    xi, z, w = np.empty(n1), np.empty(n1), np.empty(n1)
    S, Dm = np.empty((n1, n1)), np.empty((n1, n1))
    _check(lib().mfq_reference_tables(degree, xi.ctypes.data, z.ctypes.data, w.ctypes.data, S.ctypes.data,
                                      Dm.ctypes.data))
    return xi, z, w, S, Dm


def mfq_mesh_create(n_cells_1d, amplitude):
    return _handle(lib().mfq_mesh_create, n_cells_1d, amplitude)


def mfq_mesh_destroy(mesh):
    lib().mfq_mesh_destroy(mesh)


def mfq_space_create(mesh, degree, bc):
    return _handle(lib().mfq_space_create, mesh, degree, bc)


def mfq_space_destroy(space):
    lib().mfq_space_destroy(space)


def mfq_space_n_dofs(space):
    return lib().mfq_space_n_dofs(space)


def mfq_space_n_cells(space):
    return lib().mfq_space_n_cells(space)


def mfq_space_random(space, precision, x, seed, stream):
    _check(lib().mfq_space_random(space, precision, x, seed, stream))


def mfq_space_apply_mask(space, precision, x, stream):
    _check(lib().mfq_space_apply_mask(space, precision, x, stream))


def mfq_op_create(space, alpha, precision):
    return _handle(lib().mfq_op_create, space, alpha, precision)


def mfq_op_destroy(op):
    lib().mfq_op_destroy(op)


def mfq_op_device_bytes(op):
    n = SZ()
    _check(lib().mfq_op_device_bytes(op, C.byref(n)))
    return n.value


def mfq_op_set_fused_updates(op, enable):
    _check(lib().mfq_op_set_fused_updates(op, 1 if enable else 0))


def mfq_op_bind(op, dev_buf, nbytes, stream):
    _check(lib().mfq_op_bind(op, dev_buf, nbytes, stream))


def mfq_vmult(op, src, dst, stream):
    _check(lib().mfq_vmult(op, src, dst, stream))


def mfq_vmult_add(op, src, dst, stream):
    _check(lib().mfq_vmult_add(op, src, dst, stream))


def mfq_op_get_layout(op):
    """Work decomposition of the cell loop as a dict (brick, launches, workgroups)."""
    r = OpLayout()
    _check(lib().mfq_op_get_layout(op, C.byref(r)))
    return {"brick": tuple(r.brick), "launches": r.launches, "workgroups": r.workgroups}


def mfq_op_diagonal(op, diag, stream):
    _check(lib().mfq_op_diagonal(op, diag, stream))


def mfq_op_geometry(op, out, stream):
    _check(lib().mfq_op_geometry(op, out, stream))


def mfq_rhs_manufactured(op, b, stream):
    _check(lib().mfq_rhs_manufactured(op, b, stream))


def mfq_csr_create(op, precision=MFQ_FP64):
    return _handle(lib().mfq_csr_create, op, precision)


def mfq_csr_destroy(a):
    lib().mfq_csr_destroy(a)


def mfq_csr_size(a):
    """(n_rows, nnz, device_bytes)."""
    r, z, b = I64(), I64(), SZ()
    _check(lib().mfq_csr_size(a, C.byref(r), C.byref(z), C.byref(b)))
    return r.value, z.value, b.value


def mfq_csr_bind(a, dev_buf, nbytes, stream):
    _check(lib().mfq_csr_bind(a, dev_buf, nbytes, stream))


def mfq_csr_arrays(a):
    """Device addresses (rowptr, cols, vals) inside the bound buffer."""
    r, c, v = C.c_void_p(), C.c_void_p(), C.c_void_p()
    _check(lib().mfq_csr_arrays(a, C.byref(r), C.byref(c), C.byref(v)))
    return r.value, c.value, v.value


def mfq_csr_spmv(a, src, dst, stream):
    _check(lib().mfq_csr_spmv(a, src, dst, stream))


def mfq_dg_create(mesh, degree):
    return _handle(lib().mfq_dg_create, mesh, degree)


def mfq_dg_destroy(op):
    lib().mfq_dg_destroy(op)


def mfq_dg_n_dofs(op):
    return lib().mfq_dg_n_dofs(op)


def mfq_dg_vmult(op, src, dst, stream):
    _check(lib().mfq_dg_vmult(op, src, dst, stream))


def mfq_dg_vmult_prec(op, precision, src, dst, stream):
    _check(lib().mfq_dg_vmult_prec(op, precision, src, dst, stream))


def mfq_dg_diagonal(op, precision, diag, stream):
    _check(lib().mfq_dg_diagonal(op, precision, diag, stream))


def mfq_dg_cg_n_dofs(op):
    return lib().mfq_dg_cg_n_dofs(op)


def mfq_dg_transfer(op, precision, to_dg, src, dst, stream):
    _check(lib().mfq_dg_transfer(op, precision, int(bool(to_dg)), src, dst, stream))


def mfq_dg_solver_create(op, params=None):
    return _handle(lib().mfq_dg_solver_create, op, C.byref(params) if params is not None else None)


def mfq_dg_solver_destroy(s):
    lib().mfq_dg_solver_destroy(s)


def mfq_dg_solver_device_bytes(s):
    n = SZ()
    _check(lib().mfq_dg_solver_device_bytes(s, C.byref(n)))
    return n.value


def mfq_dg_solver_bind(s, dev_buf, nbytes, stream):
    _check(lib().mfq_dg_solver_bind(s, dev_buf, nbytes, stream))


def mfq_dg_precondition(s, r, z, stream):
    _check(lib().mfq_dg_precondition(s, r, z, stream))


def mfq_dg_solve(s, b, x, rtol, max_iter, stream, check=True):
    """Returns (status, SolveInfo).  With check=True a status other than MFQ_OK raises."""
    info = SolveInfo()
    st = lib().mfq_dg_solve(s, b, x, rtol, max_iter, stream, C.byref(info))
    if check:
        _check(st)
    return st, info


def mfq_transfer_create(coarse, fine):
    return _handle(lib().mfq_transfer_create, coarse, fine)


def mfq_transfer_destroy(t):
    lib().mfq_transfer_destroy(t)


def mfq_prolongate(t, precision, coarse, fine, stream):
    _check(lib().mfq_prolongate(t, precision, coarse, fine, stream))


def mfq_restrict(t, precision, fine, coarse, stream):
    _check(lib().mfq_restrict(t, precision, fine, coarse, stream))


def mfq_chebyshev(op, inv_diag, b, x, x_is_zero, degree, lmin, lmax, work, stream):
    _check(lib().mfq_chebyshev(op, inv_diag, b, x, int(bool(x_is_zero)), degree, lmin, lmax, work, stream))


def mfq_chebyshev_noalloc(op, inv_diag, b, x, x_is_zero, degree, lmin, lmax, stream):
    _check(lib().mfq_chebyshev_noalloc(op, inv_diag, b, x, int(bool(x_is_zero)), degree, lmin, lmax, stream))


def mfq_chebyshev_noalloc_max_bytes():
    return int(lib().mfq_chebyshev_noalloc_max_bytes())


def mfq_solver_default_params():
    prm = SolverParams()
    lib().mfq_solver_default_params(C.byref(prm))
    return prm


def mfq_solver_create(op64, kind, params=None):
    return _handle(lib().mfq_solver_create, op64, kind, C.byref(params) if params is not None else None)


def mfq_solver_destroy(s):
    lib().mfq_solver_destroy(s)


def mfq_solver_device_bytes(s):
    n = SZ()
    _check(lib().mfq_solver_device_bytes(s, C.byref(n)))
    return n.value


def mfq_solver_bind(s, dev_buf, nbytes, stream):
    _check(lib().mfq_solver_bind(s, dev_buf, nbytes, stream))


def mfq_solver_bind_lazy(s, dev_buf, nbytes, stream):
    _check(lib().mfq_solver_bind_lazy(s, dev_buf, nbytes, stream))


def mfq_solve(s, b, x, rtol, max_iter, stream, check=True):
    """Returns (status, SolveInfo).  With check=True a status other than MFQ_OK raises."""
    info = SolveInfo()
    st = lib().mfq_solve(s, b, x, rtol, max_iter, stream, C.byref(info))
    if check:
        _check(st)
    return st, info


def mfq_solve_begin(s, b, x, rtol, max_iter, stream):
    _check(lib().mfq_solve_begin(s, b, x, rtol, max_iter, stream))


def mfq_batch_step(solvers, iters):
    """One step of the running solves `solvers` (handles); returns their done flags."""
    n = len(solvers)
    arr = (C.c_void_p * max(n, 1))(*solvers)
    done = (C.c_int * max(n, 1))()
    _check(lib().mfq_batch_step(arr, n, iters, done))
    return [bool(done[i]) for i in range(n)]


def mfq_solve_step_async(s, iters):
    _check(lib().mfq_solve_step_async(s, iters))


def mfq_solve_step_poll(s):
    """(ready, done) of the solve's last asynchronous step; never waits."""
    ready, done = C.c_int(), C.c_int()
    _check(lib().mfq_solve_step_poll(s, C.byref(ready), C.byref(done)))
    return bool(ready.value), bool(done.value)


def mfq_solve_end(s, check=True):
    """Returns (status, SolveInfo) of a finished solve; check=True raises on a status other than MFQ_OK."""
    info = SolveInfo()
    st = lib().mfq_solve_end(s, C.byref(info))
    if check:
        _check(st)
    return st, info


def mfq_solver_lambdas(s, n):
    arr = (C.c_double * max(n, 1))()
    _check(lib().mfq_solver_lambdas(s, arr, n))
    return [arr[i] for i in range(n)]


def mfq_solver_precondition(s, r, z, stream):
    _check(lib().mfq_solver_precondition(s, r, z, stream))


def mfq_hang_create(n_coarse, amplitude, degree, alpha, precision=MFQ_FP64):
    return _handle(lib().mfq_hang_create, n_coarse, amplitude, degree, alpha, precision)


def mfq_hang_destroy(h):
    lib().mfq_hang_destroy(h)


def mfq_hang_n_dofs(h):
    return int(lib().mfq_hang_n_dofs(h))


def mfq_hang_device_bytes(h):
    n = SZ()
    _check(lib().mfq_hang_device_bytes(h, C.byref(n)))
    return n.value


def mfq_hang_bind(h, dev_buf, nbytes, stream):
    _check(lib().mfq_hang_bind(h, dev_buf, nbytes, stream))


def mfq_hang_vmult(h, src, dst, stream):
    _check(lib().mfq_hang_vmult(h, src, dst, stream))


def mfq_hang_cg_work_bytes(h):
    return int(lib().mfq_hang_cg_work_bytes(h))


def mfq_hang_cg(h, b, x, rtol, max_iter, work, work_bytes, stream, check=True):
    """Returns (status, SolveInfo).  With check=True a status other than MFQ_OK raises."""
    info = SolveInfo()
    st = lib().mfq_hang_cg(h, b, x, rtol, max_iter, work, work_bytes, stream, C.byref(info))
    if check:
        _check(st)
    return st, info


def mfq_batch_create(max_solvers):
    return _handle(lib().mfq_batch_create, max_solvers)


def mfq_batch_destroy(b):
    lib().mfq_batch_destroy(b)


def mfq_batch_device_bytes(b):
    n = SZ()
    _check(lib().mfq_batch_device_bytes(b, C.byref(n)))
    return n.value


def mfq_batch_bind(b, dev_buf, nbytes, stream):
    _check(lib().mfq_batch_bind(b, dev_buf, nbytes, stream))


def mfq_batch_run(b, solvers, iters, stream):
    """Advances every listed running solve (batched launches where they qualify); returns the
    list of done flags."""
    n = len(solvers)
    arr = (C.c_void_p * max(n, 1))(*solvers)
    done = (C.c_int * max(n, 1))()
    _check(lib().mfq_batch_run(b, arr, n, iters, stream, done))
    return [bool(done[i]) for i in range(n)]
