"""Matrix-free Q_p finite elements on AMD MI355X (gfx950).

The compute path is libmfq.so (hand-written HIP kernels behind a C ABI, see include/mfq.h);
this package is its Python binding.  ``_lib`` has one function per C entry point with the
same name; the classes below only add ownership: device memory comes from PyTorch (caching
allocator, current stream), the library works inside those buffers.

Objects mirror the problem statement of the deal.II paper (arXiv 1910.13247, Fig. 1 and
Sec. 3.1-3.7): a mesh, a finite element space on it, the operator of the weak form applied
matrix-free, level transfers, and solvers (CG, geometric multigrid).
"""
from . import _lib
from ._lib import (MfqError, MFQ_FP64, MFQ_FP32, MFQ_FP32_MFMA, MFQ_BC_NONE, MFQ_BC_DIRICHLET0, MFQ_SOLVER_CG,
                   MFQ_SOLVER_GMG_FP64, MFQ_SOLVER_GMG_MIXED, MFQ_SOLVER_GMG_MIXED_IR, MFQ_OK, MFQ_EINVAL,
                   MFQ_ENOMEM, MFQ_EHIP, MFQ_ENOCONV, MFQ_ENONFINITE, MFQ_EBUSY)

__all__ = ["Mesh", "Space", "Operator", "HangingOperator", "Transfer", "Solver", "Batch", "MfqError", "MFQ_FP64", "MFQ_FP32", "MFQ_FP32_MFMA",
           "MFQ_BC_NONE", "MFQ_BC_DIRICHLET0", "MFQ_SOLVER_CG", "MFQ_SOLVER_GMG_FP64",
           "MFQ_SOLVER_GMG_MIXED", "MFQ_SOLVER_GMG_MIXED_IR", "MFQ_OK", "MFQ_EINVAL", "MFQ_ENOMEM",
           "MFQ_EHIP", "MFQ_ENOCONV", "MFQ_ENONFINITE", "MFQ_EBUSY", "batch_step", "SparseMatrix", "DGOperator",
           "DGSolver"]


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dtype(precision):
    torch = _torch()
    return torch.float64 if precision == MFQ_FP64 else torch.float32


def _release(obj, destroy):
    """Destroy obj's library handle once.  At interpreter shutdown the binding module may already
    be torn down; the process is ending, so the handle is left to it then.  (Each __del__ binds
    this function as a default argument, which outlives the module's globals.)"""
    h = getattr(obj, "handle", None)
    obj.handle = None
    if h and _lib is not None and getattr(_lib, "_lib", None) is not None:
        getattr(_lib, destroy)(h)


def _check_vec(t, n, precision, name):
    torch = _torch()
    if not t.is_cuda or t.dtype != _dtype(precision) or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need a contiguous CUDA tensor of {n} {_dtype(precision)} values")
    return t.data_ptr()


class Mesh:
    """n^3 cells on the unit cube, deformed by x + A*sin(pi x)sin(pi y)sin(pi z)*(1,1,1)."""

    def __init__(self, n_cells_1d, amplitude=0.0):
        self.n = int(n_cells_1d)
        self.amplitude = float(amplitude)
        self.handle = _lib.mfq_mesh_create(self.n, self.amplitude)

    def __del__(self, _release=_release):
        _release(self, "mfq_mesh_destroy")


class Space:
    """Continuous Q_p space (GLL nodes) on a mesh, optionally with homogeneous Dirichlet rows."""

    def __init__(self, mesh, degree, bc=MFQ_BC_DIRICHLET0):
        self.mesh = mesh
        self.degree = int(degree)
        self.bc = int(bc)
        self.handle = _lib.mfq_space_create(mesh.handle, self.degree, self.bc)
        self.n_dofs = _lib.mfq_space_n_dofs(self.handle)
        self.n_cells = _lib.mfq_space_n_cells(self.handle)

    def random(self, seed, precision=MFQ_FP64, x=None, stream=None):
        """Counter-based (SplitMix64) uniform[-1,1) vector, zero on Dirichlet nodes."""
        torch = _torch()
        if x is None:
            x = torch.empty(self.n_dofs, dtype=torch.float64 if precision == MFQ_FP64 else torch.float32,
                            device="cuda")
        _lib.mfq_space_random(self.handle, precision, _check_vec(x, self.n_dofs, precision, "x"), int(seed),
                              _stream(stream))
        return x

    def apply_mask(self, x, precision=MFQ_FP64, stream=None):
        _lib.mfq_space_apply_mask(self.handle, precision, _check_vec(x, self.n_dofs, precision, "x"), _stream(stream))
        return x

    def __del__(self, _release=_release):
        _release(self, "mfq_space_destroy")


class Operator:
    """Matrix-free variable-coefficient Laplacian on a space; device data in a torch buffer."""

    def __init__(self, space, alpha=0.0, precision=MFQ_FP64, device="cuda", stream=None):
        torch = _torch()
        self.space = space
        self.alpha = float(alpha)
        self.precision = int(precision)
        self.dtype = _dtype(self.precision)
        self.handle = _lib.mfq_op_create(space.handle, self.alpha, self.precision)
        self.device_bytes = _lib.mfq_op_device_bytes(self.handle)
        self.buffer = torch.empty(self.device_bytes, dtype=torch.uint8, device=device)
        _lib.mfq_op_bind(self.handle, self.buffer.data_ptr(), self.device_bytes, _stream(stream))

    @property
    def n_dofs(self):
        return self.space.n_dofs

    def new_vector(self):
        torch = _torch()
        return torch.empty(self.n_dofs, dtype=self.dtype, device=self.buffer.device)

    def vmult(self, src, dst=None, stream=None):
        if dst is None:
            dst = self.new_vector()
        _lib.mfq_vmult(self.handle, _check_vec(src, self.n_dofs, self.precision, "src"),
                       _check_vec(dst, self.n_dofs, self.precision, "dst"), _stream(stream))
        return dst

    def layout(self):
        """Work decomposition of the cell loop: brick shape, launches per vmult, workgroups."""
        return _lib.mfq_op_get_layout(self.handle)

    def set_fused_updates(self, enable):
        """Smoother steps and multigrid residuals fused into the operator application (default on)."""
        _lib.mfq_op_set_fused_updates(self.handle, enable)

    def vmult_add(self, src, dst, stream=None):
        _lib.mfq_vmult_add(self.handle, _check_vec(src, self.n_dofs, self.precision, "src"),
                           _check_vec(dst, self.n_dofs, self.precision, "dst"), _stream(stream))
        return dst

    def diagonal(self, stream=None):
        d = self.new_vector()
        _lib.mfq_op_diagonal(self.handle, d.data_ptr(), _stream(stream))
        return d

    def geometry(self, stream=None):
        torch = _torch()
        out = torch.empty((self.space.n_cells, (self.space.degree + 1) ** 3, 6), dtype=torch.float64,
                          device=self.buffer.device)
        _lib.mfq_op_geometry(self.handle, out.data_ptr(), _stream(stream))
        return out

    def rhs_manufactured(self, stream=None):
        torch = _torch()
        b = torch.empty(self.n_dofs, dtype=torch.float64, device=self.buffer.device)
        _lib.mfq_rhs_manufactured(self.handle, b.data_ptr(), _stream(stream))
        return b

    def chebyshev(self, inv_diag, b, x, x_is_zero, degree, lmin, lmax, work=None, stream=None):
        torch = _torch()
        if work is None:
            work = torch.empty(3 * self.n_dofs, dtype=self.dtype, device=self.buffer.device)
        _lib.mfq_chebyshev(self.handle, _check_vec(inv_diag, self.n_dofs, self.precision, "inv_diag"),
                           _check_vec(b, self.n_dofs, self.precision, "b"),
                           _check_vec(x, self.n_dofs, self.precision, "x"), x_is_zero, degree, lmin, lmax,
                           work.data_ptr(), _stream(stream))
        return x

    def chebyshev_noalloc(self, inv_diag, b, x, x_is_zero, degree, lmin, lmax, stream=None):
        """mfq_chebyshev with the library's fixed per-device work array (no allocation)."""
        _lib.mfq_chebyshev_noalloc(self.handle, _check_vec(inv_diag, self.n_dofs, self.precision, "inv_diag"),
                                   _check_vec(b, self.n_dofs, self.precision, "b"),
                                   _check_vec(x, self.n_dofs, self.precision, "x"), x_is_zero, degree, lmin, lmax,
                                   _stream(stream))
        return x

    def __del__(self, _release=_release):
        _release(self, "mfq_op_destroy")


class HangingOperator:
    """The operator on the two-block mesh with a 2:1 interface (hanging nodes on the fine side):
    the unit cube in n^3 cells joined at X1 = 1 to [1,2] x [0,1]^2 in (2n)^3 cells (mfq_hang_*).
    Vectors: block 0's lattice, then block 1's; device data in a torch buffer."""

    def __init__(self, n_coarse, degree, amplitude=0.0, alpha=0.0, precision=MFQ_FP64, device="cuda", stream=None):
        torch = _torch()
        self.precision = int(precision)
        self.dtype = _dtype(self.precision)
        self.handle = _lib.mfq_hang_create(int(n_coarse), float(amplitude), int(degree), float(alpha),
                                           self.precision)
        self.n_dofs = _lib.mfq_hang_n_dofs(self.handle)
        self.device_bytes = _lib.mfq_hang_device_bytes(self.handle)
        self.buffer = torch.empty(self.device_bytes, dtype=torch.uint8, device=device)
        _lib.mfq_hang_bind(self.handle, self.buffer.data_ptr(), self.device_bytes, _stream(stream))

    def vmult(self, src, dst=None, stream=None):
        torch = _torch()
        if dst is None:
            dst = torch.empty(self.n_dofs, dtype=self.dtype, device=self.buffer.device)
        _lib.mfq_hang_vmult(self.handle, _check_vec(src, self.n_dofs, self.precision, "src"),
                            _check_vec(dst, self.n_dofs, self.precision, "dst"), _stream(stream))
        return dst

    def cg(self, b, rtol=1e-10, max_iter=10000, stream=None, check=True):
        """(x, status, info): unpreconditioned FP64 CG from zero (mfq_hang_cg)."""
        torch = _torch()
        x = torch.empty(self.n_dofs, dtype=torch.float64, device=self.buffer.device)
        nb = _lib.mfq_hang_cg_work_bytes(self.handle)
        work = torch.empty(nb, dtype=torch.uint8, device=self.buffer.device)
        st, info = _lib.mfq_hang_cg(self.handle, _check_vec(b, self.n_dofs, MFQ_FP64, "b"),
                                    _check_vec(x, self.n_dofs, MFQ_FP64, "x"), rtol, max_iter, work.data_ptr(), nb,
                                    _stream(stream), check=check)
        return x, st, info

    def __del__(self, _release=_release):
        _release(self, "mfq_hang_destroy")


class DGOperator:
    """Symmetric interior penalty DG Laplacian of degree p on the undeformed n^3 mesh (no device
    storage); vectors are float64, cell-major."""

    def __init__(self, mesh, degree):
        self.mesh = mesh
        self.degree = int(degree)
        self.handle = _lib.mfq_dg_create(mesh.handle, self.degree)
        self.n_dofs = _lib.mfq_dg_n_dofs(self.handle)

        self.cg_n_dofs = _lib.mfq_dg_cg_n_dofs(self.handle)

    def vmult(self, src, dst=None, stream=None):
        """dst = A src; float64 vectors use mfq_dg_vmult, float32 ones the FP32 product."""
        torch = _torch()
        if dst is None:
            dst = torch.empty(self.n_dofs, dtype=src.dtype, device=src.device)
        if src.dtype == torch.float64:
            _lib.mfq_dg_vmult(self.handle, _check_vec(src, self.n_dofs, MFQ_FP64, "src"),
                              _check_vec(dst, self.n_dofs, MFQ_FP64, "dst"), _stream(stream))
        else:
            _lib.mfq_dg_vmult_prec(self.handle, MFQ_FP32, _check_vec(src, self.n_dofs, MFQ_FP32, "src"),
                                   _check_vec(dst, self.n_dofs, MFQ_FP32, "dst"), _stream(stream))
        return dst

    def diagonal(self, precision=MFQ_FP64, device="cuda", stream=None):
        torch = _torch()
        d = torch.empty(self.n_dofs, dtype=_dtype(precision), device=device)
        _lib.mfq_dg_diagonal(self.handle, int(precision), _check_vec(d, self.n_dofs, precision, "diag"),
                             _stream(stream))
        return d

    def from_cg(self, cg, stream=None):
        """DG vector of the continuous lattice vector cg (every cell takes its nodes' values)."""
        torch = _torch()
        prec = MFQ_FP64 if cg.dtype == torch.float64 else MFQ_FP32
        out = torch.empty(self.n_dofs, dtype=cg.dtype, device=cg.device)
        _lib.mfq_dg_transfer(self.handle, prec, 1, _check_vec(cg, self.cg_n_dofs, prec, "cg"),
                             _check_vec(out, self.n_dofs, prec, "out"), _stream(stream))
        return out

    def to_cg(self, dg, stream=None):
        """Transpose of from_cg: each lattice node sums its cell copies; zero on the boundary."""
        torch = _torch()
        prec = MFQ_FP64 if dg.dtype == torch.float64 else MFQ_FP32
        out = torch.empty(self.cg_n_dofs, dtype=dg.dtype, device=dg.device)
        _lib.mfq_dg_transfer(self.handle, prec, 0, _check_vec(dg, self.n_dofs, prec, "dg"),
                             _check_vec(out, self.cg_n_dofs, prec, "out"), _stream(stream))
        return out

    def __del__(self, _release=_release):
        _release(self, "mfq_dg_destroy")


class DGSolver:
    """FP64 CG on a DGOperator preconditioned by the FP32 V-cycle DG -> continuous Q_p -> the
    continuous hierarchy (see mfq_dg_solver_create)."""

    def __init__(self, dg, stream=None, device="cuda", lambda_override=None, **params):
        torch = _torch()
        import ctypes
        self.op = dg
        prm = _lib.mfq_solver_default_params()
        params.setdefault("smoother_degree", 6)     # the Chebyshev degree of the paper's DG runs
        for k, v in params.items():
            setattr(prm, k, v)
        if lambda_override is not None:
            # lmax of the continuous levels 1.. (finest last), then of the DG level
            self._lam = (ctypes.c_double * len(lambda_override))(*lambda_override)
            prm.n_lambda_override = len(lambda_override)
            prm.lambda_override = ctypes.cast(self._lam, ctypes.POINTER(ctypes.c_double))
        self.params = prm
        self.handle = _lib.mfq_dg_solver_create(dg.handle, prm)
        self.device_bytes = _lib.mfq_dg_solver_device_bytes(self.handle)
        self.buffer = torch.empty(max(self.device_bytes, 256), dtype=torch.uint8, device=device)
        _lib.mfq_dg_solver_bind(self.handle, self.buffer.data_ptr(), self.device_bytes, _stream(stream))

    def new_vector(self):
        torch = _torch()
        return torch.zeros(self.op.n_dofs, dtype=torch.float64, device=self.buffer.device)

    def solve(self, b, x=None, rtol=1e-10, max_iter=1000, stream=None, check=True):
        if x is None:
            x = self.new_vector()
        st, info = _lib.mfq_dg_solve(self.handle, _check_vec(b, self.op.n_dofs, MFQ_FP64, "b"),
                                     _check_vec(x, self.op.n_dofs, MFQ_FP64, "x"), rtol, max_iter,
                                     _stream(stream), check=check)
        return x, info, st

    def precondition(self, r, z=None, stream=None):
        if z is None:
            z = self.new_vector()
        _lib.mfq_dg_precondition(self.handle, _check_vec(r, self.op.n_dofs, MFQ_FP64, "r"),
                                 _check_vec(z, self.op.n_dofs, MFQ_FP64, "z"), _stream(stream))
        return z

    def __del__(self, _release=_release):
        _release(self, "mfq_dg_solver_destroy")


class SparseMatrix:
    """The operator assembled as a CSR matrix on the device (for comparison with the matrix-free
    action); device data in a torch buffer.  rowptr int64, cols int32, vals float64 or float32
    (`precision`, also the precision of the product's vectors)."""

    def __init__(self, op, precision=MFQ_FP64, stream=None):
        torch = _torch()
        if op.precision != MFQ_FP64:
            raise ValueError("the assembled matrix needs an FP64 operator")
        self.op = op
        self.precision = int(precision)
        self.dtype = _dtype(self.precision)
        self.handle = _lib.mfq_csr_create(op.handle, self.precision)
        self.n_rows, self.nnz, self.device_bytes = _lib.mfq_csr_size(self.handle)
        self.buffer = torch.empty(self.device_bytes, dtype=torch.uint8, device=op.buffer.device)
        _lib.mfq_csr_bind(self.handle, self.buffer.data_ptr(), self.device_bytes, _stream(stream))

    def arrays(self):
        """(rowptr, cols, vals) as torch views of the bound buffer."""
        torch = _torch()
        r, c, v = _lib.mfq_csr_arrays(self.handle)
        base = self.buffer.data_ptr()

        def view(addr, count, dtype, size):
            off = addr - base
            return self.buffer[off:off + count * size].view(dtype)

        vs = 8 if self.precision == MFQ_FP64 else 4
        return (view(r, self.n_rows + 1, torch.int64, 8), view(c, self.nnz, torch.int32, 4),
                view(v, self.nnz, self.dtype, vs))

    def spmv(self, src, dst=None, stream=None):
        torch = _torch()
        if dst is None:
            dst = torch.empty(self.n_rows, dtype=self.dtype, device=self.buffer.device)
        _lib.mfq_csr_spmv(self.handle, _check_vec(src, self.n_rows, self.precision, "src"),
                          _check_vec(dst, self.n_rows, self.precision, "dst"), _stream(stream))
        return dst

    def __del__(self, _release=_release):
        _release(self, "mfq_csr_destroy")


class Transfer:
    """Interpolation between nested spaces (h: fine mesh halves coarse cells; p: lower degree)."""

    def __init__(self, coarse, fine):
        self.coarse, self.fine = coarse, fine
        self.handle = _lib.mfq_transfer_create(coarse.handle, fine.handle)

    def prolongate(self, coarse_vec, fine_vec, precision=MFQ_FP64, stream=None):
        _lib.mfq_prolongate(self.handle, precision, _check_vec(coarse_vec, self.coarse.n_dofs, precision, "coarse"),
                            _check_vec(fine_vec, self.fine.n_dofs, precision, "fine"), _stream(stream))
        return fine_vec

    def restrict(self, fine_vec, coarse_vec, precision=MFQ_FP64, stream=None):
        _lib.mfq_restrict(self.handle, precision, _check_vec(fine_vec, self.fine.n_dofs, precision, "fine"),
                          _check_vec(coarse_vec, self.coarse.n_dofs, precision, "coarse"), _stream(stream))
        return coarse_vec

    def __del__(self, _release=_release):
        _release(self, "mfq_transfer_destroy")


def batch_step(solvers, iters=2):
    """Advance every running solve in `solvers` by up to `iters` CG iterations (each on the stream
    it was begun on), wait once for all of them, and return their done flags."""
    return _lib.mfq_batch_step([s.handle for s in solvers], iters)


class Batch:
    """Batched steps over many running solves (mfq_batch_*): one launch per (kernel, degree) covers
    every qualifying solve; device workspace in a torch buffer."""

    def __init__(self, max_solvers=256, device="cuda", stream=None):
        torch = _torch()
        self.max_solvers = int(max_solvers)
        self.handle = _lib.mfq_batch_create(self.max_solvers)
        self.device_bytes = _lib.mfq_batch_device_bytes(self.handle)
        self.buffer = torch.empty(self.device_bytes, dtype=torch.uint8, device=device)
        _lib.mfq_batch_bind(self.handle, self.buffer.data_ptr(), self.device_bytes, _stream(stream))

    def run(self, solvers, iters=2, stream=None):
        """Advance every running solve in `solvers` (all begun on `stream`); returns done flags."""
        return _lib.mfq_batch_run(self.handle, [s.handle if hasattr(s, "handle") else s for s in solvers], iters,
                                  _stream(stream))

    def __del__(self, _release=_release):
        _release(self, "mfq_batch_destroy")


class Solver:
    """CG / GMG-preconditioned CG on an FP64 operator (see mfq_solver_kind).  lazy=True binds with
    mfq_solver_bind_lazy: the eigenvalue bounds are estimated by the first solve step."""

    def __init__(self, op64, kind=MFQ_SOLVER_GMG_MIXED, stream=None, lambda_override=None, lazy=False, **params):
        torch = _torch()
        import ctypes
        self.op = op64
        self.kind = int(kind)
        prm = _lib.mfq_solver_default_params()
        for k, v in params.items():
            setattr(prm, k, v)
        if lambda_override is not None:
            self._lam = (ctypes.c_double * len(lambda_override))(*lambda_override)
            prm.n_lambda_override = len(lambda_override)
            prm.lambda_override = ctypes.cast(self._lam, ctypes.POINTER(ctypes.c_double))
        self.params = prm
        self.handle = _lib.mfq_solver_create(op64.handle, self.kind, prm)
        self.device_bytes = _lib.mfq_solver_device_bytes(self.handle)
        self.buffer = torch.empty(max(self.device_bytes, 256), dtype=torch.uint8, device=op64.buffer.device)
        bind = _lib.mfq_solver_bind_lazy if lazy else _lib.mfq_solver_bind
        bind(self.handle, self.buffer.data_ptr(), self.device_bytes, _stream(stream))

    def solve(self, b, x=None, rtol=1e-10, max_iter=10000, stream=None, check=True):
        if x is None:
            x = self.op.new_vector()
        st, info = _lib.mfq_solve(self.handle, _check_vec(b, self.op.n_dofs, MFQ_FP64, "b"),
                                  _check_vec(x, self.op.n_dofs, MFQ_FP64, "x"), rtol, max_iter, _stream(stream),
                                  check=check)
        return x, info, st

    def begin(self, b, x, rtol=1e-10, max_iter=10000, stream=None):
        """Start a resumable solve (advance it with batch_step, finish with end)."""
        _lib.mfq_solve_begin(self.handle, _check_vec(b, self.op.n_dofs, MFQ_FP64, "b"),
                             _check_vec(x, self.op.n_dofs, MFQ_FP64, "x"), rtol, max_iter, _stream(stream))

    def end(self, check=True):
        """(status, SolveInfo) of a solve that batch_step reported done."""
        return _lib.mfq_solve_end(self.handle, check=check)

    def precondition(self, r, z=None, stream=None):
        if z is None:
            z = self.op.new_vector()
        _lib.mfq_solver_precondition(self.handle, _check_vec(r, self.op.n_dofs, MFQ_FP64, "r"),
                                     _check_vec(z, self.op.n_dofs, MFQ_FP64, "z"), _stream(stream))
        return z

    def lambdas(self, n_levels):
        return _lib.mfq_solver_lambdas(self.handle, max(n_levels - 1, 0))

    def __del__(self, _release=_release):
        _release(self, "mfq_solver_destroy")
