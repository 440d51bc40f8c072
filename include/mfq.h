/*
 * mfq.h — C ABI of the matrix-free Q_p finite element library for AMD MI355X (gfx950).
 *
 * What it computes (section numbers refer to the deal.II paper, arXiv 1910.13247):
 *   The action y = A x of the operator of the weak form of eq. (1), generalised to a
 *   variable coefficient, a(u,v) = int a(x) grad u . grad v dx, discretised with continuous
 *   tensor-product Lagrange elements Q_p on a hexahedral mesh (Sec. 3.1, 3.4), integrated
 *   with shape-function gradients and JxW at quadrature points as in the cell loop of
 *   Sec. 2.4, and applied without assembling a matrix, by evaluating the integrals on the
 *   fly with the tensor-product (sum factorisation) structure of the shape functions
 *   (Sec. 3.6) on the GPU (Sec. 3.7).  The operator is used inside conjugate gradients and a
 *   geometric multigrid preconditioner with Chebyshev smoothing (Sec. 3.5) whose V-cycle runs
 *   in single precision under a double-precision correction (Sec. 6.1).
 *
 * Problem statement fixed by this library (readings where the paper is silent):
 *   - mesh: n^3 cells on the unit cube, optionally deformed by the exact map
 *     x = X + A*sin(pi X1) sin(pi X2) sin(pi X3)*(1,1,1) evaluated at every quadrature point;
 *   - element: Q_p, p = 1..8, nodes at the Gauss-Lobatto-Legendre points, lexicographic
 *     numbering (x fastest) of the (p*n+1)^3 lattice nodes;
 *   - quadrature: (p+1)^3-point tensor Gauss-Legendre;
 *   - coefficient: a(x) = 1 + alpha*sin(2 pi x1) sin(2 pi x2) sin(2 pi x3) at the physical point;
 *   - Dirichlet (bc = MFQ_BC_DIRICHLET0): y = m*A(m*x) + (1-m)*x with m = 0 on boundary nodes.
 *
 * Conventions
 *   - Every function returns an mfq_status (0 = MFQ_OK, < 0 = error).  On error the
 *     out-parameters are left untouched and mfq_last_error() returns a message
 *     (thread-local).  Arguments are validated on the host before any launch.
 *   - Device memory is owned by the caller.  Objects that need device storage report its size
 *     (*_device_bytes) and are bound to a caller-provided buffer (*_bind); the library never
 *     allocates device memory on the hot path.  The buffer must stay alive and unmodified while
 *     the object is used.  All device pointers are plain device addresses (e.g. torch
 *     data_ptr()); alignment of 256 bytes is required for bound buffers and 16 bytes for vectors.
 *   - Streams are hipStream_t passed as void* (NULL = the null stream).  Launch functions are
 *     asynchronous and do not synchronise the host unless stated.  Kernel faults surface at
 *     the next synchronising call as MFQ_EHIP.
 *   - Handles are not thread-safe.  Host handles are owned by the caller and freed with the
 *     matching *_destroy (NULL is accepted).
 *   - Vectors have length mfq_space_n_dofs() and hold boundary entries.  Their element type is
 *     the precision of the object that consumes them: double for MFQ_FP64, float for MFQ_FP32.
 */
#ifndef MFQ_H
#define MFQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MFQ_OK = 0,
  MFQ_EINVAL = -1,      /* invalid argument (sizes, degree, NULL, unbound object, ...) */
  MFQ_ENOMEM = -2,      /* caller buffer too small / host allocation failed */
  MFQ_EHIP = -3,        /* HIP runtime error (message in mfq_last_error) */
  MFQ_ENOCONV = -4,     /* solver did not reach the tolerance within max_iter (info is valid) */
  MFQ_ENONFINITE = -5,  /* NaN or Inf met in a solver residual */
  MFQ_EBUSY = -6        /* object in use by an unfinished batched solve */
} mfq_status;

/* MFQ_FP32_MFMA: an FP32 operator (FP32 storage and arithmetic, same results within the FP32
 * bound) whose cell loop runs its 1D contractions on the matrix cores (v_mfma_f32_16x16x4f32);
 * as a vector precision it means float, like MFQ_FP32. */
typedef enum { MFQ_FP64 = 0, MFQ_FP32 = 1, MFQ_FP32_MFMA = 2 } mfq_precision;
typedef enum { MFQ_BC_NONE = 0, MFQ_BC_DIRICHLET0 = 1 } mfq_bc;

typedef struct mfq_mesh mfq_mesh;
typedef struct mfq_space mfq_space;
typedef struct mfq_op mfq_op;
typedef struct mfq_transfer mfq_transfer;
typedef struct mfq_csr mfq_csr;
typedef struct mfq_dg mfq_dg;
typedef struct mfq_solver mfq_solver;
typedef struct mfq_dg_solver mfq_dg_solver;
typedef struct mfq_hang mfq_hang;
typedef struct mfq_batch mfq_batch;

/* Library version string and the message of the last failed call on this thread. */
const char* mfq_version(void);
const char* mfq_last_error(void);

/* Host copies of the 1D reference data of Q_p (Sec. 3.4: reference-cell data computed once and
 * cached): GLL nodes xi[p+1], Gauss points zeta[p+1] and weights omega[p+1] on [0,1] (weights sum
 * to 1), S[q*(p+1)+a] = l_a(zeta_q), D[q*(p+1)+a] = l_a'(zeta_q).  Host pointers, caller-owned. */
int mfq_reference_tables(int degree, double* xi, double* zeta, double* omega, double* S, double* D);

/* ---------------------------------------------------------------- mesh / space (Sec. 3.1, 3.4)
 * Mesh of n_cells_1d^3 cells on [0,1]^3 (1 <= n_cells_1d <= 1024), deformed with the given
 * amplitude (0 = affine; |amplitude| < 1/(3 pi) keeps the map invertible). */
int mfq_mesh_create(int n_cells_1d, double amplitude, mfq_mesh** out);
void mfq_mesh_destroy(mfq_mesh* mesh);

/* Q_p space on a mesh: degree 1..8, bc one of mfq_bc.  The space keeps a reference to the
 * mesh, which must outlive it.  Fails with MFQ_EINVAL when (p*n+1)^3 >= 2^31. */
int mfq_space_create(const mfq_mesh* mesh, int degree, int bc, mfq_space** out);
void mfq_space_destroy(mfq_space* space);
int64_t mfq_space_n_dofs(const mfq_space* space);   /* (p*n+1)^3, -1 on NULL */
int64_t mfq_space_n_cells(const mfq_space* space);  /* n^3, -1 on NULL */

/* b = m*x in place on `n_dofs` entries (zero on Dirichlet nodes): the algebraic right-hand side
 * of a nodal load vector.  precision selects double/float. */
int mfq_space_apply_mask(const mfq_space* space, int precision, void* x, void* hip_stream);

/* x_i = 2 u_i - 1 with u_i = (z_i >> 11) 2^-53 and z_i the SplitMix64 output (Steele, Lea and
 * Flood, OOPSLA 2014) of the state seed + (i+1) 0x9E3779B97F4A7C15, for i = 0..n_dofs-1; zero on
 * Dirichlet nodes when the space has MFQ_BC_DIRICHLET0.  A counter-based random load vector
 * (independent of launch shape), e.g. the right-hand sides of a stream of solve requests. */
int mfq_space_random(const mfq_space* space, int precision, void* x, uint64_t seed, void* hip_stream);

/* ---------------------------------------------------------------- operator (Sec. 3.6, 3.7)
 * The variable-coefficient operator on a space, computed in `precision` (MFQ_FP64, MFQ_FP32 or
 * MFQ_FP32_MFMA).
 * Device storage: the cell index maps (int32, (p+1)^3 per cell) and the merged
 * quadrature-point tensor G_q = w_q a(x_q) det(J_q) J_q^{-1} J_q^{-T} (6 values per quadrature
 * point, stored in `precision`, always computed in FP64 from the analytic Jacobian). */
int mfq_op_create(const mfq_space* space, double alpha, int precision, mfq_op** out);
void mfq_op_destroy(mfq_op* op);
int mfq_op_device_bytes(const mfq_op* op, size_t* bytes);
/* Binds `bytes` of device memory at dev_buf (256-byte aligned) and fills the index maps and
 * G on the stream (asynchronous). */
int mfq_op_bind(mfq_op* op, void* dev_buf, size_t bytes, void* hip_stream);

/* dst = A src (Dirichlet rows as identity).  src, dst: device vectors of n_dofs elements of
 * the operator's precision; they must not overlap.  Asynchronous, no host synchronisation. */
int mfq_vmult(const mfq_op* op, const void* src, void* dst, void* hip_stream);

/* dst += A src (same operator, Dirichlet rows add src): the cell loop alone, without clearing dst.
 * Both are deterministic (fixed summation order, no atomics): equal inputs give bitwise equal
 * outputs.  One launch per non-empty colour of the work decomposition (mfq_op_get_layout). */
int mfq_vmult_add(const mfq_op* op, const void* src, void* dst, void* hip_stream);

/* Work decomposition of the cell loop, for callers that time or profile it: the mesh is cut into
 * bricks of brick[0] x brick[1] x brick[2] cells, one workgroup each; `launches` kernel launches
 * (one per non-empty brick colour) make one mfq_vmult or mfq_vmult_add, with `workgroups`
 * workgroups (bricks) over all of them.  Host only; valid before mfq_op_bind. */
typedef struct {
  int brick[3];
  int launches;
  int64_t workgroups;
} mfq_op_layout;
int mfq_op_get_layout(const mfq_op* op, mfq_op_layout* out);

/* diag = diagonal of A (1 on Dirichlet rows), computed matrix-free from the same quadrature. */
int mfq_op_diagonal(const mfq_op* op, void* diag, void* hip_stream);

/* Copies G to out as double [n_cells][(p+1)^3][6] in the order (xx, xy, xz, yy, yz, zz),
 * quadrature points lexicographic (x fastest).  For tests of the geometry precompute. */
int mfq_op_geometry(const mfq_op* op, double* out_device, void* hip_stream);

/* b_i = sum_K sum_q f(x_q) phi_i(x_q) JxW_q (Sec. 2.4 right-hand-side term) for the manufactured
 * solution u* = sin(pi x1) sin(pi x2) sin(pi x3), f = -div(a grad u*); zero on Dirichlet rows.
 * b is a double device vector; computed in FP64 for either operator precision. */
int mfq_rhs_manufactured(const mfq_op* op, double* b, void* hip_stream);

/* ---------------------------------------------------------------- assembled matrix (Sec. 3.6)
 * The same operator stored as a global sparse matrix, the representation that the matrix-free
 * action replaces (Sec. 3.6 weighs the memory transfer of a matrix that couples every unknown
 * to its neighbours against computing the integrals on the fly).  For measuring the two side
 * by side on one device; the solvers never use it.
 * Layout (CSR, in the caller's buffer): rowptr int64 [n_rows+1], cols int32 [nnz] increasing
 * within each row, vals [nnz] of the value precision (double or float); n_rows = n_dofs.  Row (I,J,K) holds every node that
 * shares a cell with it (the tensor product of the 1D neighbour ranges), so
 * nnz = (n(p+1)^2 - n + 1)^3.  Entries are sum_K A^K_ij over the cells holding both nodes,
 * computed in FP64 from the operator's stored G (FP32 values: each cell colour's FP64 sum is
 * added into the stored value with one rounding, at most 8 per entry).  With MFQ_BC_DIRICHLET0
 * the couplings of
 * Dirichlet nodes are stored as zeros and their diagonal as 1, so the matrix applies
 * m*A(m*x) + (1-m)*x exactly as mfq_vmult does. */
/* op: an MFQ_FP64 operator; precision: of the stored values and of the product's vectors,
 * MFQ_FP64 or MFQ_FP32 (MFQ_EINVAL otherwise).  Host only; nothing is read from the device. */
int mfq_csr_create(const mfq_op* op, int precision, mfq_csr** out);
void mfq_csr_destroy(mfq_csr* a);
/* Rows, stored entries and the device bytes mfq_csr_bind needs (any output may be NULL). */
int mfq_csr_size(const mfq_csr* a, int64_t* n_rows, int64_t* nnz, size_t* device_bytes);
/* Binds the buffer (256-byte aligned, at least the reported bytes) and assembles the matrix on
 * the stream (asynchronous).  The operator must be bound, its G complete before the work on
 * this stream runs, and unchanged until this work has finished; after that the matrix no
 * longer reads the operator. */
int mfq_csr_bind(mfq_csr* a, void* dev_buf, size_t bytes, void* hip_stream);
/* Device addresses of the three arrays inside the bound buffer (MFQ_EINVAL when unbound). */
int mfq_csr_arrays(const mfq_csr* a, void** rowptr, void** cols, void** vals);
/* dst = A src for device vectors of n_rows elements of the value precision (double or float,
 * accumulated in that precision) that must not overlap.  Asynchronous, no host synchronisation,
 * deterministic (fixed summation order per row). */
int mfq_csr_spmv(const mfq_csr* a, const void* src, void* dst, void* hip_stream);

/* ---------------------------------------------------------------- discontinuous Galerkin operator (Sec. 6.1)
 * The symmetric interior penalty DG discretisation of the Laplacian of the paper's multigrid
 * experiment (Laplace equation, DG of degree p on a hyper-rectangle), applied matrix-free.
 * Readings (the paper gives none of them): the undeformed n^3 mesh of the unit cube, coefficient
 * 1; per cell the discontinuous Q_p basis on the GLL nodes, DoF (a,b,c) of cell K = i + n j +
 * n^2 k at index K (p+1)^3 + a + (p+1) b + (p+1)^2 c; (p+1)-point Gauss rules on cells and
 * faces;
 *   a(u,v) = sum_K int_K grad u . grad v + sum_F int_F ( -{d_n u}[v] - {d_n v}[u] + sigma [u][v] )
 * with [u] = u_L - u_R and {.} the mean across an interior face (n from the lower to the upper
 * cell), the outside values zero and the inside value for the mean on boundary faces
 * (homogeneous Dirichlet data imposed weakly), sigma = 2 (p+1)^2 / h.  No device storage: the
 * affine cells need no stored geometry. */
/* mesh: amplitude 0 (MFQ_EINVAL otherwise); degree 1..8.  Host only. */
int mfq_dg_create(const mfq_mesh* mesh, int degree, mfq_dg** out);
void mfq_dg_destroy(mfq_dg* op);
int64_t mfq_dg_n_dofs(const mfq_dg* op);  /* n^3 (p+1)^3; -1 for NULL */
/* dst = A src for double device vectors of n_dofs elements that must not overlap: one launch in
 * which each cell forms, along every 1D line of each direction, the line's stiffness term and the
 * terms of its two faces (from its own line and the neighbours' lines through those faces), then
 * applies the Gauss rule's mass matrix in the two tangential directions, and stores its result
 * once (an interior face is evaluated by both of its cells, each keeping its own half).
 * Asynchronous, deterministic. */
int mfq_dg_vmult(const mfq_dg* op, const double* src, double* dst, void* hip_stream);
/* The same product in MFQ_FP64 or MFQ_FP32 (vectors and arithmetic of that precision; the FP32
 * form is the smoother operator of the multigrid below). */
int mfq_dg_vmult_prec(const mfq_dg* op, int precision, const void* src, void* dst, void* hip_stream);
/* diag[i] = A_ii of the DG-SIPG matrix (n_dofs device values of `precision`), evaluated in closed
 * form per cell: the cell term is separable in the three directions and each face adds its
 * penalty, consistency and symmetry terms of the node's trace.  Overwrites diag. */
int mfq_dg_diagonal(const mfq_dg* op, int precision, void* diag, void* hip_stream);
/* Number of nodes (n p + 1)^3 of the continuous Q_p space with Dirichlet nodes on the same mesh
 * (lattice order, as mfq_space_create with MFQ_BC_DIRICHLET0); -1 for NULL. */
int64_t mfq_dg_cg_n_dofs(const mfq_dg* op);
/* Transfer between the continuous space (cg, mfq_dg_cg_n_dofs values) and the DG space (dg,
 * n_dofs values), the change of space inside the multigrid hierarchy (Sec. 6.1).  to_dg = 1:
 * dg = E cg, every cell takes the values of its lattice nodes (the continuous function is also a
 * discontinuous one).  to_dg = 0: cg = E^T dg, each node sums its copies in the cells holding it
 * in a fixed cell order (deterministic), zero on boundary nodes.  Overwrites out; in and out must
 * not overlap.  Device vectors of `precision`. */
int mfq_dg_transfer(const mfq_dg* op, int precision, int to_dg, const void* in, void* out, void* hip_stream);

/* ---------------------------------------------------------------- transfer (Sec. 3.5, 3.1)
 * Interpolation between nested spaces on the same domain: either the fine mesh halves the
 * coarse cells (same degree) or the meshes agree and the fine degree is higher.  Both spaces
 * must have the same bc and amplitude.  No device storage. */
int mfq_transfer_create(const mfq_space* coarse, const mfq_space* fine, mfq_transfer** out);
void mfq_transfer_destroy(mfq_transfer* t);
/* fine = P coarse (overwrites fine; zero on Dirichlet nodes). */
int mfq_prolongate(const mfq_transfer* t, int precision, const void* coarse, void* fine, void* hip_stream);
/* coarse = P^T fine (overwrites coarse; zero on Dirichlet nodes). */
int mfq_restrict(const mfq_transfer* t, int precision, const void* fine, void* coarse, void* hip_stream);

/* ---------------------------------------------------------------- smoother (Sec. 3.5, 6.1)
 * `degree` Chebyshev updates of x for A x = b with the Jacobi preconditioner inv_diag on the
 * interval [lmin, lmax] of D^{-1}A (Chebyshev semi-iteration).  x_is_zero != 0 starts from
 * x = 0 (x is overwritten).  work must hold 3*n_dofs elements of the operator's precision.
 * With fused updates enabled on the operator (mfq_op_set_fused_updates), each update that
 * follows an operator application is done inside it. */
int mfq_chebyshev(const mfq_op* op, const void* inv_diag, const void* b, void* x, int x_is_zero,
                  int degree, double lmin, double lmax, void* work, void* hip_stream);
/* Fused vector updates (not in the paper; its smoother steps are separate vector operations):
 * with enable != 0 a Chebyshev step of mfq_chebyshev, and the multigrid residual r = b - A x of
 * the V-cycles of solvers created afterwards from this operator, is done inside the operator
 * application: the brick that completes a node's product applies the update there, so the
 * product is never stored or read back (the third work vector keeps only partial sums of nodes
 * shared between bricks).  enable = 0 (the default) issues the application and a separate vector
 * kernel.  Both give bitwise equal results; on MI355X the separate form is the faster one (the
 * cell loop is bound by per-brick latency at its occupancy, and the update's operands lengthen
 * it more than a streaming vector kernel costs).  Matrix-core operators never fuse.  Host only. */
int mfq_op_set_fused_updates(mfq_op* op, int enable);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops or
 * harnesses that forbid the allocator): mfq_chebyshev without the `work` argument.  The three
 * work vectors live in a fixed array of this library on each device (its address looked up once
 * per device on the first call there, with that device current), so the call allocates nothing;
 * the caller still passes the inputs and x.  The current device must be the one that holds the
 * operator and the vectors.  Limit: 3 n_dofs elements of the operator's precision must fit in
 * mfq_chebyshev_noalloc_max_bytes() (64 MiB: 2,796,202 DoFs in FP64, 5,592,405 in FP32); larger
 * operators get MFQ_EINVAL.  Every call on a device shares that device's array (its contents are
 * the last call's work vectors; nothing in it has to start at zero): calls that overlap in time
 * on one device, on any streams, race and must not be issued.  Same kernels and arithmetic as
 * mfq_chebyshev (bitwise equal results). */
int mfq_chebyshev_noalloc(const mfq_op* op, const void* inv_diag, const void* b, void* x, int x_is_zero,
                          int degree, double lmin, double lmax, void* hip_stream);
size_t mfq_chebyshev_noalloc_max_bytes(void);

/* ---------------------------------------------------------------- solvers (Sec. 3.5, 6.1)
 * Kinds: CG: unpreconditioned FP64 CG.  GMG_FP64: FP64 CG preconditioned by an FP64 V-cycle.
 * GMG_MIXED: FP64 CG (FP64 operator, vectors and dot products) preconditioned by an FP32
 * V-cycle.  GMG_MIXED_IR: FP64 iterative refinement (FP64 residual and correction) around an
 * inner CG on FP32 operators preconditioned by the FP32 V-cycle.
 * The solver is built on an FP64 operator with MFQ_BC_DIRICHLET0; the hierarchy halves n
 * while n is even and the level has more than coarse_dofs free DoFs (default 4096), then
 * lowers p to ceil(p/2) while more than coarse_dofs free DoFs remain.  Coarsest level:
 *   coarse_mode 0 (default): solved in FP64 by a dense inverse (<= coarse_dofs free DoFs) or by
 *     Jacobi-CG to 1e-12 (which polls the host);
 *   coarse_mode 1: coarse_degree Chebyshev updates from zero on [lmax/coarse_ratio, lmax] with
 *     the V-cycle's precision, so a V-cycle never waits on the host (used when many solves share
 *     the device, see mfq_batch_step).
 * Every solve ends with an FP64 true-residual check; while it exceeds rtol, another CG pass on
 * the residual equation (FP64 correction) follows, within max_iter iterations in total. */
typedef enum { MFQ_SOLVER_CG = 0, MFQ_SOLVER_GMG_FP64 = 1, MFQ_SOLVER_GMG_MIXED = 2,
               MFQ_SOLVER_GMG_MIXED_IR = 3 } mfq_solver_kind;

typedef struct {
  int smoother_degree;     /* Chebyshev degree (default 3) */
  int lanczos_iters;       /* CG-Lanczos steps for the largest eigenvalue (default 12) */
  double lambda_factor;    /* lmax = factor * estimate (default 1.2) */
  double lambda_ratio;     /* lmin = lmax / ratio (default 15) */
  double inner_rtol;       /* inner tolerance of GMG_MIXED_IR (default 1e-4) */
  int check_every;         /* host convergence poll period in iterations (default 4) */
  int n_lambda_override;   /* if > 0: lmax of levels 1..n (finest last) taken from lambda_override */
  const double* lambda_override;
  int coarse_mode;         /* 0: dense inverse or Jacobi-CG; 1: Chebyshev, no host round trip */
  int coarse_degree;       /* Chebyshev degree on the coarsest level in coarse_mode 1 (default 16) */
  double coarse_ratio;     /* its interval [lmax/coarse_ratio, lmax] (default 30) */
  int coarse_dofs;         /* coarsening stops at this many free DoFs (default 4096, at most 4096) */
  int use_graphs;          /* 1 (default): on a non-default stream, each CG iteration is captured
                              once as a HIP graph and replayed (not when a Jacobi-CG coarse solve
                              must poll the host); 0: launches issued one by one */
} mfq_solver_params;

typedef struct {
  int iterations;          /* CG iterations (summed over inner solves for IR) */
  int outer_iterations;    /* IR steps (1 for non-IR kinds) */
  double rel_residual;     /* final true relative residual ||b - A x|| / ||b||, FP64 */
  double seconds;          /* wall time of mfq_solve */
  int n_levels;
} mfq_solve_info;

void mfq_solver_default_params(mfq_solver_params* params);
int mfq_solver_create(const mfq_op* op_fp64, int kind, const mfq_solver_params* params, mfq_solver** out);
void mfq_solver_destroy(mfq_solver* s);
int mfq_solver_device_bytes(const mfq_solver* s, size_t* bytes);
/* Binds the buffer; builds the level operators, diagonals, eigenvalue bounds and the coarse
 * inverse.  Synchronises the stream.  May be called again (another buffer, or after the operator
 * was re-bound): captured HIP graphs are dropped. */
int mfq_solver_bind(mfq_solver* s, void* dev_buf, size_t bytes, void* hip_stream);
/* As mfq_solver_bind, but the eigenvalue bounds of the Chebyshev levels are not estimated here:
 * the first step of the first solve estimates them (the same Lanczos runs, so the same bounds
 * bitwise).  mfq_batch_run estimates those of all lazily bound solves that start in one call with
 * one set of launches; mfq_batch_step and the asynchronous step estimate them per solve and wait
 * for the stream there.  Until then mfq_solver_lambdas fails (MFQ_EINVAL) and
 * mfq_solver_precondition estimates them first.  A solve whose estimate fails ends with
 * MFQ_ENONFINITE.  For serving, where set-up of many requests would otherwise be one small
 * launch sequence and one stream wait per request (not in the paper). */
int mfq_solver_bind_lazy(mfq_solver* s, void* dev_buf, size_t bytes, void* hip_stream);
/* Solves A x = b to ||b - A x||_2 <= rtol ||b||_2 from x = 0 (x overwritten).  b, x: double
 * device vectors.  Blocks until done.  MFQ_ENOCONV when max_iter is reached (info valid).
 * Equivalent to mfq_solve_begin, mfq_batch_step on this solver alone (check_every iterations
 * per step) until it reports done, and mfq_solve_end. */
int mfq_solve(mfq_solver* s, const double* b, double* x, double rtol, int max_iter,
              void* hip_stream, mfq_solve_info* info);

/* Resumable solves, for serving many requests on one device (continuous batching; not in the
 * paper).  mfq_solve_begin validates the arguments like mfq_solve and records the solve (on
 * GMG_MIXED_IR it enqueues x = 0 on hip_stream); the first step enqueues its start.  The solver
 * remembers b, x and the stream, which must stay valid until mfq_solve_end.  A solver runs one
 * solve at a time (MFQ_EBUSY otherwise). */
int mfq_solve_begin(mfq_solver* s, const double* b, double* x, double rtol, int max_iter, void* hip_stream);

/* One step of `count` running solves: enqueues up to `iters` CG iterations of each (or its
 * residual check) on its own stream, then waits once for all of them and reads every solve's
 * convergence state from pinned host memory (one device-to-host copy per solve per step).
 * done[i] is set to 1 once solve i has finished (converged, out of iterations or non-finite).
 * Solves on different streams overlap on the device. */
int mfq_batch_step(mfq_solver* const* solvers, int count, int iters, int* done);

/* Non-blocking form of a step of one solve.  mfq_solve_step_async enqueues up to `iters` CG
 * iterations (or the residual check) and the status copy on the solve's stream and records an
 * event; MFQ_EBUSY while the previous asynchronous step has not been polled to completion, MFQ_OK
 * without work once the solve is done.  mfq_solve_step_poll never waits: *ready = 0 while that
 * work runs; otherwise it reads the outcome, sets *ready = 1 and *done = 1 once the solve has
 * finished.  Lets a caller advance each solve at its own pace instead of waiting for all of them
 * at every step.  Not to be mixed with mfq_batch_step on a solve with a step in flight. */
/* Batched serving step (not part of the paper's method: continuous batching of many solves).
 * mfq_batch_run advances every running solve in `solvers` like mfq_batch_step (the start of a CG
 * pass, iters CG iterations, or the residual check between CG passes; done[i] = 1 once solve i
 * has finished), but for the solves that qualify (GMG_MIXED with coarse_mode 1, FP32 V-cycle) the
 * work is issued as one launch per (kernel, degree) over all of them: the eigenvalue estimates of
 * lazily bound solves (mfq_solver_bind_lazy; every level's Lanczos run at once, traces read back
 * in one copy and one extra stream wait), then one plan of the pass starts and residual checks
 * (once) and of one CG iteration (the FP64 operator, the CG updates, the FP32 V-cycle level by
 * level from the finest; replayed `iters` times for the solves within their iteration budget),
 * planned once per call as work tables in device memory (one host-to-device copy); the solves'
 * scalar states and residual norms come back in one device-to-host copy; one stream wait.  Each
 * solve's kernels see its own operands with the grids of its own launches, so results are bitwise
 * those of mfq_batch_step.  Every listed solve must run on hip_stream (mfq_solve_begin) and the
 * qualifying ones must share smoother_degree and coarse_degree.  mfq_batch_create: up to
 * max_solvers solves per call; device workspace of mfq_batch_device_bytes (tables, states,
 * traces; mfq_batch_bind), pinned host staging owned by the handle.  One call at a time per
 * handle. */
int mfq_batch_create(int max_solvers, mfq_batch** out);
void mfq_batch_destroy(mfq_batch* b);
int mfq_batch_device_bytes(const mfq_batch* b, size_t* bytes);
int mfq_batch_bind(mfq_batch* b, void* dev_buf, size_t bytes, void* hip_stream);
int mfq_batch_run(mfq_batch* b, mfq_solver* const* solvers, int count, int iters, void* hip_stream, int* done);

int mfq_solve_step_async(mfq_solver* s, int iters);
int mfq_solve_step_poll(mfq_solver* s, int* ready, int* done);

/* Finishes a solve reported done (by mfq_batch_step or mfq_solve_step_poll): fills info and
 * returns the solve's status (MFQ_OK, MFQ_ENOCONV or MFQ_ENONFINITE); the solver can then begin
 * another solve.  MFQ_EINVAL if no solve has finished. */
int mfq_solve_end(mfq_solver* s, mfq_solve_info* info);
/* z = M r: one application of the solver's preconditioner (the V-cycle; identity for CG) to
 * the double device vector r.  Asynchronous. */
int mfq_solver_precondition(mfq_solver* s, const double* r, double* z, void* hip_stream);
/* Largest-eigenvalue estimates of D^{-1}A per level (finest last); n_out >= n_levels - 1. */
int mfq_solver_lambdas(const mfq_solver* s, double* out, int n_out);

/* ---------------------------------------------------------------- DG multigrid solver (Sec. 6.1)
 * FP64 CG on the DG-SIPG operator preconditioned by an FP32 V-cycle whose finest level is the DG
 * space and whose next level is the continuous Q_p space on the same mesh: Chebyshev smoothing
 * (smoother_degree, Jacobi with the exact DG diagonal, largest eigenvalue from lanczos_iters
 * Jacobi-PCG steps on the DG level), the residual moved to the continuous space by
 * mfq_dg_transfer(to_dg = 0), one V-cycle of a GMG_MIXED solver of the continuous Q_p Laplacian
 * (Dirichlet nodes, coefficient 1) with the same parameters, the correction moved back by
 * mfq_dg_transfer(to_dg = 1), post-smoothing.  lambda_override, if given, lists lmax of the
 * continuous levels 1.. (finest last, as for mfq_solver_create) followed by the DG level's.
 * params NULL: mfq_solver_default_params with
 * smoother_degree 6, the Chebyshev degree of the paper's experiment.  Needs p n >= 2 (the
 * continuous level must have an interior node; MFQ_EINVAL otherwise).  The DG operator must
 * outlive the solver. */
int mfq_dg_solver_create(const mfq_dg* op, const mfq_solver_params* params, mfq_dg_solver** out);
void mfq_dg_solver_destroy(mfq_dg_solver* s);
int mfq_dg_solver_device_bytes(const mfq_dg_solver* s, size_t* bytes);
/* Binds a 256-byte aligned device buffer of at least device_bytes; builds the continuous
 * hierarchy, the DG diagonal and the eigenvalue bound.  Synchronises the stream. */
int mfq_dg_solver_bind(mfq_dg_solver* s, void* dev_buf, size_t bytes, void* hip_stream);
/* z = M r: one V-cycle on the double device vector r (n_dofs).  Asynchronous.  With use_graphs
 * (default) on a non-default stream, the V-cycle is captured once per (stream, r, z) as a HIP
 * graph and replayed (the last two captures are kept); mfq_dg_solve uses this too. */
int mfq_dg_precondition(mfq_dg_solver* s, const double* r, double* z, void* hip_stream);
/* Solves A x = b to ||b - A x||_2 <= rtol ||b||_2 from x = 0, with FP64 correction passes on the
 * residual equation while the FP64 true residual exceeds rtol (as mfq_solve).  Blocks until done;
 * MFQ_ENOCONV when max_iter is reached (info valid).  info->n_levels counts the DG level. */
int mfq_dg_solve(mfq_dg_solver* s, const double* b, double* x, double rtol, int max_iter, void* hip_stream,
                 mfq_solve_info* info);

/* ---------------------------------------------------------------- hanging nodes (Sec. 3.3)
 * The variable-coefficient operator of mfq_op_create on a two-block mesh with a 2:1 interface,
 * the smallest mesh with hanging nodes (adaptive refinement, Sec. 3.3; Fig. 3) that keeps each
 * part a tensor-product lattice.  Block 0: the unit cube in n^3 cells of side 1/n; block 1:
 * [1,2] x [0,1]^2 in (2n)^3 cells of side 1/(2n); the deformation x = X + A s(X)(1,1,1),
 * s = sin(pi X1) sin(pi X2) sin(pi X3), and the coefficient a(x) = 1 + alpha sin(2 pi x1)
 * sin(2 pi x2) sin(2 pi x3) are evaluated on the whole domain [0,2] x [0,1]^2.
 * Vectors: block 0's lattice ((pn+1)^3 nodes, x fastest), then block 1's ((2pn+1)^3, x fastest).
 * Block 1's nodes on X1 = 1 are hanging: their conforming values are the coarse face's trace,
 * interpolated in each face direction (the 1D h-transfer table); they are not unknowns.
 * Homogeneous Dirichlet data on the domain's boundary (X1 in {0, 2}, X2, X3 in {0, 1}).
 * The operator is y = m C^T blockdiag(A_0, A_1) C (m x) + (1 - m) x on the independent entries
 * and y = x on the hanging entries (C: identity on independent entries, interpolation on the
 * hanging ones; m: Dirichlet mask).  Precision MFQ_FP64 or MFQ_FP32 (G stored as in mfq_op).
 * Device storage (mfq_hang_device_bytes): both blocks' index lattices and G, and two face arrays
 * of (2pn+1)^2 values that every application uses: applications of one operator must not overlap
 * in time (on any streams). */
int mfq_hang_create(int n_coarse, double amplitude, int degree, double alpha, int precision, mfq_hang** out);
void mfq_hang_destroy(mfq_hang* h);
int64_t mfq_hang_n_dofs(const mfq_hang* h);     /* (pn+1)^3 + (2pn+1)^3; -1 on NULL */
int mfq_hang_device_bytes(const mfq_hang* h, size_t* bytes);
/* Binds a 256-byte aligned buffer of at least device_bytes and fills both blocks' data on the
 * stream (asynchronous). */
int mfq_hang_bind(mfq_hang* h, void* dev_buf, size_t bytes, void* hip_stream);
/* dst = A src on the device vectors above (n_dofs elements of the operator's precision, not
 * overlapping).  Asynchronous: interpolation to the hanging face, the two blocks' cell loops,
 * the transposed interpolation added to the coarse face (deterministic, no atomics). */
int mfq_hang_vmult(const mfq_hang* h, const void* src, void* dst, void* hip_stream);
/* Unpreconditioned FP64 CG on an MFQ_FP64 operator from x = 0 to ||b - A x||_2 <= rtol ||b||_2
 * (b zero on Dirichlet and hanging entries for a solution of the constrained problem; the hanging
 * entries of x are then zero: their conforming values are the interpolated coarse trace).  work:
 * 256-byte aligned device memory of mfq_hang_cg_work_bytes.  Blocks; MFQ_ENOCONV when the true
 * residual exceeds rtol after max_iter iterations (info valid). */
size_t mfq_hang_cg_work_bytes(const mfq_hang* h);
int mfq_hang_cg(const mfq_hang* h, const double* b, double* x, double rtol, int max_iter, void* work,
                size_t work_bytes, void* hip_stream, mfq_solve_info* info);

#ifdef __cplusplus
}
#endif
#endif /* MFQ_H */
