// Internal declarations of the matrix-free Q_p library (host side + kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/mfq.h"

namespace mfq {

constexpr int kMaxDegree = 8;
constexpr int kBlock = 256;  // threads per workgroup of the cell kernels

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);
#define MFQ_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return ::mfq::fail(MFQ_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                         __FILE__, __LINE__);                                               \
  } while (0)

// ---------------------------------------------------------------- 1D tables (host, FP64)
// Nodes of Q_p: Gauss-Lobatto-Legendre points on [0,1]; quadrature: (p+1)-point Gauss on [0,1].
struct Tables1D {
  int p = 0;
  std::vector<double> xi;     // p+1 nodes
  std::vector<double> zeta;   // p+1 Gauss points
  std::vector<double> omega;  // p+1 Gauss weights (sum 1)
  std::vector<double> S;      // S[q*(p+1)+a] = l_a(zeta_q)
  std::vector<double> D;      // D[q*(p+1)+a] = l_a'(zeta_q)
};
const Tables1D& tables(int p);
std::vector<double> gll_points(int p);
double lagrange_value(const std::vector<double>& nodes, int a, double t);
double lagrange_derivative(const std::vector<double>& nodes, int a, double t);
// 1D transfer matrix [nf1][pc+1]: coarse basis (degree pc) at the fine nodes lying in one coarse
// cell: h-transfer (fine degree pc, two fine cells) when h_transfer, else the GLL nodes of pf.
std::vector<double> transfer_matrix_1d(int pc, int pf, bool h_transfer, int* nf1);

// Work decomposition of the cell kernels: the mesh is cut into bricks of bx x by x bz cells, one
// workgroup per brick and one lane per 1D pencil of a cell ((p+1)^2 lanes per cell).  Bricks are
// coloured by the parities of their (x, y, z) brick coordinates: bricks of one colour share no
// node, so a colour is one launch whose workgroups write their nodes without atomics, and the
// colours run in order 0..7.
struct BrickDims {
  int bx, by, bz;
};
// Brick shapes (cells in x, y, z) per degree, chosen by timing the operator on MI355X among the
// shapes that fill a 256-lane workgroup; a build can override one, e.g. -DMFQ_BRICK_P4=4,1,2.
#ifndef MFQ_BRICK_P1
#define MFQ_BRICK_P1 32, 2, 1
#endif
#ifndef MFQ_BRICK_P2
#define MFQ_BRICK_P2 14, 2, 1
#endif
#ifndef MFQ_BRICK_P3
#define MFQ_BRICK_P3 16, 1, 1
#endif
#ifndef MFQ_BRICK_P4
#define MFQ_BRICK_P4 5, 2, 1
#endif
#ifndef MFQ_BRICK_P5
#define MFQ_BRICK_P5 7, 1, 1
#endif
#ifndef MFQ_BRICK_P6
#define MFQ_BRICK_P6 4, 1, 1
#endif
#ifndef MFQ_BRICK_P7
#define MFQ_BRICK_P7 4, 1, 1
#endif
#ifndef MFQ_BRICK_P8
#define MFQ_BRICK_P8 3, 1, 1
#endif
constexpr BrickDims brick_dims(int p) {
  return p == 1 ? BrickDims{MFQ_BRICK_P1} : p == 2 ? BrickDims{MFQ_BRICK_P2} : p == 3 ? BrickDims{MFQ_BRICK_P3}
       : p == 4 ? BrickDims{MFQ_BRICK_P4} : p == 5 ? BrickDims{MFQ_BRICK_P5} : p == 6 ? BrickDims{MFQ_BRICK_P6}
       : p == 7 ? BrickDims{MFQ_BRICK_P7} : BrickDims{MFQ_BRICK_P8};
}
inline int threads_per_cell(int p) { return (p + 1) * (p + 1); }
inline int cells_per_brick(int p) {
  const BrickDims b = brick_dims(p);
  return b.bx * b.by * b.bz;
}
inline int lanes_per_brick(int p) { return cells_per_brick(p) * threads_per_cell(p); }
inline int64_t lattice_per_brick(int p) {
  const BrickDims b = brick_dims(p);
  return (int64_t)(b.bx * p + 1) * (b.by * p + 1) * (b.bz * p + 1);
}

constexpr int kColours = 8;

// Brick grid of a mesh.  Colour c = (x parity) + 2 (y parity) + 4 (z parity) of the brick
// coordinates.  Per-brick data is stored colour-major, bricks of a colour x-fastest, so each
// launch streams one contiguous range.
struct Bricks {
  int n;                     // cells per direction of the mesh
  int bx, by, bz;            // cells per brick
  int nbx, nby, nbz;         // bricks per direction
  int cxn[kColours];         // bricks of colour c along x
  int cyn[kColours];         // bricks of colour c along y
  int64_t count[kColours];   // bricks of colour c
  int64_t offset[kColours];  // first brick ordinal of colour c
  int64_t n_bricks;
};
inline Bricks make_bricks(int p, int n) {
  Bricks b{};
  const BrickDims d = brick_dims(p);
  b.n = n;
  b.bx = d.bx;
  b.by = d.by;
  b.bz = d.bz;
  b.nbx = (n + d.bx - 1) / d.bx;
  b.nby = (n + d.by - 1) / d.by;
  b.nbz = (n + d.bz - 1) / d.bz;
  int64_t off = 0;
  for (int c = 0; c < kColours; ++c) {
    const int cx = (b.nbx + 1 - (c & 1)) / 2, cy = (b.nby + 1 - ((c >> 1) & 1)) / 2, cz = (b.nbz + 1 - (c >> 2)) / 2;
    b.cxn[c] = cx;
    b.cyn[c] = cy;
    b.count[c] = (int64_t)cx * cy * cz;
    b.offset[c] = off;
    off += b.count[c];
  }
  b.n_bricks = off;
  return b;
}

}  // namespace mfq

// ---------------------------------------------------------------- opaque handles
struct mfq_mesh {
  int n;
  double amplitude;
  double x0 = 0.0;            // X1 of the mesh's first cell face (1 for the fine block of the two-block mesh)
};

struct mfq_space {
  const mfq_mesh* mesh;
  int p;
  int bc;
  int64_t n_dofs;
  int64_t n_cells;
  int bc_faces = -1;          // Dirichlet faces (bit 2d: X_d low, 2d+1: X_d high); -1: all six when bc
  bool side = false;          // nodes on the X1-low face are hanging (read from / written to face arrays)
};

// Fused vector updates are off by default: measured slower on MI355X (the cell loop is bound by
// per-brick latency at its occupancy; the separate vector kernel streams at full bandwidth).
#ifndef MFQ_FUSE_DEFAULT
#define MFQ_FUSE_DEFAULT 0
#endif

struct mfq_op {
  const mfq_space* space;
  double alpha;
  int precision;              // MFQ_FP64 or MFQ_FP32 (storage and arithmetic)
  bool mfma = false;          // FP32 cell loop on the matrix cores (created as MFQ_FP32_MFMA)
  bool fuse = MFQ_FUSE_DEFAULT != 0;  // vector updates fused into the cell loop (mfq_op_set_fused_updates)
  mfq::Bricks bricks;
  size_t idx_bytes, geo_bytes;
  void* buf = nullptr;        // caller-owned device memory
  int* idx = nullptr;         // [n_bricks][lattice]: global node of each brick-lattice node,
                              // ~g on Dirichlet nodes, INT_MIN outside the mesh
  void* geo = nullptr;        // [n_bricks][p+1][3][lanes][2] of the precision's type
  // undeformed mesh with a variable coefficient: G_q = a(x_q) h w_q I, so the cell loop reads
  // only its diagonal, kept once more as [n_bricks][p+1][lanes] (the other kernels read geo)
  size_t coef_bytes = 0;
  void* coef = nullptr;
};

struct mfq_csr {
  const mfq_op* op;           // FP64 operator whose stored geometry the values are assembled from
  int precision;              // of the stored values and the product's vectors (MFQ_FP64 or MFQ_FP32)
  int p, n, bc;
  int64_t n_rows, nnz;
  bool long_rows;             // product by lane groups per row (long rows) instead of row blocks
  int lanes_per_row;          // lanes that share one row in the product
  int64_t window;             // entries per row block of the product
  int64_t n_blocks;           // row blocks: ceil(nnz / window)
  int64_t max_row;            // longest row
  size_t rowptr_bytes, cols_bytes, vals_bytes, blk_bytes;
  void* buf = nullptr;        // caller-owned device memory
  int64_t* rowptr = nullptr;  // [n_rows + 1]
  int* cols = nullptr;        // [nnz], increasing within a row
  void* vals = nullptr;       // [nnz] of the value precision
  int64_t* blk = nullptr;     // [n_blocks + 1]: first row of each row block
};

struct mfq_dg {
  int p, n;
  int64_t n_dofs;
};

struct mfq_transfer {
  const mfq_space* coarse;
  const mfq_space* fine;
  bool h_transfer;
  int nf1;
  std::vector<double> P1;     // [nf1][pc+1]
};

namespace mfq {

// Plain-struct view of an operator handed to launchers.
struct OpView {
  int p, n, bc;
  int64_t n_cells, n_dofs;
  double amplitude, alpha;
  Bricks bricks;
  const int* idx;
  const void* geo;
  bool mfma;
  double x0;                  // X1 offset of the mesh
  int bc_faces;               // Dirichlet faces, bit 2d: X_d low, 2d+1: X_d high
  int side_base;              // >= 0: index-lattice entries >= side_base are X1-low face nodes read from
                              // side_in[g - side_base] and written to side_out[g - side_base]
  const void* side_in;        // set by the caller of a cell loop on a space with hanging nodes
  void* side_out;
  const void* coef;           // diagonal of G per quadrature point (undeformed mesh, variable coefficient) or null
};
inline OpView view(const mfq_op* op) {
  const mfq_space* s = op->space;
  const int faces = s->bc_faces >= 0 ? s->bc_faces : (s->bc ? 0b111111 : 0);
  return OpView{s->p, s->mesh->n, s->bc, s->n_cells, s->n_dofs, s->mesh->amplitude, op->alpha, op->bricks,
                op->idx, op->geo, op->mfma, s->mesh->x0, faces, s->side ? (int)s->n_dofs : -1, nullptr, nullptr,
                op->coef};
}

// precision of a vector argument: MFQ_FP32_MFMA means float; -1 if unknown
inline int vector_precision(int precision) {
  if (precision == MFQ_FP32_MFMA) return MFQ_FP32;
  return (precision == MFQ_FP64 || precision == MFQ_FP32) ? precision : -1;
}

// ---------------------------------------------------------------- launchers (kernels_*.hip)
hipError_t launch_fill_index(const OpView& v, int* idx, hipStream_t st);
hipError_t launch_geometry(const OpView& v, int precision, void* geo, hipStream_t st);
hipError_t launch_geometry_export(const OpView& v, int precision, double* out, hipStream_t st);
// dst = A src (accumulate = false: every node written, no clearing needed) or dst += A src.
hipError_t launch_coef_from_geo(const OpView& v, int precision, const void* geo, void* coef, hipStream_t st);
hipError_t launch_vmult_cells(const OpView& v, int precision, const void* src, void* dst, bool accumulate,
                              hipStream_t st);
// diag = diagonal of A (1 on Dirichlet rows); every node written, no clearing needed.
hipError_t launch_diagonal_cells(const OpView& v, int precision, void* diag, hipStream_t st);
// Setup-time cell loops: the manufactured load vector (every entry written) and the dense coarse
// matrix (added into mat, which the caller zeroes first); colour-ordered, no atomics.
hipError_t launch_rhs_cells(const OpView& v, double* b, hipStream_t st);
hipError_t launch_assemble_dense(const OpView& v, double* mat, int64_t ld, hipStream_t st);
hipError_t launch_transfer(const mfq_transfer* t, int precision, bool prolongate, const void* in,
                           void* out, hipStream_t st);

// assembled sparse matrix (kernels_csr.hip)
hipError_t launch_csr_pattern(int p, int n, int64_t* rowptr, int* cols, hipStream_t st);
hipError_t launch_csr_values(const OpView& v, int precision, const int64_t* rowptr, void* vals, hipStream_t st);
hipError_t launch_csr_blocks(const int64_t* rowptr, int64_t* blk, int64_t n_rows, int64_t n_blocks, int64_t window,
                             hipStream_t st);
hipError_t launch_csr_spmv(const mfq_csr* a, const void* x, void* y, hipStream_t st);
int64_t csr_row_start_host(int64_t I, int64_t J, int64_t K, int p, int n);

// DG-SIPG operator (kernels_dg.hip): dst = A src (cell term stored, face terms added), its
// Jacobi diagonal, and the transfer between the continuous Q_p lattice and DG on the same mesh
hipError_t launch_dg_vmult(int p, int n, int precision, const void* src, void* dst, hipStream_t st);
// Chebyshev step fused with the DG product (vectors of `precision`, n_dofs each): r -= A d;
// dnew = c1 d + c2 dinv r; x += dnew.  dnew must not alias d, x or r.
hipError_t launch_dg_cheb_step(int p, int n, int precision, const void* d, const void* dinv, void* x, void* r,
                               void* dnew, double c1, double c2, hipStream_t st);
// r = b - A x with the DG product
hipError_t launch_dg_residual(int p, int n, int precision, const void* b, const void* x, void* r, hipStream_t st);
hipError_t launch_dg_diagonal(int p, int n, int precision, void* diag, hipStream_t st);
hipError_t launch_dg_transfer(int p, int n, int precision, bool to_dg, const void* in, void* out, hipStream_t st);

// vector kernels (kernels_vector.hip)
hipError_t launch_fill(int precision, void* x, int64_t n, double value, hipStream_t st);
hipError_t launch_mask(int precision, int p, int n, void* x, hipStream_t st);
hipError_t launch_cast(int from_precision, const void* in, int to_precision, void* out, int64_t n,
                       hipStream_t st);

struct SolverState;
hipError_t launch_cg_start(const double* b, double* x, double* r, double* p, int64_t n, SolverState* s, bool copy_p,
                           double tol2, hipStream_t st);
hipError_t launch_cg_alpha(const double* p, const double* Ap, int64_t n, SolverState* s, hipStream_t st);
hipError_t launch_cg_update(double* x, double* r, const double* p, const double* Ap, int64_t n, SolverState* s,
                            bool unprec, hipStream_t st);
hipError_t launch_cg_beta(const double* r, const double* z, int64_t n, SolverState* s, hipStream_t st);
hipError_t launch_cg_direction(const double* z, double* p, int64_t n, SolverState* s, bool first, hipStream_t st);
hipError_t launch_residual_norm(const double* b, const double* t, double* r, int64_t n, SolverState* s, double* out,
                                hipStream_t st);
hipError_t launch_add(int precision, void* x, int cor_precision, const void* c, int64_t n, hipStream_t st);
hipError_t launch_cheb_first(int precision, const void* b, const void* t, const void* dinv, void* x, void* r, void* d,
                             int64_t n, double inv_theta, bool x_is_zero, hipStream_t st);
hipError_t launch_cheb_step(int precision, const void* Ad, const void* dinv, void* x, void* r, void* d, int64_t n,
                            double c1, double c2, hipStream_t st);
hipError_t launch_sub(int precision, const void* b, const void* t, void* r, int64_t n, hipStream_t st);
hipError_t launch_dense_solve(int precision, const double* Ainv, int nf, int64_t N1, const void* b, void* x,
                              hipStream_t st);
hipError_t launch_dot(int precision, const void* x, const void* y, int64_t n, SolverState* s, double* out,
                      hipStream_t st);
hipError_t launch_axpby(int precision, double a, const void* x, double b, void* y, int64_t n, hipStream_t st);
hipError_t launch_mul(int precision, const void* d, const void* r, void* z, int64_t n, hipStream_t st);
hipError_t launch_reciprocal(int precision, void* x, int64_t n, hipStream_t st);
hipError_t launch_splitmix(int precision, void* x, int64_t N1, uint64_t seed, bool masked, hipStream_t st);
// device-side Lanczos (Jacobi-PCG) steps; trace[2j], trace[2j+1] = alpha_j, beta_j; trace[count_slot] = steps
hipError_t launch_lz_init(int precision, const void* r, const void* dinv, void* z, void* p, int64_t n, SolverState* s,
                          double* trace, int count_slot, hipStream_t st);
hipError_t launch_lz_alpha(int precision, const void* p, const void* Ap, int64_t n, SolverState* s, double* trace,
                           hipStream_t st);
hipError_t launch_lz_update(int precision, void* r, void* z, const void* Ap, const void* dinv, int64_t n,
                            SolverState* s, double* trace, int count_slot, hipStream_t st);
hipError_t launch_lz_direction(int precision, const void* z, void* p, int64_t n, SolverState* s, hipStream_t st);

// two-block mesh with hanging nodes (kernels_hang.hip): f = (Pi x Pi)(m x0) on the interface and
// y1 = x1 on block 1's hanging rows; y0 += (Pi x Pi)^T g on block 0's interface nodes
hipError_t launch_hang_interp(int precision, int p, int n, int bc, const void* x0, const void* x1, void* f, void* y1,
                              hipStream_t st);
hipError_t launch_hang_restrict(int precision, int p, int n, int bc, const void* g, void* y0, hipStream_t st);

// ---------------------------------------------------------------- host-side operator helpers (api.cpp)
int op_vmult(const mfq_op* op, const void* src, void* dst, hipStream_t st);      // zero dst + cell loop

// Unpreconditioned FP64 CG from x = 0 with any operator (solver.cpp): work holds r, p, A p and the
// device-resident scalars (cg_work_bytes); info gets the iterations and the true relative residual
// ||b - A x|| / ||b|| (MFQ_ENOCONV when it exceeds rtol).
using Apply = std::function<int(const double* in, double* out)>;
size_t cg_work_bytes(int64_t n);
int cg_unpreconditioned(const Apply& apply, const double* b, double* x, int64_t n, double rtol, int max_iter,
                        void* work, hipStream_t st, mfq_solve_info* info);
int op_diagonal(const mfq_op* op, void* diag, hipStream_t st);
const char* last_error_cstr();

}  // namespace mfq
