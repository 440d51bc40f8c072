// C ABI: mesh, space, operator, transfer and smoother entry points (see include/mfq.h).
#include <cmath>
#include <cstring>
#include <new>

#include "batch.hpp"
#include "mfq_internal.hpp"

using namespace mfq;

namespace {

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }
size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
size_t real_size(int precision) { return precision == MFQ_FP64 ? 8 : 4; }

int check_vec(const void* v, const char* name) {
  if (!v) return fail(MFQ_EINVAL, "%s is NULL", name);
  if (!aligned(v, 16)) return fail(MFQ_EINVAL, "%s is not 16-byte aligned", name);
  return MFQ_OK;
}

int check_op(const mfq_op* op) {
  if (!op) return fail(MFQ_EINVAL, "operator is NULL");
  if (!op->buf) return fail(MFQ_EINVAL, "operator is not bound to device memory (call mfq_op_bind)");
  return MFQ_OK;
}

}  // namespace

namespace mfq {

int op_vmult(const mfq_op* op, const void* src, void* dst, hipStream_t st) {
  const OpView v = view(op);
  MFQ_HIP(launch_vmult_cells(v, op->precision, src, dst, false, st));
  return MFQ_OK;
}

int op_diagonal(const mfq_op* op, void* diag, hipStream_t st) {
  MFQ_HIP(launch_diagonal_cells(view(op), op->precision, diag, st));
  return MFQ_OK;
}

}  // namespace mfq

extern "C" {

const char* mfq_version(void) { return "mfq 0.1 (gfx950)"; }
const char* mfq_last_error(void) { return last_error_cstr(); }

int mfq_reference_tables(int degree, double* xi, double* zeta, double* omega, double* S, double* D) {
  if (degree < 1 || degree > kMaxDegree) return fail(MFQ_EINVAL, "degree %d outside [1,%d]", degree, kMaxDegree);
  if (!xi || !zeta || !omega || !S || !D) return fail(MFQ_EINVAL, "NULL output");
  const Tables1D& t = tables(degree);
  const int n1 = degree + 1;
  std::memcpy(xi, t.xi.data(), n1 * sizeof(double));
  std::memcpy(zeta, t.zeta.data(), n1 * sizeof(double));
  std::memcpy(omega, t.omega.data(), n1 * sizeof(double));
  std::memcpy(S, t.S.data(), n1 * n1 * sizeof(double));
  std::memcpy(D, t.D.data(), n1 * n1 * sizeof(double));
  return MFQ_OK;
}

int mfq_mesh_create(int n_cells_1d, double amplitude, mfq_mesh** out) {
  if (!out) return fail(MFQ_EINVAL, "out is NULL");
  if (n_cells_1d < 1 || n_cells_1d > 1024) return fail(MFQ_EINVAL, "n_cells_1d=%d outside [1,1024]", n_cells_1d);
  if (!std::isfinite(amplitude) || std::fabs(amplitude) * 3.0 * M_PI >= 1.0)
    return fail(MFQ_EINVAL, "amplitude %g would make the deformation non-invertible", amplitude);
  mfq_mesh* m = new (std::nothrow) mfq_mesh{n_cells_1d, amplitude};
  if (!m) return fail(MFQ_ENOMEM, "host allocation failed");
  *out = m;
  return MFQ_OK;
}

void mfq_mesh_destroy(mfq_mesh* mesh) { delete mesh; }

int mfq_space_create(const mfq_mesh* mesh, int degree, int bc, mfq_space** out) {
  if (!mesh || !out) return fail(MFQ_EINVAL, "mesh or out is NULL");
  if (degree < 1 || degree > kMaxDegree) return fail(MFQ_EINVAL, "degree %d outside [1,%d]", degree, kMaxDegree);
  if (bc != MFQ_BC_NONE && bc != MFQ_BC_DIRICHLET0) return fail(MFQ_EINVAL, "unknown bc %d", bc);
  const int64_t N1 = (int64_t)degree * mesh->n + 1;
  const int64_t ndofs = N1 * N1 * N1;
  if (ndofs >= ((int64_t)1 << 31)) return fail(MFQ_EINVAL, "space has %lld DoFs (limit 2^31-1)", (long long)ndofs);
  const int64_t ncells = (int64_t)mesh->n * mesh->n * mesh->n;
  mfq_space* s = new (std::nothrow) mfq_space{mesh, degree, bc, ndofs, ncells};
  if (!s) return fail(MFQ_ENOMEM, "host allocation failed");
  *out = s;
  return MFQ_OK;
}

void mfq_space_destroy(mfq_space* space) { delete space; }
int64_t mfq_space_n_dofs(const mfq_space* space) { return space ? space->n_dofs : -1; }
int64_t mfq_space_n_cells(const mfq_space* space) { return space ? space->n_cells : -1; }

int mfq_space_apply_mask(const mfq_space* space, int precision, void* x, void* hip_stream) {
  if (!space) return fail(MFQ_EINVAL, "space is NULL");
  const int vp = vector_precision(precision);
  if (vp < 0) return fail(MFQ_EINVAL, "unknown precision %d", precision);
  if (int rc = check_vec(x, "x")) return rc;
  if (space->bc == MFQ_BC_NONE) return MFQ_OK;
  MFQ_HIP(launch_mask(vp, space->p, space->mesh->n, x, (hipStream_t)hip_stream));
  return MFQ_OK;
}

int mfq_space_random(const mfq_space* space, int precision, void* x, uint64_t seed, void* hip_stream) {
  if (!space) return fail(MFQ_EINVAL, "space is NULL");
  const int vp = vector_precision(precision);
  if (vp < 0) return fail(MFQ_EINVAL, "unknown precision %d", precision);
  if (int rc = check_vec(x, "x")) return rc;
  const int64_t N1 = (int64_t)space->p * space->mesh->n + 1;
  MFQ_HIP(launch_splitmix(vp, x, N1, seed, space->bc == MFQ_BC_DIRICHLET0, (hipStream_t)hip_stream));
  return MFQ_OK;
}

int mfq_op_create(const mfq_space* space, double alpha, int precision, mfq_op** out) {
  if (!space || !out) return fail(MFQ_EINVAL, "space or out is NULL");
  if (vector_precision(precision) < 0) return fail(MFQ_EINVAL, "unknown precision %d", precision);
  if (!std::isfinite(alpha) || std::fabs(alpha) >= 1.0)
    return fail(MFQ_EINVAL, "alpha %g must satisfy |alpha| < 1 (coefficient stays positive)", alpha);
  mfq_op* op = new (std::nothrow) mfq_op();
  if (!op) return fail(MFQ_ENOMEM, "host allocation failed");
  op->space = space;
  op->alpha = alpha;
  op->precision = vector_precision(precision);
  op->mfma = precision == MFQ_FP32_MFMA;
  const int p = space->p;
  op->bricks = make_bricks(p, space->mesh->n);
  const size_t nb = (size_t)op->bricks.n_bricks;
  const size_t lanes = (size_t)lanes_per_brick(p);
  op->idx_bytes = round_up(nb * (size_t)lattice_per_brick(p) * sizeof(int), 256);
  op->geo_bytes = round_up(nb * (p + 1) * 3 * lanes * 2 * real_size(precision), 256);
  if (space->mesh->amplitude == 0.0 && alpha != 0.0 && !op->mfma && !space->side)
    op->coef_bytes = round_up(nb * (p + 1) * lanes * real_size(precision), 256);
  *out = op;
  return MFQ_OK;
}

void mfq_op_destroy(mfq_op* op) { delete op; }

int mfq_op_device_bytes(const mfq_op* op, size_t* bytes) {
  if (!op || !bytes) return fail(MFQ_EINVAL, "op or bytes is NULL");
  *bytes = op->idx_bytes + op->geo_bytes + op->coef_bytes;
  return MFQ_OK;
}

int mfq_op_get_layout(const mfq_op* op, mfq_op_layout* out) {
  if (!op || !out) return fail(MFQ_EINVAL, "op or out is NULL");
  const Bricks& b = op->bricks;
  mfq_op_layout r{};
  r.brick[0] = b.bx;
  r.brick[1] = b.by;
  r.brick[2] = b.bz;
  for (int c = 0; c < kColours; ++c) {
    r.launches += b.count[c] > 0 ? 1 : 0;
    r.workgroups += b.count[c];
  }
  *out = r;
  return MFQ_OK;
}

int mfq_op_bind(mfq_op* op, void* dev_buf, size_t bytes, void* hip_stream) {
  if (!op) return fail(MFQ_EINVAL, "op is NULL");
  if (!dev_buf || !aligned(dev_buf, 256)) return fail(MFQ_EINVAL, "buffer NULL or not 256-byte aligned");
  const size_t need = op->idx_bytes + op->geo_bytes + op->coef_bytes;
  if (bytes < need) return fail(MFQ_ENOMEM, "buffer of %zu bytes, operator needs %zu", bytes, need);
  hipStream_t st = (hipStream_t)hip_stream;
  op->buf = dev_buf;
  op->idx = (int*)dev_buf;
  op->geo = (char*)dev_buf + op->idx_bytes;
  op->coef = op->coef_bytes ? (char*)op->geo + op->geo_bytes : nullptr;
  const OpView v = view(op);
  hipError_t e = launch_fill_index(v, op->idx, st);
  if (e == hipSuccess) e = launch_geometry(v, op->precision, op->geo, st);
  if (e == hipSuccess && op->coef) e = launch_coef_from_geo(v, op->precision, op->geo, op->coef, st);
  if (e != hipSuccess) {
    op->buf = nullptr;
    return fail(MFQ_EHIP, "operator setup launch failed: %s", hipGetErrorString(e));
  }
  return MFQ_OK;
}

int mfq_vmult(const mfq_op* op, const void* src, void* dst, void* hip_stream) {
  if (int rc = check_op(op)) return rc;
  if (int rc = check_vec(src, "src")) return rc;
  if (int rc = check_vec(dst, "dst")) return rc;
  const size_t bytes = (size_t)op->space->n_dofs * real_size(op->precision);
  const char* s = (const char*)src;
  const char* d = (const char*)dst;
  if (s < d + bytes && d < s + bytes) return fail(MFQ_EINVAL, "src and dst overlap");
  return op_vmult(op, src, dst, (hipStream_t)hip_stream);
}

int mfq_vmult_add(const mfq_op* op, const void* src, void* dst, void* hip_stream) {
  if (int rc = check_op(op)) return rc;
  if (int rc = check_vec(src, "src")) return rc;
  if (int rc = check_vec(dst, "dst")) return rc;
  const size_t bytes = (size_t)op->space->n_dofs * real_size(op->precision);
  const char* s = (const char*)src;
  const char* d = (const char*)dst;
  if (s < d + bytes && d < s + bytes) return fail(MFQ_EINVAL, "src and dst overlap");
  MFQ_HIP(launch_vmult_cells(view(op), op->precision, src, dst, true, (hipStream_t)hip_stream));
  return MFQ_OK;
}

int mfq_op_diagonal(const mfq_op* op, void* diag, void* hip_stream) {
  if (int rc = check_op(op)) return rc;
  if (int rc = check_vec(diag, "diag")) return rc;
  return op_diagonal(op, diag, (hipStream_t)hip_stream);
}

int mfq_op_geometry(const mfq_op* op, double* out_device, void* hip_stream) {
  if (int rc = check_op(op)) return rc;
  if (int rc = check_vec(out_device, "out")) return rc;
  MFQ_HIP(launch_geometry_export(view(op), op->precision, out_device, (hipStream_t)hip_stream));
  return MFQ_OK;
}

int mfq_rhs_manufactured(const mfq_op* op, double* b, void* hip_stream) {
  if (int rc = check_op(op)) return rc;
  if (int rc = check_vec(b, "b")) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  MFQ_HIP(launch_rhs_cells(view(op), b, st));  // writes every entry
  return MFQ_OK;
}

int mfq_transfer_create(const mfq_space* coarse, const mfq_space* fine, mfq_transfer** out) {
  if (!coarse || !fine || !out) return fail(MFQ_EINVAL, "coarse, fine or out is NULL");
  if (coarse->bc != fine->bc) return fail(MFQ_EINVAL, "spaces have different bc");
  if (coarse->mesh->amplitude != fine->mesh->amplitude) return fail(MFQ_EINVAL, "meshes have different deformation");
  bool h;
  if (fine->mesh->n == 2 * coarse->mesh->n && fine->p == coarse->p)
    h = true;
  else if (fine->mesh->n == coarse->mesh->n && fine->p > 1 && coarse->p == (fine->p + 1) / 2)
    h = false;
  else
    return fail(MFQ_EINVAL, "spaces (p=%d,n=%d) -> (p=%d,n=%d) are not an h- or p-coarsening pair", coarse->p,
                coarse->mesh->n, fine->p, fine->mesh->n);
  mfq_transfer* t = new (std::nothrow) mfq_transfer();
  if (!t) return fail(MFQ_ENOMEM, "host allocation failed");
  t->coarse = coarse;
  t->fine = fine;
  t->h_transfer = h;
  t->P1 = transfer_matrix_1d(coarse->p, fine->p, h, &t->nf1);
  *out = t;
  return MFQ_OK;
}

void mfq_transfer_destroy(mfq_transfer* t) { delete t; }

int mfq_prolongate(const mfq_transfer* t, int precision, const void* coarse, void* fine, void* hip_stream) {
  if (!t) return fail(MFQ_EINVAL, "transfer is NULL");
  const int vp = vector_precision(precision);
  if (vp < 0) return fail(MFQ_EINVAL, "unknown precision %d", precision);
  if (int rc = check_vec(coarse, "coarse")) return rc;
  if (int rc = check_vec(fine, "fine")) return rc;
  MFQ_HIP(launch_transfer(t, vp, true, coarse, fine, (hipStream_t)hip_stream));
  return MFQ_OK;
}

int mfq_restrict(const mfq_transfer* t, int precision, const void* fine, void* coarse, void* hip_stream) {
  if (!t) return fail(MFQ_EINVAL, "transfer is NULL");
  const int vp = vector_precision(precision);
  if (vp < 0) return fail(MFQ_EINVAL, "unknown precision %d", precision);
  if (int rc = check_vec(coarse, "coarse")) return rc;
  if (int rc = check_vec(fine, "fine")) return rc;
  MFQ_HIP(launch_transfer(t, vp, false, fine, coarse, (hipStream_t)hip_stream));
  return MFQ_OK;
}

int mfq_op_set_fused_updates(mfq_op* op, int enable) {
  if (!op) return fail(MFQ_EINVAL, "op is NULL");
  op->fuse = enable != 0;
  return MFQ_OK;
}

int mfq_chebyshev(const mfq_op* op, const void* inv_diag, const void* b, void* x, int x_is_zero, int degree,
                  double lmin, double lmax, void* work, void* hip_stream) {
  if (int rc = check_op(op)) return rc;
  if (int rc = check_vec(inv_diag, "inv_diag")) return rc;
  if (int rc = check_vec(b, "b")) return rc;
  if (int rc = check_vec(x, "x")) return rc;
  if (int rc = check_vec(work, "work")) return rc;
  if (degree < 1 || degree > 64) return fail(MFQ_EINVAL, "degree %d outside [1,64]", degree);
  if (!(lmin > 0) || !(lmax > lmin)) return fail(MFQ_EINVAL, "need 0 < lmin < lmax (got %g, %g)", lmin, lmax);
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t n = op->space->n_dofs;
  const size_t rs = real_size(op->precision);
  char* w = (char*)work;
  void* r = w;
  void* d = w + n * rs;
  void* t = w + 2 * n * rs;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  // With fused updates enabled on the operator, each step's vector update is done inside the
  // operator application (applied where a node's product completes; t keeps only partial sums);
  // otherwise, and always on the matrix cores and with hanging nodes, the product is stored and a
  // vector kernel follows.
  const OpView v = view(op);
  const bool fuse = op->fuse && !op->mfma && v.side_base < 0;
  CellEpilogue ep;
  ep.b = b;
  ep.dinv = inv_diag;
  ep.x = x;
  ep.r = r;
  ep.d = d;
  if (x_is_zero) {
    MFQ_HIP(launch_cheb_first(op->precision, b, t, inv_diag, x, r, d, n, 1.0 / theta, true, st));
  } else if (fuse) {
    ep.mode = kEpiChebFirst;
    ep.s0 = 1.0 / theta;
    MFQ_HIP(launch_vmult_epilogue(v, op->precision, x, t, ep, st));
  } else {
    if (int rc = op_vmult(op, x, t, st)) return rc;
    MFQ_HIP(launch_cheb_first(op->precision, b, t, inv_diag, x, r, d, n, 1.0 / theta, false, st));
  }
  for (int k = 1; k < degree; ++k) {
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    const double c1 = rho_new * rho, c2 = 2.0 * rho_new / delta;
    if (fuse) {
      ep.mode = kEpiChebStep;
      ep.s0 = c1;
      ep.s1 = c2;
      MFQ_HIP(launch_vmult_epilogue(v, op->precision, d, t, ep, st));
    } else {
      if (int rc = op_vmult(op, d, t, st)) return rc;
      MFQ_HIP(launch_cheb_step(op->precision, t, inv_diag, x, r, d, n, c1, c2, st));
    }
    rho = rho_new;
  }
  return MFQ_OK;
}

}  // extern "C"
