// C ABI: the Q_p operator on the two-block mesh with hanging nodes, and CG on it (see
// include/mfq.h).  Sec. 3.3 (hanging nodes), Sec. 3.6 (matrix-free action).
#include <cmath>
#include <new>

#include "mfq_internal.hpp"

using namespace mfq;

struct mfq_hang {
  int p = 0, n = 0, precision = 0, bc = 0;
  mfq_mesh mesh0{}, mesh1{};
  mfq_space space0{}, space1{};
  mfq_op* op0 = nullptr;       // coarse block: n^3 cells of [0,1]^3
  mfq_op* op1 = nullptr;       // fine block: (2n)^3 cells of [1,2] x [0,1]^2, face X1 = 1 hanging
  int64_t n0 = 0, n1 = 0;      // lattice sizes of the blocks (vector = block 0, then block 1)
  size_t op0_bytes = 0, op1_bytes = 0, face_bytes = 0;
  void* buf = nullptr;
  void* f = nullptr;           // (2pn+1)^2: the coarse trace interpolated at the fine face nodes
  void* g = nullptr;           // (2pn+1)^2: the fine block's results at its face nodes
};

namespace {

size_t round256(size_t x) { return (x + 255) / 256 * 256; }
size_t rsize(int precision) { return precision == MFQ_FP64 ? 8 : 4; }

// Dirichlet faces (bit 2d: X_d = 0, bit 2d+1: X_d = 1) of each block on the domain [0,2] x [0,1]^2
constexpr int kFacesBlock0 = 0b111101;  // all but X1 = 1 (the interface)
constexpr int kFacesBlock1 = 0b111110;  // all but X1 = 1 (its X1-low face: the hanging nodes)

}  // namespace

namespace mfq {

int hang_vmult(const mfq_hang* h, const void* src, void* dst, hipStream_t st) {
  const size_t rs = rsize(h->precision);
  const char* s = (const char*)src;
  char* d = (char*)dst;
  const char* s1 = s + h->n0 * rs;
  char* d1 = d + h->n0 * rs;
  MFQ_HIP(launch_hang_interp(h->precision, h->p, h->n, h->bc, s, s1, h->f, d1, st));
  MFQ_HIP(launch_vmult_cells(view(h->op0), h->precision, s, d, false, st));
  OpView v1 = view(h->op1);
  v1.side_in = h->f;
  v1.side_out = h->g;
  MFQ_HIP(launch_vmult_cells(v1, h->precision, s1, d1, false, st));
  MFQ_HIP(launch_hang_restrict(h->precision, h->p, h->n, h->bc, h->g, d, st));
  return MFQ_OK;
}

}  // namespace mfq

extern "C" {

int mfq_hang_create(int n_coarse, double amplitude, int degree, double alpha, int precision, mfq_hang** out) {
  if (!out) return fail(MFQ_EINVAL, "out is NULL");
  if (n_coarse < 1 || n_coarse > 512) return fail(MFQ_EINVAL, "n_coarse=%d outside [1,512]", n_coarse);
  if (degree < 1 || degree > kMaxDegree) return fail(MFQ_EINVAL, "degree %d outside [1,%d]", degree, kMaxDegree);
  if (precision != MFQ_FP64 && precision != MFQ_FP32)
    return fail(MFQ_EINVAL, "precision %d: the hanging-node operator runs in MFQ_FP64 or MFQ_FP32", precision);
  if (!std::isfinite(amplitude) || std::fabs(amplitude) * 3.0 * M_PI >= 1.0)
    return fail(MFQ_EINVAL, "amplitude %g would make the deformation non-invertible", amplitude);
  const int64_t L1 = 2 * (int64_t)degree * n_coarse + 1;
  const int64_t n0 = ((int64_t)degree * n_coarse + 1) * ((int64_t)degree * n_coarse + 1) * ((int64_t)degree * n_coarse + 1);
  const int64_t n1 = L1 * L1 * L1;
  if (n0 + n1 + L1 * L1 >= ((int64_t)1 << 31))
    return fail(MFQ_EINVAL, "two-block mesh of %lld DoFs (limit 2^31 minus one face)", (long long)(n0 + n1));
  mfq_hang* h = new (std::nothrow) mfq_hang();
  if (!h) return fail(MFQ_ENOMEM, "host allocation failed");
  h->p = degree;
  h->n = n_coarse;
  h->precision = precision;
  h->bc = MFQ_BC_DIRICHLET0;
  h->mesh0 = mfq_mesh{n_coarse, amplitude, 0.0};
  h->mesh1 = mfq_mesh{2 * n_coarse, amplitude, 1.0};
  h->space0 = mfq_space{&h->mesh0, degree, MFQ_BC_DIRICHLET0, n0, (int64_t)n_coarse * n_coarse * n_coarse,
                        kFacesBlock0, false};
  h->space1 = mfq_space{&h->mesh1, degree, MFQ_BC_DIRICHLET0, n1, 8 * (int64_t)n_coarse * n_coarse * n_coarse,
                        kFacesBlock1, true};
  h->n0 = n0;
  h->n1 = n1;
  int rc = mfq_op_create(&h->space0, alpha, precision, &h->op0);
  if (!rc) rc = mfq_op_create(&h->space1, alpha, precision, &h->op1);
  if (rc) {
    mfq_op_destroy(h->op0);
    delete h;
    return rc;
  }
  mfq_op_device_bytes(h->op0, &h->op0_bytes);
  mfq_op_device_bytes(h->op1, &h->op1_bytes);
  h->face_bytes = round256((size_t)(L1 * L1) * rsize(precision));
  *out = h;
  return MFQ_OK;
}

void mfq_hang_destroy(mfq_hang* h) {
  if (!h) return;
  mfq_op_destroy(h->op0);
  mfq_op_destroy(h->op1);
  delete h;
}

int64_t mfq_hang_n_dofs(const mfq_hang* h) { return h ? h->n0 + h->n1 : -1; }

int mfq_hang_device_bytes(const mfq_hang* h, size_t* bytes) {
  if (!h || !bytes) return fail(MFQ_EINVAL, "h or bytes is NULL");
  *bytes = h->op0_bytes + h->op1_bytes + 2 * h->face_bytes;
  return MFQ_OK;
}

int mfq_hang_bind(mfq_hang* h, void* dev_buf, size_t bytes, void* hip_stream) {
  if (!h) return fail(MFQ_EINVAL, "h is NULL");
  size_t need = 0;
  mfq_hang_device_bytes(h, &need);
  if (!dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) % 256) != 0)
    return fail(MFQ_EINVAL, "buffer NULL or not 256-byte aligned");
  if (bytes < need) return fail(MFQ_ENOMEM, "buffer of %zu bytes, the two-block operator needs %zu", bytes, need);
  char* b = (char*)dev_buf;
  h->buf = nullptr;
  if (int rc = mfq_op_bind(h->op0, b, h->op0_bytes, hip_stream)) return rc;
  if (int rc = mfq_op_bind(h->op1, b + h->op0_bytes, h->op1_bytes, hip_stream)) return rc;
  h->f = b + h->op0_bytes + h->op1_bytes;
  h->g = (char*)h->f + h->face_bytes;
  h->buf = dev_buf;
  return MFQ_OK;
}

int mfq_hang_vmult(const mfq_hang* h, const void* src, void* dst, void* hip_stream) {
  if (!h) return fail(MFQ_EINVAL, "h is NULL");
  if (!h->buf) return fail(MFQ_EINVAL, "the two-block operator is not bound (call mfq_hang_bind)");
  if (!src || !dst || (reinterpret_cast<uintptr_t>(src) % 16) || (reinterpret_cast<uintptr_t>(dst) % 16))
    return fail(MFQ_EINVAL, "src or dst NULL or not 16-byte aligned");
  const size_t bytes = (size_t)(h->n0 + h->n1) * rsize(h->precision);
  const char* s = (const char*)src;
  const char* d = (const char*)dst;
  if (s < d + bytes && d < s + bytes) return fail(MFQ_EINVAL, "src and dst overlap");
  return hang_vmult(h, src, dst, (hipStream_t)hip_stream);
}

size_t mfq_hang_cg_work_bytes(const mfq_hang* h) {
  return h ? cg_work_bytes(h->n0 + h->n1) : 0;
}

int mfq_hang_cg(const mfq_hang* h, const double* b, double* x, double rtol, int max_iter, void* work,
                size_t work_bytes, void* hip_stream, mfq_solve_info* info) {
  if (!h) return fail(MFQ_EINVAL, "h is NULL");
  if (!h->buf) return fail(MFQ_EINVAL, "the two-block operator is not bound (call mfq_hang_bind)");
  if (h->precision != MFQ_FP64) return fail(MFQ_EINVAL, "mfq_hang_cg needs an MFQ_FP64 operator");
  if (!b || !x || !work) return fail(MFQ_EINVAL, "b, x or work is NULL");
  if ((reinterpret_cast<uintptr_t>(work) % 256) != 0) return fail(MFQ_EINVAL, "work is not 256-byte aligned");
  const int64_t n = h->n0 + h->n1;
  if (work_bytes < cg_work_bytes(n)) return fail(MFQ_ENOMEM, "work of %zu bytes, CG needs %zu", work_bytes, cg_work_bytes(n));
  if (!(rtol > 0) || max_iter < 1) return fail(MFQ_EINVAL, "need rtol > 0 and max_iter >= 1");
  hipStream_t st = (hipStream_t)hip_stream;
  Apply A = [h, st](const double* in, double* out) { return hang_vmult(h, in, out, st); };
  return cg_unpreconditioned(A, b, x, n, rtol, max_iter, work, st, info);
}

}  // extern "C"
