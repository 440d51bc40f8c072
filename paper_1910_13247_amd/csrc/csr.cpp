// C ABI of the assembled sparse matrix (see include/mfq.h, "assembled matrix").
#include <new>

#include "mfq_internal.hpp"

using namespace mfq;

namespace {

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Product kernels: matrices whose mean row holds at least MFQ_CSR_LONG_ROW entries use lane
// groups per row (enough independent loads per row); shorter rows use row blocks whose products
// are staged in LDS (window entries plus the longest row must fit 64 KiB of values).
#ifndef MFQ_CSR_LONG_ROW
#define MFQ_CSR_LONG_ROW 384
#endif
// window of a row block in bytes of staged products: 2048 FP64 or 4096 FP32 entries
#ifndef MFQ_CSR_WINDOW_BYTES
#define MFQ_CSR_WINDOW_BYTES 16384
#endif
// lanes per row: 0 = from the mean row length (a build may fix it, e.g. -DMFQ_CSR_LPR=32)
#ifndef MFQ_CSR_LPR
#define MFQ_CSR_LPR 0
#endif
constexpr int64_t kLdsBytes = 65536;

}  // namespace

extern "C" {

int mfq_csr_create(const mfq_op* op, int precision, mfq_csr** out) {
  if (!op || !out) return fail(MFQ_EINVAL, "op or out is NULL");
  if (op->precision != MFQ_FP64 || op->mfma) return fail(MFQ_EINVAL, "the assembled matrix needs an MFQ_FP64 operator");
  if (precision != MFQ_FP64 && precision != MFQ_FP32)
    return fail(MFQ_EINVAL, "value precision %d is not MFQ_FP64 or MFQ_FP32", precision);
  const size_t vsize = precision == MFQ_FP64 ? sizeof(double) : sizeof(float);
  const mfq_space* s = op->space;
  const int p = s->p, n = s->mesh->n;
  const int64_t S = (int64_t)n * (p + 1) * (p + 1) - n + 1;
  mfq_csr* a = new (std::nothrow) mfq_csr();
  if (!a) return fail(MFQ_ENOMEM, "host allocation failed");
  a->op = op;
  a->precision = precision;
  a->p = p;
  a->n = n;
  a->bc = s->bc;
  a->n_rows = s->n_dofs;
  a->nnz = S * S * S;
  const double avg = (double)a->nnz / (double)a->n_rows;
  a->long_rows = avg >= MFQ_CSR_LONG_ROW;
  a->lanes_per_row = MFQ_CSR_LPR ? MFQ_CSR_LPR : a->long_rows ? 64 : avg >= 160 ? 32 : avg >= 40 ? 16 : 8;
  const int64_t len1 = n >= 2 ? 2 * p + 1 : p + 1;  // longest 1D neighbour range
  a->max_row = len1 * len1 * len1;
  int64_t w = MFQ_CSR_WINDOW_BYTES / (int64_t)vsize;
  if (w + a->max_row > kLdsBytes / (int64_t)vsize) w = (kLdsBytes / (int64_t)vsize - a->max_row) / 256 * 256;
  a->window = w;
  a->n_blocks = (a->nnz + w - 1) / w;
  a->rowptr_bytes = round_up((size_t)(a->n_rows + 1) * sizeof(int64_t), 256);
  a->cols_bytes = round_up((size_t)a->nnz * sizeof(int), 256);
  a->vals_bytes = round_up((size_t)a->nnz * vsize, 256);
  a->blk_bytes = round_up((size_t)(a->n_blocks + 1) * sizeof(int64_t), 256);
  *out = a;
  return MFQ_OK;
}

void mfq_csr_destroy(mfq_csr* a) { delete a; }

int mfq_csr_size(const mfq_csr* a, int64_t* n_rows, int64_t* nnz, size_t* device_bytes) {
  if (!a) return fail(MFQ_EINVAL, "matrix is NULL");
  if (n_rows) *n_rows = a->n_rows;
  if (nnz) *nnz = a->nnz;
  if (device_bytes) *device_bytes = a->rowptr_bytes + a->cols_bytes + a->vals_bytes + a->blk_bytes;
  return MFQ_OK;
}

int mfq_csr_bind(mfq_csr* a, void* dev_buf, size_t bytes, void* hip_stream) {
  if (!a) return fail(MFQ_EINVAL, "matrix is NULL");
  if (!a->op->buf) return fail(MFQ_EINVAL, "operator is not bound to device memory (call mfq_op_bind)");
  if (!dev_buf || !aligned(dev_buf, 256)) return fail(MFQ_EINVAL, "buffer NULL or not 256-byte aligned");
  const size_t need = a->rowptr_bytes + a->cols_bytes + a->vals_bytes + a->blk_bytes;
  if (bytes < need) return fail(MFQ_ENOMEM, "buffer of %zu bytes, matrix needs %zu", bytes, need);
  hipStream_t st = (hipStream_t)hip_stream;
  char* b = (char*)dev_buf;
  int64_t* rowptr = (int64_t*)b;
  int* cols = (int*)(b + a->rowptr_bytes);
  void* vals = b + a->rowptr_bytes + a->cols_bytes;
  int64_t* blk = (int64_t*)(b + a->rowptr_bytes + a->cols_bytes + a->vals_bytes);
  hipError_t e = launch_csr_pattern(a->p, a->n, rowptr, cols, st);
  if (e == hipSuccess) e = launch_csr_blocks(rowptr, blk, a->n_rows, a->n_blocks, a->window, st);
  if (e == hipSuccess) e = launch_fill(a->precision, vals, a->nnz, 0.0, st);
  if (e == hipSuccess) e = launch_csr_values(view(a->op), a->precision, rowptr, vals, st);
  if (e != hipSuccess) return fail(MFQ_EHIP, "matrix assembly launch failed: %s", hipGetErrorString(e));
  a->buf = dev_buf;
  a->rowptr = rowptr;
  a->cols = cols;
  a->vals = vals;
  a->blk = blk;
  return MFQ_OK;
}

int mfq_csr_arrays(const mfq_csr* a, void** rowptr, void** cols, void** vals) {
  if (!a) return fail(MFQ_EINVAL, "matrix is NULL");
  if (!a->buf) return fail(MFQ_EINVAL, "matrix is not bound (call mfq_csr_bind)");
  if (rowptr) *rowptr = a->rowptr;
  if (cols) *cols = a->cols;
  if (vals) *vals = a->vals;
  return MFQ_OK;
}

int mfq_csr_spmv(const mfq_csr* a, const void* src, void* dst, void* hip_stream) {
  if (!a) return fail(MFQ_EINVAL, "matrix is NULL");
  if (!a->buf) return fail(MFQ_EINVAL, "matrix is not bound (call mfq_csr_bind)");
  if (!src || !dst) return fail(MFQ_EINVAL, "src or dst is NULL");
  if (!aligned(src, 16) || !aligned(dst, 16)) return fail(MFQ_EINVAL, "src or dst is not 16-byte aligned");
  const size_t bytes = (size_t)a->n_rows * (a->precision == MFQ_FP64 ? sizeof(double) : sizeof(float));
  const char* s = (const char*)src;
  const char* d = (const char*)dst;
  if (s < d + bytes && d < s + bytes) return fail(MFQ_EINVAL, "src and dst overlap");
  MFQ_HIP(launch_csr_spmv(a, src, dst, (hipStream_t)hip_stream));
  return MFQ_OK;
}

}  // extern "C"
