// C ABI of the DG-SIPG operator (see include/mfq.h, "discontinuous Galerkin operator").
#include <new>

#include "mfq_internal.hpp"

using namespace mfq;

extern "C" {

int mfq_dg_create(const mfq_mesh* mesh, int degree, mfq_dg** out) {
  if (!mesh || !out) return fail(MFQ_EINVAL, "mesh or out is NULL");
  if (degree < 1 || degree > kMaxDegree) return fail(MFQ_EINVAL, "degree %d outside [1,%d]", degree, kMaxDegree);
  if (mesh->amplitude != 0.0) return fail(MFQ_EINVAL, "the DG operator needs the undeformed mesh (amplitude 0)");
  const int64_t nloc = (int64_t)(degree + 1) * (degree + 1) * (degree + 1);
  const int64_t cells = (int64_t)mesh->n * mesh->n * mesh->n;
  if (cells * nloc >= ((int64_t)1 << 31)) return fail(MFQ_EINVAL, "space has %lld DoFs (limit 2^31-1)", (long long)(cells * nloc));
  mfq_dg* g = new (std::nothrow) mfq_dg{degree, mesh->n, cells * nloc};
  if (!g) return fail(MFQ_ENOMEM, "host allocation failed");
  *out = g;
  return MFQ_OK;
}

void mfq_dg_destroy(mfq_dg* g) { delete g; }

int64_t mfq_dg_n_dofs(const mfq_dg* g) { return g ? g->n_dofs : -1; }

int mfq_dg_vmult(const mfq_dg* g, const double* src, double* dst, void* hip_stream) {
  if (!g) return fail(MFQ_EINVAL, "operator is NULL");
  if (!src || !dst) return fail(MFQ_EINVAL, "src or dst is NULL");
  if ((reinterpret_cast<uintptr_t>(src) % 16) || (reinterpret_cast<uintptr_t>(dst) % 16))
    return fail(MFQ_EINVAL, "src or dst is not 16-byte aligned");
  const size_t bytes = (size_t)g->n_dofs * sizeof(double);
  const char* s = (const char*)src;
  const char* d = (const char*)dst;
  if (s < d + bytes && d < s + bytes) return fail(MFQ_EINVAL, "src and dst overlap");
  MFQ_HIP(launch_dg_vmult(g->p, g->n, MFQ_FP64, src, dst, (hipStream_t)hip_stream));
  return MFQ_OK;
}

int mfq_dg_vmult_prec(const mfq_dg* g, int precision, const void* src, void* dst, void* hip_stream) {
  if (!g) return fail(MFQ_EINVAL, "operator is NULL");
  if (precision != MFQ_FP64 && precision != MFQ_FP32) return fail(MFQ_EINVAL, "precision must be FP64 or FP32");
  if (!src || !dst) return fail(MFQ_EINVAL, "src or dst is NULL");
  if ((reinterpret_cast<uintptr_t>(src) % 16) || (reinterpret_cast<uintptr_t>(dst) % 16))
    return fail(MFQ_EINVAL, "src or dst is not 16-byte aligned");
  const size_t bytes = (size_t)g->n_dofs * (precision == MFQ_FP64 ? 8 : 4);
  const char* s = (const char*)src;
  const char* d = (const char*)dst;
  if (s < d + bytes && d < s + bytes) return fail(MFQ_EINVAL, "src and dst overlap");
  MFQ_HIP(launch_dg_vmult(g->p, g->n, precision, src, dst, (hipStream_t)hip_stream));
  return MFQ_OK;
}

int mfq_dg_diagonal(const mfq_dg* g, int precision, void* diag, void* hip_stream) {
  if (!g) return fail(MFQ_EINVAL, "operator is NULL");
  if (precision != MFQ_FP64 && precision != MFQ_FP32) return fail(MFQ_EINVAL, "precision must be FP64 or FP32");
  if (!diag) return fail(MFQ_EINVAL, "diag is NULL");
  MFQ_HIP(launch_dg_diagonal(g->p, g->n, precision, diag, (hipStream_t)hip_stream));
  return MFQ_OK;
}

int64_t mfq_dg_cg_n_dofs(const mfq_dg* g) {
  if (!g) return -1;
  const int64_t m = (int64_t)g->n * g->p + 1;
  return m * m * m;
}

int mfq_dg_transfer(const mfq_dg* g, int precision, int to_dg, const void* in, void* out, void* hip_stream) {
  if (!g) return fail(MFQ_EINVAL, "operator is NULL");
  if (precision != MFQ_FP64 && precision != MFQ_FP32) return fail(MFQ_EINVAL, "precision must be FP64 or FP32");
  if (!in || !out) return fail(MFQ_EINVAL, "in or out is NULL");
  const size_t w = precision == MFQ_FP64 ? 8 : 4;
  const size_t bin = (size_t)(to_dg ? mfq_dg_cg_n_dofs(g) : g->n_dofs) * w;
  const size_t bout = (size_t)(to_dg ? g->n_dofs : mfq_dg_cg_n_dofs(g)) * w;
  const char* s = (const char*)in;
  const char* d = (const char*)out;
  if (s < d + bout && d < s + bin) return fail(MFQ_EINVAL, "in and out overlap");
  MFQ_HIP(launch_dg_transfer(g->p, g->n, precision, to_dg != 0, in, out, (hipStream_t)hip_stream));
  return MFQ_OK;
}

}  // extern "C"
