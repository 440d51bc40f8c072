// C ABI of the DG-SIPG operator (see include/mfq.h, "discontinuous Galerkin operator").
#include <new>

#include "mfq_internal.hpp"

using namespace mfq;

struct mfq_dg {
  int p, n;
  int64_t n_dofs;
};

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
  MFQ_HIP(launch_dg_vmult(g->p, g->n, src, dst, (hipStream_t)hip_stream));
  return MFQ_OK;
}

}  // extern "C"
