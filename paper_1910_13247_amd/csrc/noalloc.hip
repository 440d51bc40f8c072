// Chebyshev smoother without a caller workspace: the three work vectors live in a fixed device
// array of this library, for callers that cannot allocate device memory (code under HIP graph
// capture, serving loops that must not call the allocator).  Same kernels and the same arithmetic
// as mfq_chebyshev, so both give bitwise equal results on equal inputs.
#include <mutex>

#include "mfq_internal.hpp"

using namespace mfq;

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

// The work vectors r, d, t (3 n elements of the operator's precision).  Its host-side name is not
// a device address: host code uses only the per-device pointer that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per device with that device
// current (the caller's current device); nullptr and an error message on failure.
void* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    fail(MFQ_EHIP, "no current HIP device (or device ordinal %d beyond %d)", dev, kMaxDevices);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      fail(MFQ_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
      return nullptr;
    }
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" {

size_t mfq_chebyshev_noalloc_max_bytes(void) { return kScratchBytes; }

int mfq_chebyshev_noalloc(const mfq_op* op, const void* inv_diag, const void* b, void* x, int x_is_zero, int degree,
                          double lmin, double lmax, void* hip_stream) {
  if (!op) return fail(MFQ_EINVAL, "operator is NULL");
  const size_t rs = op->precision == MFQ_FP64 ? 8 : 4;
  const size_t need = 3 * (size_t)op->space->n_dofs * rs;
  if (need > kScratchBytes)
    return fail(MFQ_EINVAL, "mfq_chebyshev_noalloc: 3 work vectors of %lld DoFs need %zu bytes, more than the %zu "
                "bytes of its fixed device array (use mfq_chebyshev with a workspace)",
                (long long)op->space->n_dofs, need, kScratchBytes);
  if (!op->buf) return fail(MFQ_EINVAL, "operator is not bound to device memory (call mfq_op_bind)");
  void* work = scratch_on_current_device();
  if (!work) return MFQ_EHIP;
  return mfq_chebyshev(op, inv_diag, b, x, x_is_zero, degree, lmin, lmax, work, hip_stream);
}

}  // extern "C"
