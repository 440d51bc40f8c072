// Hanging-node constraints of the two-block mesh (Sec. 3.3: adaptive refinement with hanging
// nodes).  Block 0 is the unit cube in n^3 cells, block 1 the cube [1,2] x [0,1]^2 in (2n)^3 cells;
// on their common face X1 = 1 every coarse cell face meets 2 x 2 fine ones.  Block 1's nodes on that
// face are not unknowns: the conforming function takes there the coarse side's trace, interpolated
// from the coarse face nodes by the 1D h-transfer table in each face direction.  The operator is
// C^T A C: the fine block's cell loop reads those nodes from an interpolated face array f = C x and
// writes their results to a face array g, whose transpose-interpolation is added to the coarse face
// nodes.  Both face kernels run on one face of nodes only (O(N^(2/3)) work).
#include "kernels_common.hpp"

namespace mfq {

namespace {

// t.w[jl (p+1) + a]: coarse basis function a of one coarse cell at fine node jl in [0, 2p] of
// that cell (the 1D h-transfer table).
struct HangTable {
  double w[(2 * kMaxDegree + 1) * (kMaxDegree + 1)];
};

__device__ __forceinline__ bool on_ring(int i, int L) { return i == 0 || i == L - 1; }

// f[J + L1 K] = (Pi x Pi) (m x0) on the X1 = 1 face, and the hanging rows of block 1 are identity
// rows: y1 = x1 there.  Coarse face nodes on the domain boundary are Dirichlet nodes and count as
// zero (bc != 0).  Accumulated in FP64, rounded once.
template <typename Real>
__global__ __launch_bounds__(kBlock) void hang_interp_kernel(const Real* __restrict__ x0, const Real* __restrict__ x1,
                                                             Real* __restrict__ f, Real* __restrict__ y1, int p,
                                                             int n, int bc, HangTable t) {
  const int L0 = p * n + 1, L1 = 2 * p * n + 1;
  const int64_t total = (int64_t)L1 * L1;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
    const int J = (int)(k % L1), K = (int)(k / L1);
    const int cj = min(J / (2 * p), n - 1), ck = min(K / (2 * p), n - 1);
    const int jl = J - 2 * p * cj, kl = K - 2 * p * ck;
    double s = 0.0;
    for (int b = 0; b <= p; ++b) {
      const int Kc = p * ck + b;
      if (bc && on_ring(Kc, L0)) continue;
      double row = 0.0;
      for (int a = 0; a <= p; ++a) {
        const int Jc = p * cj + a;
        if (bc && on_ring(Jc, L0)) continue;
        row += t.w[jl * (p + 1) + a] * (double)x0[(L0 - 1) + (int64_t)L0 * (Jc + (int64_t)L0 * Kc)];
      }
      s += t.w[kl * (p + 1) + b] * row;
    }
    f[k] = (Real)s;
    const int64_t g1 = (int64_t)L1 * (J + (int64_t)L1 * K);
    y1[g1] = x1[g1];
  }
}

// y0 += (Pi x Pi)^T g on the coarse X1 = 1 face nodes that are not Dirichlet nodes: each coarse node
// sums the fine face nodes of its (at most 2 x 2) coarse cells in a fixed order (gather form, no
// atomics).  Fine node J belongs to coarse cell min(J / 2p, n - 1); its weight for coarse node Jc is
// the table entry of that cell, zero when Jc is not a node of it.
template <typename Real>
__global__ __launch_bounds__(kBlock) void hang_restrict_kernel(const Real* __restrict__ g, Real* __restrict__ y0, int p,
                                                               int n, int bc, HangTable t) {
  const int L0 = p * n + 1, L1 = 2 * p * n + 1;
  const int64_t total = (int64_t)L0 * L0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
    const int Jc = (int)(k % L0), Kc = (int)(k / L0);
    if (bc && (on_ring(Jc, L0) || on_ring(Kc, L0))) continue;
    const int jlo = 2 * p * (Jc > p ? (Jc - 1) / p : 0), jhi = 2 * p * min(n - 1, Jc / p) + 2 * p;
    const int klo = 2 * p * (Kc > p ? (Kc - 1) / p : 0), khi = 2 * p * min(n - 1, Kc / p) + 2 * p;
    double s = 0.0;
    for (int K = klo; K <= khi; ++K) {
      const int ck = min(K / (2 * p), n - 1), b = Kc - p * ck;
      // fine face nodes on the domain boundary are Dirichlet nodes: g holds nothing there (their
      // weight for a coarse node off the boundary is zero, and 0 times an unset value is not 0)
      if (b < 0 || b > p || (bc && on_ring(K, L1))) continue;
      const double wk = t.w[(K - 2 * p * ck) * (p + 1) + b];
      double row = 0.0;
      for (int J = jlo; J <= jhi; ++J) {
        const int cj = min(J / (2 * p), n - 1), a = Jc - p * cj;
        if (a < 0 || a > p || (bc && on_ring(J, L1))) continue;
        row += t.w[(J - 2 * p * cj) * (p + 1) + a] * (double)g[J + (int64_t)L1 * K];
      }
      s += wk * row;
    }
    const int64_t i0 = (L0 - 1) + (int64_t)L0 * (Jc + (int64_t)L0 * Kc);
    y0[i0] = (Real)((double)y0[i0] + s);
  }
}

unsigned face_grid(int64_t total) {
  const int64_t b = (total + kBlock - 1) / kBlock;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

HangTable make_hang_table(int p) {
  HangTable t{};
  int nf1 = 0;
  const std::vector<double> P1 = transfer_matrix_1d(p, p, true, &nf1);
  for (size_t i = 0; i < P1.size(); ++i) t.w[i] = P1[i];
  return t;
}

}  // namespace

hipError_t launch_hang_interp(int precision, int p, int n, int bc, const void* x0, const void* x1, void* f, void* y1,
                              hipStream_t st) {
  const HangTable t = make_hang_table(p);
  const unsigned g = face_grid((int64_t)(2 * p * n + 1) * (2 * p * n + 1));
  if (precision == MFQ_FP64)
    hang_interp_kernel<double><<<g, kBlock, 0, st>>>((const double*)x0, (const double*)x1, (double*)f, (double*)y1, p,
                                                    n, bc, t);
  else
    hang_interp_kernel<float><<<g, kBlock, 0, st>>>((const float*)x0, (const float*)x1, (float*)f, (float*)y1, p, n,
                                                   bc, t);
  return hipGetLastError();
}

hipError_t launch_hang_restrict(int precision, int p, int n, int bc, const void* g, void* y0, hipStream_t st) {
  const HangTable t = make_hang_table(p);
  const unsigned gr = face_grid((int64_t)(p * n + 1) * (p * n + 1));
  if (precision == MFQ_FP64)
    hang_restrict_kernel<double><<<gr, kBlock, 0, st>>>((const double*)g, (double*)y0, p, n, bc, t);
  else
    hang_restrict_kernel<float><<<gr, kBlock, 0, st>>>((const float*)g, (float*)y0, p, n, bc, t);
  return hipGetLastError();
}

}  // namespace mfq
