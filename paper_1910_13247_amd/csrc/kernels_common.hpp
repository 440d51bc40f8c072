// Device-side helpers shared by the CDNA4 kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mfq_internal.hpp"

namespace mfq {

// 1D shape tables at the Gauss points, S[q*(P+1)+a] = l_a(zeta_q), D[q*(P+1)+a] = l_a'(zeta_q).
// Passed by value as a kernel argument: with fully unrolled loops every entry is a
// compile-time offset into the kernel-argument segment and lands in scalar registers.
template <int P, typename Real>
struct Shape {
  Real S[(P + 1) * (P + 1)];
  Real D[(P + 1) * (P + 1)];
};

template <int P, typename Real>
Shape<P, Real> make_shape() {
  Shape<P, Real> sh;
  const Tables1D& t = tables(P);
  for (int k = 0; k < (P + 1) * (P + 1); ++k) {
    sh.S[k] = (Real)t.S[k];
    sh.D[k] = (Real)t.D[k];
  }
  return sh;
}

// Compile-time geometry of the cell kernels: one thread per 1D pencil ((P+1)^2 per cell),
// CPB cells per 256-lane workgroup, NT lanes carry work (the rest idle).
template <int P>
struct Cell {
  static constexpr int N1 = P + 1;
  static constexpr int T = N1 * N1;
  static constexpr int NQ = N1 * T;
  static constexpr int CPB = kBlock / T;
  static constexpr int NT = CPB * T;
};

// Workgroup barrier that orders LDS only: global loads issued before it stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename Real>
using Real2 = Real __attribute__((ext_vector_type(2)));

// out[q] = sum_a M[q][a] in[a]
template <int N1, typename Real>
__device__ __forceinline__ void apply(const Real* M, const Real (&in)[N1], Real (&out)[N1]) {
#pragma unroll
  for (int q = 0; q < N1; ++q) {
    Real s = M[q * N1] * in[0];
#pragma unroll
    for (int a = 1; a < N1; ++a) s = __builtin_fma(M[q * N1 + a], in[a], s);
    out[q] = s;
  }
}

// out[a] = sum_q M[q][a] in[q]
template <int N1, typename Real>
__device__ __forceinline__ void apply_t(const Real* M, const Real (&in)[N1], Real (&out)[N1]) {
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    Real s = M[a] * in[0];
#pragma unroll
    for (int q = 1; q < N1; ++q) s = __builtin_fma(M[q * N1 + a], in[q], s);
    out[a] = s;
  }
}

// out[a] = sum_q M1[q][a] in1[q] + M2[q][a] in2[q]
template <int N1, typename Real>
__device__ __forceinline__ void apply_t2(const Real* M1, const Real (&in1)[N1], const Real* M2,
                                         const Real (&in2)[N1], Real (&out)[N1]) {
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    Real s = M1[a] * in1[0];
    s = __builtin_fma(M2[a], in2[0], s);
#pragma unroll
    for (int q = 1; q < N1; ++q) {
      s = __builtin_fma(M1[q * N1 + a], in1[q], s);
      s = __builtin_fma(M2[q * N1 + a], in2[q], s);
    }
    out[a] = s;
  }
}

__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }

// Quadrature-point geometry of the deformed cube (FP64): the exact map
// x = X + A sin(pi X1) sin(pi X2) sin(pi X3) (1,1,1) evaluated at the point, X = h*(cell + xhat).
struct QGeo {
  double x[3];      // physical point
  double Jinv[3][3];
  double detJ;      // det of dx/dxhat
};

__device__ __forceinline__ void qpoint_geometry(int n, double amp, int64_t cell, double xh0, double xh1,
                                                double xh2, QGeo& g) {
  const double h = 1.0 / n;
  const int64_t i = cell % n, j = (cell / n) % n, k = cell / ((int64_t)n * n);
  const double X[3] = {h * ((double)i + xh0), h * ((double)j + xh1), h * ((double)k + xh2)};
  double s[3], c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) sincospi(X[d], &s[d], &c[d]);
  const double sv = s[0] * s[1] * s[2];
  const double gs[3] = {M_PI * c[0] * s[1] * s[2], M_PI * s[0] * c[1] * s[2], M_PI * s[0] * s[1] * c[2]};
  double J[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) J[r][cc] = h * ((r == cc ? 1.0 : 0.0) + amp * gs[cc]);
#pragma unroll
  for (int d = 0; d < 3; ++d) g.x[d] = X[d] + amp * sv;
  // inverse by cofactors
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  const double id = 1.0 / det;
  g.detJ = det;
  g.Jinv[0][0] = c00 * id;
  g.Jinv[1][0] = c01 * id;
  g.Jinv[2][0] = c02 * id;
  g.Jinv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  g.Jinv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  g.Jinv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  g.Jinv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  g.Jinv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  g.Jinv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
}

__device__ __forceinline__ double coefficient(double alpha, const double (&x)[3]) {
  return 1.0 + alpha * sinpi(2.0 * x[0]) * sinpi(2.0 * x[1]) * sinpi(2.0 * x[2]);
}

}  // namespace mfq
