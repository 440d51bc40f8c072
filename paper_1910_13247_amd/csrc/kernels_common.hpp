// Device-side helpers shared by the CDNA4 kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mfq_internal.hpp"
#include "tables_ct.hpp"

namespace mfq {

// fused multiply-add in the operand's own precision (no promotion of float to double)
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// 1D shape tables at the Gauss points, S[q*(P+1)+a] = l_a(zeta_q), D[q*(P+1)+a] = l_a'(zeta_q).
// Passed by value as a kernel argument: with fully unrolled loops every entry is a
// compile-time offset into the kernel-argument segment and lands in scalar registers.
template <int P, typename Real>
struct Shape {
  Real S[(P + 1) * (P + 1)];
  Real D[(P + 1) * (P + 1)];
};

template <int P, typename Real>
constexpr Shape<P, Real> make_shape() {
  Shape<P, Real> sh{};
  for (int k = 0; k < (P + 1) * (P + 1); ++k) {
    sh.S[k] = (Real)ct::kTab<P>.S[k];
    sh.D[k] = (Real)ct::kTab<P>.D[k];
  }
  return sh;
}

// Even-odd form of a 1D table M (N1 x N1) with M[N1-1-q][N1-1-a] = sgn M[q][a]: S is symmetric
// and D antisymmetric under this reflection because the nodes and the Gauss points are symmetric
// about 1/2.  With e_k = x_k + x_{N1-1-k}, o_k = x_k - x_{N1-1-k} (k < H = N1/2):
//   y_q = E_q + O_q,  y_{N1-1-q} = sgn (E_q - O_q),  E_q = sum_k A[q][k] e_k (+ mc[q] x_H),
//   O_q = sum_k B[q][k] o_k, A = (M[q][k] + M[q][N1-1-k])/2, B = (M[q][k] - M[q][N1-1-k])/2, and
//   for odd N1 the middle row y_H = sum_k mr[k] e_k + cc x_H (sgn +1) or sum_k mr[k] o_k (sgn -1).
// The transpose reuses the same numbers (A^T, B^T, mid row <-> mid column; A and B swap for the
// antisymmetric table), so one set of about N1^2/2 constants per table serves both directions:
// few enough to stay in scalar registers for p <= 5 in FP64.
template <int N1, typename Real>
struct EvenOdd {
  static constexpr int H = N1 / 2;
  Real A[H * H];
  Real B[H * H];
  Real mc[H];
  Real mr[H];
  Real cc;
};

template <int P, typename Real>
struct ShapeEO {
  EvenOdd<P + 1, Real> S, D;
};

template <int N1, typename Real>
EvenOdd<N1, Real> make_even_odd(const double* M) {
  EvenOdd<N1, Real> t{};
  constexpr int H = N1 / 2;
  for (int q = 0; q < H; ++q)
    for (int k = 0; k < H; ++k) {
      t.A[q * H + k] = (Real)(0.5 * (M[q * N1 + k] + M[q * N1 + N1 - 1 - k]));
      t.B[q * H + k] = (Real)(0.5 * (M[q * N1 + k] - M[q * N1 + N1 - 1 - k]));
    }
  if (N1 % 2 == 1) {
    for (int q = 0; q < H; ++q) {
      t.mc[q] = (Real)M[q * N1 + H];
      t.mr[q] = (Real)M[H * N1 + q];
    }
    t.cc = (Real)M[H * N1 + H];
  }
  return t;
}

template <int P, typename Real>
ShapeEO<P, Real> make_shape_eo() {
  ShapeEO<P, Real> s;
  s.S = make_even_odd<P + 1, Real>(ct::kTab<P>.S);
  s.D = make_even_odd<P + 1, Real>(ct::kTab<P>.D);
  return s;
}

// y = M x (TR = false) or y = M^T x (TR = true) for a table in even-odd form; SGN = +1 for S,
// -1 for D.
template <int N1, int SGN, bool TR, typename Real>
__device__ __forceinline__ void eo_apply(const EvenOdd<N1, Real>& m, const Real (&x)[N1], Real (&y)[N1]) {
  constexpr int H = N1 / 2;
  constexpr bool odd = (N1 % 2) == 1;
  Real e[H > 0 ? H : 1], o[H > 0 ? H : 1];
#pragma unroll
  for (int k = 0; k < H; ++k) {
    e[k] = x[k] + x[N1 - 1 - k];
    o[k] = x[k] - x[N1 - 1 - k];
  }
#pragma unroll
  for (int q = 0; q < H; ++q) {
    Real E = 0, O = 0;
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const Real a = !TR ? m.A[q * H + k] : (SGN > 0 ? m.A[k * H + q] : m.B[k * H + q]);
      const Real b = !TR ? m.B[q * H + k] : (SGN > 0 ? m.B[k * H + q] : m.A[k * H + q]);
      E = fmad(a, e[k], E);
      O = fmad(b, o[k], O);
    }
    if constexpr (odd) E = fmad(TR ? m.mr[q] : m.mc[q], x[H], E);
    y[q] = E + O;
    y[N1 - 1 - q] = SGN > 0 ? E - O : O - E;
  }
  if constexpr (odd) {
    Real s = 0;
#pragma unroll
    for (int k = 0; k < H; ++k) s = fmad(TR ? m.mc[k] : m.mr[k], SGN > 0 ? e[k] : o[k], s);
    if constexpr (SGN > 0) s = fmad(m.cc, x[H], s);
    y[H] = s;
  }
}

// y = S^T x1 + D^T x2 in even-odd form
template <int N1, typename Real>
__device__ __forceinline__ void eo_apply_t2(const EvenOdd<N1, Real>& S, const Real (&x1)[N1],
                                            const EvenOdd<N1, Real>& D, const Real (&x2)[N1], Real (&y)[N1]) {
  Real y1[N1], y2[N1];
  eo_apply<N1, 1, true>(S, x1, y1);
  eo_apply<N1, -1, true>(D, x2, y2);
#pragma unroll
  for (int a = 0; a < N1; ++a) y[a] = y1[a] + y2[a];
}

// Compile-time geometry of the cell kernels: a workgroup works on a brick of BX*BY*BZ cells, one
// lane per 1D pencil of a cell (T = (P+1)^2 lanes per cell, NT lanes carry work), and the brick's
// node lattice LX*LY*LZ (shared nodes of neighbouring cells appear once).
template <int P>
struct Cell {
  static constexpr int N1 = P + 1;
  static constexpr int T = N1 * N1;
  static constexpr int NQ = N1 * T;
  static constexpr BrickDims BD = brick_dims(P);
  static constexpr int BX = BD.bx, BY = BD.by, BZ = BD.bz;
  static constexpr int NCELL = BX * BY * BZ;
  static constexpr int NT = NCELL * T;
  static constexpr int LX = BX * P + 1, LY = BY * P + 1, LZ = BZ * P + 1;
  static constexpr int NL = LX * LY * LZ;
  // workgroup of the per-brick kernels: 256 lanes, or 512 for bricks of more than 256 pencils
  static constexpr int BLOCK = NT <= kBlock ? kBlock : 2 * kBlock;
  static_assert(NT <= BLOCK, "a brick must fit one workgroup");
};

// Brick coordinates of brick b (counted within colour c, x fastest).
__host__ __device__ inline void brick_of(const Bricks& bk, int c, int64_t b64, int& bi, int& bj, int& bz) {
  const unsigned b = (unsigned)b64, cxn = (unsigned)bk.cxn[c], cyn = (unsigned)bk.cyn[c];
  const unsigned r = b / cxn, q = r / cyn;
  bi = 2 * (int)(b - r * cxn) + (c & 1);
  bj = 2 * (int)(r - q * cyn) + ((c >> 1) & 1);
  bz = 2 * (int)q + (c >> 2);
}

// Brick coordinates of a storage ordinal (colour-major order).
__host__ __device__ inline void brick_of_ordinal(const Bricks& bk, int64_t ord, int& bi, int& bj, int& bz) {
  int c = 0;
  while (c < kColours - 1 && ord >= bk.offset[c] + bk.count[c]) ++c;
  brick_of(bk, c, ord - bk.offset[c], bi, bj, bz);
}

// Storage ordinal of the brick holding cell (ci, cj, ck), and the cell's index inside it.
__host__ __device__ inline int64_t ordinal_of_cell(const Bricks& bk, int64_t ci, int64_t cj, int64_t ck, int& lc) {
  const int bi = (int)(ci / bk.bx), bj = (int)(cj / bk.by), bz = (int)(ck / bk.bz);
  lc = (int)(ci - (int64_t)bi * bk.bx) + bk.bx * ((int)(cj - (int64_t)bj * bk.by) + bk.by * (int)(ck - (int64_t)bz * bk.bz));
  const int c = (bi & 1) + 2 * (bj & 1) + 4 * (bz & 1);
  return bk.offset[c] + (bi / 2) + (int64_t)bk.cxn[c] * ((bj / 2) + (int64_t)bk.cyn[c] * (bz / 2));
}

// Workgroup barrier that orders LDS only: global loads issued before it stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One entry of the Chebyshev smoother's updates, written once for the vector kernels and the cell
// loop's fused epilogue.  Contraction is off and the one fused multiply-add is written out, so the
// rounding does not depend on how the compiler fuses the surrounding code (left to it, the two
// kernels round apart).
// First step: r = b - t (b when x = 0), d = dinv r / theta, x = x + d (d when x = 0).
template <typename Real>
__device__ __forceinline__ void cheb_first_entry(Real b, Real t, Real dinv, Real inv_theta, bool x_is_zero, Real& r,
                                                 Real& d, Real& x) {
#pragma clang fp contract(off)
  const Real rv = x_is_zero ? b : b - t;
  const Real dv = dinv * rv * inv_theta;
  r = rv;
  d = dv;
  x = x_is_zero ? dv : x + dv;
}
// Later steps: r = r - t, d = c1 d + c2 dinv r, x = x + d.
template <typename Real>
__device__ __forceinline__ void cheb_step_entry(Real t, Real dinv, Real c1, Real c2, Real& r, Real& d, Real& x) {
#pragma clang fp contract(off)
  const Real rv = r - t;
  Real dv;
  if constexpr (sizeof(Real) == 8)
    dv = __builtin_fma(c1, d, c2 * dinv * rv);
  else
    dv = __builtin_fmaf(c1, d, c2 * dinv * rv);
  r = rv;
  d = dv;
  x = x + dv;
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
    for (int a = 1; a < N1; ++a) s = fmad(M[q * N1 + a], in[a], s);
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
    for (int q = 1; q < N1; ++q) s = fmad(M[q * N1 + a], in[q], s);
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
    s = fmad(M2[a], in2[0], s);
#pragma unroll
    for (int q = 1; q < N1; ++q) {
      s = fmad(M1[q * N1 + a], in1[q], s);
      s = fmad(M2[q * N1 + a], in2[q], s);
    }
    out[a] = s;
  }
}

// Quadrature-point geometry of the deformed cube (FP64): the exact map
// x = X + A sin(pi X1) sin(pi X2) sin(pi X3) (1,1,1) evaluated at the point, X = h*(cell + xhat)
// (shifted by x0 along X1 for a mesh that starts at X1 = x0).
struct QGeo {
  double x[3];      // physical point
  double Jinv[3][3];
  double detJ;      // det of dx/dxhat
};

__device__ __forceinline__ void qpoint_geometry(int n, double amp, int64_t cell, double xh0, double xh1,
                                                double xh2, QGeo& g, double x0 = 0.0) {
  const double h = 1.0 / n;
  const int64_t i = cell % n, j = (cell / n) % n, k = cell / ((int64_t)n * n);
  const double X[3] = {x0 + h * ((double)i + xh0), h * ((double)j + xh1), h * ((double)k + xh2)};
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
