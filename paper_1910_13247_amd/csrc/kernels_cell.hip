// Cell kernels of the matrix-free Q_p operator on CDNA4 (gfx950).
//
// The operator is the variable-coefficient weak Laplacian of eq. (1), integrated cell by cell
// with shape-function gradients and JxW at the (p+1)^3 Gauss points (Sec. 2.4 cell loop) and
// applied without a matrix (Sec. 3.6): gather the cell's DoFs, evaluate reference gradients at
// the quadrature points by sum factorisation, multiply by the stored quadrature-point tensor
// G_q = w_q a(x_q) det(J_q) J_q^{-1} J_q^{-T}, test with the reference gradients (transposed sum
// factorisation), scatter-add.
//
// Work decomposition (MI355X-first): one lane per 1D pencil of a cell ((p+1)^2 lanes per cell,
// 256 // (p+1)^2 cells per workgroup), each lane contracting its pencil in registers; the
// pencils change direction through LDS.  Gradients are formed directly from the 1D value and
// derivative tables in the order x (S, D) -> y (S, D on the S-branch) -> z, so all three
// components arrive at the same lane and point without extra transposes; the backward pass is
// the exact transpose.  The G stream (the dominant HBM traffic) is laid out so that every wave
// load is 1 KiB contiguous and is issued at kernel start to overlap the forward contractions.
#include "kernels_common.hpp"

namespace mfq {

namespace {

// ---------------------------------------------------------------- index maps
// idx[blk][a][lane]: lane = lc*T + e, e = e0 + N1*e1, holds the global DoF of local DoF
// (a, e0, e1) of cell blk*CPB + lc; Dirichlet nodes are stored as ~g (negative).
template <int P>
__global__ __launch_bounds__(kBlock) void fill_index_kernel(int* __restrict__ idx, int64_t n_cells, int64_t n_blocks,
                                                            int n, int bc) {
  using C = Cell<P>;
  const int64_t total = n_blocks * C::N1 * C::NT;
  const int64_t N1g = (int64_t)P * n + 1;
  for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < total; L += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = L / (C::N1 * C::NT);
    const int rem = (int)(L - blk * (C::N1 * C::NT));
    const int a = rem / C::NT;
    const int lane = rem - a * C::NT;
    const int lc = lane / C::T;
    const int e = lane - lc * C::T;
    const int e0 = e % C::N1, e1 = e / C::N1;
    const int64_t cell = blk * C::CPB + lc;
    int val = 0;
    if (cell < n_cells) {
      const int64_t ci = cell % n, cj = (cell / n) % n, ck = cell / ((int64_t)n * n);
      const int64_t I = P * ci + a, J = P * cj + e0, K = P * ck + e1;
      const int64_t g = I + N1g * (J + N1g * K);
      const bool bnd = bc && (I == 0 || J == 0 || K == 0 || I == N1g - 1 || J == N1g - 1 || K == N1g - 1);
      val = bnd ? ~(int)g : (int)g;
    }
    idx[L] = val;
  }
}

// ---------------------------------------------------------------- geometry precompute (FP64)
// geo[blk][t][m][lane][2]: for lane = lc*T + (r + N1*s), quadrature point (r, s, t) of cell
// blk*CPB+lc; pairs m = (G00,G01), (G02,G11), (G12,G22).
template <int P>
struct QuadRule {
  double z[P + 1];
  double w[P + 1];
};

template <int P>
QuadRule<P> make_rule() {
  QuadRule<P> q;
  const Tables1D& t = tables(P);
  for (int k = 0; k <= P; ++k) {
    q.z[k] = t.zeta[k];
    q.w[k] = t.omega[k];
  }
  return q;
}

__device__ __forceinline__ void merged_tensor(const QGeo& g, double wa, double (&G)[6]) {
  const double f = wa * g.detJ;
  double K[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      K[i][j] = g.Jinv[i][0] * g.Jinv[j][0] + g.Jinv[i][1] * g.Jinv[j][1] + g.Jinv[i][2] * g.Jinv[j][2];
  G[0] = f * K[0][0];
  G[1] = f * K[0][1];
  G[2] = f * K[0][2];
  G[3] = f * K[1][1];
  G[4] = f * K[1][2];
  G[5] = f * K[2][2];
}

template <int P, typename Real>
__global__ __launch_bounds__(kBlock) void geometry_kernel(Real* __restrict__ geo, int64_t n_cells, int64_t n_blocks,
                                                          int n, double amp, double alpha, QuadRule<P> qr) {
  using C = Cell<P>;
  const int64_t total = n_blocks * C::N1 * C::NT;
  for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < total; L += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = L / (C::N1 * C::NT);
    const int rem = (int)(L - blk * (C::N1 * C::NT));
    const int t = rem / C::NT;
    const int lane = rem - t * C::NT;
    const int lc = lane / C::T;
    const int e = lane - lc * C::T;
    const int r = e % C::N1, s = e / C::N1;
    const int64_t cell = blk * C::CPB + lc;
    double G[6] = {0, 0, 0, 0, 0, 0};
    if (cell < n_cells) {
      QGeo g;
      qpoint_geometry(n, amp, cell, qr.z[r], qr.z[s], qr.z[t], g);
      merged_tensor(g, qr.w[r] * qr.w[s] * qr.w[t] * coefficient(alpha, g.x), G);
    }
    Real2<Real>* out = reinterpret_cast<Real2<Real>*>(geo) + (blk * C::N1 + t) * 3 * C::NT + lane;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      Real2<Real> v;
      v.x = (Real)G[2 * m];
      v.y = (Real)G[2 * m + 1];
      out[m * C::NT] = v;
    }
  }
}

template <int P, typename Real>
__global__ __launch_bounds__(kBlock) void geometry_export_kernel(const Real* __restrict__ geo, double* __restrict__ out,
                                                                 int64_t n_cells) {
  using C = Cell<P>;
  const int64_t total = n_cells * C::NQ;
  for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < total; L += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = L / C::NQ;
    const int q = (int)(L - cell * C::NQ);
    const int t = q / C::T, e = q - t * C::T;
    const int64_t blk = cell / C::CPB;
    const int lc = (int)(cell - blk * C::CPB);
    const Real2<Real>* in = reinterpret_cast<const Real2<Real>*>(geo) + (blk * C::N1 + t) * 3 * C::NT + lc * C::T + e;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      Real2<Real> v = in[m * C::NT];
      out[L * 6 + 2 * m] = (double)v.x;
      out[L * 6 + 2 * m + 1] = (double)v.y;
    }
  }
}

// ---------------------------------------------------------------- operator application
template <int P, typename Real>
__global__ __launch_bounds__(kBlock) void vmult_kernel(const int* __restrict__ idx, const Real* __restrict__ geo,
                                                       const Real* __restrict__ src, Real* __restrict__ dst,
                                                       int64_t n_cells, int n1d, Shape<P, Real> sh) {
  using C = Cell<P>;
  constexpr int N1 = C::N1, T = C::T, NQ = C::NQ, CPB = C::CPB, NT = C::NT;
  constexpr bool kPrefetch = (P <= 5);
  __shared__ Real lds[CPB * 3 * NQ];

  const int tid = threadIdx.x;
  const int lc = tid / T;
  const int e = tid - lc * T;
  const int e0 = e % N1, e1 = e / N1;
  const int64_t blk = blockIdx.x;
  const bool lane_ok = lc < CPB;
  const bool active = lane_ok && (blk * CPB + lc) < n_cells;
  const int lane = lane_ok ? lc * T + e : 0;
  Real* L0 = lds + (lane_ok ? lc : 0) * 3 * NQ;
  Real* L1 = L0 + NQ;
  Real* L2 = L1 + NQ;

  // quadrature-point tensor of this lane's z-pencil (points (e0, e1, t))
  const Real2<Real>* gp = reinterpret_cast<const Real2<Real>*>(geo) + blk * (int64_t)(N1 * 3 * NT) + lane;
  Real2<Real> g[kPrefetch ? N1 : 1][3];
#pragma unroll
  for (int t = 0; t < (kPrefetch ? N1 : 1); ++t)
#pragma unroll
    for (int m = 0; m < 3; ++m) g[t][m] = (kPrefetch && active) ? __builtin_nontemporal_load(gp + (t * 3 + m) * NT)
                                                                 : Real2<Real>{0, 0};

  // gather the x-pencil (a, e0, e1); Dirichlet nodes enter as zero
  int gi[N1];
  Real u[N1];
  const int* ip = idx + blk * (int64_t)(N1 * NT) + lane;
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    gi[a] = active ? ip[a * NT] : 0;
  }
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    Real v = 0;
    if (active && gi[a] >= 0) v = src[gi[a]];
    u[a] = v;
  }

  // x: values and x-derivatives at (q, e0, e1)
  {
    Real A[N1], B[N1];
    apply<N1>(sh.S, u, A);
    apply<N1>(sh.D, u, B);
    if (lane_ok) {
#pragma unroll
      for (int q = 0; q < N1; ++q) {
        L0[q + N1 * e] = A[q];
        L1[q + N1 * e] = B[q];
      }
    }
  }
  lds_barrier();
  // y: lane (r=e0, c=e1) holds y-pencils
  {
    Real a1[N1], b1[N1];
#pragma unroll
    for (int b = 0; b < N1; ++b) {
      a1[b] = L0[e0 + N1 * b + T * e1];
      b1[b] = L1[e0 + N1 * b + T * e1];
    }
    Real A2[N1], B2[N1], C2[N1];
    apply<N1>(sh.S, a1, A2);
    apply<N1>(sh.D, a1, C2);
    apply<N1>(sh.S, b1, B2);
    lds_barrier();
    if (lane_ok) {
#pragma unroll
      for (int s = 0; s < N1; ++s) {
        L0[e0 + N1 * s + T * e1] = A2[s];
        L1[e0 + N1 * s + T * e1] = B2[s];
        L2[e0 + N1 * s + T * e1] = C2[s];
      }
    }
  }
  lds_barrier();
  // z: lane (r=e0, s=e1) holds z-pencils; gradient, G, and the transposed z contraction
  {
    Real a2[N1], b2[N1], c2[N1];
#pragma unroll
    for (int c = 0; c < N1; ++c) {
      a2[c] = L0[e + T * c];
      b2[c] = L1[e + T * c];
      c2[c] = L2[e + T * c];
    }
    Real Az[N1], Bz[N1], Cz[N1];
#pragma unroll
    for (int c = 0; c < N1; ++c) Az[c] = Bz[c] = Cz[c] = 0;
#pragma unroll
    for (int t = 0; t < N1; ++t) {
      Real gx = 0, gy = 0, gz = 0;
#pragma unroll
      for (int c = 0; c < N1; ++c) {
        gx = __builtin_fma(sh.S[t * N1 + c], b2[c], gx);
        gy = __builtin_fma(sh.S[t * N1 + c], c2[c], gy);
        gz = __builtin_fma(sh.D[t * N1 + c], a2[c], gz);
      }
      Real2<Real> G0, G1, G2;
      if constexpr (kPrefetch) {
        G0 = g[t][0];
        G1 = g[t][1];
        G2 = g[t][2];
      } else {
        if (active) {
          G0 = __builtin_nontemporal_load(gp + (t * 3 + 0) * NT);
          G1 = __builtin_nontemporal_load(gp + (t * 3 + 1) * NT);
          G2 = __builtin_nontemporal_load(gp + (t * 3 + 2) * NT);
        } else {
          G0 = G1 = G2 = Real2<Real>{0, 0};
        }
      }
      // (G00 G01 G02; G01 G11 G12; G02 G12 G22) = (G0.x G0.y G1.x; . G1.y G2.x; . . G2.y)
      const Real vx = G0.x * gx + G0.y * gy + G1.x * gz;
      const Real vy = G0.y * gx + G1.y * gy + G2.x * gz;
      const Real vz = G1.x * gx + G2.x * gy + G2.y * gz;
#pragma unroll
      for (int c = 0; c < N1; ++c) {
        Bz[c] = __builtin_fma(sh.S[t * N1 + c], vx, Bz[c]);
        Cz[c] = __builtin_fma(sh.S[t * N1 + c], vy, Cz[c]);
        Az[c] = __builtin_fma(sh.D[t * N1 + c], vz, Az[c]);
      }
    }
    lds_barrier();
    if (lane_ok) {
#pragma unroll
      for (int c = 0; c < N1; ++c) {
        L0[e + T * c] = Az[c];
        L1[e + T * c] = Bz[c];
        L2[e + T * c] = Cz[c];
      }
    }
  }
  lds_barrier();
  // transposed y: lane (r=e0, c=e1)
  {
    Real az[N1], bz[N1], cz[N1];
#pragma unroll
    for (int s = 0; s < N1; ++s) {
      az[s] = L0[e0 + N1 * s + T * e1];
      bz[s] = L1[e0 + N1 * s + T * e1];
      cz[s] = L2[e0 + N1 * s + T * e1];
    }
    Real Ap[N1], Bp[N1];
    apply_t2<N1>(sh.S, az, sh.D, cz, Ap);
    apply_t<N1>(sh.S, bz, Bp);
    lds_barrier();
    if (lane_ok) {
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        L0[e0 + N1 * b + T * e1] = Ap[b];
        L1[e0 + N1 * b + T * e1] = Bp[b];
      }
    }
  }
  lds_barrier();
  // transposed x: lane (b=e0, c=e1) owns the DoFs it gathered
  {
    Real ap[N1], bp[N1], y[N1];
#pragma unroll
    for (int r = 0; r < N1; ++r) {
      ap[r] = L0[r + N1 * e];
      bp[r] = L1[r + N1 * e];
    }
    apply_t2<N1>(sh.S, ap, sh.D, bp, y);
    if (active) {
      // Dirichlet rows add src once: by the cell that holds the node at a non-lower face in
      // every direction (no lower-indexed neighbour shares it)
      const int64_t cell = blk * CPB + lc;
      const int64_t ci = cell % n1d, cj = (cell / n1d) % n1d, ck = cell / ((int64_t)n1d * n1d);
      const bool own_yz = (e0 > 0 || cj == 0) && (e1 > 0 || ck == 0);
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        if (gi[a] >= 0)
          atomic_add(dst + gi[a], y[a]);
        else if (own_yz && (a > 0 || ci == 0))
          atomic_add(dst + ~gi[a], src[~gi[a]]);
      }
    }
  }
}

// ---------------------------------------------------------------- diagonal
// diag_i = sum_K sum_q grad phi_i(q)^T G_q grad phi_i(q); one thread per (cell, i).
template <int P, typename Real>
__global__ __launch_bounds__(kBlock) void diagonal_kernel(const int* __restrict__ idx, const Real* __restrict__ geo,
                                                          Real* __restrict__ diag, int64_t n_cells, Shape<P, Real> sh) {
  using C = Cell<P>;
  constexpr int N1 = C::N1, T = C::T, NQ = C::NQ, CPB = C::CPB, NT = C::NT;
  const int64_t blk = blockIdx.x;
  for (int k = threadIdx.x; k < CPB * NQ; k += kBlock) {
    const int lc = k / NQ;
    const int i = k - lc * NQ;
    if (blk * CPB + lc >= n_cells) continue;
    const int a = i % N1, b = (i / N1) % N1, c = i / T;
    // idx layout: local DoF (a, b, c) is lane lc*T + (b + N1*c), row a
    const int g = idx[blk * (int64_t)(N1 * NT) + a * NT + lc * T + b + N1 * c];
    if (g < 0) {
      diag[~g] = (Real)1;
      continue;
    }
    const Real2<Real>* gp = reinterpret_cast<const Real2<Real>*>(geo) + blk * (int64_t)(N1 * 3 * NT) + lc * T;
    Real sum = 0;
    for (int t = 0; t < N1; ++t)
      for (int s = 0; s < N1; ++s)
        for (int r = 0; r < N1; ++r) {
          const Real bx = sh.D[r * N1 + a] * sh.S[s * N1 + b] * sh.S[t * N1 + c];
          const Real by = sh.S[r * N1 + a] * sh.D[s * N1 + b] * sh.S[t * N1 + c];
          const Real bz = sh.S[r * N1 + a] * sh.S[s * N1 + b] * sh.D[t * N1 + c];
          const Real2<Real> G0 = gp[(t * 3 + 0) * NT + r + N1 * s];
          const Real2<Real> G1 = gp[(t * 3 + 1) * NT + r + N1 * s];
          const Real2<Real> G2 = gp[(t * 3 + 2) * NT + r + N1 * s];
          sum += bx * (G0.x * bx + 2 * (G0.y * by + G1.x * bz)) + by * (G1.y * by + 2 * G2.x * bz) + G2.y * bz * bz;
        }
    atomic_add(diag + g, sum);
  }
}

// ---------------------------------------------------------------- right-hand side
// b_i += sum_q f(x_q) JxW_q phi_i(q) for u* = sin(pi x) sin(pi y) sin(pi z), f = -div(a grad u*).
template <int P>
__global__ __launch_bounds__(kBlock) void rhs_kernel(const int* __restrict__ idx, double* __restrict__ b, int64_t n_cells,
                                                     int n, double amp, double alpha, Shape<P, double> sh,
                                                     QuadRule<P> qr) {
  using C = Cell<P>;
  constexpr int N1 = C::N1, T = C::T, NQ = C::NQ, CPB = C::CPB, NT = C::NT;
  __shared__ double lds[CPB * NQ];
  const int tid = threadIdx.x;
  const int lc = tid / T;
  const int e = tid - lc * T;
  const int e0 = e % N1, e1 = e / N1;
  const int64_t blk = blockIdx.x;
  const bool lane_ok = lc < CPB;
  const int64_t cell = blk * CPB + lc;
  const bool active = lane_ok && cell < n_cells;
  double* L0 = lds + (lane_ok ? lc : 0) * NQ;
  // z-pencil of f*JxW at points (e0, e1, t), tested with S^T in z
  double fz[N1];
  for (int t = 0; t < N1; ++t) {
    double v = 0;
    if (active) {
      QGeo g;
      qpoint_geometry(n, amp, cell, qr.z[e0], qr.z[e1], qr.z[t], g);
      const double* x = g.x;
      double s1[3], c1[3], s2[3], c2[3];
      for (int d = 0; d < 3; ++d) {
        sincospi(x[d], &s1[d], &c1[d]);
        sincospi(2.0 * x[d], &s2[d], &c2[d]);
      }
      const double uu = s1[0] * s1[1] * s1[2];
      const double gu[3] = {M_PI * c1[0] * s1[1] * s1[2], M_PI * s1[0] * c1[1] * s1[2], M_PI * s1[0] * s1[1] * c1[2]};
      const double aa = 1.0 + alpha * s2[0] * s2[1] * s2[2];
      const double ga[3] = {2 * M_PI * alpha * c2[0] * s2[1] * s2[2], 2 * M_PI * alpha * s2[0] * c2[1] * s2[2],
                            2 * M_PI * alpha * s2[0] * s2[1] * c2[2]};
      const double f = -(ga[0] * gu[0] + ga[1] * gu[1] + ga[2] * gu[2]) + 3.0 * M_PI * M_PI * aa * uu;
      v = f * g.detJ * qr.w[e0] * qr.w[e1] * qr.w[t];
    }
    fz[t] = v;
  }
  double bz[N1];
  apply_t<N1>(sh.S, fz, bz);
  if (lane_ok)
    for (int c = 0; c < N1; ++c) L0[e + T * c] = bz[c];
  lds_barrier();
  double by[N1], tmp[N1];
  for (int s = 0; s < N1; ++s) tmp[s] = L0[e0 + N1 * s + T * e1];
  apply_t<N1>(sh.S, tmp, by);
  lds_barrier();
  if (lane_ok)
    for (int bb = 0; bb < N1; ++bb) L0[e0 + N1 * bb + T * e1] = by[bb];
  lds_barrier();
  double bx[N1];
  for (int r = 0; r < N1; ++r) tmp[r] = L0[r + N1 * e];
  apply_t<N1>(sh.S, tmp, bx);
  if (active) {
    const int* ip = idx + blk * (int64_t)(N1 * NT) + lc * T + e;
    for (int a = 0; a < N1; ++a) {
      const int g = ip[a * NT];
      if (g >= 0) atomic_add(b + g, bx[a]);
    }
  }
}

// ---------------------------------------------------------------- dense assembly (coarse levels)
// Free-free block of the assembled matrix: mat[f_i*ld + f_j] += A^K_ij, f = interior lattice index
// (I-1) + m*((J-1) + m*(K-1)), m = N1-2.  One thread per (cell, i, j).
template <int P>
__global__ __launch_bounds__(kBlock) void assemble_dense_kernel(const int* __restrict__ idx, const double* __restrict__ geo,
                                                                double* __restrict__ mat, int64_t ld, int64_t n_cells,
                                                                int64_t N1g, Shape<P, double> sh) {
  using C = Cell<P>;
  constexpr int N1 = C::N1, T = C::T, NQ = C::NQ, CPB = C::CPB, NT = C::NT;
  const int64_t total = n_cells * NQ * NQ;
  const int64_t m = N1g - 2;
  for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < total; L += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = L / (NQ * NQ);
    const int ij = (int)(L - cell * NQ * NQ);
    const int i = ij / NQ, j = ij - (ij / NQ) * NQ;
    const int64_t blk = cell / CPB;
    const int lc = (int)(cell - blk * CPB);
    const int ai = i % N1, bi = (i / N1) % N1, ci = i / T;
    const int aj = j % N1, bj = (j / N1) % N1, cj = j / T;
    const int gi = idx[blk * (int64_t)(N1 * NT) + ai * NT + lc * T + bi + N1 * ci];
    const int gj = idx[blk * (int64_t)(N1 * NT) + aj * NT + lc * T + bj + N1 * cj];
    if (gi < 0 || gj < 0) continue;
    const Real2<double>* gp = reinterpret_cast<const Real2<double>*>(geo) + blk * (int64_t)(N1 * 3 * NT) + lc * T;
    double sum = 0;
    for (int t = 0; t < N1; ++t)
      for (int s = 0; s < N1; ++s)
        for (int r = 0; r < N1; ++r) {
          const double ux = sh.D[r * N1 + ai] * sh.S[s * N1 + bi] * sh.S[t * N1 + ci];
          const double uy = sh.S[r * N1 + ai] * sh.D[s * N1 + bi] * sh.S[t * N1 + ci];
          const double uz = sh.S[r * N1 + ai] * sh.S[s * N1 + bi] * sh.D[t * N1 + ci];
          const double vx = sh.D[r * N1 + aj] * sh.S[s * N1 + bj] * sh.S[t * N1 + cj];
          const double vy = sh.S[r * N1 + aj] * sh.D[s * N1 + bj] * sh.S[t * N1 + cj];
          const double vz = sh.S[r * N1 + aj] * sh.S[s * N1 + bj] * sh.D[t * N1 + cj];
          const Real2<double> G0 = gp[(t * 3 + 0) * NT + r + N1 * s];
          const Real2<double> G1 = gp[(t * 3 + 1) * NT + r + N1 * s];
          const Real2<double> G2 = gp[(t * 3 + 2) * NT + r + N1 * s];
          sum += ux * (G0.x * vx + G0.y * vy + G1.x * vz) + uy * (G0.y * vx + G1.y * vy + G2.x * vz) +
                 uz * (G1.x * vx + G2.x * vy + G2.y * vz);
        }
    const int64_t Ii = gi % N1g, Ji = (gi / N1g) % N1g, Ki = gi / (N1g * N1g);
    const int64_t Ij = gj % N1g, Jj = (gj / N1g) % N1g, Kj = gj / (N1g * N1g);
    const int64_t fi = (Ii - 1) + m * ((Ji - 1) + m * (Ki - 1));
    const int64_t fj = (Ij - 1) + m * ((Jj - 1) + m * (Kj - 1));
    atomic_add(mat + fi * ld + fj, sum);
  }
}

int grid_for(int64_t work) {
  int64_t g = (work + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

template <int P>
hipError_t fill_index_p(const OpView& v, int* idx, hipStream_t st) {
  using C = Cell<P>;
  fill_index_kernel<P><<<grid_for(v.n_blocks * C::N1 * C::NT), kBlock, 0, st>>>(idx, v.n_cells, v.n_blocks, v.n, v.bc);
  return hipGetLastError();
}

template <int P>
hipError_t geometry_p(const OpView& v, int precision, void* geo, hipStream_t st) {
  using C = Cell<P>;
  const int g = grid_for(v.n_blocks * C::N1 * C::NT);
  if (precision == MFQ_FP64)
    geometry_kernel<P, double><<<g, kBlock, 0, st>>>((double*)geo, v.n_cells, v.n_blocks, v.n, v.amplitude, v.alpha,
                                                     make_rule<P>());
  else
    geometry_kernel<P, float><<<g, kBlock, 0, st>>>((float*)geo, v.n_cells, v.n_blocks, v.n, v.amplitude, v.alpha,
                                                    make_rule<P>());
  return hipGetLastError();
}

template <int P>
hipError_t geometry_export_p(const OpView& v, int precision, double* out, hipStream_t st) {
  using C = Cell<P>;
  const int g = grid_for(v.n_cells * C::NQ);
  if (precision == MFQ_FP64)
    geometry_export_kernel<P, double><<<g, kBlock, 0, st>>>((const double*)v.geo, out, v.n_cells);
  else
    geometry_export_kernel<P, float><<<g, kBlock, 0, st>>>((const float*)v.geo, out, v.n_cells);
  return hipGetLastError();
}

template <int P>
hipError_t vmult_p(const OpView& v, int precision, const void* src, void* dst, hipStream_t st) {
  if (v.n_blocks == 0) return hipSuccess;
  if (precision == MFQ_FP64)
    vmult_kernel<P, double><<<(unsigned)v.n_blocks, kBlock, 0, st>>>(v.idx, (const double*)v.geo, (const double*)src,
                                                                   (double*)dst, v.n_cells, v.n, make_shape<P, double>());
  else
    vmult_kernel<P, float><<<(unsigned)v.n_blocks, kBlock, 0, st>>>(v.idx, (const float*)v.geo, (const float*)src,
                                                                  (float*)dst, v.n_cells, v.n, make_shape<P, float>());
  return hipGetLastError();
}

template <int P>
hipError_t diagonal_p(const OpView& v, int precision, void* diag, hipStream_t st) {
  if (v.n_blocks == 0) return hipSuccess;
  if (precision == MFQ_FP64)
    diagonal_kernel<P, double><<<(unsigned)v.n_blocks, kBlock, 0, st>>>(v.idx, (const double*)v.geo, (double*)diag,
                                                                      v.n_cells, make_shape<P, double>());
  else
    diagonal_kernel<P, float><<<(unsigned)v.n_blocks, kBlock, 0, st>>>(v.idx, (const float*)v.geo, (float*)diag,
                                                                     v.n_cells, make_shape<P, float>());
  return hipGetLastError();
}

template <int P>
hipError_t rhs_p(const OpView& v, double* b, hipStream_t st) {
  if (v.n_blocks == 0) return hipSuccess;
  rhs_kernel<P><<<(unsigned)v.n_blocks, kBlock, 0, st>>>(v.idx, b, v.n_cells, v.n, v.amplitude, v.alpha,
                                                         make_shape<P, double>(), make_rule<P>());
  return hipGetLastError();
}

template <int P>
hipError_t assemble_dense_p(const OpView& v, double* mat, int64_t ld, hipStream_t st) {
  using C = Cell<P>;
  assemble_dense_kernel<P><<<grid_for(v.n_cells * C::NQ * C::NQ), kBlock, 0, st>>>(
      v.idx, (const double*)v.geo, mat, ld, v.n_cells, (int64_t)P * v.n + 1, make_shape<P, double>());
  return hipGetLastError();
}

#define MFQ_DISPATCH(p, fn, ...)                 \
  switch (p) {                                   \
    case 1: return fn<1>(__VA_ARGS__);           \
    case 2: return fn<2>(__VA_ARGS__);           \
    case 3: return fn<3>(__VA_ARGS__);           \
    case 4: return fn<4>(__VA_ARGS__);           \
    case 5: return fn<5>(__VA_ARGS__);           \
    case 6: return fn<6>(__VA_ARGS__);           \
    case 7: return fn<7>(__VA_ARGS__);           \
    case 8: return fn<8>(__VA_ARGS__);           \
    default: return hipErrorInvalidValue;        \
  }

}  // namespace

hipError_t launch_fill_index(const OpView& v, int* idx, hipStream_t st) { MFQ_DISPATCH(v.p, fill_index_p, v, idx, st); }

hipError_t launch_geometry(const OpView& v, int precision, void* geo, hipStream_t st) {
  MFQ_DISPATCH(v.p, geometry_p, v, precision, geo, st);
}

hipError_t launch_geometry_export(const OpView& v, int precision, double* out, hipStream_t st) {
  MFQ_DISPATCH(v.p, geometry_export_p, v, precision, out, st);
}

hipError_t launch_vmult_cells(const OpView& v, int precision, const void* src, void* dst, hipStream_t st) {
  MFQ_DISPATCH(v.p, vmult_p, v, precision, src, dst, st);
}

hipError_t launch_diagonal_cells(const OpView& v, int precision, void* diag, hipStream_t st) {
  MFQ_DISPATCH(v.p, diagonal_p, v, precision, diag, st);
}

hipError_t launch_rhs_cells(const OpView& v, double* b, hipStream_t st) { MFQ_DISPATCH(v.p, rhs_p, v, b, st); }

hipError_t launch_assemble_dense(const OpView& v, double* mat, int64_t ld, hipStream_t st) {
  MFQ_DISPATCH(v.p, assemble_dense_p, v, mat, ld, st);
}

}  // namespace mfq
