// Symmetric interior penalty DG Laplacian, matrix-free, on the affine n^3 mesh (the
// discretisation of the paper's multigrid experiment, Sec. 6.1).  Per cell the discontinuous
// Q_p basis on the GLL nodes; DoF (a,b,c) of cell K at K (p+1)^3 + a + (p+1) b + (p+1)^2 c.
//
//   a(u,v) = sum_K int_K grad u . grad v
//          + sum_F int_F ( -{d_n u}[v] - {d_n v}[u] + sigma [u][v] ),   sigma = 2 (p+1)^2 / h,
//
// interior faces with n from the lower cell L to the upper cell R, [u] = u_L - u_R, {w} the mean;
// boundary faces with the outside values zero and the inside value instead of the mean
// (homogeneous Dirichlet data imposed weakly).
//
// Cell term: one lane per 1D pencil of a cell, the sum factorisation of the continuous operator
// (even-odd forms of the 1D tables) with the quadrature tensor h w_r w_s w_t I of the affine cube; a cell's DoFs are contiguous, so
// loads and stores are plain coalesced reads and writes (no lattice, no colours).
// Face terms: one launch per normal direction d and parity of the face position along d (faces of
// one parity touch disjoint cells, so their adds need no atomics), one lane per tangential node
// of a face.  The lane reads the normal lines of both cells (the trace is the end node on the GLL
// nodes, the normal derivative a dot product with l'_a at the end point), forms the jump and the
// mean normal derivative, interpolates both to the face Gauss points through LDS (two 1D passes),
// applies weight and penalty there, interpolates back and adds the value part to the face node and
// the derivative part along the whole normal line of each cell.
#include "kernels_common.hpp"

namespace mfq {
namespace {

template <int P>
struct DgTables {
  double S[(P + 1) * (P + 1)];  // [q*(P+1)+a]: l_a(zeta_q)
  double D[(P + 1) * (P + 1)];  // l_a'(zeta_q)
  double w[P + 1];              // Gauss weights on [0,1]
  double d0[P + 1];             // l_a'(0)
  double d1[P + 1];             // l_a'(1)
};

template <int P>
DgTables<P> make_dg_tables() {
  DgTables<P> t{};
  const Tables1D& tb = tables(P);
  for (int k = 0; k < (P + 1) * (P + 1); ++k) {
    t.S[k] = tb.S[k];
    t.D[k] = tb.D[k];
  }
  for (int a = 0; a <= P; ++a) {
    t.w[a] = tb.omega[a];
    t.d0[a] = lagrange_derivative(tb.xi, a, 0.0);
    t.d1[a] = lagrange_derivative(tb.xi, a, 1.0);
  }
  return t;
}

template <int P>
struct DgWeights {
  double w[P + 1];  // Gauss weights on [0,1]
};

template <int P>
struct DgCell {
  static constexpr int N1 = P + 1;
  static constexpr int T = N1 * N1;
  static constexpr int NQ = N1 * T;
  static constexpr int CPW = 256 / T > 0 ? 256 / T : 1;  // cells (or faces) per workgroup
  static constexpr int THREADS = CPW * T;
};

template <int P>
__global__ __launch_bounds__(DgCell<P>::THREADS) void dg_cell_kernel(const double* __restrict__ src,
                                                                     double* __restrict__ dst, int64_t n_cells,
                                                                     double h, ShapeEO<P, double> sh,
                                                                     DgWeights<P> tb) {
  using C = DgCell<P>;
  constexpr int N1 = C::N1, T = C::T, NQ = C::NQ, CPW = C::CPW;
  __shared__ double lds[3 * CPW * NQ];
  const int tid = threadIdx.x;
  const int lc = tid / T, e = tid - lc * T;
  const int e0 = e % N1, e1 = e / N1;
  const int64_t cell = (int64_t)blockIdx.x * CPW + lc;
  const bool live = cell < n_cells;
  const int64_t base = (live ? cell : 0) * NQ;
  double* L0 = lds + lc * NQ;
  double* L1 = L0 + CPW * NQ;
  double* L2 = L1 + CPW * NQ;
  {  // x: values and x-derivatives at (q, e0, e1)
    double u[N1], A[N1], B[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) u[a] = live ? src[base + a + N1 * e] : 0.0;
    eo_apply<N1, 1, false>(sh.S, u, A);
    eo_apply<N1, -1, false>(sh.D, u, B);
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      L0[q + N1 * e] = A[q];
      L1[q + N1 * e] = B[q];
    }
  }
  __syncthreads();
  {  // y: lane (r = e0, c = e1)
    double a1[N1], b1[N1], A2[N1], B2[N1], C2[N1];
#pragma unroll
    for (int b = 0; b < N1; ++b) {
      a1[b] = L0[e0 + N1 * b + T * e1];
      b1[b] = L1[e0 + N1 * b + T * e1];
    }
    eo_apply<N1, 1, false>(sh.S, a1, A2);
    eo_apply<N1, -1, false>(sh.D, a1, C2);
    eo_apply<N1, 1, false>(sh.S, b1, B2);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < N1; ++s) {
      L0[e0 + N1 * s + T * e1] = A2[s];
      L1[e0 + N1 * s + T * e1] = B2[s];
      L2[e0 + N1 * s + T * e1] = C2[s];
    }
  }
  __syncthreads();
  {  // z: lane (r = e0, s = e1): gradient, weight, transposed z contraction
    double a2[N1], b2[N1], c2[N1], gx[N1], gy[N1], gz[N1];
#pragma unroll
    for (int c = 0; c < N1; ++c) {
      a2[c] = L0[e + T * c];
      b2[c] = L1[e + T * c];
      c2[c] = L2[e + T * c];
    }
    eo_apply<N1, 1, false>(sh.S, b2, gx);
    eo_apply<N1, 1, false>(sh.S, c2, gy);
    eo_apply<N1, -1, false>(sh.D, a2, gz);
    double w0 = 0, w1 = 0;  // weights of this lane's (r, s), selected with compile-time indices
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      w0 = e0 == k ? tb.w[k] : w0;
      w1 = e1 == k ? tb.w[k] : w1;
    }
    const double wrs = h * w0 * w1;
#pragma unroll
    for (int t = 0; t < N1; ++t) {
      const double w = wrs * tb.w[t];
      gx[t] *= w;
      gy[t] *= w;
      gz[t] *= w;
    }
    double Az[N1], Bz[N1], Cz[N1];
    eo_apply<N1, -1, true>(sh.D, gz, Az);
    eo_apply<N1, 1, true>(sh.S, gx, Bz);
    eo_apply<N1, 1, true>(sh.S, gy, Cz);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < N1; ++c) {
      L0[e + T * c] = Az[c];
      L1[e + T * c] = Bz[c];
      L2[e + T * c] = Cz[c];
    }
  }
  __syncthreads();
  {  // transposed y: lane (r = e0, c = e1)
    double az[N1], bz[N1], cz[N1], Ap[N1], Bp[N1];
#pragma unroll
    for (int s = 0; s < N1; ++s) {
      az[s] = L0[e0 + N1 * s + T * e1];
      bz[s] = L1[e0 + N1 * s + T * e1];
      cz[s] = L2[e0 + N1 * s + T * e1];
    }
    eo_apply_t2<N1>(sh.S, az, sh.D, cz, Ap);
    eo_apply<N1, 1, true>(sh.S, bz, Bp);
    __syncthreads();
#pragma unroll
    for (int b = 0; b < N1; ++b) {
      L0[e0 + N1 * b + T * e1] = Ap[b];
      L1[e0 + N1 * b + T * e1] = Bp[b];
    }
  }
  __syncthreads();
  {  // transposed x: lane (b = e0, c = e1) writes its x-pencil of the cell result
    double ap[N1], bp[N1], y[N1];
#pragma unroll
    for (int r = 0; r < N1; ++r) {
      ap[r] = L0[r + N1 * e];
      bp[r] = L1[r + N1 * e];
    }
    eo_apply_t2<N1>(sh.S, ap, sh.D, bp, y);
    if (live)
#pragma unroll
      for (int a = 0; a < N1; ++a) dst[base + a + N1 * e] = y[a];
  }
}

// local index of node a_d along the normal direction d at tangential node (a1, a2)
template <int N1>
__device__ __forceinline__ int face_local(int d, int ad, int a1, int a2) {
  return d == 0 ? ad + N1 * a1 + N1 * N1 * a2 : d == 1 ? a1 + N1 * ad + N1 * N1 * a2 : a1 + N1 * a2 + N1 * N1 * ad;
}

template <int P>
__global__ __launch_bounds__(DgCell<P>::THREADS) void dg_face_kernel(const double* __restrict__ src,
                                                                     double* __restrict__ dst, int n, int d, int parity,
                                                                     int64_t n_faces, double h, double sigma,
                                                                     DgTables<P> tb) {
  using C = DgCell<P>;
  constexpr int N1 = C::N1, T = C::T, NQ = C::NQ, FPW = C::CPW;
  __shared__ double lds[4 * FPW * T];
  const int tid = threadIdx.x;
  const int lf = tid / T, e = tid - lf * T;
  const int e0 = e % N1, e1 = e / N1;
  const int64_t face = (int64_t)blockIdx.x * FPW + lf;
  const bool live = face < n_faces;
  const int64_t fc = live ? face : 0;
  // face = (f index along d) * n^2 + tangential cell (ta + n tb), f = parity + 2 * (face / n^2)
  const int64_t nn = (int64_t)n * n;
  const int f = parity + 2 * (int)(fc / nn);
  const int ta = (int)(fc % nn) % n, tb2 = (int)(fc % nn) / n;
  int64_t cL = -1, cR = -1;
  {
    int64_t ijk[3];
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    ijk[t1] = ta;
    ijk[t2] = tb2;
    ijk[d] = f;
    if (f < n) cR = ijk[0] + n * (ijk[1] + (int64_t)n * ijk[2]);
    ijk[d] = f - 1;
    if (f > 0) cL = ijk[0] + n * (ijk[1] + (int64_t)n * ijk[2]);
  }
  const bool hasL = live && cL >= 0, hasR = live && cR >= 0;
  const double ih = 1.0 / h;
  double uL[N1], uR[N1];
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    uL[a] = hasL ? src[cL * NQ + face_local<N1>(d, a, e0, e1)] : 0.0;
    uR[a] = hasR ? src[cR * NQ + face_local<N1>(d, a, e0, e1)] : 0.0;
  }
  double dnL = 0, dnR = 0;
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    dnL = fmad(tb.d1[a], uL[a], dnL);
    dnR = fmad(tb.d0[a], uR[a], dnR);
  }
  dnL *= ih;
  dnR *= ih;
  const bool interior = hasL && hasR;
  const double jump = uL[N1 - 1] - uR[0];
  const double mean = interior ? 0.5 * (dnL + dnR) : dnL + dnR;  // one of them is zero on a boundary face
  const double dfac = interior ? 0.5 : 1.0;
  double* F0 = lds + lf * T;
  double* F1 = F0 + FPW * T;
  double* G0 = F1 + FPW * T;
  double* G1 = G0 + FPW * T;
  // nodes -> Gauss points, first tangential direction: lane (q1 = e0, a2 = e1)
  F0[e] = jump;
  F1[e] = mean;
  __syncthreads();
  {
    double sj = 0, sm = 0;
#pragma unroll
    for (int a1 = 0; a1 < N1; ++a1) {
      sj = fmad(tb.S[e0 * N1 + a1], F0[a1 + N1 * e1], sj);
      sm = fmad(tb.S[e0 * N1 + a1], F1[a1 + N1 * e1], sm);
    }
    G0[e] = sj;
    G1[e] = sm;
  }
  __syncthreads();
  // second tangential direction: lane (q1 = e0, q2 = e1) at its Gauss point
  double jq = 0, mq = 0;
#pragma unroll
  for (int a2 = 0; a2 < N1; ++a2) {
    jq = fmad(tb.S[e1 * N1 + a2], G0[e0 + N1 * a2], jq);
    mq = fmad(tb.S[e1 * N1 + a2], G1[e0 + N1 * a2], mq);
  }
  double w0 = 0, w1 = 0;
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    w0 = e0 == k ? tb.w[k] : w0;
    w1 = e1 == k ? tb.w[k] : w1;
  }
  const double W = h * h * w0 * w1;
  const double cval = W * (sigma * jq - mq);
  const double cder = -dfac * W * jq;
  __syncthreads();
  // Gauss points -> nodes (transposed), second direction first: lane (q1 = e0, a2 = e1)
  F0[e] = cval;
  F1[e] = cder;
  __syncthreads();
  {
    double sv = 0, sd = 0;
#pragma unroll
    for (int q2 = 0; q2 < N1; ++q2) {
      sv = fmad(tb.S[q2 * N1 + e1], F0[e0 + N1 * q2], sv);
      sd = fmad(tb.S[q2 * N1 + e1], F1[e0 + N1 * q2], sd);
    }
    G0[e] = sv;
    G1[e] = sd;
  }
  __syncthreads();
  // first direction: lane (a1 = e0, a2 = e1) gets its face node's coefficients
  double V = 0, Dd = 0;
#pragma unroll
  for (int q1 = 0; q1 < N1; ++q1) {
    V = fmad(tb.S[q1 * N1 + e0], G0[q1 + N1 * e1], V);
    Dd = fmad(tb.S[q1 * N1 + e0], G1[q1 + N1 * e1], Dd);
  }
  Dd *= ih;
  // add: value part on the face node, derivative part along the normal line
  if (hasL)
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      double* p = dst + cL * NQ + face_local<N1>(d, a, e0, e1);
      *p += (a == N1 - 1 ? V : 0.0) + Dd * tb.d1[a];
    }
  if (hasR)
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      double* p = dst + cR * NQ + face_local<N1>(d, a, e0, e1);
      *p += (a == 0 ? -V : 0.0) + Dd * tb.d0[a];
    }
}

template <int P>
hipError_t dg_vmult_p(int n, const double* src, double* dst, hipStream_t st) {
  using C = DgCell<P>;
  static const DgTables<P> tb = make_dg_tables<P>();
  static const ShapeEO<P, double> sh = make_shape_eo<P, double>();
  DgWeights<P> wt;
  for (int a = 0; a <= P; ++a) wt.w[a] = tb.w[a];
  const double h = 1.0 / n;
  const double sigma = 2.0 * (P + 1) * (P + 1) / h;
  const int64_t cells = (int64_t)n * n * n;
  const int64_t g = (cells + C::CPW - 1) / C::CPW;
  if (g > 0x7fffffff) return hipErrorInvalidValue;
  dg_cell_kernel<P><<<(unsigned)g, C::THREADS, 0, st>>>(src, dst, cells, h, sh, wt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int d = 0; d < 3; ++d)
    for (int parity = 0; parity < 2; ++parity) {
      if (parity > n) continue;
      const int64_t nf = (int64_t)((n - parity) / 2 + 1) * n * n;
      const int64_t gf = (nf + C::CPW - 1) / C::CPW;
      dg_face_kernel<P><<<(unsigned)gf, C::THREADS, 0, st>>>(src, dst, n, d, parity, nf, h, sigma, tb);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

}  // namespace

hipError_t launch_dg_vmult(int p, int n, const double* src, double* dst, hipStream_t st) {
  switch (p) {
    case 1: return dg_vmult_p<1>(n, src, dst, st);
    case 2: return dg_vmult_p<2>(n, src, dst, st);
    case 3: return dg_vmult_p<3>(n, src, dst, st);
    case 4: return dg_vmult_p<4>(n, src, dst, st);
    case 5: return dg_vmult_p<5>(n, src, dst, st);
    case 6: return dg_vmult_p<6>(n, src, dst, st);
    case 7: return dg_vmult_p<7>(n, src, dst, st);
    case 8: return dg_vmult_p<8>(n, src, dst, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mfq
