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
// One kernel computes the whole operator per cell in tensor-product form (dg_kron_kernel, below):
// CPW consecutive cells of an x-row per workgroup, one lane per 1D line of a cell; each cell's
// result is written once.
#include "kernels_common.hpp"

// Lanes per workgroup that the cells fill (one lane per 1D line): 128 up to degree 4 (5 cells of
// 25 lanes at p = 4), 256 above (at p >= 6 a 128-lane workgroup would hold a single cell).
#ifndef MFQ_DG_LANES
#define MFQ_DG_LANES(P) ((P) <= 4 ? 128 : 256)
#endif

namespace mfq {
namespace {

template <int P>
struct DgCell {
  static constexpr int N1 = P + 1;
  static constexpr int T = N1 * N1;
  static constexpr int NQ = N1 * T;
  static constexpr int CPW = MFQ_DG_LANES(P) / T > 0 ? MFQ_DG_LANES(P) / T : 1;  // cells per workgroup
  static constexpr int THREADS = CPW * T;
};

// local index of node a_d along the normal direction d at tangential node (a1, a2)
template <int N1>
__device__ __forceinline__ int face_local(int d, int ad, int a1, int a2) {
  return d == 0 ? ad + N1 * a1 + N1 * N1 * a2 : d == 1 ? a1 + N1 * ad + N1 * N1 * a2 : a1 + N1 * a2 + N1 * N1 * ad;
}

// What the kernel does with its result v = (A src)_i before storing (one pass over the vectors,
// fused with the operator):
//   kStore:    dst = v
//   kChebStep: r -= v; dnew = c1 src + c2 dinv r; x += dnew   (a Chebyshev step, src = d; dnew
//              must be another buffer since other cells still read src)
//   kResidual: r = b - v
enum DgEpilogueMode { kStore = 0, kChebStep = 1, kResidual = 2 };
template <typename Real>
struct DgEpilogue {
  int mode;
  Real* dst;
  const Real* b;
  const Real* dinv;
  Real* x;
  Real* r;
  Real* dnew;
  Real c1, c2;
};

// Tensor-product form of the whole operator.  On the affine cube mesh every term of a(u, v)
// factorises over the three directions: with the Gauss rule's 1D mass matrix M = S^T diag(w) S
// and stiffness matrix K = D^T diag(w) D on the reference interval,
//
//   A u = sum_d (M x M)_{tangential to d} w_d,   w_d = h K u + (face terms of the faces normal to d)
//
// along every line of the cell in direction d: the cell term of direction d is h (K x M x M)
// (h^3 from the cell measure, h^-2 from the two derivatives), and the terms of a face normal to d
// are h^2 (M x M) applied to sigma [u] - {d_n u} at the face layer and, from d_n v = l'_a / h, to
// -f h [u] times l'_a at the face end along the line (f = 1/2 on interior faces, 1 on boundary
// faces).  The trace of a line on a face is its GLL end node and its normal derivative a dot
// product with l'_a at the end point, so w_d needs only the cell's own line and the two
// neighbours' lines through the faces it touches.  Per cell one lane per 1D line forms w_d for the
// three directions, and the tangential mass matrices act in five 1D passes,
//
//   A u = M_y (M_z w_x + M_x w_z) + M_x M_z w_y,
//
// in place in two LDS arrays per cell (each pass reads and writes only its own lane's line, with a
// barrier between passes).  K and M are symmetric about their centre, so every 1D contraction
// uses the even-odd form: eight per line in all.
template <int P, typename Real>
struct DgKron {
  EvenOdd<P + 1, Real> K;  // sum_q w_q l_a'(zeta_q) l_b'(zeta_q)
  EvenOdd<P + 1, Real> M;  // sum_q w_q l_a(zeta_q) l_b(zeta_q)
  Real d0[P + 1];          // l_a'(0)
  Real d1[P + 1];          // l_a'(1)
};

template <int P, typename Real>
DgKron<P, Real> make_dg_kron() {
  constexpr int N1 = P + 1;
  const Tables1D& tb = tables(P);
  double K[N1 * N1], M[N1 * N1];
  for (int a = 0; a < N1; ++a)
    for (int b = 0; b < N1; ++b) {
      double k = 0, m = 0;
      for (int q = 0; q < N1; ++q) {
        k += tb.omega[q] * tb.D[q * N1 + a] * tb.D[q * N1 + b];
        m += tb.omega[q] * tb.S[q * N1 + a] * tb.S[q * N1 + b];
      }
      K[a * N1 + b] = k;
      M[a * N1 + b] = m;
    }
  DgKron<P, Real> t{};
  t.K = make_even_odd<N1, Real>(K);
  t.M = make_even_odd<N1, Real>(M);
  for (int a = 0; a < N1; ++a) {
    t.d0[a] = (Real)lagrange_derivative(tb.xi, a, 0.0);
    t.d1[a] = (Real)lagrange_derivative(tb.xi, a, 1.0);
  }
  return t;
}

// w = h K u + the face terms of one line's two faces, from the line u of the cell and the lines
// uLo, uHi of its neighbours below and above along the line (zero where absent)
template <int N1, typename Real, typename KT>
__device__ __forceinline__ void dg_line_terms(const Real (&u)[N1], const Real (&uLo)[N1], const Real (&uHi)[N1],
                                              bool hasLo, bool hasHi, Real h, Real ih, Real h2, Real sigma,
                                              const KT& kt, Real (&w)[N1]) {
  Real dK0 = 0, dK1 = 0, dLo = 0, dHi = 0;
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    dK0 = fmad(kt.d0[a], u[a], dK0);
    dK1 = fmad(kt.d1[a], u[a], dK1);
    dLo = fmad(kt.d1[a], uLo[a], dLo);
    dHi = fmad(kt.d0[a], uHi[a], dHi);
  }
  // jump and mean normal derivative on the lower face (this cell its upper side) and the upper
  // face; on a boundary face the outside is zero and the inside derivative replaces the mean
  const Real jLo = uLo[N1 - 1] - u[0], jHi = u[N1 - 1] - uHi[0];
  const Real mLo = hasLo ? (Real)0.5 * ih * (dLo + dK0) : ih * dK0;
  const Real mHi = hasHi ? (Real)0.5 * ih * (dK1 + dHi) : ih * dK1;
  const Real fLo = hasLo ? (Real)0.5 : (Real)1, fHi = hasHi ? (Real)0.5 : (Real)1;
  const Real VLo = h2 * (sigma * jLo - mLo), DLo = -fLo * h * jLo;
  const Real VHi = h2 * (sigma * jHi - mHi), DHi = -fHi * h * jHi;
  Real ku[N1];
  eo_apply<N1, 1, false>(kt.K, u, ku);
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    Real v = h * ku[a];
    if (a == 0) v -= VLo;
    if (a == N1 - 1) v += VHi;
    v = fmad(DLo, kt.d0[a], v);
    w[a] = fmad(DHi, kt.d1[a], v);
  }
}

// Waves per SIMD the tensor-product kernel asks for: 5 where that fits its registers without
// spilling, fewer at the high FP64 degrees
constexpr int dg_kron_waves(int p, bool fp64) { return !fp64 ? 5 : p <= 5 ? 5 : p <= 7 ? 4 : 1; }

template <int P, typename Real>
__global__ __launch_bounds__(DgCell<P>::THREADS) __attribute__((amdgpu_waves_per_eu(dg_kron_waves(P, sizeof(Real) == 8))))
void dg_kron_kernel(const Real* __restrict__ src, int n, int slab_planes, Real h, Real sigma, DgKron<P, Real> kt,
                    DgEpilogue<Real> ep) {
  using C = DgCell<P>;
  constexpr int N1 = C::N1, T = C::T, NQ = C::NQ, CPW = C::CPW;
  __shared__ Real lds[2 * CPW * NQ];
  const int tid = threadIdx.x;
  const int lc = tid / T, e = tid - lc * T;
  const int e0 = e % N1, e1 = e / N1;
  // A workgroup takes CPW consecutive cells of one x-row of cells.  Its place in the launch order
  // (XCD-contiguous: block b runs on XCD b % 8 and takes the (b / 8)-th item of that XCD's
  // contiguous share) walks slabs of slab_planes z-planes (n/8 rounded up: about one slab per
  // XCD): within a slab z fastest, then the row segments along x, then y.  The z- and
  // x-neighbours' lines are then read a few workgroups after they were fetched, the
  // y-neighbours' one slab-row later, from the XCD's L2; only the lines across a slab boundary
  // come from HBM again.
  const int64_t G = gridDim.x, q8 = G / 8, r8 = G % 8;
  const int64_t x8 = blockIdx.x % 8, i8 = blockIdx.x / 8;
  const int64_t blk = (x8 < r8 ? x8 * (q8 + 1) : r8 * (q8 + 1) + (x8 - r8) * q8) + i8;
  const int nxb = (n + CPW - 1) / CPW;                 // row segments per x-row
  const int64_t slab = (int64_t)slab_planes * n * nxb;  // workgroups per full slab
  const int kb = (int)(blk / slab);
  const int64_t rs = blk - kb * slab;
  const int tz = min(slab_planes, n - kb * slab_planes);  // planes of this slab (the last may be thinner)
  const int jrow = (int)(rs / ((int64_t)nxb * tz));
  const int r2 = (int)(rs - (int64_t)jrow * nxb * tz);
  const int xb = r2 / tz;
  const int kz = kb * slab_planes + (r2 - xb * tz);
  const int i0 = xb * CPW;
  const int cnt = min(CPW, n - i0);                    // cells of this row segment
  const int64_t nn = (int64_t)n * n;
  const int64_t cell0 = i0 + (int64_t)n * jrow + nn * kz;
  const bool live = lc < cnt;
  const int64_t K = live ? cell0 + lc : cell0;
  const int64_t base = K * NQ;
  const int64_t ijk[3] = {i0 + (live ? lc : 0), jrow, kz};
  const Real ih = (Real)1 / h, h2 = h * h;
  // two arrays of this cell, node order (a + N1 b + T c)
  Real* W0 = lds + lc * NQ;
  Real* W1 = W0 + CPW * NQ;
  // The own cells through LDS: each lane loads its z-line (contiguous across lanes) into
  // registers and W1, and the x- and y-lines of the own cells, and of the x-neighbours inside the
  // row segment, are read back from W1.  The other neighbours' lines come from global memory (the
  // z-neighbours' z-lines contiguous across lanes).
  Real uz[N1];
#pragma unroll
  for (int c = 0; c < N1; ++c) uz[c] = live ? src[base + e + T * c] : (Real)0;
#pragma unroll
  for (int c = 0; c < N1; ++c) W1[e + T * c] = uz[c];
  __syncthreads();
  Real w[N1], wy[N1], wz[N1];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t stride = d == 0 ? 1 : d == 1 ? n : nn;
    const bool hasLo = live && ijk[d] > 0, hasHi = live && ijk[d] < n - 1;
    Real u[N1], uLo[N1], uHi[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int loc = face_local<N1>(d, a, e0, e1);
      u[a] = d == 2 ? uz[a] : W1[loc];
      if (d == 0) {
        uLo[a] = lc > 0 ? W1[loc - NQ] : hasLo ? src[base - NQ + loc] : (Real)0;
        uHi[a] = lc + 1 < cnt ? W1[loc + NQ] : hasHi ? src[base + NQ + loc] : (Real)0;
      } else {
        uLo[a] = hasLo ? src[base - stride * NQ + loc] : (Real)0;
        uHi[a] = hasHi ? src[base + stride * NQ + loc] : (Real)0;
      }
    }
    dg_line_terms<N1>(u, uLo, uHi, hasLo, hasHi, h, ih, h2, sigma, kt, w);
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      if (d == 0) W0[a + N1 * e] = w[a];  // nobody reads W0 before the passes
      if (d == 1) wy[a] = w[a];
      if (d == 2) wz[a] = w[a];
    }
  }
  // A u = M_y (M_z w_x + M_x w_z) + M_x M_z w_y: w_y replaces the copy of the source once every
  // lane has read it; w_z enters after M_z w_y has been read out of its array
  __syncthreads();
#pragma unroll
  for (int b = 0; b < N1; ++b) W1[e0 + N1 * b + T * e1] = wy[b];
  __syncthreads();
  {  // z-lines, lane (a, b): W0 <- M_z w_x, W1 <- M_z w_y
    Real v[N1], r[N1];
#pragma unroll
    for (int c = 0; c < N1; ++c) v[c] = W0[e + T * c];
    eo_apply<N1, 1, false>(kt.M, v, r);
#pragma unroll
    for (int c = 0; c < N1; ++c) W0[e + T * c] = r[c];
#pragma unroll
    for (int c = 0; c < N1; ++c) v[c] = W1[e + T * c];
    eo_apply<N1, 1, false>(kt.M, v, r);
#pragma unroll
    for (int c = 0; c < N1; ++c) W1[e + T * c] = r[c];
  }
  __syncthreads();
  Real r1[N1];  // x-lines, lane (b, c): M_x M_z w_y
  {
    Real v[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) v[a] = W1[a + N1 * e];
    eo_apply<N1, 1, false>(kt.M, v, r1);
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < N1; ++c) W1[e + T * c] = wz[c];  // z-line (a, b) of w_z
  __syncthreads();
  {  // x-lines, lane (b, c): W0 <- M_x w_z + W0
    Real v[N1], r[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) v[a] = W1[a + N1 * e];
    eo_apply<N1, 1, false>(kt.M, v, r);
#pragma unroll
    for (int a = 0; a < N1; ++a) W0[a + N1 * e] += r[a];
  }
  __syncthreads();
  {  // y-lines, lane (a, c): W0 <- M_y W0
    Real v[N1], r[N1];
#pragma unroll
    for (int b = 0; b < N1; ++b) v[b] = W0[e0 + N1 * b + T * e1];
    eo_apply<N1, 1, false>(kt.M, v, r);
#pragma unroll
    for (int b = 0; b < N1; ++b) W0[e0 + N1 * b + T * e1] = r[b];
  }
  __syncthreads();
  Real y[N1];  // x-line (b, c) of the result
#pragma unroll
  for (int a = 0; a < N1; ++a) y[a] = W0[a + N1 * e] + r1[a];
  if (ep.mode == kStore) {
    if (!live) return;
    const int64_t g0i = base + N1 * e;
#pragma unroll
    for (int a = 0; a < N1; ++a) ep.dst[g0i + a] = y[a];
    return;
  }
  // smoother step or residual: the result goes through LDS in node order (this lane's own x-line
  // of W0, which no other lane reads) and a coalesced pass covers the workgroup's cells
#pragma unroll
  for (int a = 0; a < N1; ++a) W0[a + N1 * e] = y[a];
  __syncthreads();
  const int64_t limit = (int64_t)cnt * NQ;
  const int64_t gb = cell0 * NQ;
  if (ep.mode == kChebStep) {
    for (int i = tid; i < CPW * NQ; i += C::THREADS)
      if (i < limit) {
        const int64_t gi = gb + i;
        const Real rv = ep.r[gi] - lds[i];
        const Real dv = ep.c1 * src[gi] + ep.c2 * ep.dinv[gi] * rv;
        ep.r[gi] = rv;
        ep.dnew[gi] = dv;
        ep.x[gi] += dv;
      }
  } else {
    for (int i = tid; i < CPW * NQ; i += C::THREADS)
      if (i < limit) ep.r[gb + i] = ep.b[gb + i] - lds[i];
  }
}

struct DgApplyArgs {
  int mode;
  void* dst;
  const void* b;
  const void* dinv;
  void* x;
  void* r;
  void* dnew;
  double c1, c2;
};

template <int P, typename Real>
hipError_t dg_apply_pr(int n, const Real* src, const DgEpilogue<Real>& ep, hipStream_t st) {
  using C = DgCell<P>;
  static const DgKron<P, Real> kt = make_dg_kron<P, Real>();
  const Real h = (Real)(1.0 / n);
  const Real sigma = (Real)(2.0 * (P + 1) * (P + 1) * n);
  const int64_t g = (int64_t)((n + C::CPW - 1) / C::CPW) * n * n;  // row segments of CPW cells
  if (g > 0x7fffffff) return hipErrorInvalidValue;
  const int slab_planes = (n + 7) / 8;
  dg_kron_kernel<P, Real><<<(unsigned)g, C::THREADS, 0, st>>>(src, n, slab_planes, h, sigma, kt, ep);
  return hipGetLastError();
}

template <int P>
hipError_t dg_apply_p(int n, int precision, const void* src, const DgApplyArgs& a, hipStream_t st) {
  if (precision == MFQ_FP64) {
    const DgEpilogue<double> ep{a.mode, (double*)a.dst, (const double*)a.b, (const double*)a.dinv, (double*)a.x,
                                (double*)a.r, (double*)a.dnew, a.c1, a.c2};
    return dg_apply_pr<P, double>(n, (const double*)src, ep, st);
  }
  const DgEpilogue<float> ep{a.mode, (float*)a.dst, (const float*)a.b, (const float*)a.dinv, (float*)a.x,
                             (float*)a.r, (float*)a.dnew, (float)a.c1, (float)a.c2};
  return dg_apply_pr<P, float>(n, (const float*)src, ep, st);
}

hipError_t dg_apply(int p, int n, int precision, const void* src, const DgApplyArgs& a, hipStream_t st) {
  switch (p) {
    case 1: return dg_apply_p<1>(n, precision, src, a, st);
    case 2: return dg_apply_p<2>(n, precision, src, a, st);
    case 3: return dg_apply_p<3>(n, precision, src, a, st);
    case 4: return dg_apply_p<4>(n, precision, src, a, st);
    case 5: return dg_apply_p<5>(n, precision, src, a, st);
    case 6: return dg_apply_p<6>(n, precision, src, a, st);
    case 7: return dg_apply_p<7>(n, precision, src, a, st);
    case 8: return dg_apply_p<8>(n, precision, src, a, st);
    default: return hipErrorInvalidValue;
  }
}

// Jacobi diagonal of the DG-SIPG matrix in closed form.  With m_a = sum_q w_q S_qa^2 and
// k_a = sum_q w_q D_qa^2 (1D Gauss sums), the cell part of DoF (a,b,c) is
// h (k_a m_b m_c + m_a k_b m_c + m_a m_b k_c); a face of normal d adds, at the cell's face-layer
// nodes only (the trace of every other basis function vanishes on the GLL end points),
// h^2 m_a1 m_a2 (sigma + c l'_end(end) / h) with c = -1 for the upper face and +1 for the lower one
// of an interior face (the mean halves the two cross terms), doubled on boundary faces.
struct DgDiag1D {
  double m[kMaxDegree + 1];
  double k[kMaxDegree + 1];
  double dp1;  // l_p'(1)
  double d00;  // l_0'(0)
};

template <typename Real>
__global__ __launch_bounds__(256) void dg_diag_kernel(Real* __restrict__ diag, int p, int n, DgDiag1D t) {
  const int N1 = p + 1;
  const int64_t nloc = (int64_t)N1 * N1 * N1;
  const int64_t N = (int64_t)n * n * n * nloc;
  const double h = 1.0 / n, sigma = 2.0 * N1 * N1 * n;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < N; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t K = g / nloc;
    const int i = (int)(g - K * nloc);
    const int ai[3] = {i % N1, (i / N1) % N1, i / (N1 * N1)};
    const int64_t ck[3] = {K % n, (K / n) % n, K / ((int64_t)n * n)};
    double v = h * (t.k[ai[0]] * t.m[ai[1]] * t.m[ai[2]] + t.m[ai[0]] * t.k[ai[1]] * t.m[ai[2]] +
                    t.m[ai[0]] * t.m[ai[1]] * t.k[ai[2]]);
    for (int d = 0; d < 3; ++d) {
      const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      const double mm = h * h * t.m[ai[t1]] * t.m[ai[t2]];
      if (ai[d] == 0) v += mm * (sigma + (ck[d] == 0 ? 2.0 : 1.0) * t.d00 / h);
      if (ai[d] == p) v += mm * (sigma - (ck[d] == n - 1 ? 2.0 : 1.0) * t.dp1 / h);
    }
    diag[g] = (Real)v;
  }
}

// Continuous Q_p (lattice of (pn+1)^3 nodes, Dirichlet nodes zero) <-> DG on the same mesh and
// nodes.  Prolongation copies each lattice node into every cell that holds it; restriction (its
// transpose) sums, per free lattice node, the entries of the cells that hold it in a fixed order.
template <typename Real>
__global__ __launch_bounds__(256) void dg_from_cg_kernel(const Real* __restrict__ cg, Real* __restrict__ dg, int p,
                                                         int n) {
  const int N1 = p + 1;
  const int64_t nloc = (int64_t)N1 * N1 * N1, L1 = (int64_t)p * n + 1;
  const int64_t N = (int64_t)n * n * n * nloc;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < N; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t K = g / nloc;
    const int i = (int)(g - K * nloc);
    const int64_t I = p * (K % n) + i % N1, J = p * ((K / n) % n) + (i / N1) % N1,
                  Kz = p * (K / ((int64_t)n * n)) + i / (N1 * N1);
    dg[g] = cg[I + L1 * (J + L1 * Kz)];
  }
}

template <typename Real>
__global__ __launch_bounds__(256) void cg_from_dg_kernel(const Real* __restrict__ dg, Real* __restrict__ cg, int p,
                                                         int n) {
  const int N1 = p + 1;
  const int64_t nloc = (int64_t)N1 * N1 * N1, L1 = (int64_t)p * n + 1, pn = L1 - 1;
  const int64_t M = L1 * L1 * L1;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < M; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t X[3] = {g % L1, (g / L1) % L1, g / (L1 * L1)};
    if (X[0] == 0 || X[0] == pn || X[1] == 0 || X[1] == pn || X[2] == 0 || X[2] == pn) {
      cg[g] = (Real)0;
      continue;
    }
    // per direction the cells holding the node: one, or two when it is a cell vertex
    int64_t c0[3], c1[3];
    int cnt[3];
    for (int d = 0; d < 3; ++d) {
      const int64_t c = X[d] / p;
      if (X[d] % p == 0) {
        c0[d] = c - 1;
        c1[d] = c;
        cnt[d] = 2;
      } else {
        c0[d] = c;
        cnt[d] = 1;
      }
    }
    Real s = 0;
    for (int kz = 0; kz < cnt[2]; ++kz)
      for (int ky = 0; ky < cnt[1]; ++ky)
        for (int kx = 0; kx < cnt[0]; ++kx) {
          const int64_t ci = kx ? c1[0] : c0[0], cj = ky ? c1[1] : c0[1], ck = kz ? c1[2] : c0[2];
          const int64_t K = ci + n * (cj + (int64_t)n * ck);
          const int li = (int)(X[0] - p * ci) + N1 * ((int)(X[1] - p * cj) + N1 * (int)(X[2] - p * ck));
          s += dg[K * nloc + li];
        }
    cg[g] = s;
  }
}

int dg_grid(int64_t work) {
  int64_t g = (work + 255) / 256;
  return (int)(g > 65536 ? 65536 : g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_dg_vmult(int p, int n, int precision, const void* src, void* dst, hipStream_t st) {
  DgApplyArgs a{};
  a.mode = kStore;
  a.dst = dst;
  return dg_apply(p, n, precision, src, a, st);
}

hipError_t launch_dg_cheb_step(int p, int n, int precision, const void* d, const void* dinv, void* x, void* r,
                               void* dnew, double c1, double c2, hipStream_t st) {
  DgApplyArgs a{};
  a.mode = kChebStep;
  a.dinv = dinv;
  a.x = x;
  a.r = r;
  a.dnew = dnew;
  a.c1 = c1;
  a.c2 = c2;
  return dg_apply(p, n, precision, d, a, st);
}

hipError_t launch_dg_residual(int p, int n, int precision, const void* b, const void* x, void* r, hipStream_t st) {
  DgApplyArgs a{};
  a.mode = kResidual;
  a.b = b;
  a.r = r;
  return dg_apply(p, n, precision, x, a, st);
}

hipError_t launch_dg_diagonal(int p, int n, int precision, void* diag, hipStream_t st) {
  const Tables1D& tb = tables(p);
  DgDiag1D t{};
  for (int a = 0; a <= p; ++a) {
    double m = 0, k = 0;
    for (int q = 0; q <= p; ++q) {
      m += tb.omega[q] * tb.S[q * (p + 1) + a] * tb.S[q * (p + 1) + a];
      k += tb.omega[q] * tb.D[q * (p + 1) + a] * tb.D[q * (p + 1) + a];
    }
    t.m[a] = m;
    t.k[a] = k;
  }
  t.dp1 = lagrange_derivative(tb.xi, p, 1.0);
  t.d00 = lagrange_derivative(tb.xi, 0, 0.0);
  const int64_t N = (int64_t)n * n * n * (p + 1) * (p + 1) * (p + 1);
  if (precision == MFQ_FP64)
    dg_diag_kernel<double><<<dg_grid(N), 256, 0, st>>>((double*)diag, p, n, t);
  else
    dg_diag_kernel<float><<<dg_grid(N), 256, 0, st>>>((float*)diag, p, n, t);
  return hipGetLastError();
}

hipError_t launch_dg_transfer(int p, int n, int precision, bool to_dg, const void* in, void* out, hipStream_t st) {
  const int64_t N = (int64_t)n * n * n * (p + 1) * (p + 1) * (p + 1);
  const int64_t L1 = (int64_t)p * n + 1;
  if (to_dg) {
    if (precision == MFQ_FP64)
      dg_from_cg_kernel<double><<<dg_grid(N), 256, 0, st>>>((const double*)in, (double*)out, p, n);
    else
      dg_from_cg_kernel<float><<<dg_grid(N), 256, 0, st>>>((const float*)in, (float*)out, p, n);
  } else {
    if (precision == MFQ_FP64)
      cg_from_dg_kernel<double><<<dg_grid(L1 * L1 * L1), 256, 0, st>>>((const double*)in, (double*)out, p, n);
    else
      cg_from_dg_kernel<float><<<dg_grid(L1 * L1 * L1), 256, 0, st>>>((const float*)in, (float*)out, p, n);
  }
  return hipGetLastError();
}

}  // namespace mfq
