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
// One kernel computes everything, cell by cell: CPW consecutive cells per workgroup, one lane per
// 1D pencil of a cell.  Cell term: the sum factorisation of the continuous operator (even-odd forms
// of the 1D tables) with the quadrature tensor h w_r w_s w_t I of the affine cube.  Face terms: the
// cell evaluates all six of its faces itself (an interior face is evaluated by both its cells, each
// keeping its own half), one lane per tangential node: it reads its own and the neighbour's normal
// line (the trace is the end node of the GLL line, the normal derivative a dot product with l'_a
// at the end point), forms jump and mean normal derivative at the face nodes, applies the face
// rule's tensor-product mass matrix in two 1D passes through LDS, and adds the value part at the
// face node and the derivative part along the normal line.  A cell's DoFs are contiguous, so the
// result is written once with coalesced stores; the neighbours' lines come from the caches.
#include "kernels_common.hpp"

// Ask for at least 5 waves per SIMD: the register allocation then fits 5 workgroups per CU at
// p = 4 FP64 (96 instead of 126 VGPRs, no spills at any degree), which the LDS use also allows.
// Lanes per workgroup that the cells fill (one lane per 1D pencil): 128 up to degree 4 (5 cells of
// 25 lanes at p = 4; fewer waves wait at each of the kernel's barriers), 256 above (at p >= 6 a
// 128-lane workgroup holds a single cell).
#ifndef MFQ_DG_LANES
#define MFQ_DG_LANES(P) ((P) <= 4 ? 128 : 256)
#endif

#ifndef MFQ_DG_WAVES
#define MFQ_DG_WAVES __attribute__((amdgpu_waves_per_eu(5, 8)))
#endif

namespace mfq {
namespace {

template <int P, typename Real>
struct DgTables {
  Real S[(P + 1) * (P + 1)];  // [q*(P+1)+a]: l_a(zeta_q)
  Real D[(P + 1) * (P + 1)];  // l_a'(zeta_q)
  Real w[P + 1];              // Gauss weights on [0,1]
  Real d0[P + 1];             // l_a'(0)
  Real d1[P + 1];             // l_a'(1)
  Real M[(P + 1) * (P + 1)];  // 1D mass matrix of the face rule: M[a*(P+1)+b] = sum_q w_q l_a(zeta_q) l_b(zeta_q)
};

template <int P, typename Real>
DgTables<P, Real> make_dg_tables() {
  DgTables<P, Real> t{};
  const Tables1D& tb = tables(P);
  for (int k = 0; k < (P + 1) * (P + 1); ++k) {
    t.S[k] = (Real)tb.S[k];
    t.D[k] = (Real)tb.D[k];
  }
  for (int a = 0; a <= P; ++a) {
    t.w[a] = (Real)tb.omega[a];
    t.d0[a] = (Real)lagrange_derivative(tb.xi, a, 0.0);
    t.d1[a] = (Real)lagrange_derivative(tb.xi, a, 1.0);
  }
  for (int a = 0; a <= P; ++a)
    for (int b = 0; b <= P; ++b) {
      double m = 0;
      for (int q = 0; q <= P; ++q) m += tb.omega[q] * tb.S[q * (P + 1) + a] * tb.S[q * (P + 1) + b];
      t.M[a * (P + 1) + b] = (Real)m;
    }
  return t;
}

template <int P>
struct DgCell {
  static constexpr int N1 = P + 1;
  static constexpr int T = N1 * N1;
  static constexpr int NQ = N1 * T;
  static constexpr int CPW = MFQ_DG_LANES(P) / T > 0 ? MFQ_DG_LANES(P) / T : 1;  // cells per workgroup
  static constexpr int THREADS = CPW * T;
};

// Cell term of one cell per T lanes: on return, lane e = b + N1 c holds the x-pencil (b, c) of the
// cell's result in y.  lds holds 3 CPW NQ values (three arrays of CPW cells); ends after its last
// read of the first two arrays (the caller synchronises before reusing them).
template <int P, typename Real>
__device__ __forceinline__ void dg_cell_term(const Real* __restrict__ src, int64_t base, bool live, Real* lds,
                                             int lc, int e, Real h, const ShapeEO<P, Real>& sh,
                                             const Real (&wq)[P + 1], Real (&y)[P + 1]) {
  using C = DgCell<P>;
  constexpr int N1 = C::N1, T = C::T, NQ = C::NQ, CPW = C::CPW;
  const int e0 = e % N1, e1 = e / N1;
  Real* L0 = lds + lc * NQ;
  Real* L1 = L0 + CPW * NQ;
  Real* L2 = L1 + CPW * NQ;
  {  // x: values and x-derivatives at (q, e0, e1)
    Real u[N1], A[N1], B[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) u[a] = live ? src[base + a + N1 * e] : (Real)0;
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
    Real a1[N1], b1[N1], A2[N1], B2[N1], C2[N1];
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
    Real a2[N1], b2[N1], c2[N1], gx[N1], gy[N1], gz[N1];
#pragma unroll
    for (int c = 0; c < N1; ++c) {
      a2[c] = L0[e + T * c];
      b2[c] = L1[e + T * c];
      c2[c] = L2[e + T * c];
    }
    eo_apply<N1, 1, false>(sh.S, b2, gx);
    eo_apply<N1, 1, false>(sh.S, c2, gy);
    eo_apply<N1, -1, false>(sh.D, a2, gz);
    Real w0 = 0, w1 = 0;  // weights of this lane's (r, s), selected with compile-time indices
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      w0 = e0 == k ? wq[k] : w0;
      w1 = e1 == k ? wq[k] : w1;
    }
    const Real wrs = h * w0 * w1;
#pragma unroll
    for (int t = 0; t < N1; ++t) {
      const Real w = wrs * wq[t];
      gx[t] *= w;
      gy[t] *= w;
      gz[t] *= w;
    }
    Real Az[N1], Bz[N1], Cz[N1];
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
    Real az[N1], bz[N1], cz[N1], Ap[N1], Bp[N1];
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
  {  // transposed x: lane (b = e0, c = e1) forms its x-pencil of the cell result
    Real ap[N1], bp[N1];
#pragma unroll
    for (int r = 0; r < N1; ++r) {
      ap[r] = L0[r + N1 * e];
      bp[r] = L1[r + N1 * e];
    }
    eo_apply_t2<N1>(sh.S, ap, sh.D, bp, y);
  }
}

// local index of node a_d along the normal direction d at tangential node (a1, a2)
template <int N1>
__device__ __forceinline__ int face_local(int d, int ad, int a1, int a2) {
  return d == 0 ? ad + N1 * a1 + N1 * N1 * a2 : d == 1 ? a1 + N1 * ad + N1 * N1 * a2 : a1 + N1 * a2 + N1 * N1 * ad;
}

// Cell-centric form of the whole operator: one workgroup per CPW consecutive cells computes each
// cell's volume term and all six of its face terms (every interior face is evaluated by both of its
// cells, each keeping its own half), then writes each cell's result once with coalesced stores.
// The neighbours' normal lines are read from the caches (they are the same workgroup's or a
// nearby one's cells); the result is never re-read.  Workgroups are mapped so that each XCD runs
// a contiguous range of cells, keeping the y and z neighbours in that XCD's L2 more often.
// Two forms of the face terms, equal bitwise (same operations in the same order per entry):
//  direction by direction: per direction each lane forms its node's four face values, and the
//    two 1D passes of the face mass matrix run one lane per face node (two barriers per
//    direction); the result is kept in LDS and written by a coalesced pass;
//  all directions at once (LEAN): the twelve face arrays of a cell are formed together (the
//    neighbour loads of all three directions in flight at once), the 1D passes run one lane per
//    row (then column) of an array, a whole 1D contraction each (about half the LDS accesses, two
//    barriers in all), and each lane writes its x-pencil of the result from registers.
// Timed per degree and precision on MI355X (ms, direction by direction -> all at once), the
// faster form is used: FP32 p=3 0.059 -> 0.053, p=4 0.232 -> 0.209, p=5 0.181 -> 0.158,
// p=6 0.190 -> 0.157, p=8 0.204 -> 0.182 (p=1 0.026 -> 0.030, p=2 and 7 equal); FP64 p=1
// 0.042 -> 0.041, p=4 0.385 -> 0.367, p=5 0.294 -> 0.277, p=6 0.316 -> 0.289 (p=2 0.086 -> 0.093,
// p=3 0.093 -> 0.097, p=7 0.240 -> 0.371, p=8 0.447 -> 0.588: more registers and LDS per cell).
constexpr bool dg_lean_faces(int p, bool fp64) {
  return fp64 ? (p == 1 || p == 4 || p == 5 || p == 6) : (p == 3 || p == 4 || p == 5 || p == 6 || p == 8);
}

template <int P, bool LEAN = false>
struct DgFused {
  static constexpr int N1 = P + 1, T = N1 * N1, NQ = N1 * T, CPW = DgCell<P>::CPW;
  // per cell: the cell term's three arrays, or
  //   direction by direction: the result plus 8 face arrays (the 4 inputs of one direction's two
  //   faces and the 4 outputs of the first 1D pass);
  //   all at once: region A (12 face arrays, later the second pass's outputs) and region B (the
  //   first pass's outputs, later two arrays of line contributions)
  static constexpr int REGB = 12 * T > 2 * NQ ? 12 * T : 2 * NQ;
  static constexpr int FACE = LEAN ? 12 * T + REGB : NQ + 8 * T;
  static constexpr int PER_CELL = 3 * NQ > FACE ? 3 * NQ : FACE;
};

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

template <int P, typename Real>
__global__ __launch_bounds__(DgCell<P>::THREADS) MFQ_DG_WAVES void dg_fused_kernel(const Real* __restrict__ src, int n,
                                                                      int64_t n_cells, Real h, Real sigma,
                                                                      ShapeEO<P, Real> sh, DgTables<P, Real> tb,
                                                                      DgEpilogue<Real> ep) {
  constexpr bool LEAN = dg_lean_faces(P, sizeof(Real) == 8);
  using F = DgFused<P, LEAN>;
  constexpr int N1 = F::N1, T = F::T, NQ = F::NQ, CPW = F::CPW;
  __shared__ Real lds[CPW * F::PER_CELL];
  const int tid = threadIdx.x;
  const int lc = tid / T, e = tid - lc * T;
  const int e0 = e % N1, e1 = e / N1;
  // XCD-contiguous block order: block b runs on XCD b % 8 and takes the (b / 8)-th block of that
  // XCD's contiguous share (a bijection for any grid size)
  const int64_t G = gridDim.x, q8 = G / 8, r8 = G % 8;
  const int64_t x8 = blockIdx.x % 8, i8 = blockIdx.x / 8;
  const int64_t blk = (x8 < r8 ? x8 * (q8 + 1) : r8 * (q8 + 1) + (x8 - r8) * q8) + i8;
  const int64_t cell0 = blk * CPW;
  const int64_t cell = cell0 + lc;
  const bool live = cell < n_cells;
  const int64_t K = live ? cell : 0;
  const int64_t base = K * NQ;
  Real y[N1];
  dg_cell_term<P, Real>(src, base, live, lds, lc, e, h, sh, tb.w, y);
  __syncthreads();
  if constexpr (LEAN) {
    // Face terms of all three directions at once.  Lane (e0, e1) is the tangential node of each
    // direction: it forms the jump and mean normal derivative of both faces from its own and the
    // neighbours' normal lines (12 face arrays per cell).  The face mass matrix h^2 (M x M) is then
    // applied to all 12 arrays in two 1D passes whose work items are rows (then columns) of an
    // array, a 1D contraction each, spread over all lanes; the last pass leaves the results where
    // the face arrays were.
    Real* FA = lds + lc * F::PER_CELL;  // region A: face arrays, later the results of both passes
    const int64_t ijk[3] = {K % n, (K / n) % n, K / ((int64_t)n * n)};
    const int64_t nn = (int64_t)n * n;
    const Real ih = (Real)1 / h;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t stride = d == 0 ? 1 : d == 1 ? n : nn;
      const bool hasLo = live && ijk[d] > 0, hasHi = live && ijk[d] < n - 1;
      Real uK[N1], uLo[N1], uHi[N1];
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const int loc = face_local<N1>(d, a, e0, e1);
        uK[a] = live ? src[base + loc] : (Real)0;
        uLo[a] = hasLo ? src[base - stride * NQ + loc] : (Real)0;
        uHi[a] = hasHi ? src[base + stride * NQ + loc] : (Real)0;
      }
      Real dK0 = 0, dK1 = 0, dLo = 0, dHi = 0;
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        dK0 = fmad(tb.d0[a], uK[a], dK0);
        dK1 = fmad(tb.d1[a], uK[a], dK1);
        dLo = fmad(tb.d1[a], uLo[a], dLo);
        dHi = fmad(tb.d0[a], uHi[a], dHi);
      }
      // lower face (this cell on its upper side) and upper face (this cell on its lower side): jump
      // and mean normal derivative at the face nodes
      Real* Fd = FA + 4 * d * T;
      Fd[e] = uLo[N1 - 1] - uK[0];
      Fd[T + e] = hasLo ? (Real)0.5 * ih * (dLo + dK0) : ih * dK0;
      Fd[2 * T + e] = uK[N1 - 1] - uHi[0];
      Fd[3 * T + e] = hasHi ? (Real)0.5 * ih * (dK1 + dHi) : ih * dK1;
    }
    __syncthreads();
    // The face terms are the face mass matrix h^2 (M x M) applied to sigma [u] - {d_n u} (value
    // part) and to [u] (derivative part); M = S^T diag(w) S is the Gauss rule's 1D mass matrix,
    // so the interpolation to the face points and back collapses into one 1D pass per direction.
    // First tangential direction: item (cell, array, row a2) contracts the row into region B.
    constexpr int ITEMS = CPW * 12 * N1;
    for (int w = tid; w < ITEMS; w += DgCell<P>::THREADS) {
      const int wc = w / (12 * N1), rem = w - wc * 12 * N1;
      const int arr = rem / N1, a2 = rem - arr * N1;
      const Real* in = lds + wc * F::PER_CELL + arr * T + N1 * a2;
      Real* out = lds + wc * F::PER_CELL + 12 * T + arr * T + N1 * a2;
      Real f[N1];
#pragma unroll
      for (int b1 = 0; b1 < N1; ++b1) f[b1] = in[b1];
#pragma unroll
      for (int a1 = 0; a1 < N1; ++a1) {
        Real acc = 0;
#pragma unroll
        for (int b1 = 0; b1 < N1; ++b1) acc = fmad(tb.M[a1 * N1 + b1], f[b1], acc);
        out[a1] = acc;
      }
    }
    __syncthreads();
    // second tangential direction: item (cell, array, column a1), back into region A
    for (int w = tid; w < ITEMS; w += DgCell<P>::THREADS) {
      const int wc = w / (12 * N1), rem = w - wc * 12 * N1;
      const int arr = rem / N1, a1 = rem - arr * N1;
      const Real* in = lds + wc * F::PER_CELL + 12 * T + arr * T + a1;
      Real* out = lds + wc * F::PER_CELL + arr * T + a1;
      Real gcol[N1];
#pragma unroll
      for (int b2 = 0; b2 < N1; ++b2) gcol[b2] = in[N1 * b2];
#pragma unroll
      for (int a2 = 0; a2 < N1; ++a2) {
        Real acc = 0;
#pragma unroll
        for (int b2 = 0; b2 < N1; ++b2) acc = fmad(tb.M[a2 * N1 + b2], gcol[b2], acc);
        out[N1 * a2] = acc;
      }
    }
    __syncthreads();
    // Value part on the face layer, derivative part along the normal line.  Direction 0: the
    // lane's normal line is the x-pencil of the result it holds in y.  Directions 1 and 2: lines
    // through other lanes' pencils, written to two arrays in region B (one writer per node) and
    // added by the pencils' lanes after a barrier, in the order of the directions.
    Real* R1 = lds + lc * F::PER_CELL + 12 * T;
    Real* R2 = R1 + NQ;
    const Real h2 = h * h;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const bool hasLo = live && ijk[d] > 0, hasHi = live && ijk[d] < n - 1;
      const Real* Gd = FA + 4 * d * T;
      const Real g0 = Gd[e], g1 = Gd[T + e], g2 = Gd[2 * T + e], g3 = Gd[3 * T + e];
      const Real fLo = hasLo ? (Real)0.5 : (Real)1, fHi = hasHi ? (Real)0.5 : (Real)1;
      const Real VLo = h2 * (sigma * g0 - g1), DLo = -fLo * h * g0;
      const Real VHi = h2 * (sigma * g2 - g3), DHi = -fHi * h * g2;
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const Real c = (a == 0 ? -VLo : (Real)0) + (a == N1 - 1 ? VHi : (Real)0) + DLo * tb.d0[a] + DHi * tb.d1[a];
        if (d == 0)
          y[a] += c;
        else
          (d == 1 ? R1 : R2)[face_local<N1>(d, a, e0, e1)] = c;
      }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < N1; ++a) y[a] += R1[a + N1 * e];
#pragma unroll
    for (int a = 0; a < N1; ++a) y[a] += R2[a + N1 * e];
    if (ep.mode == kStore) {
      if (!live) return;
      // this lane's x-pencil of the cell result, N1 consecutive entries
      const int64_t g0i = base + N1 * e;
#pragma unroll
      for (int a = 0; a < N1; ++a) ep.dst[g0i + a] = y[a];
      return;
    }
    // smoother step or residual (several vectors read and written per entry): the result goes
    // through LDS in node order and a coalesced pass covers the workgroup's cells
    __syncthreads();
    Real* Rc = lds + lc * NQ;
#pragma unroll
    for (int a = 0; a < N1; ++a) Rc[a + N1 * e] = y[a];
    __syncthreads();
    const int64_t limit = (n_cells - cell0) * NQ;
    const int64_t gb = cell0 * NQ;
    if (ep.mode == kChebStep) {
      for (int i = tid; i < CPW * NQ; i += DgCell<P>::THREADS)
        if (i < limit) {
          const int64_t gi = gb + i;
          const Real rv = ep.r[gi] - lds[i];
          const Real dv = ep.c1 * src[gi] + ep.c2 * ep.dinv[gi] * rv;
          ep.r[gi] = rv;
          ep.dnew[gi] = dv;
          ep.x[gi] += dv;
        }
    } else {
      for (int i = tid; i < CPW * NQ; i += DgCell<P>::THREADS)
        if (i < limit) ep.r[gb + i] = ep.b[gb + i] - lds[i];
    }
  } else {
    Real* R = lds + lc * NQ;  // this cell's result, node order (contiguous over the workgroup's cells)
#pragma unroll
    for (int a = 0; a < N1; ++a) R[a + N1 * e] = y[a];
    Real* Fa = lds + CPW * NQ + lc * 4 * T;  // four face arrays of this cell
    Real* Ga = lds + CPW * NQ + CPW * 4 * T + lc * 4 * T;
    const int64_t ijk[3] = {K % n, (K / n) % n, K / ((int64_t)n * n)};
    const int64_t nn = (int64_t)n * n;
    const Real ih = (Real)1 / h;
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
      const int64_t stride = d == 0 ? 1 : d == 1 ? n : nn;
      const bool hasLo = live && ijk[d] > 0, hasHi = live && ijk[d] < n - 1;
      Real uK[N1], uLo[N1], uHi[N1];
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const int loc = face_local<N1>(d, a, e0, e1);
        uK[a] = live ? src[base + loc] : (Real)0;
        uLo[a] = hasLo ? src[base - stride * NQ + loc] : (Real)0;
        uHi[a] = hasHi ? src[base + stride * NQ + loc] : (Real)0;
      }
      Real dK0 = 0, dK1 = 0, dLo = 0, dHi = 0;
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        dK0 = fmad(tb.d0[a], uK[a], dK0);
        dK1 = fmad(tb.d1[a], uK[a], dK1);
        dLo = fmad(tb.d1[a], uLo[a], dLo);
        dHi = fmad(tb.d0[a], uHi[a], dHi);
      }
      // lower face (this cell on its upper side) and upper face (this cell on its lower side): jump
      // and mean normal derivative at the face nodes
      Fa[e] = uLo[N1 - 1] - uK[0];
      Fa[T + e] = hasLo ? (Real)0.5 * ih * (dLo + dK0) : ih * dK0;
      Fa[2 * T + e] = uK[N1 - 1] - uHi[0];
      Fa[3 * T + e] = hasHi ? (Real)0.5 * ih * (dK1 + dHi) : ih * dK1;
      __syncthreads();
      // The face terms are the face mass matrix h^2 (M x M) applied to sigma [u] - {d_n u} (value
      // part) and to [u] (derivative part); M = S^T diag(w) S is the Gauss rule's 1D mass matrix,
      // so the interpolation to the face points and back collapses into one 1D pass per direction.
      // First tangential direction: lane (a1 = e0, a2 = e1)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Real acc = 0;
#pragma unroll
        for (int b1 = 0; b1 < N1; ++b1) acc = fmad(tb.M[e0 * N1 + b1], Fa[k * T + b1 + N1 * e1], acc);
        Ga[k * T + e] = acc;
      }
      __syncthreads();
      Real g[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Real acc = 0;
#pragma unroll
        for (int b2 = 0; b2 < N1; ++b2) acc = fmad(tb.M[e1 * N1 + b2], Ga[k * T + e0 + N1 * b2], acc);
        g[k] = acc;
      }
      const Real fLo = hasLo ? (Real)0.5 : (Real)1, fHi = hasHi ? (Real)0.5 : (Real)1;
      const Real h2 = h * h;
      const Real VLo = h2 * (sigma * g[0] - g[1]), DLo = -fLo * h * g[0];
      const Real VHi = h2 * (sigma * g[2] - g[3]), DHi = -fHi * h * g[2];
      // value part on the face layer, derivative part along the normal line (this lane's own line:
      // no other lane touches it in this direction)
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const int loc = face_local<N1>(d, a, e0, e1);
        R[loc] += (a == 0 ? -VLo : (Real)0) + (a == N1 - 1 ? VHi : (Real)0) + DLo * tb.d0[a] + DHi * tb.d1[a];
      }
    }
    __syncthreads();
    // coalesced pass over the workgroup's cells
    const int64_t limit = (n_cells - cell0) * NQ;
    const int64_t g0 = cell0 * NQ;
    if (ep.mode == kStore) {
      for (int i = tid; i < CPW * NQ; i += DgCell<P>::THREADS)
        if (i < limit) ep.dst[g0 + i] = lds[i];
    } else if (ep.mode == kChebStep) {
      for (int i = tid; i < CPW * NQ; i += DgCell<P>::THREADS)
        if (i < limit) {
          const int64_t gi = g0 + i;
          const Real rv = ep.r[gi] - lds[i];
          const Real dv = ep.c1 * src[gi] + ep.c2 * ep.dinv[gi] * rv;
          ep.r[gi] = rv;
          ep.dnew[gi] = dv;
          ep.x[gi] += dv;
        }
    } else {
      for (int i = tid; i < CPW * NQ; i += DgCell<P>::THREADS)
        if (i < limit) ep.r[g0 + i] = ep.b[g0 + i] - lds[i];
    }
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
  static const DgTables<P, Real> tb = make_dg_tables<P, Real>();
  static const ShapeEO<P, Real> sh = make_shape_eo<P, Real>();
  const Real h = (Real)(1.0 / n);
  const Real sigma = (Real)(2.0 * (P + 1) * (P + 1) * n);
  const int64_t cells = (int64_t)n * n * n;
  const int64_t g = (cells + C::CPW - 1) / C::CPW;
  if (g > 0x7fffffff) return hipErrorInvalidValue;
  dg_fused_kernel<P, Real><<<(unsigned)g, C::THREADS, 0, st>>>(src, n, cells, h, sigma, sh, tb, ep);
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
