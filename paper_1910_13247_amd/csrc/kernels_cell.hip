// Cell kernels of the matrix-free Q_p operator on CDNA4 (gfx950).
//
// The operator is the variable-coefficient weak Laplacian of eq. (1), integrated cell by cell
// with shape-function gradients and JxW at the (p+1)^3 Gauss points (Sec. 2.4 cell loop) and
// applied without a matrix (Sec. 3.6): gather the cell's DoFs, evaluate reference gradients at
// the quadrature points by sum factorisation, multiply by the stored quadrature-point tensor
// G_q = w_q a(x_q) det(J_q) J_q^{-1} J_q^{-T}, test with the reference gradients (transposed sum
// factorisation), add into the result.
//
// Work decomposition (MI355X-first):
//  * one workgroup per brick of cells (e.g. 5x2x1 at p=4), one lane per 1D pencil of a
//    cell, each lane contracting its pencil in registers; pencils change direction through LDS.
//    Gradients are formed from the 1D value and derivative tables in the order x (S, D) ->
//    y (S, D on the S-branch) -> z, so all three components arrive at the same lane and
//    quadrature point without extra transposes; the backward pass is the exact transpose.
//  * the brick's node lattice is gathered once into LDS (shared nodes of neighbouring cells
//    read once) and the cells' results are summed per lattice node in LDS in a fixed order;
//  * bricks are coloured by the parities of their coordinates: one launch per colour, colours
//    in order, so a workgroup owns its lattice nodes during its launch and writes them with plain
//    stores (the first colour touching a node stores, later colours add).  No atomics (device
//    atomics across the 8 XCDs are resolved at the memory side and cost several times the
//    whole operator), no clearing of the result, bitwise reproducible.
//  * per-brick data (index lattice, G) is stored colour-major so each launch streams a
//    contiguous range; every wave's G load is 1 KiB contiguous and issued at kernel start.
#include <climits>

#include "batch.hpp"
#include "kernels_common.hpp"

namespace mfq {

namespace {

constexpr int kAbsent = INT_MIN;  // lattice node outside the mesh (ragged last bricks)

// ---------------------------------------------------------------- index lattices
// idx[ord][k]: global node of lattice node k = li + LX*(lj + LY*lk) of brick `ord`;
// ~g on Dirichlet nodes (nodes on a face whose bit is set in `faces`, bit 2d: X_d low, 2d+1: X_d
// high), kAbsent outside the mesh; with side_base >= 0 the other nodes of the X1-low face are
// hanging nodes, side_base + J + N1 K (entries of the face arrays).
template <int P>
__global__ __launch_bounds__(kBlock) void fill_index_kernel(int* __restrict__ idx, Bricks bk, int n, int faces,
                                                            int side_base) {
  using C = Cell<P>;
  const int64_t total = bk.n_bricks * C::NL;
  const int64_t N1g = (int64_t)P * n + 1;
  for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < total; L += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ord = L / C::NL;
    const int k = (int)(L - ord * C::NL);
    const int li = k % C::LX, lj = (k / C::LX) % C::LY, lk = k / (C::LX * C::LY);
    int bi, bj, bz;
    brick_of_ordinal(bk, ord, bi, bj, bz);
    const int64_t I = (int64_t)bi * C::BX * P + li, J = (int64_t)bj * C::BY * P + lj, K = (int64_t)bz * C::BZ * P + lk;
    int val = kAbsent;
    if (I < N1g && J < N1g && K < N1g) {
      const int64_t g = I + N1g * (J + N1g * K);
      const int e = N1g - 1;
      const bool bnd = ((faces & 1) && I == 0) || ((faces & 2) && I == e) || ((faces & 4) && J == 0) ||
                       ((faces & 8) && J == e) || ((faces & 16) && K == 0) || ((faces & 32) && K == e);
      val = bnd ? ~(int)g : (side_base >= 0 && I == 0) ? side_base + (int)(J + N1g * K) : (int)g;
    }
    idx[L] = val;
  }
}

// lattice index of local node (a, b, c) of cell lc of a brick
template <int P>
__host__ __device__ inline int lattice_of(int lc, int a, int b, int c) {
  using C = Cell<P>;
  const int cx = lc % C::BX, cy = (lc / C::BX) % C::BY, cz = lc / (C::BX * C::BY);
  return (cx * P + a) + C::LX * ((cy * P + b) + C::LY * (cz * P + c));
}

// ---------------------------------------------------------------- geometry precompute (FP64)
// geo[ord][t][m][lane][2]: for lane = lc*T + (r + N1*s), quadrature point (r, s, t) of cell lc of
// brick ord; pairs m = (G00,G01), (G02,G11), (G12,G22); zero for cells outside the mesh.
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

// global cell (ci, cj, ck) of cell lc in brick (bi, bj, bz); false when outside the mesh
template <int P>
__device__ __forceinline__ bool cell_of(int bi, int bj, int bz, int lc, int n, int64_t& ci, int64_t& cj, int64_t& ck) {
  using C = Cell<P>;
  ci = (int64_t)bi * C::BX + lc % C::BX;
  cj = (int64_t)bj * C::BY + (lc / C::BX) % C::BY;
  ck = (int64_t)bz * C::BZ + lc / (C::BX * C::BY);
  return ci < n && cj < n && ck < n;
}

template <int P, typename Real>
__global__ __launch_bounds__(kBlock) void geometry_kernel(Real* __restrict__ geo, Bricks bk, int n, double amp,
                                                          double alpha, QuadRule<P> qr, double x0) {
  using C = Cell<P>;
  const int64_t total = bk.n_bricks * C::N1 * C::NT;
  for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < total; L += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ord = L / (C::N1 * C::NT);
    const int rem = (int)(L - ord * (C::N1 * C::NT));
    const int t = rem / C::NT;
    const int lane = rem - t * C::NT;
    const int lc = lane / C::T;
    const int e = lane - lc * C::T;
    const int r = e % C::N1, s = e / C::N1;
    int bi, bj, bz;
    brick_of_ordinal(bk, ord, bi, bj, bz);
    int64_t ci, cj, ck;
    double G[6] = {0, 0, 0, 0, 0, 0};
    if (cell_of<P>(bi, bj, bz, lc, n, ci, cj, ck)) {
      QGeo g;
      qpoint_geometry(n, amp, ci + (int64_t)n * (cj + (int64_t)n * ck), qr.z[r], qr.z[s], qr.z[t], g, x0);
      merged_tensor(g, qr.w[r] * qr.w[s] * qr.w[t] * coefficient(alpha, g.x), G);
    }
    Real2<Real>* out = reinterpret_cast<Real2<Real>*>(geo) + (ord * C::N1 + t) * 3 * C::NT + lane;
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
                                                                 Bricks bk, int n) {
  using C = Cell<P>;
  const int64_t total = (int64_t)n * n * n * C::NQ;
  for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < total; L += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = L / C::NQ;
    const int q = (int)(L - cell * C::NQ);
    const int t = q / C::T, e = q - t * C::T;
    int lc;
    const int64_t ord = ordinal_of_cell(bk, cell % n, (cell / n) % n, cell / ((int64_t)n * n), lc);
    const Real2<Real>* in = reinterpret_cast<const Real2<Real>*>(geo) + (ord * C::N1 + t) * 3 * C::NT + lc * C::T + e;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      Real2<Real> v = in[m * C::NT];
      out[L * 6 + 2 * m] = (double)v.x;
      out[L * 6 + 2 * m + 1] = (double)v.y;
    }
  }
}

// ---------------------------------------------------------------- operator application
// Gather of a brick's node lattice by BLOCK threads (KPT nodes each), in two steps so that other
// loads can be issued in between (vector-memory loads complete in issue order, so a load issued
// before the index lattice would delay the dependent source gather):
//  lattice_index: global index of each node from the index lattice (~g on Dirichlet nodes,
//    kAbsent outside the mesh) and its store/add bit (bit j of `first`, in a vector register);
//  lattice_values: source values into `lat` (zero on Dirichlet and absent nodes) and the dst
//    values this launch adds to.
// A node shared with neighbouring bricks is written by each of them, each in its own launch: the
// brick that is even in every direction in which the node is shared stores (its colour comes
// first), the others add to what is there.
template <int P, int BLOCK, int KPT>
__device__ __forceinline__ void lattice_index(const int* __restrict__ ip, const Bricks& bk, int bi, int bj, int bz,
                                              int (&gk)[KPT], unsigned& first) {
  using C = Cell<P>;
  constexpr int LX = C::LX, LY = C::LY, NL = C::NL;
  const int tid = threadIdx.x;
  // loads only: the loaded indices are first used in lattice_values
#pragma unroll
  for (int j = 0; j < KPT; ++j) gk[j] = __builtin_nontemporal_load(ip + min(tid + j * BLOCK, NL - 1));
  // bitwise logic (no short-circuit branches: a branch here would also force a wait for the loads)
  first = 0;
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int kk = min(tid + j * BLOCK, NL - 1);
    const int li = kk % LX, lj = (kk / LX) % LY, lk = kk / (LX * LY);
    const bool sx = ((li == 0) & (bi > 0)) | ((li == LX - 1) & (bi < bk.nbx - 1));
    const bool sy = ((lj == 0) & (bj > 0)) | ((lj == LY - 1) & (bj < bk.nby - 1));
    const bool sz = ((lk == 0) & (bz > 0)) | ((lk == C::LZ - 1) & (bz < bk.nbz - 1));
    const bool fj = ((!sx) | !(bi & 1)) & ((!sy) | !(bj & 1)) & ((!sz) | !(bz & 1));
    first |= fj ? 1u << j : 0u;
  }
}

// lattice_index for spaces without hanging nodes, the indices computed instead of loaded: the
// numbering is structural (node (I, J, K) of the (pn+1)^3 lattice is I + (pn+1)(J + (pn+1) K), ~g on
// the Dirichlet faces in `faces`, kAbsent outside the mesh), exactly what fill_index_kernel stores.
template <int P, int BLOCK, int KPT>
__device__ __forceinline__ void lattice_index_computed(const Bricks& bk, int bi, int bj, int bz, int faces,
                                                       int (&gk)[KPT], unsigned& first) {
  using C = Cell<P>;
  constexpr int LX = C::LX, LY = C::LY, NL = C::NL;
  const int tid = threadIdx.x;
  const int N1g = P * bk.n + 1, e = N1g - 1;
  first = 0;
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int kk = min(tid + j * BLOCK, NL - 1);
    const int li = kk % LX, lj = (kk / LX) % LY, lk = kk / (LX * LY);
    const int I = bi * C::BX * P + li, J = bj * C::BY * P + lj, K = bz * C::BZ * P + lk;
    const int g = I + N1g * (J + N1g * K);
    const bool bnd = ((faces & 1) && I == 0) || ((faces & 2) && I == e) || ((faces & 4) && J == 0) ||
                     ((faces & 8) && J == e) || ((faces & 16) && K == 0) || ((faces & 32) && K == e);
    gk[j] = (I < N1g && J < N1g && K < N1g) ? (bnd ? ~g : g) : kAbsent;
    const bool sx = ((li == 0) & (bi > 0)) | ((li == LX - 1) & (bi < bk.nbx - 1));
    const bool sy = ((lj == 0) & (bj > 0)) | ((lj == LY - 1) & (bj < bk.nby - 1));
    const bool sz = ((lk == 0) & (bz > 0)) | ((lk == C::LZ - 1) & (bz < bk.nbz - 1));
    const bool fj = ((!sx) | !(bi & 1)) & ((!sy) | !(bj & 1)) & ((!sz) | !(bz & 1));
    first |= fj ? 1u << j : 0u;
  }
}

// Face arrays of a space with hanging nodes: index-lattice entries g >= base are nodes of the
// hanging face, read from in[g - base] and written to out[g - base] instead of the vectors.
template <typename Real>
struct Side {
  const Real* in = nullptr;
  Real* out = nullptr;
  int base = 0;
};

// MASK: nodes this brick stores (first writer) do not read dst (their lanes read entry 0
// instead, a line every brick touches and the cache keeps), so the lines of stored-only nodes are
// not fetched; otherwise every node's dst value is loaded and the unneeded ones dropped.
template <typename Real, bool ACC, int BLOCK, int KPT, int NL, bool HANG = false, bool MASK = true>
__device__ __forceinline__ void lattice_values(const Real* __restrict__ src, const Real* __restrict__ dst,
                                               int (&gk)[KPT], unsigned first, Real* lat, Real (&dv)[KPT],
                                               const Side<Real>& sd = {}) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int g0 = tid + j * BLOCK < NL ? gk[j] : kAbsent;
    gk[j] = g0;
    const bool live = g0 >= 0;
    int gs = live ? g0 : 0;
    const bool need = live && (ACC || !(first >> j & 1u));
    const Real* sp = src;
    const Real* dp = dst;
    if constexpr (HANG) {
      if (gs >= sd.base) {
        sp = sd.in;
        dp = sd.out;
        gs -= sd.base;
      }
    }
    const Real s = sp[gs];
    const Real d = dp[(MASK && !need) ? 0 : gs];
    lat[tid + j * BLOCK] = live ? s : (Real)0;
    dv[j] = need ? d : (Real)0;
  }
}

// Result values this launch adds to (nodes whose `first` bit is clear), for kernels that only
// write the result (no source lattice).
template <typename Real, int BLOCK, int KPT, int NL>
__device__ __forceinline__ void lattice_dst(const Real* __restrict__ dst, int (&gk)[KPT], unsigned first,
                                            Real (&dv)[KPT]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int g0 = tid + j * BLOCK < NL ? gk[j] : kAbsent;
    gk[j] = g0;
    const bool need = g0 >= 0 && !(first >> j & 1u);
    const Real d = dst[need ? g0 : 0];
    dv[j] = need ? d : (Real)0;
  }
}

// What scatter_lattice writes on Dirichlet rows: the source value (operator: identity rows), 1
// (diagonal) or 0 (load vector).
enum DirichletRow { kDirSource = 0, kDirUnit = 1, kDirZero = 2 };

// Sum the cells' results per lattice node in a fixed order (cell c's result at res + c * cstride,
// local lexicographic order) and write the brick's nodes: store or add per the `first` bit,
// Dirichlet nodes get the DIR value (src added to dst when accumulating) from the brick that stores.
template <int P, typename Real, bool ACC, int BLOCK, int KPT, int DIR = kDirSource, bool HANG = false>
__device__ __forceinline__ void scatter_lattice(const Real* res, int cstride, const Real* __restrict__ src,
                                                Real* __restrict__ dst, const int (&gk)[KPT], unsigned first,
                                                const Real (&dv)[KPT], const Side<Real>& sd = {}) {
  using C = Cell<P>;
  constexpr int N1 = C::N1, LX = C::LX, LY = C::LY;
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int k = tid + j * BLOCK;
    const int g0 = gk[j];
    if (g0 == kAbsent) continue;
    const int li = k % LX, lj = (k / LX) % LY, lk = k / (LX * LY);
    const int xhi = min(li / P, C::BX - 1), xlo = (li % P == 0 && li > 0) ? li / P - 1 : xhi;
    const int yhi = min(lj / P, C::BY - 1), ylo = (lj % P == 0 && lj > 0) ? lj / P - 1 : yhi;
    const int zhi = min(lk / P, C::BZ - 1), zlo = (lk % P == 0 && lk > 0) ? lk / P - 1 : zhi;
    Real sum = 0;
    for (int ccz = zlo; ccz <= zhi; ++ccz)
      for (int ccy = ylo; ccy <= yhi; ++ccy)
        for (int ccx = xlo; ccx <= xhi; ++ccx) {
          const int cell = ccx + C::BX * (ccy + C::BY * ccz);
          sum += res[cell * cstride + (li - ccx * P) + N1 * ((lj - ccy * P) + N1 * (lk - ccz * P))];
        }
    const bool fj = first >> j & 1u;
    if (g0 >= 0) {
      Real* dp = dst;
      int gl = g0;
      if constexpr (HANG) {
        if (gl >= sd.base) {
          dp = sd.out;
          gl -= sd.base;
        }
      }
      dp[gl] = (ACC || !fj) ? dv[j] + sum : sum;
    } else if (fj) {
      const int gg = ~g0;
      if constexpr (DIR == kDirUnit)
        dst[gg] = (Real)1;
      else if constexpr (DIR == kDirZero)
        dst[gg] = (Real)0;
      else
        dst[gg] = ACC ? dst[gg] + src[gg] : src[gg];
    }
  }
}

// Fused form of scatter_lattice (ACC = false, no hanging nodes): a node's last writer, the brick
// that is odd in every direction in which the node is shared (its colour comes last), completes
// t = (A src)_i and applies the epilogue there (Dirichlet rows: t = src_i) instead of storing t;
// the other bricks store or add their partial sums into dst as scatter_lattice does.  No later
// launch touches a completed node, so the epilogue may overwrite src there.  The epilogue's
// operands are loaded with the source lattice (epilogue_prefetch), so their latency hides behind
// the cell computation instead of lengthening the brick's store pass.
template <typename Real, int KPT>
struct EpiRegs {
  unsigned last;     // bit j: this brick completes node j
  int gi[KPT];       // vector index of node j (Dirichlet nodes included), 0 when not completed here
  Real a[KPT];       // r (step) or b (first step, residual)
  Real dinv[KPT];
  Real x[KPT];       // x (step)
  Real s[KPT];       // src: d (step) or x (first step); t itself on Dirichlet rows
};

template <int P, typename Real, int BLOCK, int KPT>
__device__ __forceinline__ void epilogue_prefetch(const CellEpilogue& ep, const Real* src, const int (&gk)[KPT],
                                                  const Bricks& bk, int bi, int bj, int bz, EpiRegs<Real, KPT>& e) {
  using C = Cell<P>;
  constexpr int LX = C::LX, LY = C::LY;
  const int tid = threadIdx.x;
  const Real* b = (const Real*)ep.b;
  const Real* dinv = (const Real*)ep.dinv;
  const Real* x = (const Real*)ep.x;
  const Real* r = (const Real*)ep.r;
  e.last = 0;
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int k = tid + j * BLOCK;
    const int g0 = gk[j];
    const int li = k % LX, lj = (k / LX) % LY, lk = k / (LX * LY);
    const bool sx = ((li == 0) & (bi > 0)) | ((li == LX - 1) & (bi < bk.nbx - 1));
    const bool sy = ((lj == 0) & (bj > 0)) | ((lj == LY - 1) & (bj < bk.nby - 1));
    const bool sz = ((lk == 0) & (bz > 0)) | ((lk == C::LZ - 1) & (bz < bk.nbz - 1));
    const bool last = (g0 != kAbsent) & ((!sx) | (bi & 1)) & ((!sy) | (bj & 1)) & ((!sz) | (bz & 1));
    e.last |= last ? 1u << j : 0u;
    const int gi = last ? (g0 >= 0 ? g0 : ~g0) : 0;
    e.gi[j] = gi;
    // branch-free: nodes not completed here read entry 0 (a line every brick touches)
    if (ep.mode == kEpiChebStep) {
      e.a[j] = r[gi];
      e.dinv[j] = dinv[gi];
      e.x[j] = x[gi];
    } else if (ep.mode == kEpiChebFirst) {
      e.a[j] = b[gi];
      e.dinv[j] = dinv[gi];
    } else {
      e.a[j] = b[gi];
    }
    e.s[j] = src[gi];
  }
}

template <int P, typename Real, int BLOCK, int KPT>
__device__ __forceinline__ void scatter_epilogue(const Real* res, int cstride, Real* __restrict__ dst,
                                                 const int (&gk)[KPT], unsigned first, const Real (&dv)[KPT],
                                                 const CellEpilogue& ep, const EpiRegs<Real, KPT>& e) {
  using C = Cell<P>;
  constexpr int N1 = C::N1, LX = C::LX, LY = C::LY;
  const int tid = threadIdx.x;
  Real* x = (Real*)ep.x;
  Real* r = (Real*)ep.r;
  Real* d = (Real*)ep.d;
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int k = tid + j * BLOCK;
    const int g0 = gk[j];
    if (g0 == kAbsent) continue;
    const int li = k % LX, lj = (k / LX) % LY, lk = k / (LX * LY);
    const int xhi = min(li / P, C::BX - 1), xlo = (li % P == 0 && li > 0) ? li / P - 1 : xhi;
    const int yhi = min(lj / P, C::BY - 1), ylo = (lj % P == 0 && lj > 0) ? lj / P - 1 : yhi;
    const int zhi = min(lk / P, C::BZ - 1), zlo = (lk % P == 0 && lk > 0) ? lk / P - 1 : zhi;
    Real sum = 0;
    for (int ccz = zlo; ccz <= zhi; ++ccz)
      for (int ccy = ylo; ccy <= yhi; ++ccy)
        for (int ccx = xlo; ccx <= xhi; ++ccx) {
          const int cell = ccx + C::BX * (ccy + C::BY * ccz);
          sum += res[cell * cstride + (li - ccx * P) + N1 * ((lj - ccy * P) + N1 * (lk - ccz * P))];
        }
    const bool fj = first >> j & 1u;
    const bool last = e.last >> j & 1u;
    if (!last) {
      if (g0 >= 0) dst[g0] = fj ? sum : dv[j] + sum;
      continue;
    }
    const int i = e.gi[j];
    const Real t = g0 >= 0 ? (fj ? sum : dv[j] + sum) : e.s[j];
    if (ep.mode == kEpiChebStep) {
      Real rv = e.a[j], dd = e.s[j], xv = e.x[j];
      cheb_step_entry<Real>(t, e.dinv[j], (Real)ep.s0, (Real)ep.s1, rv, dd, xv);
      r[i] = rv;
      d[i] = dd;
      x[i] = xv;
    } else if (ep.mode == kEpiChebFirst) {
      Real rv, dd, xv = e.s[j];
      cheb_first_entry<Real>(e.a[j], t, e.dinv[j], (Real)ep.s0, false, rv, dd, xv);
      r[i] = rv;
      d[i] = dd;
      x[i] = xv;
    } else {
      r[i] = e.a[j] - t;
    }
  }
}

#ifndef MFQ_G_STAGE
#define MFQ_G_STAGE 0
#endif

// One launch per colour, one workgroup per brick of exactly NT threads (one per pencil; the
// hardware masks the lanes of a partial last wave, so no lane is idle and no LDS is set aside for
// idle lanes); ACC adds A src into dst instead of overwriting it.
// Gauss weights and cell size for the operator of undeformed (axis-parallel cube) cells with
// coefficient 1, whose quadrature tensors are G_q = h w_r w_s w_t I and need not be read.
// Undeformed cells with coefficient 1 (axis-parallel cubes of side h): the quadrature tensors are
// h w_r w_s w_t I, and the cell matrix is h (K x M x M + M x K x M + M x M x K) with the Gauss
// rule's 1D stiffness and mass matrices K = D^T diag(w) D and M = S^T diag(w) S on the reference
// interval (the rule is exact for both products), so the cell term is applied in that form.
template <int P, typename Real>
struct CartQuad {
  Real h;
  EvenOdd<P + 1, Real> K;  // sum_q w_q l_a'(zeta_q) l_b'(zeta_q)
  EvenOdd<P + 1, Real> M;  // sum_q w_q l_a(zeta_q) l_b(zeta_q)
  int faces;               // Dirichlet faces (for the computed index lattice)
};

template <int P, typename Real>
CartQuad<P, Real> make_cart_quad(double h, int faces = 0) {
  static const CartQuad<P, Real> base = [] {
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
    CartQuad<P, Real> c{};
    c.K = make_even_odd<N1, Real>(K);
    c.M = make_even_odd<N1, Real>(M);
    return c;
  }();
  CartQuad<P, Real> c = base;
  c.h = (Real)h;
  c.faces = faces;
  return c;
}

// One brick (number b of colour `colour`) of the operator application by the workgroup.  HANG: a
// space with hanging nodes (X1-low face nodes go through the face arrays `sd`).
template <int P, typename Real, bool ACC, bool CART, bool HANG, bool EPI = false, bool COEF = false,
          bool CIDX = false>
__device__ __forceinline__ void vmult_brick(const int* __restrict__ idx, const Real* __restrict__ geo,
                                            const Real* __restrict__ src, Real* __restrict__ dst, const Bricks& bk,
                                            int colour, int64_t b, const ShapeEO<P, Real>& sh,
                                            const CartQuad<P, Real>& cq, const Side<Real>& sd,
                                            const CellEpilogue& ep = CellEpilogue{},
                                            const Real* __restrict__ coef = nullptr) {
  using C = Cell<P>;
  constexpr int N1 = C::N1, T = C::T, NQ = C::NQ, NCELL = C::NCELL, NT = C::NT, LX = C::LX, LY = C::LY, NL = C::NL;
  constexpr int BLOCK = NT;                        // threads of the workgroup
  constexpr int KPT = (NL + BLOCK - 1) / BLOCK;    // lattice nodes per thread
  constexpr int SLOT = NCELL * NQ;                 // one array per cell
  constexpr int L2SZ = SLOT > KPT * BLOCK ? SLOT : KPT * BLOCK;
  // cell arrays stored array-major: [L0 of every cell][L1 ...][L2 ...]; the node lattice is only
  // read before the first write of an L2 array, so it shares the L2 block
  __shared__ Real lds[2 * SLOT + L2SZ];
  Real* const lat = lds + 2 * SLOT;

  const int tid = threadIdx.x;
  const int lc = tid / T;
  const int e = tid - lc * T;
  const int e0 = e % N1, e1 = e / N1;
  const int cx = lc % C::BX, cy = (lc / C::BX) % C::BY, cz = lc / (C::BX * C::BY);
  const int64_t ord = bk.offset[colour] + b;
  int bi, bj, bz;
  brick_of(bk, colour, b, bi, bj, bz);
  Real* L0 = lds + lc * NQ;
  Real* L1 = L0 + SLOT;
  Real* L2 = L1 + SLOT;

  // quadrature-point tensors of this lane's z-pencil (points (e0, e1, t)); lanes of cells outside
  // the mesh (ragged last bricks) load nothing.  Issued at the stage MFQ_G_STAGE selects (0: kernel
  // start, 1: after the x contraction, 2: after the y contraction): earlier hides more latency,
  // later holds the 6(p+1) values in registers for a shorter time.
  Real2<Real> g[N1][3];
  const bool cell_in = bi * C::BX + cx < bk.n && bj * C::BY + cy < bk.n && bz * C::BZ + cz < bk.n;
  // Branch-free: lanes without a cell in the mesh read lane 0's entries (inside the brick, a line
  // the wave fetches anyway) and zero them.  A branch around the loads would make the compiler wait
  // for all outstanding loads at the join, G included, before the dependent source gather.
  auto load_g = [&]() {
    if constexpr (COEF) {
      // undeformed cell, variable coefficient: G = c I with c = a(x_q) h w_q, one value per point
      const Real* cp = coef + ord * (int64_t)(N1 * NT) + (cell_in ? tid : 0);
#pragma unroll
      for (int t = 0; t < N1; ++t) {
        const Real v = __builtin_nontemporal_load(cp + t * NT);
        g[t][0] = Real2<Real>{cell_in ? v : (Real)0, 0};
      }
    } else {
      const Real2<Real>* gp = reinterpret_cast<const Real2<Real>*>(geo) + ord * (int64_t)(N1 * 3 * NT) + (cell_in ? tid : 0);
#pragma unroll
      for (int t = 0; t < N1; ++t)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const Real2<Real> v = __builtin_nontemporal_load(gp + (t * 3 + m) * NT);
          g[t][m] = cell_in ? v : Real2<Real>{0, 0};
        }
    }
  };

  // this thread's lattice nodes: index lattice first, then G (not needed before the z
  // contraction), then the source and dst values that depend on the indices
  int gk[KPT];
  unsigned first;
  Real dv[KPT];
  if constexpr (CIDX)
    lattice_index_computed<P, BLOCK, KPT>(bk, bi, bj, bz, cq.faces, gk, first);
  else
    lattice_index<P, BLOCK, KPT>(idx + ord * (int64_t)NL, bk, bi, bj, bz, gk, first);
  if (!CART && MFQ_G_STAGE == 0) load_g();
  // the masked dst gather was timed per degree on MI355X: slower only for p = 6 FP64 and p = 5 FP32
  constexpr bool MASK = !((P == 6 && sizeof(Real) == 8) || (P == 5 && sizeof(Real) == 4));
  lattice_values<Real, ACC, BLOCK, KPT, NL, HANG, MASK>(src, dst, gk, first, lat, dv, sd);
  EpiRegs<Real, EPI ? KPT : 1> er;
  if constexpr (EPI) epilogue_prefetch<P, Real, BLOCK, KPT>(ep, src, gk, bk, bi, bj, bz, er);
  lds_barrier();

  if constexpr (CART) {
    // h (M_z (K_x M_y + M_x K_y) + K_z M_x M_y) u in three passes, each lane in place on its own line
    {  // x: lane (b, c) = (e0, e1): L0 = K_x u, L1 = M_x u
      const Real* up = lat + cx * P + LX * ((cy * P + e0) + LY * (cz * P + e1));
      Real u[N1], A[N1], B[N1];
#pragma unroll
      for (int a = 0; a < N1; ++a) u[a] = up[a];
      eo_apply<N1, 1, false>(cq.K, u, A);
      eo_apply<N1, 1, false>(cq.M, u, B);
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        L0[a + N1 * e] = A[a];
        L1[a + N1 * e] = B[a];
      }
    }
    lds_barrier();
    {  // y: lane (a, c) = (e0, e1): L0 = M_y L0 + K_y L1, L1 = M_y L1
      Real a1[N1], b1[N1], r1[N1], r2[N1], r3[N1];
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        a1[b] = L0[e0 + N1 * b + T * e1];
        b1[b] = L1[e0 + N1 * b + T * e1];
      }
      eo_apply<N1, 1, false>(cq.M, a1, r1);
      eo_apply<N1, 1, false>(cq.K, b1, r2);
      eo_apply<N1, 1, false>(cq.M, b1, r3);
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        L0[e0 + N1 * b + T * e1] = r1[b] + r2[b];
        L1[e0 + N1 * b + T * e1] = r3[b];
      }
    }
    lds_barrier();
    {  // z: lane (a, b) = (e0, e1): the cell result h (M_z L0 + K_z L1) into L0 (zero for cells
       // outside the mesh, whose lattice can hold nodes of the mesh's boundary face)
      Real a2[N1], b2[N1], r1[N1], r2[N1];
#pragma unroll
      for (int c = 0; c < N1; ++c) {
        a2[c] = L0[e + T * c];
        b2[c] = L1[e + T * c];
      }
      eo_apply<N1, 1, false>(cq.M, a2, r1);
      eo_apply<N1, 1, false>(cq.K, b2, r2);
      const Real hs = cell_in ? cq.h : (Real)0;
#pragma unroll
      for (int c = 0; c < N1; ++c) L0[e + T * c] = hs * (r1[c] + r2[c]);
    }
    lds_barrier();
  } else {
  // x: values and x-derivatives at (q, e0, e1) from the lane's x-pencil
  {
    const Real* up = lat + cx * P + LX * ((cy * P + e0) + LY * (cz * P + e1));
    Real u[N1], A[N1], B[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) u[a] = up[a];
    eo_apply<N1, 1, false>(sh.S, u, A);
    eo_apply<N1, -1, false>(sh.D, u, B);
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      L0[q + N1 * e] = A[q];
      L1[q + N1 * e] = B[q];
    }
  }
  if (MFQ_G_STAGE == 1) load_g();
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
    eo_apply<N1, 1, false>(sh.S, a1, A2);
    eo_apply<N1, -1, false>(sh.D, a1, C2);
    eo_apply<N1, 1, false>(sh.S, b1, B2);
    lds_barrier();
#pragma unroll
    for (int s = 0; s < N1; ++s) {
      L0[e0 + N1 * s + T * e1] = A2[s];
      L1[e0 + N1 * s + T * e1] = B2[s];
      L2[e0 + N1 * s + T * e1] = C2[s];
    }
  }
  if (MFQ_G_STAGE == 2) load_g();
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
    Real gx[N1], gy[N1], gz[N1];
    eo_apply<N1, 1, false>(sh.S, b2, gx);
    eo_apply<N1, 1, false>(sh.S, c2, gy);
    eo_apply<N1, -1, false>(sh.D, a2, gz);
    Real vx[N1], vy[N1], vz[N1];
#pragma unroll
    for (int t = 0; t < N1; ++t) {
      if constexpr (COEF) {
        const Real c = g[t][0].x;
        vx[t] = c * gx[t];
        vy[t] = c * gy[t];
        vz[t] = c * gz[t];
      } else {
        // (G00 G01 G02; G01 G11 G12; G02 G12 G22) = (G0.x G0.y G1.x; . G1.y G2.x; . . G2.y)
        const Real2<Real> G0 = g[t][0], G1 = g[t][1], G2 = g[t][2];
        vx[t] = G0.x * gx[t] + G0.y * gy[t] + G1.x * gz[t];
        vy[t] = G0.y * gx[t] + G1.y * gy[t] + G2.x * gz[t];
        vz[t] = G1.x * gx[t] + G2.x * gy[t] + G2.y * gz[t];
      }
    }
    Real Az[N1], Bz[N1], Cz[N1];
    eo_apply<N1, 1, true>(sh.S, vx, Bz);
    eo_apply<N1, 1, true>(sh.S, vy, Cz);
    eo_apply<N1, -1, true>(sh.D, vz, Az);
    lds_barrier();
#pragma unroll
    for (int c = 0; c < N1; ++c) {
      L0[e + T * c] = Az[c];
      L1[e + T * c] = Bz[c];
      L2[e + T * c] = Cz[c];
    }
  }
  lds_barrier();
  // transposed y: lane (r=e0, c=e1)
  {
    Real az[N1], bz2[N1], cz2[N1];
#pragma unroll
    for (int s = 0; s < N1; ++s) {
      az[s] = L0[e0 + N1 * s + T * e1];
      bz2[s] = L1[e0 + N1 * s + T * e1];
      cz2[s] = L2[e0 + N1 * s + T * e1];
    }
    Real Ap[N1], Bp[N1];
    eo_apply_t2<N1>(sh.S, az, sh.D, cz2, Ap);
    eo_apply<N1, 1, true>(sh.S, bz2, Bp);
    lds_barrier();
#pragma unroll
    for (int b = 0; b < N1; ++b) {
      L0[e0 + N1 * b + T * e1] = Ap[b];
      L1[e0 + N1 * b + T * e1] = Bp[b];
    }
  }
  lds_barrier();
  // transposed x: lane (b=e0, c=e1) gets the cell result of its x-pencil, kept in L0 in local
  // lexicographic order (each lane rewrites exactly the entries it read)
  {
    Real ap[N1], bp[N1], y[N1];
#pragma unroll
    for (int r = 0; r < N1; ++r) {
      ap[r] = L0[r + N1 * e];
      bp[r] = L1[r + N1 * e];
    }
    eo_apply_t2<N1>(sh.S, ap, sh.D, bp, y);
#pragma unroll
    for (int a = 0; a < N1; ++a) L0[a + N1 * e] = y[a];
  }
  lds_barrier();
  }
  // sum the cells' results per lattice node (fixed order) and write the brick's nodes
  if constexpr (EPI)
    scatter_epilogue<P, Real, BLOCK, KPT>(lds, NQ, dst, gk, first, dv, ep, er);
  else
    scatter_lattice<P, Real, ACC, BLOCK, KPT, kDirSource, HANG>(lds, NQ, src, dst, gk, first, dv, sd);
}

// Minimum waves per SIMD asked of the register allocator for the operator kernels (1: no request).
// Degree 4 in FP64 otherwise takes 131 VGPRs, 3 waves per SIMD; the request for 4 costs no spills
// and is about 1% faster (the single-operator kernel without hanging nodes only: the others spill
// under it).  Requests that force spills (5 waves at degree 4 FP64, 8 in FP32, one
// more wave at degrees 2, 3, 5-8) were measured 10-90% slower.
#ifndef MFQ_VM_WAVES
#define MFQ_VM_WAVES(P, FP64) ((P) == 4 && (FP64) ? 4 : 1)
#endif
template <int P, typename Real>
struct VmWaves {
  static constexpr int MIN = MFQ_VM_WAVES(P, sizeof(Real) == 8);
};

template <int P, typename Real, bool ACC, bool CART = false, bool HANG = false>
__global__ __launch_bounds__(Cell<P>::NT) __attribute__((amdgpu_waves_per_eu(HANG ? 1 : VmWaves<P, Real>::MIN))) void vmult_kernel(const int* __restrict__ idx, const Real* __restrict__ geo, const Real* __restrict__ src,
                  Real* __restrict__ dst, Bricks bk, int colour, ShapeEO<P, Real> sh,
                  CartQuad<P, Real> cq = {}, Side<Real> sd = {}) {
  // Cartesian operators compute their index lattice (Q4 80^3 FP32 0.286 -> 0.278 ms, FP64 0.428 ->
  // 0.410 ms; p = 8 FP64, where the extra registers cost more, keeps the loaded lattice)
  constexpr bool CIDX = CART && !HANG && !(P == 8 && sizeof(Real) == 8);
  vmult_brick<P, Real, ACC, CART, HANG, false, false, CIDX>(idx, geo, src, dst, bk, colour, blockIdx.x, sh, cq, sd);
}

// Undeformed mesh with a variable coefficient: the diagonal of G read per quadrature point.
template <int P, typename Real, bool ACC>
__global__ __launch_bounds__(Cell<P>::NT) void vmult_coef_kernel(const int* __restrict__ idx, const Real* __restrict__ coef,
                                                                 const Real* __restrict__ src, Real* __restrict__ dst,
                                                                 Bricks bk, int colour, ShapeEO<P, Real> sh) {
  vmult_brick<P, Real, ACC, false, false, false, true>(idx, nullptr, src, dst, bk, colour, blockIdx.x, sh,
                                                       CartQuad<P, Real>{}, Side<Real>{}, CellEpilogue{}, coef);
}

// Operator application with a fused vector update (see scatter_epilogue); dst holds partial sums.
template <int P, typename Real, bool CART>
__global__ __launch_bounds__(Cell<P>::NT) void vmult_epi_kernel(const int* __restrict__ idx, const Real* __restrict__ geo,
                                                                const Real* src, Real* __restrict__ dst, Bricks bk,
                                                                int colour, ShapeEO<P, Real> sh, CartQuad<P, Real> cq,
                                                                CellEpilogue ep) {
  vmult_brick<P, Real, false, CART, false, true>(idx, geo, src, dst, bk, colour, blockIdx.x, sh, cq, Side<Real>{}, ep);
}

// Batched form (serving): one launch of colour `colour` over many operators; workgroup b belongs
// to the item whose range [first[colour], next first) holds it and computes that operator's brick
// b - first, exactly as the single-operator launch does (results bitwise equal).
template <int P, typename Real, bool CART>
__global__ __launch_bounds__(Cell<P>::NT) void batch_vmult_kernel(const CellItem* __restrict__ items, int count,
                                                                   int colour, ShapeEO<P, Real> sh,
                                                                   CartQuad<P, Real> cq) {
  int lo = 0, hi = count - 1;
  const int64_t b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first[colour] <= b) lo = mid; else hi = mid - 1;
  }
  const CellItem& it = items[lo];
  CartQuad<P, Real> cqi = cq;
  if constexpr (CART) cqi.h = (Real)(1.0 / it.bk.n);
  vmult_brick<P, Real, false, CART, false>(it.idx, (const Real*)it.geo, (const Real*)it.src, (Real*)it.dst, it.bk,
                                          colour, b - it.first[colour], sh, cqi, Side<Real>{});
}

// Batched form for operators with the coefficient diagonal (CellItem::coef).
template <int P, typename Real>
__global__ __launch_bounds__(Cell<P>::NT) void batch_vmult_coef_kernel(const CellItem* __restrict__ items, int count,
                                                                        int colour, ShapeEO<P, Real> sh) {
  int lo = 0, hi = count - 1;
  const int64_t b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first[colour] <= b) lo = mid; else hi = mid - 1;
  }
  const CellItem& it = items[lo];
  vmult_brick<P, Real, false, false, false, false, true>(it.idx, nullptr, (const Real*)it.src, (Real*)it.dst, it.bk,
                                                        colour, b - it.first[colour], sh, CartQuad<P, Real>{},
                                                        Side<Real>{}, CellEpilogue{}, (const Real*)it.coef);
}

// Batched form with each item's fused vector update.
template <int P, typename Real, bool CART>
__global__ __launch_bounds__(Cell<P>::NT) void batch_vmult_epi_kernel(const CellItem* __restrict__ items, int count,
                                                                       int colour, ShapeEO<P, Real> sh,
                                                                       CartQuad<P, Real> cq) {
  int lo = 0, hi = count - 1;
  const int64_t b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first[colour] <= b) lo = mid; else hi = mid - 1;
  }
  const CellItem& it = items[lo];
  CartQuad<P, Real> cqi = cq;
  if constexpr (CART) cqi.h = (Real)(1.0 / it.bk.n);
  vmult_brick<P, Real, false, CART, false, true>(it.idx, (const Real*)it.geo, (const Real*)it.src, (Real*)it.dst,
                                                it.bk, colour, b - it.first[colour], sh, cqi, Side<Real>{}, it.ep);
}

// ---------------------------------------------------------------- operator application, MFMA (FP32)
// The same operator with the 1D contractions on the matrix cores.  Each contraction of a cell is
// Out[m][pencil] = sum_k M[m][k] In[k][pencil] over the (p+1)^2 pencils of one direction: the 1D
// table M (S, D or their transposes, zero-padded to 16 x 4 KS) is the A operand of
// v_mfma_f32_16x16x4f32, the cell data the B operand, read from LDS with the addressing that
// transposes it to the next direction, so no explicit transposes are needed.  One wave works on one
// cell at a time; the quadrature-point tensor is applied tile by tile right after the z contraction
// and its transpose follows at once.  Brick layout, index lattice, G and the node ownership rules
// are those of the FP32 operator.
//
// Lane layout of v_mfma_f32_16x16x4f32 (wave64): A operand lane l = A[l % 16][l / 16], B operand
// lane l = B[l / 16][l % 16], result register r of lane l = D[4 (l / 16) + r][l % 16].
typedef float f32x4 __attribute__((ext_vector_type(4)));


template <int P>
struct MfmaTables {
  float S[(P + 1) * (P + 1)];  // S[q][a] = l_a(zeta_q)
  float D[(P + 1) * (P + 1)];  // D[q][a] = l_a'(zeta_q)
};

template <int P>
MfmaTables<P> make_mfma_tables() {
  MfmaTables<P> t;
  for (int k = 0; k < (P + 1) * (P + 1); ++k) {
    t.S[k] = (float)ct::kTab<P>.S[k];
    t.D[k] = (float)ct::kTab<P>.D[k];
  }
  return t;
}

template <int P>
struct MCell {
  using C = Cell<P>;
  static constexpr int N1 = P + 1, NP = N1 * N1, NQ = N1 * NP;
  static constexpr int KS = (N1 + 3) / 4;          // k-steps of 4 (K padded to 4 KS)
  static constexpr int TILES = (NP + 15) / 16;     // pencil tiles of 16 columns
  static constexpr int WAVES = C::NCELL < 8 ? C::NCELL : 8;
  static constexpr int BLOCK = 64 * WAVES;
  static constexpr int KPT = (C::NL + BLOCK - 1) / BLOCK;
  static constexpr int VROWS = 4 * KS;
  static constexpr int WORK = 3 * NQ + 3 * VROWS * 16;  // per-wave scratch (floats)
  static constexpr int LDS = KPT * BLOCK + C::NCELL * NQ + WAVES * WORK;
};

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Orders this wave's LDS accesses (data exchanged between lanes of one wave only).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// A operand of M (transpose = false) or M^T, row-major N1 x N1, zero outside N1 x N1
template <int N1, int KS>
__device__ __forceinline__ void a_operand(const float* M, bool transpose, int lane, float (&a)[KS]) {
  const int i = lane & 15, kk = lane >> 4;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = 4 * s + kk;
    a[s] = (i < N1 && k < N1) ? (transpose ? M[k * N1 + i] : M[i * N1 + k]) : 0.0f;
  }
}

template <int P, bool ACC>
__global__ __launch_bounds__(MCell<P>::BLOCK) void vmult_mfma_kernel(MfmaTables<P> tab, const int* __restrict__ idx,
                                                                     const float* __restrict__ geo,
                                                                     const float* __restrict__ src,
                                                                     float* __restrict__ dst, Bricks bk, int colour) {
  using C = Cell<P>;
  using M = MCell<P>;
  constexpr int N1 = M::N1, NP = M::NP, NQ = M::NQ, KS = M::KS, TILES = M::TILES, WAVES = M::WAVES;
  constexpr int BLOCK = M::BLOCK, KPT = M::KPT, VROWS = M::VROWS;
  constexpr int NCELL = C::NCELL, T = C::T, NT = C::NT, LX = C::LX, LY = C::LY, NL = C::NL;
  __shared__ float lds[M::LDS];
  float* const lat = lds;
  float* const res = lds + KPT * BLOCK;     // cell results, [cell][a + N1 (b + N1 c)]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int col = lane & 15, kg = lane >> 4;
  float* const A0 = res + NCELL * NQ + wave * M::WORK;
  float* const A1 = A0 + NQ;
  float* const A2 = A1 + NQ;
  float* const V = A2 + NQ;  // [3][VROWS][16]
  const int64_t ord = bk.offset[colour] + blockIdx.x;
  int bi, bj, bz;
  brick_of(bk, colour, blockIdx.x, bi, bj, bz);

  int gk[KPT];
  unsigned first;
  float dv[KPT];
  lattice_index<P, BLOCK, KPT>(idx + ord * (int64_t)NL, bk, bi, bj, bz, gk, first);
  lattice_values<float, ACC, BLOCK, KPT, NL>(src, dst, gk, first, lat, dv);

  float aS[KS], aD[KS], aSt[KS], aDt[KS];
  a_operand<N1, KS>(tab.S, false, lane, aS);
  a_operand<N1, KS>(tab.D, false, lane, aD);
  a_operand<N1, KS>(tab.S, true, lane, aSt);
  a_operand<N1, KS>(tab.D, true, lane, aDt);
  lds_barrier();

  const Real2<float>* geo2 = reinterpret_cast<const Real2<float>*>(geo) + ord * (int64_t)(N1 * 3 * NT);
  for (int lc = wave; lc < NCELL; lc += WAVES) {
    const int cx = lc % C::BX, cy = (lc / C::BX) % C::BY, cz = lc / (C::BX * C::BY);
    const bool cell_in = bi * C::BX + cx < bk.n && bj * C::BY + cy < bk.n && bz * C::BZ + cz < bk.n;
    const float* ub = lat + cx * P + LX * (cy * P + LY * (cz * P));  // u[a][b][c] = ub[a + LX (b + LY c)]

    // x: XA[q][b + N1 c] = sum_a S[q][a] u[a][b][c] -> A0, XB (D) -> A1
    {
      f32x4 xa[TILES], xb[TILES];
#pragma unroll
      for (int t = 0; t < TILES; ++t) {
        xa[t] = f32x4{0, 0, 0, 0};
        xb[t] = f32x4{0, 0, 0, 0};
        const int p = 16 * t + col;
        const bool pok = p < NP;
        const int pb = pok ? p % N1 : 0, pc = pok ? p / N1 : 0;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const int k = 4 * s + kg;
          const float bv = (pok && k < N1) ? ub[k + LX * (pb + LY * pc)] : 0.0f;
          xa[t] = mfma4(aS[s], bv, xa[t]);
          xb[t] = mfma4(aD[s], bv, xb[t]);
        }
      }
#pragma unroll
      for (int t = 0; t < TILES; ++t) {
        const int p = 16 * t + col;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = 4 * kg + r;
          if (p < NP && q < N1) {
            A0[q * NP + p] = xa[t][r];
            A1[q * NP + p] = xb[t][r];
          }
        }
      }
    }
    wave_lds_sync();
    // y: YA = S_y XA, YC = D_y XA, YB = S_y XB; Y[s][q + N1 c] (B operand k = b at q NP + b + N1 c)
    {
      f32x4 ya[TILES], yc[TILES], yb[TILES];
#pragma unroll
      for (int t = 0; t < TILES; ++t) {
        ya[t] = yc[t] = yb[t] = f32x4{0, 0, 0, 0};
        const int p = 16 * t + col;
        const bool pok = p < NP;
        const int q = pok ? p % N1 : 0, c = pok ? p / N1 : 0;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const int k = 4 * s + kg;
          const bool ok = pok && k < N1;
          const int ad = q * NP + k + N1 * c;
          const float bA = ok ? A0[ad] : 0.0f;
          const float bB = ok ? A1[ad] : 0.0f;
          ya[t] = mfma4(aS[s], bA, ya[t]);
          yc[t] = mfma4(aD[s], bA, yc[t]);
          yb[t] = mfma4(aS[s], bB, yb[t]);
        }
      }
      wave_lds_sync();
#pragma unroll
      for (int t = 0; t < TILES; ++t) {
        const int p = 16 * t + col;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int sr = 4 * kg + r;
          if (p < NP && sr < N1) {
            A2[sr * NP + p] = ya[t][r];
            A0[sr * NP + p] = yc[t][r];
            A1[sr * NP + p] = yb[t][r];
          }
        }
      }
    }
    wave_lds_sync();
    // z, quadrature point and transposed z, one tile of pencils (q, s) at a time:
    // gz = D_z YA, gx = S_z YB, gy = S_z YC (B operand k = c at s NP + q + N1 c); v = G (gx, gy, gz);
    // Az = D_z^T vz, Bz = S_z^T vx, Cz = S_z^T vy written back over the tile's Y entries
    // quadrature tensors of a tile's points, zero outside the cell's points
    Real2<float> gq[4][3];
    auto load_gq = [&](int t, Real2<float> (&dst)[4][3]) {
      const int p = 16 * t + col;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tz = 4 * kg + r;
        const bool ok = cell_in && p < NP && tz < N1;
        const Real2<float>* gp = geo2 + (int64_t)(ok ? tz : 0) * 3 * NT + lc * T + (ok ? p : 0);
#pragma unroll
        for (int m = 0; m < 3; ++m) dst[r][m] = ok ? gp[m * NT] : Real2<float>{0, 0};
      }
    };
#pragma unroll
    for (int t = 0; t < TILES; ++t) {
      load_gq(t, gq);
      const int p = 16 * t + col;
      const bool pok = p < NP;
      const int q = pok ? p % N1 : 0, sy = pok ? p / N1 : 0;
      f32x4 gx = {0, 0, 0, 0}, gy = {0, 0, 0, 0}, gz = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k = 4 * s + kg;
        const bool ok = pok && k < N1;
        const int ad = sy * NP + q + N1 * k;
        const float bA = ok ? A2[ad] : 0.0f;
        const float bB = ok ? A1[ad] : 0.0f;
        const float bC = ok ? A0[ad] : 0.0f;
        gz = mfma4(aD[s], bA, gz);
        gx = mfma4(aS[s], bB, gx);
        gy = mfma4(aS[s], bC, gy);
      }
      f32x4 vx, vy, vz;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // (G00 G01 G02; G01 G11 G12; G02 G12 G22) = (G0.x G0.y G1.x; . G1.y G2.x; . . G2.y); zero
        // outside the cell's points
        const Real2<float> G0 = gq[r][0], G1 = gq[r][1], G2 = gq[r][2];
        vx[r] = G0.x * gx[r] + G0.y * gy[r] + G1.x * gz[r];
        vy[r] = G0.y * gx[r] + G1.y * gy[r] + G2.x * gz[r];
        vz[r] = G1.x * gx[r] + G2.x * gy[r] + G2.y * gz[r];
      }
      // the tile's v to scratch ([row tz][col], VROWS = 4 KS rows per component: the rows the
      // transposed contraction reads as its K; rows N1..VROWS-1 hold zeros) and back as B operand
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 4 * kg + r;
        if (row < VROWS) {
          V[row * 16 + col] = vx[r];
          V[(VROWS + row) * 16 + col] = vy[r];
          V[(2 * VROWS + row) * 16 + col] = vz[r];
        }
      }
      wave_lds_sync();
      f32x4 az = {0, 0, 0, 0}, bzv = {0, 0, 0, 0}, czv = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int row = 4 * s + kg;
        const float bvx = V[row * 16 + col];
        const float bvy = V[(VROWS + row) * 16 + col];
        const float bvz = V[(2 * VROWS + row) * 16 + col];
        bzv = mfma4(aSt[s], bvx, bzv);
        czv = mfma4(aSt[s], bvy, czv);
        az = mfma4(aDt[s], bvz, az);
      }
      wave_lds_sync();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = 4 * kg + r;
        if (pok && c < N1) {
          const int ad = sy * NP + q + N1 * c;
          A2[ad] = az[r];
          A1[ad] = bzv[r];
          A0[ad] = czv[r];
        }
      }
    }
    wave_lds_sync();
    // transposed y: A' = S_y^T Az + D_y^T Cz, B' = S_y^T Bz (B operand k = s at s NP + q + N1 c);
    // written as X[q][b + N1 c]
    {
      f32x4 ap[TILES], bp[TILES];
#pragma unroll
      for (int t = 0; t < TILES; ++t) {
        ap[t] = bp[t] = f32x4{0, 0, 0, 0};
        const int p = 16 * t + col;
        const bool pok = p < NP;
        const int q = pok ? p % N1 : 0, c = pok ? p / N1 : 0;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const int k = 4 * s + kg;
          const bool ok = pok && k < N1;
          const int ad = k * NP + q + N1 * c;
          const float bAz = ok ? A2[ad] : 0.0f;
          const float bCz = ok ? A0[ad] : 0.0f;
          const float bBz = ok ? A1[ad] : 0.0f;
          ap[t] = mfma4(aSt[s], bAz, ap[t]);
          ap[t] = mfma4(aDt[s], bCz, ap[t]);
          bp[t] = mfma4(aSt[s], bBz, bp[t]);
        }
      }
      wave_lds_sync();
#pragma unroll
      for (int t = 0; t < TILES; ++t) {
        const int p = 16 * t + col;
        const int q = p % N1, c = p / N1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int b = 4 * kg + r;
          if (p < NP && b < N1) {
            A2[q * NP + b + N1 * c] = ap[t][r];
            A1[q * NP + b + N1 * c] = bp[t][r];
          }
        }
      }
    }
    wave_lds_sync();
    // transposed x: y[a][b + N1 c] = S_x^T A' + D_x^T B' (B operand k = q at q NP + b + N1 c)
    {
      float* out = res + lc * NQ;
#pragma unroll
      for (int t = 0; t < TILES; ++t) {
        f32x4 y = {0, 0, 0, 0};
        const int p = 16 * t + col;
        const bool pok = p < NP;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const int k = 4 * s + kg;
          const bool ok = pok && k < N1;
          const int ad = k * NP + p;
          const float bA = ok ? A2[ad] : 0.0f;
          const float bB = ok ? A1[ad] : 0.0f;
          y = mfma4(aSt[s], bA, y);
          y = mfma4(aDt[s], bB, y);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = 4 * kg + r;
          if (pok && a < N1) out[a + N1 * p] = y[r];
        }
      }
    }
    wave_lds_sync();
  }
  lds_barrier();
  scatter_lattice<P, float, ACC, BLOCK, KPT>(res, NQ, src, dst, gk, first, dv);
}

// ---------------------------------------------------------------- diagonal
// diag_i = sum_K sum_q grad phi_i(q)^T G_q grad phi_i(q), 1 on Dirichlet rows.  With
// i = (a,b,c), q = (r,s,t) the sum separates per component pair (d,e) of G into 1D factors:
// grad_d phi_i(q) grad_e phi_i(q) = X(r,a) Y(s,b) Z(t,c) with X one of S^2, D S, D^2 (D where d or
// e is x, S otherwise) and likewise Y, Z.  So each cell's diagonal is three 1D contractions per
// pair, done with the operator's brick/lane/colour layout: a lane holds the z-pencil of G at
// (r,s) and contracts t; through LDS the y-lanes contract s and group the pairs by their x table;
// the x-lanes contract r.  Results are summed per lattice node and written like the operator's
// (colour order, store then add): deterministic, no atomics, no clearing pass.
template <int P, typename Real>
struct DiagTables {
  Real SS[(P + 1) * (P + 1)];  // [q*(P+1)+a]: S^2
  Real DS[(P + 1) * (P + 1)];  // D S
  Real DD[(P + 1) * (P + 1)];  // D^2
};

template <int P, typename Real>
DiagTables<P, Real> make_diag_tables() {
  DiagTables<P, Real> t{};
  for (int k = 0; k < (P + 1) * (P + 1); ++k) {
    const double sv = ct::kTab<P>.S[k], dv = ct::kTab<P>.D[k];
    t.SS[k] = (Real)(sv * sv);
    t.DS[k] = (Real)(dv * sv);
    t.DD[k] = (Real)(dv * dv);
  }
  return t;
}

template <int P, typename Real>
__global__ __launch_bounds__(Cell<P>::NT) void diagonal_kernel(const int* __restrict__ idx, const Real* __restrict__ geo,
                                                               Real* __restrict__ diag, Bricks bk, int colour,
                                                               DiagTables<P, Real> tb) {
  using C = Cell<P>;
  constexpr int N1 = C::N1, T = C::T, NQ = C::NQ, NCELL = C::NCELL, NT = C::NT, NL = C::NL;
  constexpr int BLOCK = NT;
  constexpr int KPT = (NL + BLOCK - 1) / BLOCK;
  constexpr int SLOT = NCELL * NQ;
  __shared__ Real lds[3 * SLOT];
  const int tid = threadIdx.x;
  const int lc = tid / T;
  const int e = tid - lc * T;
  const int e0 = e % N1, e1 = e / N1;
  const int cx = lc % C::BX, cy = (lc / C::BX) % C::BY, cz = lc / (C::BX * C::BY);
  const int64_t ord = bk.offset[colour] + blockIdx.x;
  int bi, bj, bz;
  brick_of(bk, colour, blockIdx.x, bi, bj, bz);
  Real* L0 = lds + lc * NQ;
  Real* L1 = L0 + SLOT;
  Real* L2 = L1 + SLOT;
  const bool cell_in = bi * C::BX + cx < bk.n && bj * C::BY + cy < bk.n && bz * C::BZ + cz < bk.n;

  int gk[KPT];
  unsigned first;
  Real dv[KPT];
  lattice_index<P, BLOCK, KPT>(idx + ord * (int64_t)NL, bk, bi, bj, bz, gk, first);
  // G of this lane's z-pencil; lanes without a cell in the mesh read lane 0's entries and zero them
  Real gz[6][N1];
  {
    const Real2<Real>* gp = reinterpret_cast<const Real2<Real>*>(geo) + ord * (int64_t)(N1 * 3 * NT) + (cell_in ? tid : 0);
#pragma unroll
    for (int t = 0; t < N1; ++t)
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const Real2<Real> v = gp[(t * 3 + m) * NT];
        gz[2 * m][t] = cell_in ? v.x : (Real)0;      // G00, G02, G12
        gz[2 * m + 1][t] = cell_in ? v.y : (Real)0;  // G01, G11, G22
      }
  }
  lattice_dst<Real, BLOCK, KPT, NL>(diag, gk, first, dv);
  // z: H(r,s,c) = sum_t Z[t][c] G(r,s,t) per pair; pair order xx, xy, xz, yy, yz, zz with
  // (X, Y, Z) = (DD,SS,SS), (DS,DS,SS), (DS,SS,DS), (SS,DD,SS), (SS,DS,DS), (SS,SS,DD)
  Real hxx[N1], hxy[N1], hxz[N1], hyy[N1], hyz[N1], hzz[N1];
  apply_t<N1>(tb.SS, gz[0], hxx);
  apply_t<N1>(tb.SS, gz[1], hxy);
  apply_t<N1>(tb.DS, gz[2], hxz);
  apply_t<N1>(tb.SS, gz[3], hyy);
  apply_t<N1>(tb.DS, gz[4], hyz);
  apply_t<N1>(tb.DD, gz[5], hzz);
#pragma unroll
  for (int c = 0; c < N1; ++c) {
    L0[e + T * c] = hxx[c];
    L1[e + T * c] = hxy[c];
    L2[e + T * c] = hxz[c];
  }
  lds_barrier();
  // y, first round: lane (r=e0, c=e1) contracts s; K grouped by the x table
  Real kdd[N1], kds[N1], kss[N1];
  {
    Real a[N1], b[N1], c2[N1], t1[N1], t2[N1];
#pragma unroll
    for (int s2 = 0; s2 < N1; ++s2) {
      a[s2] = L0[e0 + N1 * s2 + T * e1];
      b[s2] = L1[e0 + N1 * s2 + T * e1];
      c2[s2] = L2[e0 + N1 * s2 + T * e1];
    }
    apply_t<N1>(tb.SS, a, kdd);
    apply_t<N1>(tb.DS, b, t1);
    apply_t<N1>(tb.SS, c2, t2);
#pragma unroll
    for (int k = 0; k < N1; ++k) kds[k] = 2 * (t1[k] + t2[k]);
  }
  lds_barrier();
#pragma unroll
  for (int c = 0; c < N1; ++c) {
    L0[e + T * c] = hyy[c];
    L1[e + T * c] = hyz[c];
    L2[e + T * c] = hzz[c];
  }
  lds_barrier();
  {
    Real a[N1], b[N1], c2[N1], t0[N1], t1[N1], t2[N1];
#pragma unroll
    for (int s2 = 0; s2 < N1; ++s2) {
      a[s2] = L0[e0 + N1 * s2 + T * e1];
      b[s2] = L1[e0 + N1 * s2 + T * e1];
      c2[s2] = L2[e0 + N1 * s2 + T * e1];
    }
    apply_t<N1>(tb.DD, a, t0);
    apply_t<N1>(tb.DS, b, t1);
    apply_t<N1>(tb.SS, c2, t2);
#pragma unroll
    for (int k = 0; k < N1; ++k) kss[k] = t0[k] + 2 * t1[k] + t2[k];
  }
  lds_barrier();
#pragma unroll
  for (int b = 0; b < N1; ++b) {
    L0[e0 + N1 * b + T * e1] = kdd[b];
    L1[e0 + N1 * b + T * e1] = kds[b];
    L2[e0 + N1 * b + T * e1] = kss[b];
  }
  lds_barrier();
  // x: lane (b=e0, c=e1) contracts r; the cell's diagonal in local lexicographic order in L0
  {
    Real a[N1], b[N1], c2[N1], t0[N1], t1[N1], t2[N1];
#pragma unroll
    for (int r = 0; r < N1; ++r) {
      a[r] = L0[r + N1 * e];
      b[r] = L1[r + N1 * e];
      c2[r] = L2[r + N1 * e];
    }
    apply_t<N1>(tb.DD, a, t0);
    apply_t<N1>(tb.DS, b, t1);
    apply_t<N1>(tb.SS, c2, t2);
#pragma unroll
    for (int k = 0; k < N1; ++k) L0[k + N1 * e] = t0[k] + t1[k] + t2[k];
  }
  lds_barrier();
  scatter_lattice<P, Real, false, BLOCK, KPT, kDirUnit>(lds, NQ, nullptr, diag, gk, first, dv);
}

// ---------------------------------------------------------------- right-hand side
// b_i = sum_K sum_q f(x_q) JxW_q phi_i(q) for u* = sin(pi x) sin(pi y) sin(pi z), f = -div(a grad u*):
// per cell the z-pencil of f JxW is tested with S^T in z, y and x (sum factorisation), the cells'
// results are summed per node of the brick lattice and written in colour order like the
// operator's (store, then add; 0 on Dirichlet rows): deterministic, no atomics, no clearing.
template <int P>
__global__ __launch_bounds__(Cell<P>::NT) void rhs_kernel(const int* __restrict__ idx, double* __restrict__ b,
                                                          Bricks bk, int colour, int n, double amp, double alpha,
                                                          Shape<P, double> sh, QuadRule<P> qr) {
  using C = Cell<P>;
  constexpr int N1 = C::N1, T = C::T, NQ = C::NQ, NT = C::NT, NL = C::NL;
  constexpr int BLOCK = NT;
  constexpr int KPT = (NL + BLOCK - 1) / BLOCK;
  __shared__ double lds[C::NCELL * NQ];
  const int tid = threadIdx.x;
  const int lc = tid / T;
  const int e = tid - lc * T;
  const int e0 = e % N1, e1 = e / N1;
  const int64_t ord = bk.offset[colour] + blockIdx.x;
  int bi, bj, bz;
  brick_of(bk, colour, blockIdx.x, bi, bj, bz);
  int64_t ci, cj, ck;
  const bool active = cell_of<P>(bi, bj, bz, lc, n, ci, cj, ck);
  int gk[KPT];
  unsigned first;
  double dv[KPT];
  lattice_index<P, BLOCK, KPT>(idx + ord * (int64_t)NL, bk, bi, bj, bz, gk, first);
  lattice_dst<double, BLOCK, KPT, NL>(b, gk, first, dv);
  double* L0 = lds + lc * NQ;
  // z-pencil of f*JxW at points (e0, e1, t), tested with S^T in z
  double fz[N1];
  for (int t = 0; t < N1; ++t) {
    double v = 0;
    if (active) {
      QGeo g;
      qpoint_geometry(n, amp, ci + (int64_t)n * (cj + (int64_t)n * ck), qr.z[e0], qr.z[e1], qr.z[t], g);
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
  double bzv[N1];
  apply_t<N1>(sh.S, fz, bzv);
  for (int c = 0; c < N1; ++c) L0[e + T * c] = bzv[c];
  lds_barrier();
  double by[N1], tmp[N1];
  for (int s = 0; s < N1; ++s) tmp[s] = L0[e0 + N1 * s + T * e1];
  apply_t<N1>(sh.S, tmp, by);
  lds_barrier();
  for (int bb = 0; bb < N1; ++bb) L0[e0 + N1 * bb + T * e1] = by[bb];
  lds_barrier();
  // x: lane (b=e0, c=e1) reads and rewrites its own row; the cell's vector in local lexicographic order
  double bx[N1];
  for (int r = 0; r < N1; ++r) tmp[r] = L0[r + N1 * e];
  apply_t<N1>(sh.S, tmp, bx);
  for (int a = 0; a < N1; ++a) L0[a + N1 * e] = bx[a];
  lds_barrier();
  scatter_lattice<P, double, false, BLOCK, KPT, kDirZero>(lds, NQ, nullptr, b, gk, first, dv);
}

// ---------------------------------------------------------------- dense assembly (coarse levels)
// Free-free block of the assembled matrix: mat[f_i*ld + f_j] += A^K_ij, f = interior lattice index
// (I-1) + m*((J-1) + m*(K-1)), m = N1-2.  One thread per (cell, i, j) over the cells of one parity
// colour (cell coordinates' parities; such cells share no node, so no two threads of a launch
// touch one entry): one launch per colour in order, plain adds, a fixed summation order.
template <int P>
__global__ __launch_bounds__(kBlock) void assemble_dense_kernel(const int* __restrict__ idx, const double* __restrict__ geo,
                                                                double* __restrict__ mat, int64_t ld, Bricks bk,
                                                                int colour, int64_t N1g, Shape<P, double> sh) {
  using C = Cell<P>;
  constexpr int N1 = C::N1, T = C::T, NQ = C::NQ, NT = C::NT;
  const int n = bk.n;
  const int px = colour & 1, py = (colour >> 1) & 1, pz = colour >> 2;
  const int64_t cxn = (n + 1 - px) / 2, cyn = (n + 1 - py) / 2, czn = (n + 1 - pz) / 2;
  const int64_t total = cxn * cyn * czn * NQ * NQ;
  const int64_t m = N1g - 2;
  for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < total; L += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cellc = L / (NQ * NQ);
    const int ij = (int)(L - cellc * NQ * NQ);
    const int i = ij / NQ, j = ij - (ij / NQ) * NQ;
    int lc;
    const int64_t ord = ordinal_of_cell(bk, 2 * (cellc % cxn) + px, 2 * ((cellc / cxn) % cyn) + py,
                                        2 * (cellc / (cxn * cyn)) + pz, lc);
    const int ai = i % N1, bi = (i / N1) % N1, ci = i / T;
    const int aj = j % N1, bj = (j / N1) % N1, cj = j / T;
    const int gi = idx[ord * (int64_t)C::NL + lattice_of<P>(lc, ai, bi, ci)];
    const int gj = idx[ord * (int64_t)C::NL + lattice_of<P>(lc, aj, bj, cj)];
    if (gi < 0 || gj < 0) continue;  // Dirichlet or absent
    const Real2<double>* gp = reinterpret_cast<const Real2<double>*>(geo) + ord * (int64_t)(N1 * 3 * NT) + lc * T;
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
    mat[fi * ld + fj] += sum;
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
  fill_index_kernel<P><<<grid_for(v.bricks.n_bricks * C::NL), kBlock, 0, st>>>(idx, v.bricks, v.n, v.bc_faces,
                                                                                v.side_base);
  return hipGetLastError();
}

template <int P>
hipError_t geometry_p(const OpView& v, int precision, void* geo, hipStream_t st) {
  using C = Cell<P>;
  const int g = grid_for(v.bricks.n_bricks * C::N1 * C::NT);
  if (precision == MFQ_FP64)
    geometry_kernel<P, double><<<g, kBlock, 0, st>>>((double*)geo, v.bricks, v.n, v.amplitude, v.alpha, make_rule<P>(),
                                                     v.x0);
  else
    geometry_kernel<P, float><<<g, kBlock, 0, st>>>((float*)geo, v.bricks, v.n, v.amplitude, v.alpha, make_rule<P>(),
                                                    v.x0);
  return hipGetLastError();
}

template <int P>
hipError_t geometry_export_p(const OpView& v, int precision, double* out, hipStream_t st) {
  using C = Cell<P>;
  const int g = grid_for(v.n_cells * C::NQ);
  if (precision == MFQ_FP64)
    geometry_export_kernel<P, double><<<g, kBlock, 0, st>>>((const double*)v.geo, out, v.bricks, v.n);
  else
    geometry_export_kernel<P, float><<<g, kBlock, 0, st>>>((const float*)v.geo, out, v.bricks, v.n);
  return hipGetLastError();
}

template <int P, typename Real>
hipError_t vmult_pr(const OpView& v, const void* src, void* dst, bool acc, hipStream_t st) {
  static const ShapeEO<P, Real> sh = make_shape_eo<P, Real>();
  // undeformed cells and coefficient 1: the quadrature tensors are h w_r w_s w_t I (the
  // specialised mapping of axis-parallel box cells), formed in registers instead of read
  const bool cart = v.amplitude == 0.0 && v.alpha == 0.0;
  const CartQuad<P, Real> cq = cart ? make_cart_quad<P, Real>(1.0 / v.n, v.bc_faces) : CartQuad<P, Real>{};
  if (v.side_base >= 0) {
    // space with hanging nodes: overwrite only, quadrature tensors read
    if (acc || !v.side_in || !v.side_out) return hipErrorInvalidValue;
    const Side<Real> sd{(const Real*)v.side_in, (Real*)v.side_out, v.side_base};
    for (int c = 0; c < kColours; ++c) {
      const int64_t nb = v.bricks.count[c];
      if (nb == 0) continue;
      vmult_kernel<P, Real, false, false, true><<<(unsigned)nb, Cell<P>::NT, 0, st>>>(
          v.idx, (const Real*)v.geo, (const Real*)src, (Real*)dst, v.bricks, c, sh, CartQuad<P, Real>{}, sd);
    }
    return hipGetLastError();
  }
  if (v.coef) {
    for (int c = 0; c < kColours; ++c) {
      const int64_t nb = v.bricks.count[c];
      if (nb == 0) continue;
      if (acc)
        vmult_coef_kernel<P, Real, true><<<(unsigned)nb, Cell<P>::NT, 0, st>>>(
            v.idx, (const Real*)v.coef, (const Real*)src, (Real*)dst, v.bricks, c, sh);
      else
        vmult_coef_kernel<P, Real, false><<<(unsigned)nb, Cell<P>::NT, 0, st>>>(
            v.idx, (const Real*)v.coef, (const Real*)src, (Real*)dst, v.bricks, c, sh);
    }
    return hipGetLastError();
  }
  for (int c = 0; c < kColours; ++c) {
    const int64_t nb = v.bricks.count[c];
    if (nb == 0) continue;
    if (cart && acc)
      vmult_kernel<P, Real, true, true><<<(unsigned)nb, Cell<P>::NT, 0, st>>>(
          v.idx, (const Real*)v.geo, (const Real*)src, (Real*)dst, v.bricks, c, sh, cq);
    else if (cart)
      vmult_kernel<P, Real, false, true><<<(unsigned)nb, Cell<P>::NT, 0, st>>>(
          v.idx, (const Real*)v.geo, (const Real*)src, (Real*)dst, v.bricks, c, sh, cq);
    else if (acc)
      vmult_kernel<P, Real, true><<<(unsigned)nb, Cell<P>::NT, 0, st>>>(v.idx, (const Real*)v.geo, (const Real*)src,
                                                                   (Real*)dst, v.bricks, c, sh);
    else
      vmult_kernel<P, Real, false><<<(unsigned)nb, Cell<P>::NT, 0, st>>>(v.idx, (const Real*)v.geo, (const Real*)src,
                                                                    (Real*)dst, v.bricks, c, sh);
  }
  return hipGetLastError();
}

template <int P, typename Real>
hipError_t vmult_epi_pr(const OpView& v, const void* src, void* dst, const CellEpilogue& ep, hipStream_t st) {
  static const ShapeEO<P, Real> sh = make_shape_eo<P, Real>();
  const bool cart = v.amplitude == 0.0 && v.alpha == 0.0;
  const CartQuad<P, Real> cq = cart ? make_cart_quad<P, Real>(1.0 / v.n, v.bc_faces) : CartQuad<P, Real>{};
  for (int c = 0; c < kColours; ++c) {
    const int64_t nb = v.bricks.count[c];
    if (nb == 0) continue;
    if (cart)
      vmult_epi_kernel<P, Real, true><<<(unsigned)nb, Cell<P>::NT, 0, st>>>(v.idx, (const Real*)v.geo, (const Real*)src,
                                                                         (Real*)dst, v.bricks, c, sh, cq, ep);
    else
      vmult_epi_kernel<P, Real, false><<<(unsigned)nb, Cell<P>::NT, 0, st>>>(v.idx, (const Real*)v.geo, (const Real*)src,
                                                                          (Real*)dst, v.bricks, c, sh, cq, ep);
  }
  return hipGetLastError();
}

template <int P>
hipError_t vmult_epi_p(const OpView& v, int precision, const void* src, void* dst, const CellEpilogue& ep,
                       hipStream_t st) {
  if (precision == MFQ_FP64) return vmult_epi_pr<P, double>(v, src, dst, ep, st);
  return vmult_epi_pr<P, float>(v, src, dst, ep, st);
}

template <int P>
hipError_t vmult_mfma_p(const OpView& v, const void* src, void* dst, bool acc, hipStream_t st) {
  static const MfmaTables<P> tab = make_mfma_tables<P>();
  for (int c = 0; c < kColours; ++c) {
    const int64_t nb = v.bricks.count[c];
    if (nb == 0) continue;
    if (acc)
      vmult_mfma_kernel<P, true><<<(unsigned)nb, MCell<P>::BLOCK, 0, st>>>(tab, v.idx, (const float*)v.geo,
                                                                          (const float*)src, (float*)dst, v.bricks, c);
    else
      vmult_mfma_kernel<P, false><<<(unsigned)nb, MCell<P>::BLOCK, 0, st>>>(tab, v.idx, (const float*)v.geo,
                                                                           (const float*)src, (float*)dst, v.bricks, c);
  }
  return hipGetLastError();
}

template <int P>
hipError_t vmult_p(const OpView& v, int precision, const void* src, void* dst, bool acc, hipStream_t st) {
  if (precision == MFQ_FP64) return vmult_pr<P, double>(v, src, dst, acc, st);
  if (v.mfma) return vmult_mfma_p<P>(v, src, dst, acc, st);
  return vmult_pr<P, float>(v, src, dst, acc, st);
}

template <int P, typename Real>
hipError_t batch_cells_pr(bool cart, bool coef, bool fused, const CellItem* items, int count, int colour,
                          int64_t blocks, hipStream_t st) {
  static const ShapeEO<P, Real> sh = make_shape_eo<P, Real>();
  if (coef && !fused) {
    batch_vmult_coef_kernel<P, Real><<<(unsigned)blocks, Cell<P>::NT, 0, st>>>(items, count, colour, sh);
    return hipGetLastError();
  }
  if (fused) {
    if constexpr (sizeof(Real) == 8) {
      return hipErrorInvalidValue;
    } else {
      CartQuad<P, Real> cq{};
      if (cart) {
        cq = make_cart_quad<P, Real>(1.0);
        batch_vmult_epi_kernel<P, Real, true><<<(unsigned)blocks, Cell<P>::NT, 0, st>>>(items, count, colour, sh, cq);
      } else {
        batch_vmult_epi_kernel<P, Real, false><<<(unsigned)blocks, Cell<P>::NT, 0, st>>>(items, count, colour, sh, cq);
      }
      return hipGetLastError();
    }
  }
  if (cart) {
    const CartQuad<P, Real> cq = make_cart_quad<P, Real>(1.0);
    batch_vmult_kernel<P, Real, true><<<(unsigned)blocks, Cell<P>::NT, 0, st>>>(items, count, colour, sh, cq);
  } else {
    batch_vmult_kernel<P, Real, false><<<(unsigned)blocks, Cell<P>::NT, 0, st>>>(items, count, colour, sh,
                                                                                  CartQuad<P, Real>{});
  }
  return hipGetLastError();
}

template <int P>
hipError_t batch_cells_p(int precision, bool cart, bool coef, bool fused, const CellItem* items, int count,
                         int colour, int64_t blocks, hipStream_t st) {
  if (count <= 0 || blocks <= 0) return hipSuccess;
  if (precision == MFQ_FP64) return batch_cells_pr<P, double>(cart, coef, fused, items, count, colour, blocks, st);
  return batch_cells_pr<P, float>(cart, coef, fused, items, count, colour, blocks, st);
}

template <int P>
hipError_t diagonal_p(const OpView& v, int precision, void* diag, hipStream_t st) {
  for (int c = 0; c < kColours; ++c) {
    const int64_t nb = v.bricks.count[c];
    if (nb == 0) continue;
    if (precision == MFQ_FP64)
      diagonal_kernel<P, double><<<(unsigned)nb, Cell<P>::NT, 0, st>>>(v.idx, (const double*)v.geo, (double*)diag,
                                                                     v.bricks, c, make_diag_tables<P, double>());
    else
      diagonal_kernel<P, float><<<(unsigned)nb, Cell<P>::NT, 0, st>>>(v.idx, (const float*)v.geo, (float*)diag,
                                                                    v.bricks, c, make_diag_tables<P, float>());
  }
  return hipGetLastError();
}

template <int P>
hipError_t rhs_p(const OpView& v, double* b, hipStream_t st) {
  for (int c = 0; c < kColours; ++c) {
    const int64_t nb = v.bricks.count[c];
    if (nb == 0) continue;
    rhs_kernel<P><<<(unsigned)nb, Cell<P>::NT, 0, st>>>(v.idx, b, v.bricks, c, v.n, v.amplitude, v.alpha,
                                                        make_shape<P, double>(), make_rule<P>());
  }
  return hipGetLastError();
}

template <int P>
hipError_t assemble_dense_p(const OpView& v, double* mat, int64_t ld, hipStream_t st) {
  using C = Cell<P>;
  for (int c = 0; c < kColours; ++c) {
    const int64_t cells = (int64_t)((v.n + 1 - (c & 1)) / 2) * ((v.n + 1 - ((c >> 1) & 1)) / 2) * ((v.n + 1 - (c >> 2)) / 2);
    if (cells == 0) continue;
    assemble_dense_kernel<P><<<grid_for(cells * C::NQ * C::NQ), kBlock, 0, st>>>(
        v.idx, (const double*)v.geo, mat, ld, v.bricks, c, (int64_t)P * v.n + 1, make_shape<P, double>());
  }
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

hipError_t launch_vmult_cells(const OpView& v, int precision, const void* src, void* dst, bool accumulate,
                              hipStream_t st) {
  MFQ_DISPATCH(v.p, vmult_p, v, precision, src, dst, accumulate, st);
}

hipError_t launch_vmult_epilogue(const OpView& v, int precision, const void* src, void* dst, const CellEpilogue& ep,
                                 hipStream_t st) {
  if (v.mfma || v.side_base >= 0 || ep.mode == kEpiNone) return hipErrorInvalidValue;
  MFQ_DISPATCH(v.p, vmult_epi_p, v, precision, src, dst, ep, st);
}
hipError_t launch_batch_cells(int p, int precision, bool cart, bool coef, bool fused, const CellItem* items,
                              int count, int colour, int64_t blocks, hipStream_t st) {
  MFQ_DISPATCH(p, batch_cells_p, precision, cart, coef, fused, items, count, colour, blocks, st);
}

// coef[brick][t][lane] = diagonal G_xx of the stored G (layout [brick][t][3 pairs][lane], pair 0 =
// (xx, xy)) for operators on undeformed meshes with a variable coefficient
template <typename Real>
__global__ __launch_bounds__(kBlock) void coef_from_geo_kernel(const Real2<Real>* __restrict__ geo, Real* __restrict__ coef,
                                                               int64_t total, int n1, int nt) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int64_t per = (int64_t)n1 * nt;
    const int64_t ord = i / per, rem = i - ord * per;
    const int t = (int)(rem / nt), lane = (int)(rem - (int64_t)t * nt);
    coef[i] = geo[ord * 3 * per + (int64_t)(t * 3) * nt + lane].x;
  }
}

hipError_t launch_coef_from_geo(const OpView& v, int precision, const void* geo, void* coef, hipStream_t st) {
  const int n1 = v.p + 1, nt = lanes_per_brick(v.p);
  const int64_t total = v.bricks.n_bricks * n1 * (int64_t)nt;
  const int64_t g64 = (total + kBlock - 1) / kBlock;
  const unsigned g = (unsigned)(g64 < 8192 ? (g64 > 0 ? g64 : 1) : 8192);
  if (precision == MFQ_FP64)
    coef_from_geo_kernel<double><<<g, kBlock, 0, st>>>((const Real2<double>*)geo, (double*)coef, total, n1, nt);
  else
    coef_from_geo_kernel<float><<<g, kBlock, 0, st>>>((const Real2<float>*)geo, (float*)coef, total, n1, nt);
  return hipGetLastError();
}

hipError_t launch_diagonal_cells(const OpView& v, int precision, void* diag, hipStream_t st) {
  MFQ_DISPATCH(v.p, diagonal_p, v, precision, diag, st);
}

hipError_t launch_rhs_cells(const OpView& v, double* b, hipStream_t st) { MFQ_DISPATCH(v.p, rhs_p, v, b, st); }

hipError_t launch_assemble_dense(const OpView& v, double* mat, int64_t ld, hipStream_t st) {
  MFQ_DISPATCH(v.p, assemble_dense_p, v, mat, ld, st);
}

}  // namespace mfq
