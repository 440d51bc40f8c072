// Assembled sparse matrix (CSR) of the operator and its product with a vector: the matrix-based
// counterpart of the matrix-free cell kernels, built on the device so that the two can be
// compared on the same operator and the same hardware (Sec. 3.6 sets the matrix-free action
// against a stored sparse matrix that couples every unknown to its neighbours).
//
// Pattern.  On the n^3 mesh of Q_p the nodes of one direction are 0..pn, and two nodes share a
// cell in that direction exactly when they lie in one 1D cell.  Because the cells form a tensor
// product, node (I,J,K) couples with (I',J',K') iff each pair of 1D indices shares a 1D cell, so
// a row's columns are the tensor product of three 1D ranges:
//   vertex node I = kp, 0 < k < n:  [I-p, I+p]  (2p+1 entries)
//   first / last node 0, pn:         [0, p] / [pn-p, pn]  (p+1)
//   node inside a 1D cell:            [p*floor(I/p), p*floor(I/p)+p]  (p+1)
// In increasing column order the entry of column (I',J',K') of row (I,J,K) sits at
// (I'-lo_I) + len_I*((J'-lo_J) + len_J*(K'-lo_K)), and the row starts at
//   cum(K)*S^2 + len(K)*(cum(J)*S + len(J)*cum(I)),
// cum(I) = sum of len over the 1D nodes before I, S = cum(pn+1) = n(p+1)^2 - n + 1, so that
// nnz = S^3.  The pattern is that of the unconstrained matrix; with Dirichlet rows the entries
// coupling a constrained node to another node are stored as zeros and the constrained diagonal
// as one, which is the operator m*A(m*x) + (1-m)*x of the matrix-free path.
#include "kernels_common.hpp"

namespace mfq {
namespace {

struct Range1D {
  int64_t lo;
  int len;
};

__host__ __device__ inline Range1D range_1d(int64_t I, int p, int64_t pn) {
  if (I % p == 0) {
    if (I == 0) return {0, p + 1};
    if (I == pn) return {pn - p, p + 1};
    return {I - p, 2 * p + 1};
  }
  return {I / p * p, p + 1};
}

__host__ __device__ inline int64_t cum_1d(int64_t I, int p, int n) {
  if (I == 0) return 0;
  int64_t interior_vertices = (I - 1) / p;
  if (interior_vertices > n - 1) interior_vertices = n - 1;
  return I * (p + 1) + p * interior_vertices;
}

__host__ __device__ inline int64_t row_start(int64_t I, int64_t J, int64_t K, int p, int n) {
  const int64_t pn = (int64_t)p * n;
  const int64_t S = (int64_t)n * (p + 1) * (p + 1) - n + 1;
  const int lj = range_1d(J, p, pn).len, lk = range_1d(K, p, pn).len;
  return cum_1d(K, p, n) * S * S + lk * (cum_1d(J, p, n) * S + lj * cum_1d(I, p, n));
}

constexpr int kCsrBlock = 256;

__global__ __launch_bounds__(kCsrBlock) void csr_rowptr_kernel(int64_t* __restrict__ rowptr, int p, int n) {
  const int64_t N1 = (int64_t)p * n + 1;
  const int64_t N = N1 * N1 * N1;
  for (int64_t g = blockIdx.x * (int64_t)kCsrBlock + threadIdx.x; g <= N; g += (int64_t)gridDim.x * kCsrBlock) {
    if (g == N) {
      const int64_t S = (int64_t)n * (p + 1) * (p + 1) - n + 1;
      rowptr[g] = S * S * S;
    } else {
      rowptr[g] = row_start(g % N1, (g / N1) % N1, g / (N1 * N1), p, n);
    }
  }
}

// One 64-lane group per row writes the row's column indices (coalesced).
__global__ __launch_bounds__(kCsrBlock) void csr_cols_kernel(const int64_t* __restrict__ rowptr, int* __restrict__ cols,
                                                             int p, int n) {
  const int64_t N1 = (int64_t)p * n + 1, pn = N1 - 1;
  const int64_t N = N1 * N1 * N1;
  const int lane = threadIdx.x & 63;
  const int64_t groups = (int64_t)gridDim.x * (kCsrBlock / 64);
  for (int64_t g = blockIdx.x * (int64_t)(kCsrBlock / 64) + (threadIdx.x >> 6); g < N; g += groups) {
    const Range1D rx = range_1d(g % N1, p, pn), ry = range_1d((g / N1) % N1, p, pn), rz = range_1d(g / (N1 * N1), p, pn);
    const int64_t base = rowptr[g];
    const int L = rx.len * ry.len * rz.len;
    for (int k = lane; k < L; k += 64) {
      const int kx = k % rx.len, r = k / rx.len;
      const int ky = r % ry.len, kz = r / ry.len;
      cols[base + k] = (int)((rx.lo + kx) + N1 * ((ry.lo + ky) + N1 * (rz.lo + kz)));
    }
  }
}

// Element matrices A^K_ij = sum_q grad phi_i(q)^T G_q grad phi_j(q) added into the rows of the
// cell's nodes.  One workgroup per cell of one parity colour (cells whose coordinates have the
// parities of `colour` share no node, so no two workgroups of a launch touch the same entry);
// G and the 1D tables are staged in LDS and every lane of a wave reads the same quadrature point
// at the same time.  Entries of a row are contiguous in j, and j runs fastest over the lanes.
template <int P, typename V>
__global__ __launch_bounds__(kCsrBlock) void csr_values_kernel(const double* __restrict__ geo,
                                                               const int64_t* __restrict__ rowptr,
                                                               V* __restrict__ vals, Bricks bk, int n, int bc,
                                                               int colour, Shape<P, double> sh) {
  using C = Cell<P>;
  constexpr int N1 = P + 1, T = N1 * N1, NQ = N1 * T, NT = C::NT;
  __shared__ double Gs[6][NQ];
  __shared__ double Ss[N1 * N1], Ds[N1 * N1];
  const int px = colour & 1, py = (colour >> 1) & 1, pz = colour >> 2;
  const int64_t nx = (n + 1 - px) / 2, ny = (n + 1 - py) / 2;
  const int64_t b = blockIdx.x;
  const int64_t ci = 2 * (b % nx) + px, cj = 2 * ((b / nx) % ny) + py, ck = 2 * (b / (nx * ny)) + pz;
  int lc;
  const int64_t ord = ordinal_of_cell(bk, ci, cj, ck, lc);
  const Real2<double>* gp = reinterpret_cast<const Real2<double>*>(geo) + ord * (int64_t)(N1 * 3 * NT) + lc * T;
  for (int q = threadIdx.x; q < NQ; q += kCsrBlock) {
    const int t = q / T, e = q - t * T;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const Real2<double> v = gp[(t * 3 + m) * NT + e];
      Gs[2 * m][q] = v.x;
      Gs[2 * m + 1][q] = v.y;
    }
  }
  for (int k = threadIdx.x; k < N1 * N1; k += kCsrBlock) {
    Ss[k] = sh.S[k];
    Ds[k] = sh.D[k];
  }
  __syncthreads();
  const int64_t N1g = (int64_t)P * n + 1, pn = N1g - 1;
  for (int k = threadIdx.x; k < NQ * NQ; k += kCsrBlock) {
    const int i = k / NQ, j = k - (k / NQ) * NQ;
    const int ai = i % N1, bi = (i / N1) % N1, cI = i / T;
    const int aj = j % N1, bj = (j / N1) % N1, cJ = j / T;
    const int64_t Ii = P * ci + ai, Ji = P * cj + bi, Ki = P * ck + cI;
    const int64_t Ij = P * ci + aj, Jj = P * cj + bj, Kj = P * ck + cJ;
    if (bc) {
      const bool bnd_i = Ii == 0 || Ii == pn || Ji == 0 || Ji == pn || Ki == 0 || Ki == pn;
      const bool bnd_j = Ij == 0 || Ij == pn || Jj == 0 || Jj == pn || Kj == 0 || Kj == pn;
      if (bnd_i || bnd_j) continue;
    }
    double sai[N1], dai[N1], saj[N1], daj[N1];
#pragma unroll
    for (int r = 0; r < N1; ++r) {
      sai[r] = Ss[r * N1 + ai];
      dai[r] = Ds[r * N1 + ai];
      saj[r] = Ss[r * N1 + aj];
      daj[r] = Ds[r * N1 + aj];
    }
    double sum = 0;
#pragma unroll 1
    for (int t = 0; t < N1; ++t) {
      const double sci = Ss[t * N1 + cI], dci = Ds[t * N1 + cI];
      const double scj = Ss[t * N1 + cJ], dcj = Ds[t * N1 + cJ];
#pragma unroll 1
      for (int s = 0; s < N1; ++s) {
        const double sbi = Ss[s * N1 + bi], dbi = Ds[s * N1 + bi];
        const double sbj = Ss[s * N1 + bj], dbj = Ds[s * N1 + bj];
        const double ix = sbi * sci, iy = dbi * sci, iz = sbi * dci;
        const double jx = sbj * scj, jy = dbj * scj, jz = sbj * dcj;
        const int q0 = N1 * s + T * t;
#pragma unroll
        for (int r = 0; r < N1; ++r) {
          const double ux = dai[r] * ix, uy = sai[r] * iy, uz = sai[r] * iz;
          const double vx = daj[r] * jx, vy = saj[r] * jy, vz = saj[r] * jz;
          const int q = q0 + r;
          const double g0 = Gs[0][q], g1 = Gs[1][q], g2 = Gs[2][q], g3 = Gs[3][q], g4 = Gs[4][q], g5 = Gs[5][q];
          const double wx = g0 * vx + g1 * vy + g2 * vz;
          const double wy = g1 * vx + g3 * vy + g4 * vz;
          const double wz = g2 * vx + g4 * vy + g5 * vz;
          sum += ux * wx + uy * wy + uz * wz;
        }
      }
    }
    const Range1D rx = range_1d(Ii, P, pn), ry = range_1d(Ji, P, pn), rz = range_1d(Ki, P, pn);
    const int64_t pos = (Ij - rx.lo) + rx.len * ((Jj - ry.lo) + (int64_t)ry.len * (Kj - rz.lo));
    V* const entry = vals + rowptr[Ii + N1g * (Ji + N1g * Ki)] + pos;
    *entry = (V)((double)*entry + sum);  // one rounding per colour for FP32 storage
  }
}

// Identity rows of the Dirichlet nodes: the diagonal entry is one (all others stay zero).
template <typename V>
__global__ __launch_bounds__(kCsrBlock) void csr_dirichlet_kernel(const int64_t* __restrict__ rowptr,
                                                                  V* __restrict__ vals, int p, int n) {
  const int64_t N1 = (int64_t)p * n + 1, pn = N1 - 1;
  const int64_t N = N1 * N1 * N1;
  for (int64_t g = blockIdx.x * (int64_t)kCsrBlock + threadIdx.x; g < N; g += (int64_t)gridDim.x * kCsrBlock) {
    const int64_t I = g % N1, J = (g / N1) % N1, K = g / (N1 * N1);
    if (!(I == 0 || I == pn || J == 0 || J == pn || K == 0 || K == pn)) continue;
    const Range1D rx = range_1d(I, p, pn), ry = range_1d(J, p, pn), rz = range_1d(K, p, pn);
    vals[rowptr[g] + (I - rx.lo) + rx.len * ((J - ry.lo) + (int64_t)ry.len * (K - rz.lo))] = (V)1;
  }
}

// Row blocks of the product: block b holds the rows whose first entry lies in the window
// [b W, (b+1) W) of the entry array, blk[b] = first such row (lower bound of b W in rowptr),
// blk[nb] = n_rows.  A block's entries are contiguous and number at most W + (longest row) - 1.
__global__ __launch_bounds__(kCsrBlock) void csr_blocks_kernel(const int64_t* __restrict__ rowptr,
                                                               int64_t* __restrict__ blk, int64_t n_rows,
                                                               int64_t n_blocks, int64_t window) {
  for (int64_t b = blockIdx.x * (int64_t)kCsrBlock + threadIdx.x; b <= n_blocks; b += (int64_t)gridDim.x * kCsrBlock) {
    if (b == n_blocks) {
      blk[b] = n_rows;
      continue;
    }
    const int64_t target = b * window;
    int64_t lo = 0, hi = n_rows;  // first r in [0, n_rows] with rowptr[r] >= target
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (rowptr[mid] < target)
        lo = mid + 1;
      else
        hi = mid;
    }
    blk[b] = lo;
  }
}

// y = A x for long rows: LPR lanes per row, UNROLL chunks of LPR entries (masked past the row's
// end) issued before the first use, the next row's extent fetched before the current row's
// entries.  The grid is a multiple of 8 and block b runs on XCD b % 8, so block b works on the
// b % 8-th contiguous eighth of the rows (each XCD's L2 serves the source entries that
// neighbouring rows share).
template <int LPR, int UNROLL, typename V>
__global__ __launch_bounds__(kCsrBlock) void csr_spmv_rows_kernel(const int64_t* __restrict__ rowptr,
                                                                  const int* __restrict__ cols,
                                                                  const V* __restrict__ vals,
                                                                  const V* __restrict__ x,
                                                                  V* __restrict__ y, int64_t n_rows) {
  constexpr int GPB = kCsrBlock / LPR;
  const int xcd = blockIdx.x & 7;
  const int64_t slot = blockIdx.x >> 3, per_xcd = gridDim.x >> 3;
  const int64_t chunk = (n_rows + 7) / 8;
  const int64_t r0 = xcd * chunk;
  const int64_t r1 = r0 + chunk < n_rows ? r0 + chunk : n_rows;
  const int lane = threadIdx.x % LPR;
  const int grp = threadIdx.x / LPR;
  const int64_t stride = per_xcd * GPB;
  int64_t row = r0 + slot * GPB + grp;
  int64_t beg = 0, end = 0;
  if (row < r1) {
    beg = rowptr[row];
    end = rowptr[row + 1];
  }
  while (row < r1) {
    const int64_t next = row + stride;
    int64_t nbeg = 0, nend = 0;
    if (next < r1) {
      nbeg = rowptr[next];
      nend = rowptr[next + 1];
    }
    V acc = 0;
    for (int64_t base = beg + lane; base < end; base += UNROLL * LPR) {
      int c[UNROLL];
      V v[UNROLL];
      bool ok[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int64_t k = base + u * LPR;
        ok[u] = k < end;
        c[u] = ok[u] ? cols[k] : 0;
        v[u] = ok[u] ? vals[k] : (V)0;
      }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u)
        if (ok[u]) acc = fmad(v[u], x[c[u]], acc);
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
    if (lane == 0) y[row] = acc;
    row = next;
    beg = nbeg;
    end = nend;
  }
}

// y = A x, one workgroup per row block.  The workgroup streams the block's entries with
// coalesced loads, every lane issuing UNROLL independent (value, column) loads and source
// gathers before it stores the products to LDS; then groups of LPR lanes reduce one row each
// in a fixed order (lane-strided partial sums, then a butterfly), so results are bitwise
// reproducible.  Block b of the grid (a multiple of 8) runs on XCD b % 8; it takes block
// (b % 8) * ceil(nb / 8) + b / 8, so each XCD's L2 serves a contiguous eighth of the rows and
// the source entries their columns share.
template <int LPR, int UNROLL, typename V>
__global__ __launch_bounds__(kCsrBlock) void csr_spmv_kernel(const int64_t* __restrict__ rowptr,
                                                             const int* __restrict__ cols,
                                                             const V* __restrict__ vals,
                                                             const int64_t* __restrict__ blk,
                                                             const V* __restrict__ x, V* __restrict__ y,
                                                             int64_t n_blocks) {
  extern __shared__ unsigned char smem[];
  V* const prod = reinterpret_cast<V*>(smem);
  const int64_t per_xcd = (n_blocks + 7) / 8;
  const int64_t b = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (b >= n_blocks || (blockIdx.x >> 3) >= per_xcd) return;
  const int64_t row0 = blk[b], row1 = blk[b + 1];
  if (row0 >= row1) return;
  const int64_t beg = rowptr[row0], end = rowptr[row1];
  const int cnt = (int)(end - beg);
  const int t = threadIdx.x;
  for (int base = t; base < cnt; base += UNROLL * kCsrBlock) {
    int c[UNROLL];
    V v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int k = base + u * kCsrBlock;
      c[u] = k < cnt ? cols[beg + k] : 0;
      v[u] = k < cnt ? vals[beg + k] : (V)0;
    }
    V xv[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) xv[u] = base + u * kCsrBlock < cnt ? x[c[u]] : (V)0;
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int k = base + u * kCsrBlock;
      if (k < cnt) prod[k] = v[u] * xv[u];
    }
  }
  __syncthreads();
  constexpr int GPB = kCsrBlock / LPR;
  const int lane = t % LPR, grp = t / LPR;
  for (int64_t r = row0 + grp; r < row1; r += GPB) {
    const int a = (int)(rowptr[r] - beg), e = (int)(rowptr[r + 1] - beg);
    V s = 0;
    for (int k = a + lane; k < e; k += LPR) s += prod[k];
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, LPR);
    if (lane == 0) y[r] = s;
  }
}

int csr_grid(int64_t work, int per_block) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

template <int P, typename V>
hipError_t csr_values_pv(const OpView& v, const int64_t* rowptr, V* vals, hipStream_t st) {
  const int n = v.n;
  for (int c = 0; c < kColours; ++c) {
    const int px = c & 1, py = (c >> 1) & 1, pz = c >> 2;
    const int64_t cells = (int64_t)((n + 1 - px) / 2) * ((n + 1 - py) / 2) * ((n + 1 - pz) / 2);
    if (cells == 0) continue;
    if (cells > 0x7fffffff) return hipErrorInvalidValue;
    csr_values_kernel<P, V><<<(unsigned)cells, kCsrBlock, 0, st>>>((const double*)v.geo, rowptr, vals, v.bricks, n,
                                                                   v.bc, c, make_shape<P, double>());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// (value, column) loads in flight per lane before the products are formed
#ifndef MFQ_CSR_UNROLL
#define MFQ_CSR_UNROLL 4
#endif
// chunks of a row in flight per pass in the long-row kernel
#ifndef MFQ_CSR_ROW_UNROLL
#define MFQ_CSR_ROW_UNROLL 4
#endif
// workgroups of the long-row kernel per compute unit (of 256)
#ifndef MFQ_CSR_WG_PER_CU
#define MFQ_CSR_WG_PER_CU 8
#endif

template <int LPR, typename V>
hipError_t spmv_blocks(const mfq_csr* a, const V* x, V* y, hipStream_t st) {
  const int64_t grid = 8 * ((a->n_blocks + 7) / 8);
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = (size_t)(a->window + a->max_row) * sizeof(V);
  csr_spmv_kernel<LPR, MFQ_CSR_UNROLL, V><<<(unsigned)grid, kCsrBlock, lds, st>>>(a->rowptr, a->cols, (const V*)a->vals,
                                                                               a->blk, x, y, a->n_blocks);
  return hipGetLastError();
}

template <int LPR, typename V>
hipError_t spmv_rows(const mfq_csr* a, const V* x, V* y, hipStream_t st) {
  csr_spmv_rows_kernel<LPR, MFQ_CSR_ROW_UNROLL, V><<<MFQ_CSR_WG_PER_CU * 256, kCsrBlock, 0, st>>>(
      a->rowptr, a->cols, (const V*)a->vals, x, y, a->n_rows);
  return hipGetLastError();
}

template <typename V>
hipError_t spmv_typed(const mfq_csr* a, const V* x, V* y, hipStream_t st) {
  if (a->long_rows) {
    switch (a->lanes_per_row) {
      case 32: return spmv_rows<32, V>(a, x, y, st);
      case 64: return spmv_rows<64, V>(a, x, y, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (a->lanes_per_row) {
    case 8: return spmv_blocks<8, V>(a, x, y, st);
    case 16: return spmv_blocks<16, V>(a, x, y, st);
    case 32: return spmv_blocks<32, V>(a, x, y, st);
    case 64: return spmv_blocks<64, V>(a, x, y, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename V>
hipError_t csr_values_typed(const OpView& v, const int64_t* rowptr, V* vals, hipStream_t st) {
  hipError_t e;
  switch (v.p) {
    case 1: e = csr_values_pv<1, V>(v, rowptr, vals, st); break;
    case 2: e = csr_values_pv<2, V>(v, rowptr, vals, st); break;
    case 3: e = csr_values_pv<3, V>(v, rowptr, vals, st); break;
    case 4: e = csr_values_pv<4, V>(v, rowptr, vals, st); break;
    case 5: e = csr_values_pv<5, V>(v, rowptr, vals, st); break;
    case 6: e = csr_values_pv<6, V>(v, rowptr, vals, st); break;
    case 7: e = csr_values_pv<7, V>(v, rowptr, vals, st); break;
    case 8: e = csr_values_pv<8, V>(v, rowptr, vals, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess || v.bc != MFQ_BC_DIRICHLET0) return e;
  const int64_t N1 = (int64_t)v.p * v.n + 1;
  csr_dirichlet_kernel<V><<<csr_grid(N1 * N1 * N1, kCsrBlock), kCsrBlock, 0, st>>>(rowptr, vals, v.p, v.n);
  return hipGetLastError();
}

}  // namespace

int64_t csr_row_start_host(int64_t I, int64_t J, int64_t K, int p, int n) { return row_start(I, J, K, p, n); }

hipError_t launch_csr_pattern(int p, int n, int64_t* rowptr, int* cols, hipStream_t st) {
  const int64_t N1 = (int64_t)p * n + 1;
  const int64_t N = N1 * N1 * N1;
  csr_rowptr_kernel<<<csr_grid(N + 1, kCsrBlock), kCsrBlock, 0, st>>>(rowptr, p, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  csr_cols_kernel<<<csr_grid(N, kCsrBlock / 64), kCsrBlock, 0, st>>>(rowptr, cols, p, n);
  return hipGetLastError();
}

hipError_t launch_csr_values(const OpView& v, int precision, const int64_t* rowptr, void* vals, hipStream_t st) {
  if (precision == MFQ_FP64) return csr_values_typed<double>(v, rowptr, (double*)vals, st);
  return csr_values_typed<float>(v, rowptr, (float*)vals, st);
}

hipError_t launch_csr_blocks(const int64_t* rowptr, int64_t* blk, int64_t n_rows, int64_t n_blocks, int64_t window,
                             hipStream_t st) {
  csr_blocks_kernel<<<csr_grid(n_blocks + 1, kCsrBlock), kCsrBlock, 0, st>>>(rowptr, blk, n_rows, n_blocks, window);
  return hipGetLastError();
}

hipError_t launch_csr_spmv(const mfq_csr* a, const void* x, void* y, hipStream_t st) {
  if (a->precision == MFQ_FP64) return spmv_typed<double>(a, (const double*)x, (double*)y, st);
  return spmv_typed<float>(a, (const float*)x, (float*)y, st);
}

}  // namespace mfq
