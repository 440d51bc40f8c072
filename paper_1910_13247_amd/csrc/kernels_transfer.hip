// Level transfer of the geometric multigrid (Sec. 3.5): interpolation between nested Q_p spaces.
//
// Isotropic refinement (Sec. 3.1) makes each coarse cell the union of 2^3 fine cells, and the
// hierarchy may also switch to a lower degree on the same mesh (as the paper's Sec. 6.1
// hierarchy switches spaces).  Prolongation evaluates the coarse function at the fine nodes
// inside each coarse cell: a tensor product of one 1D matrix P1 [nf1 x (pc+1)] applied in x, y
// and z.  Nodes on coarse-cell faces get bitwise equal values from every adjacent coarse cell
// (the 1D matrix is exactly the identity there); each is stored once, by the cell on its upper
// side (the mesh's last cell also stores its upper face), with plain stores.
// Restriction is the transpose: fine values are weighted by 1 / (number of coarse cells
// containing the node) so the per-cell transposes sum to P^T; each cell stages its block of fine
// values in LDS once (one global read per value) before the three 1D passes.  Coarse cells are coloured by the
// parities of their coordinates (cells of one colour share no coarse node); one launch per
// colour, colours in order, each cell adding its sums into its coarse nodes with plain stores:
// no atomics, a fixed summation order, bitwise reproducible.
#include "batch.hpp"
#include "kernels_common.hpp"

namespace mfq {

namespace {

template <int PC, int NF1>
struct Transfer1D {
  double P[NF1 * (PC + 1)];  // P[i*(PC+1)+a]
};

// Threads per coarse cell: 128, or more for the high degrees, whose fine blocks (13^3 nodes and
// up) give one cell's passes enough work for more lanes (Q8 24^3 GMG_MIXED_IR solve 0.115 s with
// 128, 0.109 with 256, 0.105 with 512 threads; 256 for the degree 4 blocks: within noise)
constexpr int tblock(int nf1) { return nf1 >= 15 ? 512 : nf1 >= 13 ? 256 : 128; }

// prolongation of coarse cell `cell` by the workgroup
template <int PC, int NF1, typename Real>
__device__ __forceinline__ void prolongate_cell(const Real* __restrict__ coarse, Real* __restrict__ fine, int nc, int bc,
                                                const Transfer1D<PC, NF1>& tr, int64_t cell) {
  constexpr int M = PC + 1;
  __shared__ Real u[M * M * M];
  __shared__ Real t1[NF1 * M * M];
  __shared__ Real t2[NF1 * NF1 * M];
  __shared__ Real Ps[NF1 * M];  // the 1D matrix, read by every pass
  const int ic = (int)(cell % nc), jc = (int)((cell / nc) % nc), kc = (int)(cell / ((int64_t)nc * nc));
  const int64_t N1c = (int64_t)PC * nc + 1;
  const int stride = NF1 - 1;
  const int64_t N1f = (int64_t)stride * nc + 1;
  for (int k = threadIdx.x; k < NF1 * M; k += tblock(NF1)) Ps[k] = (Real)tr.P[k];
  for (int k = threadIdx.x; k < M * M * M; k += tblock(NF1)) {
    const int a = k % M, b = (k / M) % M, c = k / (M * M);
    const int64_t I = (int64_t)PC * ic + a, J = (int64_t)PC * jc + b, K = (int64_t)PC * kc + c;
    const bool bnd = bc && (I == 0 || J == 0 || K == 0 || I == N1c - 1 || J == N1c - 1 || K == N1c - 1);
    u[k] = bnd ? (Real)0 : coarse[I + N1c * (J + N1c * K)];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NF1 * M * M; k += tblock(NF1)) {  // t1[i][b][c]
    const int i = k % NF1, bc2 = k / NF1;
    Real s = 0;
#pragma unroll
    for (int a = 0; a < M; ++a) s += Ps[i * M + a] * u[a + M * bc2];
    t1[k] = s;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NF1 * NF1 * M; k += tblock(NF1)) {  // t2[i][j][c]
    const int i = k % NF1, j = (k / NF1) % NF1, c = k / (NF1 * NF1);
    Real s = 0;
#pragma unroll
    for (int b = 0; b < M; ++b) s += Ps[j * M + b] * t1[i + NF1 * (b + M * c)];
    t2[k] = s;
  }
  __syncthreads();
  // each fine node written once: a cell writes the fine nodes of its lower faces and interior,
  // the mesh's last cell in a direction also its upper face (the other cells' values there are
  // bitwise equal, so the choice of writer does not change the result)
  const int ni = ic == nc - 1 ? NF1 : NF1 - 1, nj = jc == nc - 1 ? NF1 : NF1 - 1, nl = kc == nc - 1 ? NF1 : NF1 - 1;
  for (int k = threadIdx.x; k < ni * nj * nl; k += tblock(NF1)) {
    const int i = k % ni, j = (k / ni) % nj, l = k / (ni * nj);
    Real s = 0;
#pragma unroll
    for (int c = 0; c < M; ++c) s += Ps[l * M + c] * t2[i + NF1 * (j + NF1 * c)];
    const int64_t I = (int64_t)stride * ic + i, J = (int64_t)stride * jc + j, K = (int64_t)stride * kc + l;
    const bool bnd = bc && (I == 0 || J == 0 || K == 0 || I == N1f - 1 || J == N1f - 1 || K == N1f - 1);
    fine[I + N1f * (J + N1f * K)] = bnd ? (Real)0 : s;
  }
}

template <int PC, int NF1, typename Real>
__global__ __launch_bounds__(tblock(NF1)) void prolongate_kernel(const Real* __restrict__ coarse, Real* __restrict__ fine,
                                                             int nc, int bc, Transfer1D<PC, NF1> tr) {
  prolongate_cell<PC, NF1, Real>(coarse, fine, nc, bc, tr, blockIdx.x);
}

// restriction of coarse cell b of colour `colour` by the workgroup
template <int PC, int NF1, typename Real>
__device__ __forceinline__ void restrict_cell(const Real* __restrict__ fine, Real* __restrict__ coarse, int nc, int bc,
                                              int colour, const Transfer1D<PC, NF1>& tr, int64_t b) {
  constexpr int M = PC + 1;
  __shared__ Real f[NF1 * NF1 * NF1]; // the cell's fine nodes, zero on Dirichlet nodes
  __shared__ Real t1[M * NF1 * NF1];  // t1[a][j][l]
  __shared__ Real t2[M * M * NF1];    // t2[a][b][l]
  __shared__ Real Ps[NF1 * M];        // the 1D matrix, read by every pass
  // cell (ic, jc, kc) of colour (ic & 1) + 2 (jc & 1) + 4 (kc & 1), x fastest within the colour
  const int px = colour & 1, py = (colour >> 1) & 1, pz = colour >> 2;
  const int cxn = (nc + 1 - px) / 2, cyn = (nc + 1 - py) / 2;
  const int ic = 2 * (int)(b % cxn) + px, jc = 2 * (int)((b / cxn) % cyn) + py, kc = 2 * (int)(b / ((int64_t)cxn * cyn)) + pz;
  const int64_t N1c = (int64_t)PC * nc + 1;
  const int stride = NF1 - 1;
  const int64_t N1f = (int64_t)stride * nc + 1;
  auto shared_factor = [&](int i, int icell) -> Real {
    return ((i == 0 && icell > 0) || (i == NF1 - 1 && icell < nc - 1)) ? (Real)0.5 : (Real)1;
  };
  // the fine block once into LDS (rows along x coalesced), then the three 1D passes from LDS
  for (int k = threadIdx.x; k < NF1 * M; k += tblock(NF1)) Ps[k] = (Real)tr.P[k];
  for (int k = threadIdx.x; k < NF1 * NF1 * NF1; k += tblock(NF1)) {
    const int i = k % NF1, j = (k / NF1) % NF1, l = k / (NF1 * NF1);
    const int64_t I = (int64_t)stride * ic + i, J = (int64_t)stride * jc + j, K = (int64_t)stride * kc + l;
    const bool bnd = bc && (I == 0 || J == 0 || K == 0 || I == N1f - 1 || J == N1f - 1 || K == N1f - 1);
    f[k] = bnd ? (Real)0 : fine[I + N1f * (J + N1f * K)];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < M * NF1 * NF1; k += tblock(NF1)) {
    const int a = k % M, j = (k / M) % NF1, l = k / (M * NF1);
    const Real wjl = shared_factor(j, jc) * shared_factor(l, kc);
    Real s = 0;
#pragma unroll
    for (int i = 0; i < NF1; ++i) s += Ps[i * M + a] * shared_factor(i, ic) * f[i + NF1 * (j + NF1 * l)];
    t1[k] = s * wjl;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < M * M * NF1; k += tblock(NF1)) {
    const int a = k % M, b = (k / M) % M, l = k / (M * M);
    Real s = 0;
#pragma unroll
    for (int j = 0; j < NF1; ++j) s += Ps[j * M + b] * t1[a + M * (j + NF1 * l)];
    t2[k] = s;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < M * M * M; k += tblock(NF1)) {
    const int a = k % M, b = (k / M) % M, c = k / (M * M);
    Real s = 0;
#pragma unroll
    for (int l = 0; l < NF1; ++l) s += Ps[l * M + c] * t2[a + M * (b + M * l)];
    const int64_t I = (int64_t)PC * ic + a, J = (int64_t)PC * jc + b, K = (int64_t)PC * kc + c;
    const bool bnd = bc && (I == 0 || J == 0 || K == 0 || I == N1c - 1 || J == N1c - 1 || K == N1c - 1);
    // this launch's cells share no coarse node; earlier colours' sums are already in place
    if (!bnd) coarse[I + N1c * (J + N1c * K)] += s;
  }
}

template <int PC, int NF1, typename Real>
__global__ __launch_bounds__(tblock(NF1)) void restrict_kernel(const Real* __restrict__ fine, Real* __restrict__ coarse,
                                                           int nc, int bc, int colour, Transfer1D<PC, NF1> tr) {
  restrict_cell<PC, NF1, Real>(fine, coarse, nc, bc, colour, tr, blockIdx.x);
}

// Batched forms (serving): workgroup b belongs to the item whose range [first[c], next first)
// holds it (c = 0 for the prolongation, the colour for the restriction) and does that item's cell
// b - first, as the single-transfer launch does (results bitwise equal).
__device__ __forceinline__ int transfer_item(const TransferItem* __restrict__ it, int count, int c, int64_t b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (it[mid].first[c] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int PC, int NF1>
__global__ __launch_bounds__(tblock(NF1)) void batch_prolongate_kernel(const TransferItem* __restrict__ items, int count,
                                                                   Transfer1D<PC, NF1> tr) {
  const TransferItem& it = items[transfer_item(items, count, 0, blockIdx.x)];
  prolongate_cell<PC, NF1, float>((const float*)it.in, (float*)it.out, it.nc, it.bc, tr, blockIdx.x - it.first[0]);
}

template <int PC, int NF1>
__global__ __launch_bounds__(tblock(NF1)) void batch_restrict_kernel(const TransferItem* __restrict__ items, int count,
                                                                 int colour, Transfer1D<PC, NF1> tr) {
  const TransferItem& it = items[transfer_item(items, count, colour, blockIdx.x)];
  restrict_cell<PC, NF1, float>((const float*)it.in, (float*)it.out, it.nc, it.bc, colour, tr,
                                blockIdx.x - it.first[colour]);
}

template <int PC, int NF1>
hipError_t batch_transfer_pn(bool h_transfer, bool prolongate, int colour, const TransferItem* items, int count,
                             int64_t blocks, hipStream_t st) {
  int nf1 = 0;
  const std::vector<double> P1 = transfer_matrix_1d(PC, h_transfer ? PC : NF1 - 1, h_transfer, &nf1);
  if (nf1 != NF1) return hipErrorInvalidValue;
  Transfer1D<PC, NF1> tr;
  for (int k = 0; k < NF1 * (PC + 1); ++k) tr.P[k] = P1[k];
  if (prolongate)
    batch_prolongate_kernel<PC, NF1><<<(unsigned)blocks, tblock(NF1), 0, st>>>(items, count, tr);
  else
    batch_restrict_kernel<PC, NF1><<<(unsigned)blocks, tblock(NF1), 0, st>>>(items, count, colour, tr);
  return hipGetLastError();
}

template <int PC, int NF1>
hipError_t transfer_pn(const mfq_transfer* t, int precision, bool prolongate, const void* in, void* out,
                       hipStream_t st) {
  Transfer1D<PC, NF1> tr;
  for (int k = 0; k < NF1 * (PC + 1); ++k) tr.P[k] = t->P1[k];
  const int nc = t->coarse->mesh->n;
  const int bc = t->coarse->bc;
  const unsigned grid = (unsigned)t->coarse->n_cells;
  if (prolongate) {
    if (precision == MFQ_FP64)
      prolongate_kernel<PC, NF1, double><<<grid, tblock(NF1), 0, st>>>((const double*)in, (double*)out, nc, bc, tr);
    else
      prolongate_kernel<PC, NF1, float><<<grid, tblock(NF1), 0, st>>>((const float*)in, (float*)out, nc, bc, tr);
  } else {
    hipError_t e = launch_fill(precision, out, t->coarse->n_dofs, 0.0, st);
    if (e != hipSuccess) return e;
    for (int c = 0; c < 8; ++c) {
      const int64_t cells = (int64_t)((nc + 1 - (c & 1)) / 2) * ((nc + 1 - ((c >> 1) & 1)) / 2) * ((nc + 1 - (c >> 2)) / 2);
      if (cells == 0) continue;
      if (precision == MFQ_FP64)
        restrict_kernel<PC, NF1, double><<<(unsigned)cells, tblock(NF1), 0, st>>>((const double*)in, (double*)out, nc, bc, c, tr);
      else
        restrict_kernel<PC, NF1, float><<<(unsigned)cells, tblock(NF1), 0, st>>>((const float*)in, (float*)out, nc, bc, c, tr);
    }
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_transfer(const mfq_transfer* t, int precision, bool prolongate, const void* in, void* out,
                           hipStream_t st) {
  const int pc = t->coarse->p;
  if (t->h_transfer) {
    switch (pc) {
      case 1: return transfer_pn<1, 3>(t, precision, prolongate, in, out, st);
      case 2: return transfer_pn<2, 5>(t, precision, prolongate, in, out, st);
      case 3: return transfer_pn<3, 7>(t, precision, prolongate, in, out, st);
      case 4: return transfer_pn<4, 9>(t, precision, prolongate, in, out, st);
      case 5: return transfer_pn<5, 11>(t, precision, prolongate, in, out, st);
      case 6: return transfer_pn<6, 13>(t, precision, prolongate, in, out, st);
      case 7: return transfer_pn<7, 15>(t, precision, prolongate, in, out, st);
      case 8: return transfer_pn<8, 17>(t, precision, prolongate, in, out, st);
      default: return hipErrorInvalidValue;
    }
  }
  const int pf = t->fine->p;
  // degree switches of the hierarchy rule: p -> ceil(p/2)
#define MFQ_PT(a, b) \
  if (pc == a && pf == b) return transfer_pn<a, b + 1>(t, precision, prolongate, in, out, st);
  MFQ_PT(1, 2) MFQ_PT(2, 3) MFQ_PT(2, 4) MFQ_PT(3, 5) MFQ_PT(3, 6) MFQ_PT(4, 7) MFQ_PT(4, 8)
#undef MFQ_PT
  return hipErrorInvalidValue;
}

hipError_t launch_batch_transfer(int pc, int pf, bool h_transfer, bool prolongate, int colour,
                                 const TransferItem* items, int count, int64_t blocks, hipStream_t st) {
  if (count <= 0 || blocks <= 0) return hipSuccess;
  if (h_transfer) {
    switch (pc) {
      case 1: return batch_transfer_pn<1, 3>(true, prolongate, colour, items, count, blocks, st);
      case 2: return batch_transfer_pn<2, 5>(true, prolongate, colour, items, count, blocks, st);
      case 3: return batch_transfer_pn<3, 7>(true, prolongate, colour, items, count, blocks, st);
      case 4: return batch_transfer_pn<4, 9>(true, prolongate, colour, items, count, blocks, st);
      case 5: return batch_transfer_pn<5, 11>(true, prolongate, colour, items, count, blocks, st);
      case 6: return batch_transfer_pn<6, 13>(true, prolongate, colour, items, count, blocks, st);
      case 7: return batch_transfer_pn<7, 15>(true, prolongate, colour, items, count, blocks, st);
      case 8: return batch_transfer_pn<8, 17>(true, prolongate, colour, items, count, blocks, st);
      default: return hipErrorInvalidValue;
    }
  }
#define MFQ_PT(a, b) \
  if (pc == a && pf == b) return batch_transfer_pn<a, b + 1>(false, prolongate, colour, items, count, blocks, st);
  MFQ_PT(1, 2) MFQ_PT(2, 3) MFQ_PT(2, 4) MFQ_PT(3, 5) MFQ_PT(3, 6) MFQ_PT(4, 7) MFQ_PT(4, 8)
#undef MFQ_PT
  return hipErrorInvalidValue;
}

}  // namespace mfq
