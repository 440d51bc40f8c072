// Work tables of the batched launches (many independent solves advanced by one launch per kernel
// and degree).  A batched launch's grid is the concatenation of the single-solve launches' grids;
// item i owns workgroups [first_i, first_{i+1}) and each of its workgroups does exactly what the
// single-solve launch's workgroup of the same index does, so results are bitwise those of the
// solve alone.
#pragma once

#include <cstdint>

#include "mfq_internal.hpp"
#include "solver_state.hpp"

namespace mfq {

// one solve's operands of a batched vector kernel (roles per kernel, see kernels_vector.hip)
struct VecItem {
  int64_t first;       // first workgroup of the item in the batched grid
  int64_t n;           // vector length
  int nblk;            // workgroups of the single-solve launch (reductions keep its partial sums)
  int flag;            // x_is_zero (Chebyshev start) / first direction (CG)
  const void* a;
  const void* b;
  const void* c;
  void* d;
  void* e;
  void* f;
  double s0, s1;
  SolverState* st;
};

// Vector update fused into a cell loop (kernels_cell.hip): at each node the brick that completes
// the product t = (A src)_i applies it there; the other bricks leave partial sums in dst.
enum CellEpilogueMode {
  kEpiNone = 0,
  kEpiChebFirst = 1,  // src = x (not zero): r = b - t; d = dinv r / theta; x += d   (s0 = 1/theta)
  kEpiChebStep = 2,   // src = d: r -= t; d = c1 d + c2 dinv r; x += d              (s0 = c1, s1 = c2)
  kEpiResidual = 3,   // src = x: r = b - t
};
struct CellEpilogue {
  int mode = kEpiNone;
  const void* b = nullptr;
  const void* dinv = nullptr;
  void* x = nullptr;
  void* r = nullptr;
  void* d = nullptr;
  double s0 = 0, s1 = 0;
};

// one solve's operands of a batched cell loop: an operator and the vectors it reads and writes
struct CellItem {
  int64_t first[kColours];  // first workgroup of the item in colour c's launch
  const int* idx;
  const void* geo;
  const void* src;
  void* dst;
  Bricks bk;
  CellEpilogue ep;          // fused launches only
  const void* coef;         // diagonal of G per point (undeformed mesh, variable coefficient) or null
};

// one solve's operands of a batched level transfer (coarse cells of one (degree, degree) pair)
struct TransferItem {
  int64_t first[kColours];  // restriction: first workgroup per colour; prolongation: first[0]
  const void* in;
  void* out;
  int nc;                   // coarse cells per direction
  int bc;
};

enum BatchVecOp {
  kBatchCgAlpha = 0,  // a = p, b = Ap
  kBatchCgUpdate,     // d = x, e = r, a = p, b = Ap (preconditioned form); f = r rounded to FP32 (optional)
  kBatchCgBeta,       // a = r, b = z
  kBatchCgDirection,  // a = z, d = p, flag = first
  kBatchCast64To32,   // a = in (double), d = out (float)
  kBatchCast32To64,   // a = in (float), d = out (double)
  kBatchChebFirst,    // a = b, b = t, c = dinv, d = x, e = r, f = d, s0 = 1/theta, flag = x_is_zero (float)
  kBatchChebStep,     // a = A d, c = dinv, d = x, e = r, f = d, s0 = c1, s1 = c2 (float)
  kBatchSub,          // a = b, b = t, d = r (float)
  kBatchAdd,          // d = x, a = c (float)
  kBatchFill,         // d = x, s0 = value (float)
  kBatchCopy64,       // d = out, a = in (double): the solves' scalar states into one array
  kBatchCgStart,      // a = b, d = x, e = r, f = p, s0 = tol^2, flag = copy p (double)
  kBatchSplitmix,     // d = x (float), n = N1^3, flag = N1: the counter-based start vector, seed 0, masked
  kBatchLzInit,       // a = r, c = dinv, d = z, e = p, b = trace (double*), flag = count slot (float)
  kBatchLzAlpha,      // a = p, c = A p, b = trace (float)
  kBatchLzUpdate,     // d = r, e = z, a = A p, c = dinv, b = trace, flag = count slot (float)
  kBatchLzDirection,  // a = z, d = p (float)
  kBatchAdd64,        // d = x, a = c (double)
  kBatchResidualNorm, // a = b, b = t, d = r, e = out (double*): r = b - t, *out = r.r (double)
  kBatchCgBeta32,     // a = r (double), b = z (float)
  kBatchCgDirection32,// a = z (float), d = p (double), flag = first
};

// Launchers (items: device array of `count` items, `blocks` = total workgroups).
hipError_t launch_batch_vec(BatchVecOp op, const VecItem* items, int count, int64_t blocks, hipStream_t st);
// Cell loop of degree p, precision, for one colour (items' first[colour]); ACC = false.  coef: the
// items' operators read the diagonal of G (CellItem::coef); fused: with the items' epilogues (FP32
// only, stored G).
hipError_t launch_batch_cells(int p, int precision, bool cart, bool coef, bool fused, const CellItem* items,
                              int count, int colour, int64_t blocks, hipStream_t st);
// Level transfer of degree pair (pc, pf, h_transfer) in FP32: prolongation (one launch) or one
// colour of the restriction (after the coarse vectors were cleared by kBatchFill).
hipError_t launch_batch_transfer(int pc, int pf, bool h_transfer, bool prolongate, int colour,
                                 const TransferItem* items, int count, int64_t blocks, hipStream_t st);
// dst = A src with the fused update `ep` (not for matrix-core operators or spaces with hanging
// nodes); dst receives partial sums of shared nodes only.
hipError_t launch_vmult_epilogue(const OpView& v, int precision, const void* src, void* dst, const CellEpilogue& ep,
                                 hipStream_t st);
// CG steps whose preconditioner is the FP32 V-cycle: the update also writes the residual in FP32
// (the V-cycle's right-hand side), and r.z and the new direction read the V-cycle's FP32 result
// directly (widened on the fly: the values of its FP64 copy, which is never stored).
hipError_t launch_cg_update_cast(double* x, double* r, const double* p, const double* Ap, float* r32, int64_t n,
                                 SolverState* s, hipStream_t st);
hipError_t launch_cg_beta32(const double* r, const float* z, int64_t n, SolverState* s, hipStream_t st);
hipError_t launch_cg_direction32(const float* z, double* p, int64_t n, SolverState* s, bool first, hipStream_t st);
// Workgroups of the single-solve launches the batched ones reproduce.
int vec_blocks(BatchVecOp op, int64_t n);

}  // namespace mfq
