// Vector kernels of the Krylov solvers and smoothers (CDNA4, wave64).
//
// The paper leaves the solvers' vector algebra unspecified beyond running the library's own
// iterative solvers with all operations on the GPU (Sec. 3.7).  Design here: every CG / PCG
// step is a handful of fused streaming kernels; the scalars (alpha, beta, residual norms) live
// in device memory and are produced by the last workgroup of each reduction kernel
// (deterministic: partial sums per workgroup, then a fixed-order tree over the partials), so the
// host never waits inside an iteration.  Convergence is decided on the device; the host polls a
// flag every few iterations.
#include <type_traits>

#include "batch.hpp"
#include "kernels_common.hpp"
#include "solver_state.hpp"

namespace mfq {

namespace {

constexpr int kVBlock = 256;
constexpr int kMaxRedBlocks = 1024;  // partial-sum slots (fixed grid => deterministic sums)

inline int vgrid(int64_t n) {
  int64_t g = (n + kVBlock * 4 - 1) / (kVBlock * 4);
  if (g > kMaxRedBlocks) g = kMaxRedBlocks;
  if (g < 1) g = 1;
  return (int)g;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum (fixed order); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kVBlock / 64; ++k) s += sh[k];
  __syncthreads();
  return s;
}

// Stores this block's partial; returns true in the (single) last block to finish, where
// `total` then holds the fixed-order sum of all partials (valid in thread 0).
__device__ bool grid_reduce(double part, double* partials, unsigned* counter, double& total, double* sh) {
  __shared__ bool last;
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = part;
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double v = 0;
  for (int k = threadIdx.x; k < (int)gridDim.x; k += kVBlock) v += __hip_atomic_load(partials + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  total = block_sum(v, sh);
  if (threadIdx.x == 0) *counter = 0u;
  return true;
}

template <typename Real>
__global__ __launch_bounds__(kVBlock) void fill_kernel(Real* __restrict__ x, int64_t n, Real v) {
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock) x[i] = v;
}

template <typename Real>
__global__ __launch_bounds__(kVBlock) void mask_kernel(Real* __restrict__ x, int64_t N1) {
  const int64_t n = N1 * N1 * N1;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock) {
    const int64_t I = i % N1, J = (i / N1) % N1, K = i / (N1 * N1);
    if (I == 0 || J == 0 || K == 0 || I == N1 - 1 || J == N1 - 1 || K == N1 - 1) x[i] = (Real)0;
  }
}

template <typename In, typename Out>
__global__ __launch_bounds__(kVBlock) void cast_kernel(const In* __restrict__ in, Out* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    out[i] = (Out)in[i];
}

// ---------------------------------------------------------------- CG / PCG (FP64 vectors)
// start: r = b, x = 0, p = z = r (unpreconditioned) ; bb = rr = r.r
__global__ __launch_bounds__(kVBlock) void cg_start_kernel(const double* __restrict__ b, double* __restrict__ x,
                                                           double* __restrict__ r, double* __restrict__ p, int64_t n,
                                                           SolverState* st, int copy_p, double tol2) {
  __shared__ double sh[kVBlock / 64];
  double part = 0;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock) {
    const double v = b[i];
    r[i] = v;
    x[i] = 0.0;
    if (copy_p) p[i] = v;
    part += v * v;
  }
  part = block_sum(part, sh);
  double tot;
  if (grid_reduce(part, st->partials, &st->counter, tot, sh) && threadIdx.x == 0) {
    st->bb = tot;
    st->tol2 = tol2;
    st->rr = tot;
    st->rz = tot;
    st->iter = 0;
    st->done = (tot == 0.0) ? 1 : 0;
    st->converged_iter = 0;
    st->nonfinite = (tot == tot && tot < 1e308) ? 0 : 1;
    if (st->nonfinite) st->done = 1;
  }
}

// pAp = p.Ap ; alpha = rz / pAp
__global__ __launch_bounds__(kVBlock) void cg_alpha_kernel(const double* __restrict__ p, const double* __restrict__ Ap,
                                                           int64_t n, SolverState* st) {
  __shared__ double sh[kVBlock / 64];
  if (st->done) return;
  double part = 0;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    part += p[i] * Ap[i];
  part = block_sum(part, sh);
  double tot;
  if (grid_reduce(part, st->partials, &st->counter, tot, sh) && threadIdx.x == 0) {
    st->pAp = tot;
    st->alpha = (tot != 0.0) ? st->rz / tot : 0.0;
  }
}

// x += alpha p ; r -= alpha Ap ; rr = r.r ; convergence test rr <= tol2 * bb.
// Unpreconditioned (z = r): also beta = rr_new / rr_old, rz = rr_new.  r32 (optional): the new
// residual rounded to FP32 as well, the right-hand side of an FP32 V-cycle.
__global__ __launch_bounds__(kVBlock) void cg_update_kernel(double* __restrict__ x, double* __restrict__ r,
                                                            const double* __restrict__ p, const double* __restrict__ Ap,
                                                            int64_t n, SolverState* st, int unpreconditioned,
                                                            float* __restrict__ r32) {
  __shared__ double sh[kVBlock / 64];
  if (st->done) return;
  const double alpha = st->alpha;
  double part = 0;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock) {
    x[i] += alpha * p[i];
    const double v = r[i] - alpha * Ap[i];
    r[i] = v;
    if (r32) r32[i] = (float)v;
    part += v * v;
  }
  part = block_sum(part, sh);
  double tot;
  if (grid_reduce(part, st->partials, &st->counter, tot, sh) && threadIdx.x == 0) {
    st->rr = tot;
    st->iter += 1;
    if (!(tot == tot) || tot > 1e308) {
      st->nonfinite = 1;
      st->done = 1;
    } else if (tot <= st->tol2 * st->bb) {
      st->done = 1;
      st->converged_iter = st->iter;
    }
    if (unpreconditioned) {
      st->beta = (st->rz != 0.0) ? tot / st->rz : 0.0;
      st->rz = tot;
    }
  }
}

// rz_new = r.z ; beta = rz_new / rz (z in FP64, or the FP32 V-cycle's result widened on the fly:
// the same values as its FP64 copy)
template <typename ZT>
__global__ __launch_bounds__(kVBlock) void cg_beta_kernel(const double* __restrict__ r, const ZT* __restrict__ z,
                                                          int64_t n, SolverState* st) {
  __shared__ double sh[kVBlock / 64];
  if (st->done) return;
  double part = 0;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    part += r[i] * (double)z[i];
  part = block_sum(part, sh);
  double tot;
  if (grid_reduce(part, st->partials, &st->counter, tot, sh) && threadIdx.x == 0) {
    st->beta = (st->rz != 0.0) ? tot / st->rz : 0.0;
    st->rz = tot;
  }
}

// p = z + beta p; the first direction is p = z, without reading p (which holds no value yet)
template <typename ZT>
__global__ __launch_bounds__(kVBlock) void cg_direction_kernel(const ZT* __restrict__ z, double* __restrict__ p,
                                                               int64_t n, SolverState* st, int first) {
  if (st->done) return;
  const double beta = st->beta;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    p[i] = first ? (double)z[i] : (double)z[i] + beta * p[i];
}

// r = b - t (true residual), rr = r.r ; used by iterative refinement and final certificates.
__global__ __launch_bounds__(kVBlock) void residual_norm_kernel(const double* __restrict__ b, const double* __restrict__ t,
                                                                double* __restrict__ r, int64_t n, SolverState* st,
                                                                double* out) {
  __shared__ double sh[kVBlock / 64];
  double part = 0;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock) {
    const double v = b[i] - t[i];
    if (r) r[i] = v;
    part += v * v;
  }
  part = block_sum(part, sh);
  double tot;
  if (grid_reduce(part, st->partials, &st->counter, tot, sh) && threadIdx.x == 0) *out = tot;
}

// x += c
template <typename Real, typename Cor>
__global__ __launch_bounds__(kVBlock) void add_kernel(Real* __restrict__ x, const Cor* __restrict__ c, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    x[i] += (Real)c[i];
}

// ---------------------------------------------------------------- Chebyshev smoother
// first step: r = b - t (t = A x, or r = b when x = 0), d = dinv r / theta, x (+)= d
template <typename Real>
__global__ __launch_bounds__(kVBlock) void cheb_first_kernel(const Real* __restrict__ b, const Real* __restrict__ t,
                                                             const Real* __restrict__ dinv, Real* __restrict__ x,
                                                             Real* __restrict__ r, Real* __restrict__ d, int64_t n,
                                                             Real inv_theta, int x_is_zero) {
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock) {
    Real rv, dv, xv = x_is_zero ? (Real)0 : x[i];
    cheb_first_entry<Real>(b[i], x_is_zero ? (Real)0 : t[i], dinv[i], inv_theta, x_is_zero != 0, rv, dv, xv);
    r[i] = rv;
    d[i] = dv;
    x[i] = xv;
  }
}

// r -= Ad ; d = c1 d + c2 dinv r ; x += d
template <typename Real>
__global__ __launch_bounds__(kVBlock) void cheb_step_kernel(const Real* __restrict__ Ad, const Real* __restrict__ dinv,
                                                            Real* __restrict__ x, Real* __restrict__ r,
                                                            Real* __restrict__ d, int64_t n, Real c1, Real c2) {
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock) {
    Real rv = r[i], dv = d[i], xv = x[i];
    cheb_step_entry<Real>(Ad[i], dinv[i], c1, c2, rv, dv, xv);
    r[i] = rv;
    d[i] = dv;
    x[i] = xv;
  }
}

// r = b - t
template <typename Real>
__global__ __launch_bounds__(kVBlock) void sub_kernel(const Real* __restrict__ b, const Real* __restrict__ t,
                                                      Real* __restrict__ r, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    r[i] = b[i] - t[i];
}

// coarse solve on the free (interior) lattice nodes: x_f = Ainv b_f, FP64 accumulation, one wave
// per row.  Free index f <-> node (I,J,K) = (f%m+1, (f/m)%m+1, f/m^2+1), m = N1-2.
__device__ __forceinline__ int64_t free_to_global(int64_t f, int64_t N1) {
  const int64_t m = N1 - 2;
  return (f % m + 1) + N1 * ((f / m) % m + 1) + N1 * N1 * (f / (m * m) + 1);
}

template <typename Real>
__global__ __launch_bounds__(kVBlock) void dense_solve_kernel(const double* __restrict__ Ainv, int nf, int64_t N1,
                                                              const Real* __restrict__ b, Real* __restrict__ x) {
  const int wave = (blockIdx.x * kVBlock + threadIdx.x) >> 6;
  const int l = threadIdx.x & 63;
  if (wave >= nf) return;
  const double* row = Ainv + (int64_t)wave * nf;
  double s = 0;
  for (int j = l; j < nf; j += 64) s += row[j] * (double)b[free_to_global(j, N1)];
  s = wave_sum(s);
  if (l == 0) x[free_to_global(wave, N1)] = (Real)s;
}

template <typename Real>
__global__ __launch_bounds__(kVBlock) void dot_kernel(const Real* __restrict__ x, const Real* __restrict__ y, int64_t n,
                                                      SolverState* st, double* out) {
  __shared__ double sh[kVBlock / 64];
  double part = 0;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    part += (double)x[i] * (double)y[i];
  part = block_sum(part, sh);
  double tot;
  if (grid_reduce(part, st->partials, &st->counter, tot, sh) && threadIdx.x == 0) *out = tot;
}

// y = a x + b y
template <typename Real>
__global__ __launch_bounds__(kVBlock) void axpby_kernel(Real a, const Real* __restrict__ x, Real b, Real* __restrict__ y,
                                                        int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    y[i] = b == (Real)0 ? a * x[i] : a * x[i] + b * y[i];  // b = 0 never reads y
}

// z = d * r
template <typename Real>
__global__ __launch_bounds__(kVBlock) void mul_kernel(const Real* __restrict__ d, const Real* __restrict__ r,
                                                      Real* __restrict__ z, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    z[i] = d[i] * r[i];
}

// x = 1 / x
template <typename Real>
__global__ __launch_bounds__(kVBlock) void reciprocal_kernel(Real* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    x[i] = (Real)1 / x[i];
}

// Counter-based start vector: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) of counter i,
// z = seed + (i+1)*0x9E3779B97F4A7C15, two xor-shift-multiply rounds, final xor-shift; the top
// 53 bits give u in [0,1), v = 2u - 1; zero on boundary nodes of the (N1)^3 lattice when masked.
__device__ __forceinline__ double splitmix_value(int64_t i, int64_t N1, uint64_t seed, bool masked) {
  uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  const double u = (double)(z >> 11) * 0x1.0p-53;
  double v = 2.0 * u - 1.0;
  if (masked) {
    const int64_t I = i % N1, J = (i / N1) % N1, K = i / (N1 * N1);
    if (I == 0 || J == 0 || K == 0 || I == N1 - 1 || J == N1 - 1 || K == N1 - 1) v = 0.0;
  }
  return v;
}

template <typename Real>
__global__ __launch_bounds__(kVBlock) void splitmix_kernel(Real* __restrict__ x, int64_t N1, uint64_t seed, int masked) {
  const int64_t n = N1 * N1 * N1;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    x[i] = (Real)splitmix_value(i, N1, seed, masked != 0);
}

// ---------------------------------------------------------------- device-side Lanczos
// Largest-eigenvalue estimate of D^{-1} A from k steps of Jacobi-preconditioned CG (the CG
// coefficients give the Lanczos tridiagonal matrix).  Scalars stay in a SolverState (rz, alpha,
// beta, iter, done); step j records trace[2j] = alpha_j, trace[2j+1] = beta_j and the count of
// completed steps in trace[count_slot], so the host reads the whole run once at the end.
template <typename Real>
__global__ __launch_bounds__(kVBlock) void lz_init_kernel(const Real* __restrict__ r, const Real* __restrict__ dinv,
                                                          Real* __restrict__ z, Real* __restrict__ p, int64_t n,
                                                          SolverState* st, double* trace, int count_slot) {
  __shared__ double sh[kVBlock / 64];
  double part = 0;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock) {
    const Real zv = dinv[i] * r[i];
    z[i] = zv;
    p[i] = zv;
    part += (double)r[i] * (double)zv;
  }
  part = block_sum(part, sh);
  double tot;
  if (grid_reduce(part, st->partials, &st->counter, tot, sh) && threadIdx.x == 0) {
    st->rz = tot;
    st->iter = 0;
    st->done = (tot > 0) ? 0 : 1;
    trace[count_slot] = 0.0;
  }
}

template <typename Real>
__global__ __launch_bounds__(kVBlock) void lz_alpha_kernel(const Real* __restrict__ p, const Real* __restrict__ Ap,
                                                           int64_t n, SolverState* st, double* trace) {
  __shared__ double sh[kVBlock / 64];
  if (st->done) return;
  double part = 0;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    part += (double)p[i] * (double)Ap[i];
  part = block_sum(part, sh);
  double tot;
  if (grid_reduce(part, st->partials, &st->counter, tot, sh) && threadIdx.x == 0) {
    if (tot > 0) {
      st->alpha = st->rz / tot;
      trace[2 * st->iter] = st->alpha;
    } else {
      st->done = 1;
    }
  }
}

// r -= alpha Ap ; z = dinv r ; beta = r.z / rz ; rz = r.z
template <typename Real>
__global__ __launch_bounds__(kVBlock) void lz_update_kernel(Real* __restrict__ r, Real* __restrict__ z,
                                                            const Real* __restrict__ Ap, const Real* __restrict__ dinv,
                                                            int64_t n, SolverState* st, double* trace, int count_slot) {
  __shared__ double sh[kVBlock / 64];
  if (st->done) return;
  const Real alpha = (Real)st->alpha;
  double part = 0;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock) {
    const Real rv = r[i] - alpha * Ap[i];
    const Real zv = dinv[i] * rv;
    r[i] = rv;
    z[i] = zv;
    part += (double)rv * (double)zv;
  }
  part = block_sum(part, sh);
  double tot;
  if (grid_reduce(part, st->partials, &st->counter, tot, sh) && threadIdx.x == 0) {
    const double beta = tot / st->rz;
    trace[2 * st->iter + 1] = beta;
    st->beta = beta;
    st->rz = tot;
    st->iter += 1;
    trace[count_slot] = (double)st->iter;
    if (!(tot > 0)) st->done = 1;
  }
}

template <typename Real>
__global__ __launch_bounds__(kVBlock) void lz_direction_kernel(const Real* __restrict__ z, Real* __restrict__ p,
                                                               int64_t n, SolverState* st) {
  if (st->done) return;
  const Real beta = (Real)st->beta;
  for (int64_t i = blockIdx.x * (int64_t)kVBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVBlock)
    p[i] = z[i] + beta * p[i];
}

// ---------------------------------------------------------------- batched forms (serving)
// One launch covers many solves: workgroup b belongs to the item whose range [first, next first)
// holds it, and does what workgroup b - first of that item's single-solve launch does (same grid
// per item, same partial sums), so each solve's results are bitwise those it gets alone.
__device__ __forceinline__ int batch_item(const VecItem* __restrict__ it, int count, int64_t b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (it[mid].first <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// grid_reduce over the item's own workgroups (lb of nblk)
__device__ bool item_reduce(double part, SolverState* st, int lb, int nblk, double& total, double* sh) {
  __shared__ bool last;
  if (threadIdx.x == 0) {
    st->partials[lb] = part;
    __threadfence();
    const unsigned prev = atomicAdd(&st->counter, 1u);
    last = (prev == (unsigned)nblk - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double v = 0;
  for (int k = threadIdx.x; k < nblk; k += kVBlock) v += __hip_atomic_load(st->partials + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  total = block_sum(v, sh);
  if (threadIdx.x == 0) st->counter = 0u;
  return true;
}

template <int OP>
__global__ __launch_bounds__(kVBlock) void batch_vec_kernel(const VecItem* __restrict__ items, int count) {
  __shared__ double sh[kVBlock / 64];
  const VecItem& it = items[batch_item(items, count, blockIdx.x)];
  const int lb = (int)(blockIdx.x - it.first);
  const int64_t n = it.n, stride = (int64_t)it.nblk * kVBlock;
  const int64_t i0 = (int64_t)lb * kVBlock + threadIdx.x;
  SolverState* st = it.st;
  if constexpr (OP == kBatchCgAlpha) {
    if (st->done) return;
    const double* p = (const double*)it.a;
    const double* Ap = (const double*)it.b;
    double part = 0;
    for (int64_t i = i0; i < n; i += stride) part += p[i] * Ap[i];
    part = block_sum(part, sh);
    double tot;
    if (item_reduce(part, st, lb, it.nblk, tot, sh) && threadIdx.x == 0) {
      st->pAp = tot;
      st->alpha = (tot != 0.0) ? st->rz / tot : 0.0;
    }
  } else if constexpr (OP == kBatchCgUpdate) {
    if (st->done) return;
    double* x = (double*)it.d;
    double* r = (double*)it.e;
    const double* p = (const double*)it.a;
    const double* Ap = (const double*)it.b;
    const double alpha = st->alpha;
    double part = 0;
    float* r32 = (float*)it.f;
    for (int64_t i = i0; i < n; i += stride) {
      x[i] += alpha * p[i];
      const double v = r[i] - alpha * Ap[i];
      r[i] = v;
      if (r32) r32[i] = (float)v;
      part += v * v;
    }
    part = block_sum(part, sh);
    double tot;
    if (item_reduce(part, st, lb, it.nblk, tot, sh) && threadIdx.x == 0) {
      st->rr = tot;
      st->iter += 1;
      if (!(tot == tot) || tot > 1e308) {
        st->nonfinite = 1;
        st->done = 1;
      } else if (tot <= st->tol2 * st->bb) {
        st->done = 1;
        st->converged_iter = st->iter;
      }
    }
  } else if constexpr (OP == kBatchCgBeta || OP == kBatchCgBeta32) {
    if (st->done) return;
    using ZT = std::conditional_t<OP == kBatchCgBeta32, float, double>;
    const double* r = (const double*)it.a;
    const ZT* z = (const ZT*)it.b;
    double part = 0;
    for (int64_t i = i0; i < n; i += stride) part += r[i] * (double)z[i];
    part = block_sum(part, sh);
    double tot;
    if (item_reduce(part, st, lb, it.nblk, tot, sh) && threadIdx.x == 0) {
      st->beta = (st->rz != 0.0) ? tot / st->rz : 0.0;
      st->rz = tot;
    }
  } else if constexpr (OP == kBatchCgDirection || OP == kBatchCgDirection32) {
    if (st->done) return;
    using ZT = std::conditional_t<OP == kBatchCgDirection32, float, double>;
    const ZT* z = (const ZT*)it.a;
    double* p = (double*)it.d;
    const double beta = st->beta;
    for (int64_t i = i0; i < n; i += stride) p[i] = it.flag ? (double)z[i] : (double)z[i] + beta * p[i];
  } else if constexpr (OP == kBatchCast64To32) {
    const double* in = (const double*)it.a;
    float* out = (float*)it.d;
    for (int64_t i = i0; i < n; i += stride) out[i] = (float)in[i];
  } else if constexpr (OP == kBatchCast32To64) {
    const float* in = (const float*)it.a;
    double* out = (double*)it.d;
    for (int64_t i = i0; i < n; i += stride) out[i] = (double)in[i];
  } else if constexpr (OP == kBatchChebFirst) {
    const float* b = (const float*)it.a;
    const float* t = (const float*)it.b;
    const float* dinv = (const float*)it.c;
    float* x = (float*)it.d;
    float* r = (float*)it.e;
    float* d = (float*)it.f;
    const float inv_theta = (float)it.s0;
    for (int64_t i = i0; i < n; i += stride) {
      float rv, dv, xv = it.flag ? 0.0f : x[i];
      cheb_first_entry<float>(b[i], it.flag ? 0.0f : t[i], dinv[i], inv_theta, it.flag != 0, rv, dv, xv);
      r[i] = rv;
      d[i] = dv;
      x[i] = xv;
    }
  } else if constexpr (OP == kBatchChebStep) {
    const float* Ad = (const float*)it.a;
    const float* dinv = (const float*)it.c;
    float* x = (float*)it.d;
    float* r = (float*)it.e;
    float* d = (float*)it.f;
    const float c1 = (float)it.s0, c2 = (float)it.s1;
    for (int64_t i = i0; i < n; i += stride) {
      float rv = r[i], dv = d[i], xv = x[i];
      cheb_step_entry<float>(Ad[i], dinv[i], c1, c2, rv, dv, xv);
      r[i] = rv;
      d[i] = dv;
      x[i] = xv;
    }
  } else if constexpr (OP == kBatchSub) {
    const float* b = (const float*)it.a;
    const float* t = (const float*)it.b;
    float* r = (float*)it.d;
    for (int64_t i = i0; i < n; i += stride) r[i] = b[i] - t[i];
  } else if constexpr (OP == kBatchAdd) {
    float* x = (float*)it.d;
    const float* c = (const float*)it.a;
    for (int64_t i = i0; i < n; i += stride) x[i] += c[i];
  } else if constexpr (OP == kBatchFill) {
    float* x = (float*)it.d;
    const float v = (float)it.s0;
    for (int64_t i = i0; i < n; i += stride) x[i] = v;
  } else if constexpr (OP == kBatchCopy64) {
    const double* in = (const double*)it.a;
    double* out = (double*)it.d;
    for (int64_t i = i0; i < n; i += stride) out[i] = in[i];
  } else if constexpr (OP == kBatchCgStart) {
    const double* b = (const double*)it.a;
    double* x = (double*)it.d;
    double* r = (double*)it.e;
    double* p = (double*)it.f;
    double part = 0;
    for (int64_t i = i0; i < n; i += stride) {
      const double v = b[i];
      r[i] = v;
      x[i] = 0.0;
      if (it.flag) p[i] = v;
      part += v * v;
    }
    part = block_sum(part, sh);
    double tot;
    if (item_reduce(part, st, lb, it.nblk, tot, sh) && threadIdx.x == 0) {
      st->bb = tot;
      st->tol2 = it.s0;
      st->rr = tot;
      st->rz = tot;
      st->iter = 0;
      st->done = (tot == 0.0) ? 1 : 0;
      st->converged_iter = 0;
      st->nonfinite = (tot == tot && tot < 1e308) ? 0 : 1;
      if (st->nonfinite) st->done = 1;
    }
  } else if constexpr (OP == kBatchSplitmix) {
    float* x = (float*)it.d;
    const int64_t N1 = it.flag;
    for (int64_t i = i0; i < n; i += stride) x[i] = (float)splitmix_value(i, N1, 0, true);
  } else if constexpr (OP == kBatchLzInit) {
    const float* r = (const float*)it.a;
    const float* dinv = (const float*)it.c;
    float* z = (float*)it.d;
    float* p = (float*)it.e;
    double* trace = (double*)it.b;
    double part = 0;
    for (int64_t i = i0; i < n; i += stride) {
      const float zv = dinv[i] * r[i];
      z[i] = zv;
      p[i] = zv;
      part += (double)r[i] * (double)zv;
    }
    part = block_sum(part, sh);
    double tot;
    if (item_reduce(part, st, lb, it.nblk, tot, sh) && threadIdx.x == 0) {
      st->rz = tot;
      st->iter = 0;
      st->done = (tot > 0) ? 0 : 1;
      trace[it.flag] = 0.0;
    }
  } else if constexpr (OP == kBatchLzAlpha) {
    if (st->done) return;
    const float* p = (const float*)it.a;
    const float* Ap = (const float*)it.c;
    double* trace = (double*)it.b;
    double part = 0;
    for (int64_t i = i0; i < n; i += stride) part += (double)p[i] * (double)Ap[i];
    part = block_sum(part, sh);
    double tot;
    if (item_reduce(part, st, lb, it.nblk, tot, sh) && threadIdx.x == 0) {
      if (tot > 0) {
        st->alpha = st->rz / tot;
        trace[2 * st->iter] = st->alpha;
      } else {
        st->done = 1;
      }
    }
  } else if constexpr (OP == kBatchLzUpdate) {
    if (st->done) return;
    float* r = (float*)it.d;
    float* z = (float*)it.e;
    const float* Ap = (const float*)it.a;
    const float* dinv = (const float*)it.c;
    double* trace = (double*)it.b;
    const float alpha = (float)st->alpha;
    double part = 0;
    for (int64_t i = i0; i < n; i += stride) {
      const float rv = r[i] - alpha * Ap[i];
      const float zv = dinv[i] * rv;
      r[i] = rv;
      z[i] = zv;
      part += (double)rv * (double)zv;
    }
    part = block_sum(part, sh);
    double tot;
    if (item_reduce(part, st, lb, it.nblk, tot, sh) && threadIdx.x == 0) {
      const double beta = tot / st->rz;
      trace[2 * st->iter + 1] = beta;
      st->beta = beta;
      st->rz = tot;
      st->iter += 1;
      trace[it.flag] = (double)st->iter;
      if (!(tot > 0)) st->done = 1;
    }
  } else if constexpr (OP == kBatchLzDirection) {
    if (st->done) return;
    const float* z = (const float*)it.a;
    float* p = (float*)it.d;
    const float beta = (float)st->beta;
    for (int64_t i = i0; i < n; i += stride) p[i] = z[i] + beta * p[i];
  } else if constexpr (OP == kBatchAdd64) {
    double* x = (double*)it.d;
    const double* c = (const double*)it.a;
    for (int64_t i = i0; i < n; i += stride) x[i] += c[i];
  } else if constexpr (OP == kBatchResidualNorm) {
    const double* b = (const double*)it.a;
    const double* t = (const double*)it.b;
    double* r = (double*)it.d;
    double part = 0;
    for (int64_t i = i0; i < n; i += stride) {
      const double v = b[i] - t[i];
      r[i] = v;
      part += v * v;
    }
    part = block_sum(part, sh);
    double tot;
    if (item_reduce(part, st, lb, it.nblk, tot, sh) && threadIdx.x == 0) *(double*)it.e = tot;
  }
}

}  // namespace

hipError_t launch_fill(int precision, void* x, int64_t n, double value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int g = vgrid(n) * 4;
  if (precision == MFQ_FP64)
    fill_kernel<double><<<g, kVBlock, 0, st>>>((double*)x, n, value);
  else
    fill_kernel<float><<<g, kVBlock, 0, st>>>((float*)x, n, (float)value);
  return hipGetLastError();
}

hipError_t launch_mask(int precision, int p, int n, void* x, hipStream_t st) {
  const int64_t N1 = (int64_t)p * n + 1;
  const int g = vgrid(N1 * N1 * N1) * 4;
  if (precision == MFQ_FP64)
    mask_kernel<double><<<g, kVBlock, 0, st>>>((double*)x, N1);
  else
    mask_kernel<float><<<g, kVBlock, 0, st>>>((float*)x, N1);
  return hipGetLastError();
}

hipError_t launch_cast(int from, const void* in, int to, void* out, int64_t n, hipStream_t st) {
  const int g = vgrid(n) * 4;
  if (from == MFQ_FP64 && to == MFQ_FP32)
    cast_kernel<double, float><<<g, kVBlock, 0, st>>>((const double*)in, (float*)out, n);
  else if (from == MFQ_FP32 && to == MFQ_FP64)
    cast_kernel<float, double><<<g, kVBlock, 0, st>>>((const float*)in, (double*)out, n);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_cg_start(const double* b, double* x, double* r, double* p, int64_t n, SolverState* s, bool copy_p,
                           double tol2, hipStream_t st) {
  cg_start_kernel<<<vgrid(n), kVBlock, 0, st>>>(b, x, r, p, n, s, copy_p ? 1 : 0, tol2);
  return hipGetLastError();
}
hipError_t launch_cg_alpha(const double* p, const double* Ap, int64_t n, SolverState* s, hipStream_t st) {
  cg_alpha_kernel<<<vgrid(n), kVBlock, 0, st>>>(p, Ap, n, s);
  return hipGetLastError();
}
hipError_t launch_cg_update(double* x, double* r, const double* p, const double* Ap, int64_t n, SolverState* s,
                            bool unprec, hipStream_t st) {
  cg_update_kernel<<<vgrid(n), kVBlock, 0, st>>>(x, r, p, Ap, n, s, unprec ? 1 : 0, nullptr);
  return hipGetLastError();
}
hipError_t launch_cg_update_cast(double* x, double* r, const double* p, const double* Ap, float* r32, int64_t n,
                                 SolverState* s, hipStream_t st) {
  cg_update_kernel<<<vgrid(n), kVBlock, 0, st>>>(x, r, p, Ap, n, s, 0, r32);
  return hipGetLastError();
}
hipError_t launch_cg_beta(const double* r, const double* z, int64_t n, SolverState* s, hipStream_t st) {
  cg_beta_kernel<double><<<vgrid(n), kVBlock, 0, st>>>(r, z, n, s);
  return hipGetLastError();
}
hipError_t launch_cg_beta32(const double* r, const float* z, int64_t n, SolverState* s, hipStream_t st) {
  cg_beta_kernel<float><<<vgrid(n), kVBlock, 0, st>>>(r, z, n, s);
  return hipGetLastError();
}
hipError_t launch_cg_direction(const double* z, double* p, int64_t n, SolverState* s, bool first, hipStream_t st) {
  cg_direction_kernel<double><<<vgrid(n) * 4, kVBlock, 0, st>>>(z, p, n, s, first ? 1 : 0);
  return hipGetLastError();
}
hipError_t launch_cg_direction32(const float* z, double* p, int64_t n, SolverState* s, bool first, hipStream_t st) {
  cg_direction_kernel<float><<<vgrid(n) * 4, kVBlock, 0, st>>>(z, p, n, s, first ? 1 : 0);
  return hipGetLastError();
}
hipError_t launch_residual_norm(const double* b, const double* t, double* r, int64_t n, SolverState* s, double* out,
                                hipStream_t st) {
  residual_norm_kernel<<<vgrid(n), kVBlock, 0, st>>>(b, t, r, n, s, out);
  return hipGetLastError();
}
hipError_t launch_add(int precision, void* x, int cor_precision, const void* c, int64_t n, hipStream_t st) {
  const int g = vgrid(n) * 4;
  if (precision == MFQ_FP64 && cor_precision == MFQ_FP64)
    add_kernel<double, double><<<g, kVBlock, 0, st>>>((double*)x, (const double*)c, n);
  else if (precision == MFQ_FP64 && cor_precision == MFQ_FP32)
    add_kernel<double, float><<<g, kVBlock, 0, st>>>((double*)x, (const float*)c, n);
  else if (precision == MFQ_FP32 && cor_precision == MFQ_FP32)
    add_kernel<float, float><<<g, kVBlock, 0, st>>>((float*)x, (const float*)c, n);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_cheb_first(int precision, const void* b, const void* t, const void* dinv, void* x, void* r, void* d,
                             int64_t n, double inv_theta, bool x_is_zero, hipStream_t st) {
  const int g = vgrid(n) * 4;
  if (precision == MFQ_FP64)
    cheb_first_kernel<double><<<g, kVBlock, 0, st>>>((const double*)b, (const double*)t, (const double*)dinv, (double*)x,
                                                     (double*)r, (double*)d, n, inv_theta, x_is_zero ? 1 : 0);
  else
    cheb_first_kernel<float><<<g, kVBlock, 0, st>>>((const float*)b, (const float*)t, (const float*)dinv, (float*)x,
                                                    (float*)r, (float*)d, n, (float)inv_theta, x_is_zero ? 1 : 0);
  return hipGetLastError();
}
hipError_t launch_cheb_step(int precision, const void* Ad, const void* dinv, void* x, void* r, void* d, int64_t n,
                            double c1, double c2, hipStream_t st) {
  const int g = vgrid(n) * 4;
  if (precision == MFQ_FP64)
    cheb_step_kernel<double><<<g, kVBlock, 0, st>>>((const double*)Ad, (const double*)dinv, (double*)x, (double*)r,
                                                    (double*)d, n, c1, c2);
  else
    cheb_step_kernel<float><<<g, kVBlock, 0, st>>>((const float*)Ad, (const float*)dinv, (float*)x, (float*)r,
                                                   (float*)d, n, (float)c1, (float)c2);
  return hipGetLastError();
}
hipError_t launch_sub(int precision, const void* b, const void* t, void* r, int64_t n, hipStream_t st) {
  const int g = vgrid(n) * 4;
  if (precision == MFQ_FP64)
    sub_kernel<double><<<g, kVBlock, 0, st>>>((const double*)b, (const double*)t, (double*)r, n);
  else
    sub_kernel<float><<<g, kVBlock, 0, st>>>((const float*)b, (const float*)t, (float*)r, n);
  return hipGetLastError();
}
hipError_t launch_dense_solve(int precision, const double* Ainv, int nf, int64_t N1, const void* b, void* x,
                              hipStream_t st) {
  const int g = (int)(((int64_t)nf * 64 + kVBlock - 1) / kVBlock);
  if (precision == MFQ_FP64)
    dense_solve_kernel<double><<<g, kVBlock, 0, st>>>(Ainv, nf, N1, (const double*)b, (double*)x);
  else
    dense_solve_kernel<float><<<g, kVBlock, 0, st>>>(Ainv, nf, N1, (const float*)b, (float*)x);
  return hipGetLastError();
}
hipError_t launch_dot(int precision, const void* x, const void* y, int64_t n, SolverState* s, double* out,
                      hipStream_t st) {
  if (precision == MFQ_FP64)
    dot_kernel<double><<<vgrid(n), kVBlock, 0, st>>>((const double*)x, (const double*)y, n, s, out);
  else
    dot_kernel<float><<<vgrid(n), kVBlock, 0, st>>>((const float*)x, (const float*)y, n, s, out);
  return hipGetLastError();
}
hipError_t launch_axpby(int precision, double a, const void* x, double b, void* y, int64_t n, hipStream_t st) {
  const int g = vgrid(n) * 4;
  if (precision == MFQ_FP64)
    axpby_kernel<double><<<g, kVBlock, 0, st>>>(a, (const double*)x, b, (double*)y, n);
  else
    axpby_kernel<float><<<g, kVBlock, 0, st>>>((float)a, (const float*)x, (float)b, (float*)y, n);
  return hipGetLastError();
}
hipError_t launch_mul(int precision, const void* d, const void* r, void* z, int64_t n, hipStream_t st) {
  const int g = vgrid(n) * 4;
  if (precision == MFQ_FP64)
    mul_kernel<double><<<g, kVBlock, 0, st>>>((const double*)d, (const double*)r, (double*)z, n);
  else
    mul_kernel<float><<<g, kVBlock, 0, st>>>((const float*)d, (const float*)r, (float*)z, n);
  return hipGetLastError();
}
hipError_t launch_reciprocal(int precision, void* x, int64_t n, hipStream_t st) {
  const int g = vgrid(n) * 4;
  if (precision == MFQ_FP64)
    reciprocal_kernel<double><<<g, kVBlock, 0, st>>>((double*)x, n);
  else
    reciprocal_kernel<float><<<g, kVBlock, 0, st>>>((float*)x, n);
  return hipGetLastError();
}
hipError_t launch_lz_init(int precision, const void* r, const void* dinv, void* z, void* p, int64_t n, SolverState* s,
                          double* trace, int count_slot, hipStream_t st) {
  if (precision == MFQ_FP64)
    lz_init_kernel<double><<<vgrid(n), kVBlock, 0, st>>>((const double*)r, (const double*)dinv, (double*)z, (double*)p,
                                                         n, s, trace, count_slot);
  else
    lz_init_kernel<float><<<vgrid(n), kVBlock, 0, st>>>((const float*)r, (const float*)dinv, (float*)z, (float*)p, n,
                                                        s, trace, count_slot);
  return hipGetLastError();
}
hipError_t launch_lz_alpha(int precision, const void* p, const void* Ap, int64_t n, SolverState* s, double* trace,
                           hipStream_t st) {
  if (precision == MFQ_FP64)
    lz_alpha_kernel<double><<<vgrid(n), kVBlock, 0, st>>>((const double*)p, (const double*)Ap, n, s, trace);
  else
    lz_alpha_kernel<float><<<vgrid(n), kVBlock, 0, st>>>((const float*)p, (const float*)Ap, n, s, trace);
  return hipGetLastError();
}
hipError_t launch_lz_update(int precision, void* r, void* z, const void* Ap, const void* dinv, int64_t n,
                            SolverState* s, double* trace, int count_slot, hipStream_t st) {
  if (precision == MFQ_FP64)
    lz_update_kernel<double><<<vgrid(n), kVBlock, 0, st>>>((double*)r, (double*)z, (const double*)Ap,
                                                           (const double*)dinv, n, s, trace, count_slot);
  else
    lz_update_kernel<float><<<vgrid(n), kVBlock, 0, st>>>((float*)r, (float*)z, (const float*)Ap, (const float*)dinv, n,
                                                          s, trace, count_slot);
  return hipGetLastError();
}
hipError_t launch_lz_direction(int precision, const void* z, void* p, int64_t n, SolverState* s, hipStream_t st) {
  if (precision == MFQ_FP64)
    lz_direction_kernel<double><<<vgrid(n) * 4, kVBlock, 0, st>>>((const double*)z, (double*)p, n, s);
  else
    lz_direction_kernel<float><<<vgrid(n) * 4, kVBlock, 0, st>>>((const float*)z, (float*)p, n, s);
  return hipGetLastError();
}

hipError_t launch_splitmix(int precision, void* x, int64_t N1, uint64_t seed, bool masked, hipStream_t st) {
  const int g = vgrid(N1 * N1 * N1) * 4;
  if (precision == MFQ_FP64)
    splitmix_kernel<double><<<g, kVBlock, 0, st>>>((double*)x, N1, seed, masked ? 1 : 0);
  else
    splitmix_kernel<float><<<g, kVBlock, 0, st>>>((float*)x, N1, seed, masked ? 1 : 0);
  return hipGetLastError();
}

int vec_blocks(BatchVecOp op, int64_t n) {
  switch (op) {
    case kBatchCgAlpha:
    case kBatchCgUpdate:
    case kBatchCgBeta:
    case kBatchCgBeta32:
    case kBatchCgStart:
    case kBatchLzInit:
    case kBatchLzAlpha:
    case kBatchLzUpdate:
    case kBatchResidualNorm:
      return vgrid(n);      // reductions: the single-solve grid, so the partial sums agree
    default:
      return vgrid(n) * 4;  // elementwise
  }
}

hipError_t launch_batch_vec(BatchVecOp op, const VecItem* items, int count, int64_t blocks, hipStream_t st) {
  if (count <= 0 || blocks <= 0) return hipSuccess;
  const unsigned g = (unsigned)blocks;
  switch (op) {
    case kBatchCgAlpha: batch_vec_kernel<kBatchCgAlpha><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchCgUpdate: batch_vec_kernel<kBatchCgUpdate><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchCgBeta: batch_vec_kernel<kBatchCgBeta><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchCgDirection: batch_vec_kernel<kBatchCgDirection><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchCast64To32: batch_vec_kernel<kBatchCast64To32><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchCast32To64: batch_vec_kernel<kBatchCast32To64><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchChebFirst: batch_vec_kernel<kBatchChebFirst><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchChebStep: batch_vec_kernel<kBatchChebStep><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchSub: batch_vec_kernel<kBatchSub><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchAdd: batch_vec_kernel<kBatchAdd><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchFill: batch_vec_kernel<kBatchFill><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchCopy64: batch_vec_kernel<kBatchCopy64><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchCgStart: batch_vec_kernel<kBatchCgStart><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchSplitmix: batch_vec_kernel<kBatchSplitmix><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchLzInit: batch_vec_kernel<kBatchLzInit><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchLzAlpha: batch_vec_kernel<kBatchLzAlpha><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchLzUpdate: batch_vec_kernel<kBatchLzUpdate><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchLzDirection: batch_vec_kernel<kBatchLzDirection><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchAdd64: batch_vec_kernel<kBatchAdd64><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchResidualNorm: batch_vec_kernel<kBatchResidualNorm><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchCgBeta32: batch_vec_kernel<kBatchCgBeta32><<<g, kVBlock, 0, st>>>(items, count); break;
    case kBatchCgDirection32: batch_vec_kernel<kBatchCgDirection32><<<g, kVBlock, 0, st>>>(items, count); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mfq
