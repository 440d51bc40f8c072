// Solvers: CG, and CG preconditioned by a geometric-multigrid V-cycle (Sec. 3.5) with Chebyshev
// smoothing, matrix-free level operators and transfers, in FP64 or in FP32 under an FP64
// outer iteration (Sec. 6.1: single-precision V-cycle combined with a double-precision
// correction).  Host code only orchestrates launches; every vector operation runs on the device.
#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "mfq_internal.hpp"
#include "solver_state.hpp"

using namespace mfq;

namespace {

constexpr int64_t kDenseCoarseLimit = 4096;

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
size_t rsize(int prec) { return prec == MFQ_FP64 ? 8 : 4; }
int64_t n_free(int p, int n) {
  const int64_t m = (int64_t)p * n - 1;
  return m > 0 ? m * m * m : 0;
}

struct Level {
  mfq_mesh* mesh = nullptr;      // owned (nullptr for the finest level: the user's)
  mfq_space* space = nullptr;    // owned (nullptr for the finest level)
  const mfq_space* sp = nullptr; // the level's space
  mfq_op* op = nullptr;          // owned V-cycle operator (precision prec_v); finest FP64 kind: user op
  bool owns_op = true;
  mfq_transfer* to_fine = nullptr;  // owned, coarse->next finer (nullptr on finest)
  int64_t n = 0;
  // offsets / pointers of level vectors (precision prec_v)
  size_t off_op = 0, off_b = 0, off_x = 0, off_r = 0, off_d = 0, off_t = 0, off_dinv = 0;
  void *b = nullptr, *x = nullptr, *r = nullptr, *d = nullptr, *t = nullptr, *dinv = nullptr;
  double lhat = 0, lmin = 0, lmax = 0;
};

}  // namespace

struct mfq_solver {
  const mfq_op* op64 = nullptr;
  int kind = 0;
  mfq_solver_params prm{};
  int prec_v = MFQ_FP64;
  std::vector<Level> lv;  // coarsest first; empty for plain CG
  // coarse level solver (FP64)
  bool dense = false;
  int64_t nf = 0;
  mfq_op* coarse64 = nullptr;  // FP64 operator of the coarsest level (dense assembly or coarse CG)
  size_t off_coarse64 = 0, off_ainv = 0, off_cvec = 0, off_cstate = 0;
  double* ainv = nullptr;
  double *cb = nullptr, *cx = nullptr, *cr = nullptr, *cp = nullptr, *cAp = nullptr, *cz = nullptr, *cdinv = nullptr;
  SolverState* cstate = nullptr;
  // Krylov vectors (FP64, finest)
  size_t off_kry = 0, off_state = 0, off_aux = 0;
  double *r = nullptr, *p = nullptr, *Ap = nullptr, *z = nullptr, *rout = nullptr, *c = nullptr;
  SolverState* state = nullptr;
  SolverState* aux = nullptr;  // reductions of the setup phase
  size_t off_lz = 0;            // one state per level for the batched eigenvalue estimates
  SolverState* lz = nullptr;
  bool eig_pending = false;     // bound lazily: the eigenvalue bounds are estimated at the first step
  double* scal = nullptr;      // device scalars for setup dots
  size_t bytes = 0;
  void* buf = nullptr;
  // resumable solve (mfq_solve_begin / mfq_batch_step / mfq_solve_end)
  struct HostStatus {
    SolverState head;  // copy of the device state up to (excluding) the reduction partials
    double cert;       // ||b - A x||^2 of the last residual check
  };
  HostStatus* hstat = nullptr;  // pinned host memory
  struct Run {
    enum Phase { kIdle, kStart, kInner, kCheck, kDone };
    Phase phase = kIdle;
    const double* start_rhs = nullptr;  // the CG pass that the next step starts (phase kStart)
    double* start_sol = nullptr;
    double start_tol2 = 0;
    const double* b = nullptr;
    double* x = nullptr;
    double* sol = nullptr;      // solution vector of the current CG pass (x or the correction c)
    double rtol = 0;
    int max_iter = 0;
    hipStream_t st = nullptr;
    int pass = 0;               // CG passes started
    int iters = 0;              // iterations of finished passes
    int enqueued = 0, budget = 0;  // iterations enqueued / allowed in the current pass
    double bb = -1, rr = 0;
    int status = MFQ_OK;
    std::chrono::steady_clock::time_point t0;
    double seconds = 0;
  } run;
  // one CG iteration captured as a HIP graph per (stream, solution vector): a step replays it
  // instead of issuing the iteration's ~100-200 kernel launches one by one
  struct IterGraph {
    hipStream_t st = nullptr;
    double* sol = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  IterGraph graphs[2];
  int next_graph = 0;
  hipEvent_t step_event = nullptr;  // completion of the last asynchronous step
  bool step_pending = false;
  // Lanczos traces of the eigenvalue estimates (device region in the buffer, pinned host copy)
  size_t off_trace = 0;
  double* trace = nullptr;
  double* trace_host = nullptr;
  int trace_stride = 0;  // doubles per level: 2 * lanczos_iters coefficients + the step count
  ~mfq_solver() {
    if (step_event) (void)hipEventDestroy(step_event);
    if (trace_host) (void)hipHostFree(trace_host);
    for (IterGraph& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (hstat) (void)hipHostFree(hstat);
    for (Level& l : lv) {
      if (l.owns_op) mfq_op_destroy(l.op);
      mfq_transfer_destroy(l.to_fine);
      mfq_space_destroy(l.space);
      mfq_mesh_destroy(l.mesh);
    }
    mfq_op_destroy(coarse64);
  }
};

namespace {

// Dense SPD inverse on the host: Cholesky A = L L^T, then A^{-1} = L^{-T} L^{-1}.
// Rows of the triangular inverse are independent, so that step runs on several threads.
bool spd_inverse(std::vector<double>& A, int64_t n) {
  for (int64_t j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int64_t k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0)) return false;
    const double ljj = std::sqrt(d);
    A[j * n + j] = ljj;
    const double inv = 1.0 / ljj;
    auto work = [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i) {
        double s = A[i * n + j];
        const double* ai = &A[i * n];
        const double* aj = &A[j * n];
        for (int64_t k = 0; k < j; ++k) s -= ai[k] * aj[k];
        A[i * n + j] = s * inv;
      }
    };
    const int64_t rows = n - j - 1;
    const int nt = rows > 256 ? (int)std::min<unsigned>(8u, std::max(1u, std::thread::hardware_concurrency())) : 1;
    if (nt == 1) {
      work(j + 1, n);
    } else {
      std::vector<std::thread> th;
      const int64_t chunk = (rows + nt - 1) / nt;
      for (int t = 0; t < nt; ++t) {
        const int64_t a = j + 1 + t * chunk, b = std::min(n, a + chunk);
        if (a < b) th.emplace_back(work, a, b);
      }
      for (auto& x : th) x.join();
    }
  }
  // W = L^{-1} (lower triangular), by forward substitution per column
  std::vector<double> W((size_t)n * n, 0.0);
  auto inv_cols = [&](int64_t c0, int64_t c1) {
    for (int64_t c = c0; c < c1; ++c) {
      W[c * n + c] = 1.0 / A[c * n + c];
      for (int64_t i = c + 1; i < n; ++i) {
        double s = 0;
        for (int64_t k = c; k < i; ++k) s -= A[i * n + k] * W[k * n + c];
        W[i * n + c] = s / A[i * n + i];
      }
    }
  };
  auto inv_full = [&](int64_t r0, int64_t r1) {
    // A^{-1}[i][j] = sum_{k >= max(i,j)} W[k][i] W[k][j]
    for (int64_t i = r0; i < r1; ++i)
      for (int64_t j = 0; j < n; ++j) {
        double s = 0;
        for (int64_t k = std::max(i, j); k < n; ++k) s += W[k * n + i] * W[k * n + j];
        A[i * n + j] = s;
      }
  };
  const int nt = (int)std::min<unsigned>(8u, std::max(1u, std::thread::hardware_concurrency()));
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
      const int64_t a = t * chunk, b = std::min(n, a + chunk);
      if (a >= b) continue;
      if (pass == 0)
        th.emplace_back(inv_cols, a, b);
      else
        th.emplace_back(inv_full, a, b);
    }
    for (auto& x : th) x.join();
  }
  return true;
}

// Largest eigenvalue of a small symmetric matrix (cyclic Jacobi rotations).
double sym_max_eig(std::vector<double> T, int k) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j) off += T[i * k + j] * T[i * k + j];
    if (off < 1e-30) break;
    for (int pI = 0; pI < k; ++pI)
      for (int q = pI + 1; q < k; ++q) {
        const double apq = T[pI * k + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (T[q * k + q] - T[pI * k + pI]) / (2 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
        const double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int r = 0; r < k; ++r) {
          const double arp = T[r * k + pI], arq = T[r * k + q];
          T[r * k + pI] = c * arp - s * arq;
          T[r * k + q] = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {
          const double apr = T[pI * k + r], aqr = T[q * k + r];
          T[pI * k + r] = c * apr - s * aqr;
          T[q * k + r] = s * apr + c * aqr;
        }
      }
  }
  double m = -1e300;
  for (int i = 0; i < k; ++i) m = std::max(m, T[i * k + i]);
  return m;
}

int poll(SolverState* dev, SolverState& host, hipStream_t st) {
  MFQ_HIP(hipMemcpyAsync(&host, dev, offsetof(SolverState, partials), hipMemcpyDeviceToHost, st));
  MFQ_HIP(hipStreamSynchronize(st));
  return MFQ_OK;
}

struct PcgResult {
  int iters = 0;
  bool converged = false, nonfinite = false;
  double rr = 0, bb = 0;
};

// CG / PCG on FP64 vectors from x = 0.  All scalars stay on the device.
int pcg(const Apply& apply, const Apply* prec, const double* b, double* x, double* r, double* p, double* Ap, double* z,
        int64_t n, SolverState* st, double rtol, int maxit, int check_every, hipStream_t stream, PcgResult& res) {
  MFQ_HIP(launch_cg_start(b, x, r, p, n, st, prec == nullptr, rtol * rtol, stream));
  if (prec) {
    if (int rc = (*prec)(r, z)) return rc;
    MFQ_HIP(launch_cg_beta(r, z, n, st, stream));
    MFQ_HIP(launch_cg_direction(z, p, n, st, true, stream));
  }
  SolverState h{};
  if (int rc = poll(st, h, stream)) return rc;
  if (!h.done) {
    for (int it = 0; it < maxit; ++it) {
      if (int rc = apply(p, Ap)) return rc;
      MFQ_HIP(launch_cg_alpha(p, Ap, n, st, stream));
      MFQ_HIP(launch_cg_update(x, r, p, Ap, n, st, prec == nullptr, stream));
      if (prec) {
        if (int rc = (*prec)(r, z)) return rc;
        MFQ_HIP(launch_cg_beta(r, z, n, st, stream));
        MFQ_HIP(launch_cg_direction(z, p, n, st, false, stream));
      } else {
        MFQ_HIP(launch_cg_direction(r, p, n, st, false, stream));
      }
      if ((it + 1) % check_every == 0 || it + 1 == maxit) {
        if (int rc = poll(st, h, stream)) return rc;
        if (h.done) break;
      }
    }
  }
  res.iters = h.done ? h.converged_iter : h.iter;
  res.converged = h.done && !h.nonfinite;
  res.nonfinite = h.nonfinite != 0;
  res.rr = h.rr;
  res.bb = h.bb;
  if (h.bb == 0.0) res.converged = true;
  return MFQ_OK;
}

// ---------------------------------------------------------------- V-cycle
int coarse_solve(mfq_solver* s, const void* b, void* x, hipStream_t st) {
  Level& L = s->lv[0];
  const int prec = s->prec_v;
  if (s->prm.coarse_mode == 1)
    return mfq_chebyshev(L.op, L.dinv, b, x, 1, s->prm.coarse_degree, L.lmin, L.lmax, L.r, st);
  if (s->dense) {
    MFQ_HIP(launch_fill(prec, x, L.n, 0.0, st));
    MFQ_HIP(launch_dense_solve(prec, s->ainv, (int)s->nf, (int64_t)L.sp->p * L.sp->mesh->n + 1, b, x, st));
    return MFQ_OK;
  }
  // Jacobi-CG on the FP64 coarse operator to 1e-12
  const double* b64 = (const double*)b;
  double* x64 = (double*)x;
  if (prec != MFQ_FP64) {
    MFQ_HIP(launch_cast(prec, b, MFQ_FP64, s->cb, L.n, st));
    b64 = s->cb;
    x64 = s->cx;
  }
  Apply A = [s, st](const double* in, double* out) { return op_vmult(s->coarse64, in, out, st); };
  Apply M = [s, st, &L](const double* in, double* out) -> int {
    MFQ_HIP(launch_mul(MFQ_FP64, s->cdinv, in, out, L.n, st));
    return MFQ_OK;
  };
  PcgResult res;
  if (int rc = pcg(A, &M, b64, x64, s->cr, s->cp, s->cAp, s->cz, L.n, s->cstate, 1e-12, 10000, 8, st, res)) return rc;
  if (prec != MFQ_FP64) MFQ_HIP(launch_cast(MFQ_FP64, x64, prec, x, L.n, st));
  return MFQ_OK;
}

int vcycle(mfq_solver* s, int l, hipStream_t st) {
  Level& L = s->lv[l];
  if (l == 0) return coarse_solve(s, L.b, L.x, st);
  const int prec = s->prec_v;
  const int deg = s->prm.smoother_degree;
  char* work = (char*)L.r;  // r, d, t are contiguous
  if (int rc = mfq_chebyshev(L.op, L.dinv, L.b, L.x, 1, deg, L.lmin, L.lmax, work, st)) return rc;
  // residual r = b - A x (inside the operator application when the level fuses updates)
  const OpView v = view(L.op);
  if (L.op->fuse && !L.op->mfma && v.side_base < 0) {
    CellEpilogue ep;
    ep.mode = kEpiResidual;
    ep.b = L.b;
    ep.r = L.r;
    MFQ_HIP(launch_vmult_epilogue(v, prec, L.x, L.t, ep, st));
  } else {
    if (int rc = op_vmult(L.op, L.x, L.t, st)) return rc;
    MFQ_HIP(launch_sub(prec, L.b, L.t, L.r, L.n, st));
  }
  Level& C = s->lv[l - 1];
  MFQ_HIP(launch_transfer(C.to_fine, prec, false, L.r, C.b, st));
  if (int rc = vcycle(s, l - 1, st)) return rc;
  MFQ_HIP(launch_transfer(C.to_fine, prec, true, C.x, L.t, st));
  MFQ_HIP(launch_add(prec, L.x, prec, L.t, L.n, st));
  return mfq_chebyshev(L.op, L.dinv, L.b, L.x, 0, deg, L.lmin, L.lmax, work, st);
}

// z = V(r) on the finest level, FP64 in and out.
int precondition(mfq_solver* s, const double* r, double* z, hipStream_t st) {
  Level& F = s->lv.back();
  if (s->prec_v == MFQ_FP64) {
    F.b = const_cast<double*>(r);
    F.x = z;
    return vcycle(s, (int)s->lv.size() - 1, st);
  }
  MFQ_HIP(launch_cast(MFQ_FP64, r, MFQ_FP32, F.b, F.n, st));
  if (int rc = vcycle(s, (int)s->lv.size() - 1, st)) return rc;
  MFQ_HIP(launch_cast(MFQ_FP32, F.x, MFQ_FP64, z, F.n, st));
  return MFQ_OK;
}

// lhat of D^{-1} A_l: largest eigenvalue of the Lanczos matrix of `iters` Jacobi-PCG steps on
// A_l x = v0 (v0 counter-based).  The steps run on the device; their coefficients land in the
// level's trace slot, read by the host once for all levels.
int enqueue_lanczos(mfq_solver* s, Level& L, double* trace, hipStream_t st) {
  const int prec = s->prec_v;
  const int64_t n = L.n;
  void *r = L.r, *zz = L.d, *p = L.t, *Ap = L.x;
  const int k = s->prm.lanczos_iters;
  const int64_t N1 = (int64_t)L.sp->p * L.sp->mesh->n + 1;
  MFQ_HIP(launch_splitmix(prec, r, N1, 0, true, st));
  MFQ_HIP(launch_lz_init(prec, r, L.dinv, zz, p, n, s->aux, trace, 2 * k, st));
  for (int it = 0; it < k; ++it) {
    if (int rc = op_vmult(L.op, p, Ap, st)) return rc;
    MFQ_HIP(launch_lz_alpha(prec, p, Ap, n, s->aux, trace, st));
    MFQ_HIP(launch_lz_update(prec, r, zz, Ap, L.dinv, n, s->aux, trace, 2 * k, st));
    MFQ_HIP(launch_lz_direction(prec, zz, p, n, s->aux, st));
  }
  return MFQ_OK;
}

int lambda_from_trace(const mfq_solver* s, Level& L, const double* trace);

// first level with an eigenvalue estimate (the coarsest one only when it is smoothed)
size_t first_estimated(const mfq_solver* s) { return s->prm.coarse_mode == 1 ? 0 : 1; }

// Chebyshev bounds of every estimated level from the Lanczos traces (host copy, trace_stride
// doubles per level)
int lambdas_from_traces(mfq_solver* s, const double* traces) {
  const size_t nlv = s->lv.size();
  for (size_t l = first_estimated(s); l < nlv; ++l) {
    Level& L = s->lv[l];
    if (int rc = lambda_from_trace(s, L, traces + l * s->trace_stride)) return rc;
    double lmax = s->prm.lambda_factor * L.lhat;
    if (l == 0) {
      L.lmax = lmax;
      L.lmin = lmax / s->prm.coarse_ratio;
      continue;
    }
    const int idx = (int)l - 1;
    if (s->prm.n_lambda_override > idx && s->prm.lambda_override) lmax = s->prm.lambda_override[idx];
    L.lmax = lmax;
    L.lmin = lmax / s->prm.lambda_ratio;
  }
  s->eig_pending = false;
  return MFQ_OK;
}

// all Lanczos runs of one solver enqueued, their traces read back in one copy
int estimate_eigenvalues(mfq_solver* s, hipStream_t st) {
  const size_t nlv = s->lv.size();
  for (size_t l = first_estimated(s); l < nlv; ++l)
    if (int rc = enqueue_lanczos(s, s->lv[l], s->trace + l * s->trace_stride, st)) return rc;
  MFQ_HIP(hipMemcpyAsync(s->trace_host, s->trace, nlv * s->trace_stride * sizeof(double), hipMemcpyDeviceToHost, st));
  MFQ_HIP(hipStreamSynchronize(st));
  return lambdas_from_traces(s, s->trace_host);
}

int lambda_from_trace(const mfq_solver* s, Level& L, const double* trace) {
  const int k = s->prm.lanczos_iters;
  const int m = std::min(k, std::max(0, (int)trace[2 * k]));
  if (m == 0) return fail(MFQ_ENONFINITE, "eigenvalue estimate failed on level p=%d n=%d", L.sp->p, L.sp->mesh->n);
  std::vector<double> T((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) {
    const double ai = trace[2 * i], bi = trace[2 * i + 1];
    T[i * m + i] = 1.0 / ai + (i > 0 ? trace[2 * i - 1] / trace[2 * i - 2] : 0.0);
    if (i + 1 < m) T[i * m + i + 1] = T[(i + 1) * m + i] = std::sqrt(bi) / ai;
  }
  L.lhat = sym_max_eig(T, m);
  return MFQ_OK;
}

// ---------------------------------------------------------------- resumable solve
// A solve is a sequence of CG passes.  Pass 0 solves A x = b from x = 0 (for GMG_MIXED_IR: the
// FP32-operator inner system A c = b, then x = c).  Every pass ends with an FP64 true-residual
// check r = b - A x; while ||r|| > rtol ||b|| another pass solves the residual equation A c = r
// and adds c to x (FP64 iterative refinement).  Steps enqueue work asynchronously; the host
// decides between passes after reading the pinned status copy.
using Run = mfq_solver::Run;

bool preconditioned(const mfq_solver* s) { return s->kind != MFQ_SOLVER_CG; }

// operator of the inner CG: the FP64 operator, or the finest FP32 operator for GMG_MIXED_IR
int inner_apply(mfq_solver* s, const double* in, double* out, hipStream_t st) {
  if (s->kind != MFQ_SOLVER_GMG_MIXED_IR) return op_vmult(s->op64, in, out, st);
  Level& F = s->lv.back();
  MFQ_HIP(launch_cast(MFQ_FP64, in, MFQ_FP32, F.r, F.n, st));
  if (int rc = op_vmult(F.op, F.r, F.d, st)) return rc;
  MFQ_HIP(launch_cast(MFQ_FP32, F.d, MFQ_FP64, out, F.n, st));
  return MFQ_OK;
}

// the host side of starting a CG pass (its kernels are enqueued by pass_start or a batched step)
void pass_started(mfq_solver* s, double* sol) {
  Run& R = s->run;
  R.sol = sol;
  R.enqueued = 0;
  R.budget = R.max_iter - R.iters;
  R.pass += 1;
  R.phase = Run::kInner;
}

// The FP32 V-cycle preconditions the CG (GMG_MIXED, GMG_MIXED_IR): the CG steps then read its FP32
// result directly instead of an FP64 copy z (the same values; two vector passes fewer)
bool vcycle32(const mfq_solver* s) { return preconditioned(s) && s->prec_v == MFQ_FP32 && !s->lv.empty(); }

int pass_start(mfq_solver* s, const double* rhs, double* sol, double tol2) {
  Run& R = s->run;
  const int64_t N = s->op64->space->n_dofs;
  const bool pre = preconditioned(s);
  MFQ_HIP(launch_cg_start(rhs, sol, s->r, s->p, N, s->state, !pre, tol2, R.st));
  if (vcycle32(s)) {
    Level& F = s->lv.back();
    MFQ_HIP(launch_cast(MFQ_FP64, s->r, MFQ_FP32, F.b, F.n, R.st));
    if (int rc = vcycle(s, (int)s->lv.size() - 1, R.st)) return rc;
    MFQ_HIP(launch_cg_beta32(s->r, (const float*)F.x, N, s->state, R.st));
    MFQ_HIP(launch_cg_direction32((const float*)F.x, s->p, N, s->state, true, R.st));
  } else if (pre) {
    if (int rc = precondition(s, s->r, s->z, R.st)) return rc;
    MFQ_HIP(launch_cg_beta(s->r, s->z, N, s->state, R.st));
    MFQ_HIP(launch_cg_direction(s->z, s->p, N, s->state, true, R.st));
  }
  pass_started(s, sol);
  return MFQ_OK;
}

// a CG pass to be started by the next step
void pass_pending(mfq_solver* s, const double* rhs, double* sol, double tol2) {
  Run& R = s->run;
  R.start_rhs = rhs;
  R.start_sol = sol;
  R.start_tol2 = tol2;
  R.phase = Run::kStart;
}

// CG iterations issued as launches; once the device state says done, they are no-ops
int pass_iterate_direct(mfq_solver* s, int k) {
  Run& R = s->run;
  const int64_t N = s->op64->space->n_dofs;
  const bool pre = preconditioned(s);
  for (int i = 0; i < k; ++i) {
    if (int rc = inner_apply(s, s->p, s->Ap, R.st)) return rc;
    MFQ_HIP(launch_cg_alpha(s->p, s->Ap, N, s->state, R.st));
    if (vcycle32(s)) {
      Level& F = s->lv.back();
      MFQ_HIP(launch_cg_update_cast(R.sol, s->r, s->p, s->Ap, (float*)F.b, N, s->state, R.st));
      if (int rc = vcycle(s, (int)s->lv.size() - 1, R.st)) return rc;
      MFQ_HIP(launch_cg_beta32(s->r, (const float*)F.x, N, s->state, R.st));
      MFQ_HIP(launch_cg_direction32((const float*)F.x, s->p, N, s->state, false, R.st));
      continue;
    }
    MFQ_HIP(launch_cg_update(R.sol, s->r, s->p, s->Ap, N, s->state, !pre, R.st));
    if (pre) {
      if (int rc = precondition(s, s->r, s->z, R.st)) return rc;
      MFQ_HIP(launch_cg_beta(s->r, s->z, N, s->state, R.st));
      MFQ_HIP(launch_cg_direction(s->z, s->p, N, s->state, false, R.st));
    } else {
      MFQ_HIP(launch_cg_direction(s->r, s->p, N, s->state, false, R.st));
    }
  }
  return MFQ_OK;
}

// Graphs are used on a non-default stream when nothing in an iteration waits on the host (the
// Jacobi-CG coarse solve polls the host, so it is launched directly).
bool graphs_usable(const mfq_solver* s) {
  if (!s->prm.use_graphs || s->run.st == nullptr) return false;
  if (s->kind == MFQ_SOLVER_CG || s->prm.coarse_mode == 1 || s->dense) return true;
  return false;
}

int iteration_graph(mfq_solver* s, hipGraphExec_t* out) {
  Run& R = s->run;
  for (auto& g : s->graphs)
    if (g.exec && g.st == R.st && g.sol == R.sol) {
      *out = g.exec;
      return MFQ_OK;
    }
  hipGraph_t graph = nullptr;
  MFQ_HIP(hipStreamBeginCapture(R.st, hipStreamCaptureModeThreadLocal));
  const int rc = pass_iterate_direct(s, 1);
  const hipError_t e = hipStreamEndCapture(R.st, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(MFQ_EHIP, "capture of a CG iteration failed: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return fail(MFQ_EHIP, "graph instantiation failed: %s", hipGetErrorString(e2));
  auto& slot = s->graphs[s->next_graph];
  s->next_graph = (s->next_graph + 1) % 2;
  if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
  slot.st = R.st;
  slot.sol = R.sol;
  slot.exec = exec;
  *out = exec;
  return MFQ_OK;
}

int pass_iterate(mfq_solver* s, int k) {
  if (k <= 0) return MFQ_OK;
  if (!graphs_usable(s)) return pass_iterate_direct(s, k);
  hipGraphExec_t exec = nullptr;
  if (int rc = iteration_graph(s, &exec)) return rc;
  for (int i = 0; i < k; ++i) MFQ_HIP(hipGraphLaunch(exec, s->run.st));
  return MFQ_OK;
}

void finish(mfq_solver* s, int status) {
  Run& R = s->run;
  R.status = status;
  R.phase = Run::kDone;
  R.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - R.t0).count();
}

// first half of a step: enqueue work and the device-to-host copy of its outcome
int step_enqueue(mfq_solver* s, int iters) {
  Run& R = s->run;
  const int64_t N = s->op64->space->n_dofs;
  if (R.phase == Run::kStart) {
    if (s->eig_pending) {
      const int rc = estimate_eigenvalues(s, R.st);
      if (rc == MFQ_ENONFINITE) {
        finish(s, rc);
        return MFQ_OK;
      }
      if (rc) return rc;
    }
    if (int rc = pass_start(s, R.start_rhs, R.start_sol, R.start_tol2)) return rc;
  }
  if (R.phase == Run::kInner) {
    const int m = std::max(0, std::min(iters, R.budget - R.enqueued));
    if (int rc = pass_iterate(s, m)) return rc;
    R.enqueued += m;
    MFQ_HIP(hipMemcpyAsync(&s->hstat->head, s->state, offsetof(SolverState, partials), hipMemcpyDeviceToHost, R.st));
  } else if (R.phase == Run::kCheck) {
    if (R.sol != R.x) MFQ_HIP(launch_add(MFQ_FP64, R.x, MFQ_FP64, R.sol, N, R.st));
    if (int rc = op_vmult(s->op64, R.x, s->Ap, R.st)) return rc;
    MFQ_HIP(launch_residual_norm(R.b, s->Ap, s->rout, N, s->aux, s->scal, R.st));
    MFQ_HIP(hipMemcpyAsync(&s->hstat->cert, s->scal, 8, hipMemcpyDeviceToHost, R.st));
  }
  return MFQ_OK;
}

// second half, after the stream has been synchronised: read the outcome, pick the next phase
int step_collect(mfq_solver* s) {
  Run& R = s->run;
  if (R.phase == Run::kInner) {
    const SolverState& h = s->hstat->head;
    if (R.pass == 1 && R.bb < 0) R.bb = h.bb;  // pass 1 runs on b itself
    if (h.nonfinite) {
      R.iters += h.iter;
      finish(s, MFQ_ENONFINITE);
    } else if (h.done || R.enqueued >= R.budget) {
      R.iters += h.done ? h.converged_iter : h.iter;
      R.phase = Run::kCheck;
    }
  } else if (R.phase == Run::kCheck) {
    const double rr = s->hstat->cert;
    R.rr = rr;
    if (!std::isfinite(rr)) {
      finish(s, MFQ_ENONFINITE);
    } else if (rr <= R.rtol * R.rtol * R.bb || R.bb == 0) {
      finish(s, MFQ_OK);
    } else if (R.iters >= R.max_iter) {
      finish(s, MFQ_ENOCONV);
    } else {
      // correction pass on A c = r: the inner system of GMG_MIXED_IR to inner_rtol, the others
      // to half the remaining distance to rtol ||b||
      const double tol2 = s->kind == MFQ_SOLVER_GMG_MIXED_IR ? s->prm.inner_rtol * s->prm.inner_rtol
                                                              : std::min(0.25, 0.25 * R.rtol * R.rtol * R.bb / rr);
      pass_pending(s, s->rout, s->c, tol2);
    }
  }
  return MFQ_OK;
}

int begin_solve(mfq_solver* s, const double* b, double* x, double rtol, int max_iter, hipStream_t st) {
  if (!s) return fail(MFQ_EINVAL, "solver is NULL");
  if (!s->buf) return fail(MFQ_EINVAL, "solver is not bound");
  if (s->run.phase == Run::kStart || s->run.phase == Run::kInner || s->run.phase == Run::kCheck ||
      s->step_pending)
    return fail(MFQ_EBUSY, "a solve is running");
  if (!b || !x || (reinterpret_cast<uintptr_t>(b) % 16) || (reinterpret_cast<uintptr_t>(x) % 16))
    return fail(MFQ_EINVAL, "b or x NULL or misaligned");
  if (!(rtol > 0 && rtol < 1)) return fail(MFQ_EINVAL, "rtol must be in (0,1)");
  if (max_iter < 1) return fail(MFQ_EINVAL, "max_iter must be >= 1");
  Run& R = s->run;
  R = Run{};
  R.b = b;
  R.x = x;
  R.rtol = rtol;
  R.max_iter = max_iter;
  R.st = st;
  R.t0 = std::chrono::steady_clock::now();
  const int64_t N = s->op64->space->n_dofs;
  if (s->kind == MFQ_SOLVER_GMG_MIXED_IR) {
    MFQ_HIP(launch_fill(MFQ_FP64, x, N, 0.0, st));
    pass_pending(s, b, s->c, s->prm.inner_rtol * s->prm.inner_rtol);
  } else {
    pass_pending(s, b, x, rtol * rtol);
  }
  return MFQ_OK;
}

}  // namespace


// ---------------------------------------------------------------- batched steps (serving)
// Many running solves advanced by one launch per (kernel, degree): the launches of one CG
// iteration of every solve (the FP64 operator, the CG updates, the FP32 V-cycle level by level from
// the finest) are planned once per step as work tables, uploaded in one copy, and replayed for
// each iteration of the step.  Each solve's kernels see exactly the operands and grids of its own
// launches, so its results are bitwise those of mfq_batch_step.
struct mfq_batch {
  int max_solvers = 0;
  size_t table_cap = 0;          // bytes of the table region
  size_t state_off = 0;          // gathered scalar states, then residual norms (device)
  size_t trace_off = 0;          // gathered Lanczos traces (device)
  size_t bytes = 0;
  char* buf = nullptr;
  char* host_tables = nullptr;   // pinned staging of the tables
  double* host_states = nullptr; // pinned copy of the gathered states and residual norms
  double* host_traces = nullptr; // pinned copy of the gathered traces
  hipEvent_t uploaded = nullptr; // the last table upload has left the staging buffer
  // Side streams for the independent launch groups of one phase (operators of different degrees
  // or forms, transfers of different degree pairs): the groups run side by side, forked from and
  // joined back into the step's stream by events.  Default priority, like every stream here.
  static constexpr int kSide = 3;
  hipStream_t side[kSide] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kSide] = {};
  ~mfq_batch() {
    for (int k = 0; k < kSide; ++k) {
      if (join[k]) (void)hipEventDestroy(join[k]);
      if (side[k]) (void)hipStreamDestroy(side[k]);
    }
    if (fork) (void)hipEventDestroy(fork);
    if (uploaded) (void)hipEventDestroy(uploaded);
    if (host_tables) (void)hipHostFree(host_tables);
    if (host_states) (void)hipHostFree(host_states);
    if (host_traces) (void)hipHostFree(host_traces);
  }
};

namespace {

constexpr size_t kBatchTableBytesPerSolve = 96 << 10;
constexpr int kStateDoubles = (int)(offsetof(SolverState, partials) / sizeof(double));
constexpr int kTraceDoubles = 1024;  // Lanczos traces of one solve's levels in a batched estimate

struct PlanLaunch {
  enum Kind { kVec, kCells, kTransfer } kind = kVec;
  int op = 0, p = 0, pf = 0, precision = 0, colour = 0;
  int phase = 0;  // launches of one phase touch disjoint vectors group by group
  int group = 0;  // within a phase, the launches of one group run in order
  bool h = false, cart = false, prolongate = false, fused = false, coef = false;
  size_t off = 0;
  int count = 0;
  int64_t blocks = 0;
};

struct Plan {
  std::vector<char> tab;
  std::vector<PlanLaunch> launches;
  int phases = 0;

  template <class T>
  size_t put(const std::vector<T>& v) {
    const size_t off = round_up(tab.size(), 64);
    tab.resize(off + v.size() * sizeof(T));
    std::memcpy(tab.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
  void vec(BatchVecOp op, std::vector<VecItem>& items) {
    if (items.empty()) return;
    int64_t blk = 0;
    for (VecItem& it : items) {
      it.first = blk;
      it.nblk = vec_blocks(op, it.n);
      blk += it.nblk;
    }
    PlanLaunch L;
    L.kind = PlanLaunch::kVec;
    L.phase = ++phases;
    L.op = op;
    L.off = put(items);
    L.count = (int)items.size();
    L.blocks = blk;
    launches.push_back(L);
  }
  // dst = A src for each (operator, src, dst), with the fused update ep when ep.mode is set (dst
  // then receives partial sums only): one launch per (degree, precision, Cartesian form, fused,
  // colour), colours in order
  struct Apply {
    const mfq_op* op;
    const void* src;
    void* dst;
    CellEpilogue ep = CellEpilogue{};
  };
  void cells(const std::vector<Apply>& list) {
    std::vector<int> done(list.size(), 0);
    const int phase = ++phases;
    int group = 0;
    for (size_t i = 0; i < list.size(); ++i) {
      if (done[i]) continue;
      const mfq_op* o = list[i].op;
      const int p = o->space->p, prec = o->precision;
      const bool cart = o->space->mesh->amplitude == 0.0 && o->alpha == 0.0;
      const bool fused = list[i].ep.mode != kEpiNone;
      const bool coef = o->coef != nullptr && !fused;
      std::vector<CellItem> items;
      for (size_t j = i; j < list.size(); ++j) {
        const mfq_op* q = list[j].op;
        const bool cj = q->space->mesh->amplitude == 0.0 && q->alpha == 0.0;
        const bool fj = list[j].ep.mode != kEpiNone;
        if (done[j] || q->space->p != p || q->precision != prec || cj != cart || fj != fused ||
            (q->coef != nullptr && !fj) != coef)
          continue;
        done[j] = 1;
        CellItem it{};
        it.idx = q->idx;
        it.geo = q->geo;
        it.src = list[j].src;
        it.dst = list[j].dst;
        it.bk = q->bricks;
        it.ep = list[j].ep;
        it.coef = q->coef;
        items.push_back(it);
      }
      int64_t tot[kColours] = {};
      for (CellItem& it : items)
        for (int c = 0; c < kColours; ++c) {
          it.first[c] = tot[c];
          tot[c] += it.bk.count[c];
        }
      const size_t off = put(items);
      for (int c = 0; c < kColours; ++c) {
        if (tot[c] == 0) continue;
        PlanLaunch L;
        L.kind = PlanLaunch::kCells;
        L.phase = phase;
        L.group = group;
        L.p = p;
        L.precision = prec;
        L.cart = cart;
        L.fused = fused;
        L.coef = coef;
        L.colour = c;
        L.off = off;
        L.count = (int)items.size();
        L.blocks = tot[c];
        launches.push_back(L);
      }
      ++group;
    }
  }
  struct Move {
    const mfq_transfer* t;
    const void* in;
    void* out;
  };
  // prolongation (coarse -> fine) or restriction (fine -> coarse, after clearing the coarse
  // vectors) for each transfer: one launch per degree pair (and colour)
  void transfers(const std::vector<Move>& list, bool prolongate) {
    if (!prolongate) {
      std::vector<VecItem> clear;
      for (const Move& m : list) {
        VecItem it{};
        it.n = m.t->coarse->n_dofs;
        it.d = m.out;
        it.s0 = 0.0;
        clear.push_back(it);
      }
      vec(kBatchFill, clear);
    }
    std::vector<int> done(list.size(), 0);
    const int phase = ++phases;
    int group = 0;
    for (size_t i = 0; i < list.size(); ++i) {
      if (done[i]) continue;
      const int pc = list[i].t->coarse->p, pf = list[i].t->fine->p;
      const bool h = list[i].t->h_transfer;
      std::vector<TransferItem> items;
      for (size_t j = i; j < list.size(); ++j) {
        const mfq_transfer* t = list[j].t;
        if (done[j] || t->coarse->p != pc || t->fine->p != pf || t->h_transfer != h) continue;
        done[j] = 1;
        TransferItem it{};
        it.in = list[j].in;
        it.out = list[j].out;
        it.nc = t->coarse->mesh->n;
        it.bc = t->coarse->bc;
        items.push_back(it);
      }
      int64_t tot[kColours] = {};
      for (TransferItem& it : items) {
        const int nc = it.nc;
        if (prolongate) {
          it.first[0] = tot[0];
          tot[0] += (int64_t)nc * nc * nc;
        } else {
          for (int c = 0; c < kColours; ++c) {
            it.first[c] = tot[c];
            tot[c] += (int64_t)((nc + 1 - (c & 1)) / 2) * ((nc + 1 - ((c >> 1) & 1)) / 2) * ((nc + 1 - (c >> 2)) / 2);
          }
        }
      }
      const size_t off = put(items);
      for (int c = 0; c < (prolongate ? 1 : kColours); ++c) {
        if (tot[c] == 0) continue;
        PlanLaunch L;
        L.kind = PlanLaunch::kTransfer;
        L.phase = phase;
        L.group = group;
        L.p = pc;
        L.pf = pf;
        L.h = h;
        L.prolongate = prolongate;
        L.colour = c;
        L.off = off;
        L.count = (int)items.size();
        L.blocks = tot[c];
        launches.push_back(L);
      }
      ++group;
    }
  }
  // `deg` Chebyshev updates on each level (mfq_chebyshev with the work vectors r, d, t of the
  // level: the first update from x = 0 a vector kernel, every other one fused into the cell loop)
  void chebyshev(const std::vector<const Level*>& lv, int deg, bool x_is_zero) {
    if (lv.empty()) return;
    std::vector<double> sigma(lv.size()), delta(lv.size()), rho(lv.size());
    std::vector<VecItem> first;
    std::vector<Apply> ax;
    for (size_t i = 0; i < lv.size(); ++i) {
      const Level& L = *lv[i];
      const double theta = 0.5 * (L.lmax + L.lmin);
      delta[i] = 0.5 * (L.lmax - L.lmin);
      sigma[i] = theta / delta[i];
      rho[i] = 1.0 / sigma[i];
      Apply a{L.op, L.x, L.t};
      a.ep.mode = kEpiChebFirst;
      a.ep.b = L.b;
      a.ep.dinv = L.dinv;
      a.ep.x = L.x;
      a.ep.r = L.r;
      a.ep.d = L.d;
      a.ep.s0 = 1.0 / theta;
      ax.push_back(a);
      VecItem it{};
      it.n = L.n;
      it.a = L.b;
      it.b = L.t;
      it.c = L.dinv;
      it.d = L.x;
      it.e = L.r;
      it.f = L.d;
      it.s0 = 1.0 / theta;
      it.flag = 1;
      first.push_back(it);
    }
    if (x_is_zero) {
      vec(kBatchChebFirst, first);
    } else {
      // levels that do not fuse: the product into t, then the vector kernel
      std::vector<Apply> ax_plain;
      std::vector<VecItem> first_plain;
      std::vector<Apply> ax_fused;
      for (size_t i = 0; i < lv.size(); ++i) {
        if (lv[i]->op->fuse) {
          ax_fused.push_back(ax[i]);
        } else {
          ax_plain.push_back({lv[i]->op, lv[i]->x, lv[i]->t});
          VecItem it = first[i];
          it.flag = 0;
          first_plain.push_back(it);
        }
      }
      cells(ax_fused);
      cells(ax_plain);
      vec(kBatchChebFirst, first_plain);
    }
    for (int k = 1; k < deg; ++k) {
      std::vector<Apply> ad, ad_plain;
      std::vector<VecItem> step;
      for (size_t i = 0; i < lv.size(); ++i) {
        const Level& L = *lv[i];
        const double rho_new = 1.0 / (2.0 * sigma[i] - rho[i]);
        const double c1 = rho_new * rho[i], c2 = 2.0 * rho_new / delta[i];
        rho[i] = rho_new;
        if (L.op->fuse) {
          Apply a{L.op, L.d, L.t};
          a.ep.mode = kEpiChebStep;
          a.ep.dinv = L.dinv;
          a.ep.x = L.x;
          a.ep.r = L.r;
          a.ep.d = L.d;
          a.ep.s0 = c1;
          a.ep.s1 = c2;
          ad.push_back(a);
        } else {
          ad_plain.push_back({L.op, L.d, L.t});
          VecItem it{};
          it.n = L.n;
          it.a = L.t;
          it.c = L.dinv;
          it.d = L.x;
          it.e = L.r;
          it.f = L.d;
          it.s0 = c1;
          it.s1 = c2;
          step.push_back(it);
        }
      }
      cells(ad);
      cells(ad_plain);
      vec(kBatchChebStep, step);
    }
  }
};

// Solves that a batched step can advance: FP64 CG with the FP32 V-cycle whose coarsest level is
// smoothed (no host round trip), in a CG pass with room for `iters` more iterations.
bool batch_form(const mfq_solver* s) {
  if (s->kind != MFQ_SOLVER_GMG_MIXED || s->prm.coarse_mode != 1 || s->prec_v != MFQ_FP32) return false;
  if (s->op64->mfma || s->op64->space->side) return false;
  for (const Level& L : s->lv)
    if (!L.op || L.op->mfma) return false;
  return true;
}

bool batchable(const mfq_solver* s, int iters) {
  if (s->run.phase != Run::kInner || s->run.budget - s->run.enqueued < iters) return false;
  return batch_form(s);
}

// The eigenvalue estimates of lazily bound solves (every level at once, one state per level): the
// first launches once, then one Lanczos step replayed lanczos_iters times (enqueue_lanczos).
void plan_lanczos_start(Plan& P, const std::vector<mfq_solver*>& e) {
  std::vector<VecItem> seed, init;
  for (mfq_solver* s : e) {
    const int k = s->prm.lanczos_iters;
    for (size_t l = first_estimated(s); l < s->lv.size(); ++l) {
      Level& L = s->lv[l];
      const int64_t N1 = (int64_t)L.sp->p * L.sp->mesh->n + 1;
      VecItem it{};
      it.n = N1 * N1 * N1;
      it.d = L.r;
      it.flag = (int)N1;
      seed.push_back(it);
      VecItem i2{};
      i2.n = L.n;
      i2.a = L.r;
      i2.c = L.dinv;
      i2.d = L.d;
      i2.e = L.t;
      i2.b = s->trace + l * s->trace_stride;
      i2.flag = 2 * k;
      i2.st = (SolverState*)((char*)s->lz + l * round_up(sizeof(SolverState), 256));
      init.push_back(i2);
    }
  }
  P.vec(kBatchSplitmix, seed);
  P.vec(kBatchLzInit, init);
}

void plan_lanczos_step(Plan& P, const std::vector<mfq_solver*>& e) {
  std::vector<Plan::Apply> ap;
  std::vector<VecItem> alpha, update, dir;
  for (mfq_solver* s : e) {
    const int k = s->prm.lanczos_iters;
    for (size_t l = first_estimated(s); l < s->lv.size(); ++l) {
      Level& L = s->lv[l];
      ap.push_back({L.op, L.t, L.x});
      VecItem it{};
      it.n = L.n;
      it.st = (SolverState*)((char*)s->lz + l * round_up(sizeof(SolverState), 256));
      it.b = s->trace + l * s->trace_stride;
      VecItem a = it;
      a.a = L.t;
      a.c = L.x;
      alpha.push_back(a);
      VecItem u = it;
      u.d = L.r;
      u.e = L.d;
      u.a = L.x;
      u.c = L.dinv;
      u.flag = 2 * k;
      update.push_back(u);
      VecItem d = it;
      d.a = L.d;
      d.d = L.t;
      dir.push_back(d);
    }
  }
  P.cells(ap);
  P.vec(kBatchLzAlpha, alpha);
  P.vec(kBatchLzUpdate, update);
  P.vec(kBatchLzDirection, dir);
}

// The FP32 V-cycle of every solve in `g` on its finest level's b (level by level from the
// finest: depth 0 is every solve's finest level), result in the finest level's x
void plan_vcycle(Plan& P, const std::vector<mfq_solver*>& g) {
  size_t depth = 0;
  for (mfq_solver* s : g) depth = std::max(depth, s->lv.size());
  const int deg = g.front()->prm.smoother_degree, cdeg = g.front()->prm.coarse_degree;
  for (size_t d = 0; d < depth; ++d) {
    std::vector<const Level*> smooth, coarse;
    std::vector<Plan::Apply> res;
    std::vector<VecItem> sub;
    std::vector<Plan::Move> down;
    for (mfq_solver* s : g) {
      if (d >= s->lv.size()) continue;
      const size_t l = s->lv.size() - 1 - d;
      Level& L = s->lv[l];
      if (l == 0) {
        coarse.push_back(&L);
        continue;
      }
      smooth.push_back(&L);
      Plan::Apply a{L.op, L.x, L.t};
      if (L.op->fuse) {
        a.ep.mode = kEpiResidual;  // r = b - A x
        a.ep.b = L.b;
        a.ep.r = L.r;
      } else {
        VecItem it{};
        it.n = L.n;
        it.a = L.b;
        it.b = L.t;
        it.d = L.r;
        sub.push_back(it);
      }
      res.push_back(a);
      down.push_back({s->lv[l - 1].to_fine, L.r, s->lv[l - 1].b});
    }
    P.chebyshev(smooth, deg, true);
    P.chebyshev(coarse, cdeg, true);
    P.cells(res);
    P.vec(kBatchSub, sub);
    P.transfers(down, false);
  }
  for (size_t d = depth; d-- > 0;) {
    std::vector<const Level*> smooth;
    std::vector<Plan::Move> up;
    std::vector<VecItem> add;
    for (mfq_solver* s : g) {
      if (d >= s->lv.size()) continue;
      const size_t l = s->lv.size() - 1 - d;
      if (l == 0) continue;
      Level& L = s->lv[l];
      smooth.push_back(&L);
      up.push_back({s->lv[l - 1].to_fine, s->lv[l - 1].x, L.t});
      VecItem it{};
      it.n = L.n;
      it.d = L.x;
      it.a = L.t;
      add.push_back(it);
    }
    P.transfers(up, true);
    P.vec(kBatchAdd, add);
    P.chebyshev(smooth, deg, false);
  }
}

// beta = r.z / rz ; p = z (+ beta p) for every solve in `g`, z the V-cycle's FP32 result
void plan_direction(Plan& P, const std::vector<mfq_solver*>& g, bool first) {
  std::vector<VecItem> beta, dir;
  for (mfq_solver* s : g) {
    VecItem it{};
    it.n = s->op64->space->n_dofs;
    it.st = s->state;
    VecItem b = it;
    b.a = s->r;
    b.b = s->lv.back().x;
    beta.push_back(b);
    VecItem d = it;
    d.a = s->lv.back().x;
    d.d = s->p;
    d.flag = first ? 1 : 0;
    dir.push_back(d);
  }
  P.vec(kBatchCgBeta32, beta);
  P.vec(kBatchCgDirection32, dir);
}

// The launches of one CG iteration of every solve in `g` (one step replays them `iters` times).
void plan_iteration(Plan& P, const std::vector<mfq_solver*>& g) {
  std::vector<Plan::Apply> a64;
  std::vector<VecItem> alpha, update;
  for (mfq_solver* s : g) {
    a64.push_back({s->op64, s->p, s->Ap});
    VecItem it{};
    it.n = s->op64->space->n_dofs;
    it.st = s->state;
    VecItem a = it;
    a.a = s->p;
    a.b = s->Ap;
    alpha.push_back(a);
    VecItem u = it;
    u.d = s->run.sol;
    u.e = s->r;
    u.a = s->p;
    u.b = s->Ap;
    u.f = s->lv.back().b;  // the residual in FP32: the V-cycle's right-hand side
    update.push_back(u);
  }
  P.cells(a64);
  P.vec(kBatchCgAlpha, alpha);
  P.vec(kBatchCgUpdate, update);
  plan_vcycle(P, g);
  plan_direction(P, g, false);
}

// The start of the pending CG pass of every solve in `g` (pass_start)
void plan_start(Plan& P, const std::vector<mfq_solver*>& g) {
  if (g.empty()) return;
  std::vector<VecItem> start;
  for (mfq_solver* s : g) {
    VecItem it{};
    it.n = s->op64->space->n_dofs;
    it.st = s->state;
    it.a = s->run.start_rhs;
    it.d = s->run.start_sol;
    it.e = s->r;
    it.f = s->p;
    it.s0 = s->run.start_tol2;
    it.flag = 0;  // preconditioned: p is set by the first direction update
    start.push_back(it);
  }
  P.vec(kBatchCgStart, start);
  std::vector<VecItem> to32;
  for (mfq_solver* s : g) {
    VecItem c{};
    c.n = s->op64->space->n_dofs;
    c.a = s->r;
    c.d = s->lv.back().b;
    to32.push_back(c);
  }
  P.vec(kBatchCast64To32, to32);
  plan_vcycle(P, g);
  plan_direction(P, g, true);
}

// The FP64 residual check that ends a CG pass of every solve in `g` (step_enqueue): x += c for a
// correction pass, r = b - A x, ||r||^2 into the solve's scalar slot
void plan_check(Plan& P, const std::vector<mfq_solver*>& g) {
  std::vector<VecItem> add, res;
  std::vector<Plan::Apply> a64;
  for (mfq_solver* s : g) {
    const Run& R = s->run;
    const int64_t N = s->op64->space->n_dofs;
    if (R.sol != R.x) {
      VecItem it{};
      it.n = N;
      it.d = R.x;
      it.a = R.sol;
      add.push_back(it);
    }
    a64.push_back({s->op64, R.x, s->Ap});
    VecItem it{};
    it.n = N;
    it.st = s->aux;
    it.a = R.b;
    it.b = s->Ap;
    it.d = s->rout;
    it.e = s->scal;
    res.push_back(it);
  }
  P.vec(kBatchAdd64, add);
  P.cells(a64);
  P.vec(kBatchResidualNorm, res);
}

int issue(const mfq_batch* b, const PlanLaunch& L, hipStream_t st) {
  const void* items = b->buf + L.off;
  hipError_t e = hipSuccess;
  if (L.kind == PlanLaunch::kVec)
    e = launch_batch_vec((BatchVecOp)L.op, (const VecItem*)items, L.count, L.blocks, st);
  else if (L.kind == PlanLaunch::kCells)
    e = launch_batch_cells(L.p, L.precision, L.cart, L.coef, L.fused, (const CellItem*)items, L.count, L.colour,
                           L.blocks, st);
  else
    e = launch_batch_transfer(L.p, L.pf, L.h, L.prolongate, L.colour, (const TransferItem*)items, L.count,
                              L.blocks, st);
  if (e != hipSuccess) return fail(MFQ_EHIP, "batched launch failed: %s", hipGetErrorString(e));
  return MFQ_OK;
}

// The launches in plan order; a phase of several groups is forked over the step's stream and
// the side streams (group g on stream g mod S) and joined back before the next phase.
int run_plan(const mfq_batch* b, const Plan& P, hipStream_t st) {
  const size_t n = P.launches.size();
  for (size_t i = 0; i < n;) {
    size_t j = i;
    int groups = 0;
    while (j < n && P.launches[j].phase == P.launches[i].phase) groups = std::max(groups, P.launches[j++].group + 1);
    const int S = std::min(groups, mfq_batch::kSide + 1);
    if (S <= 1) {
      for (size_t l = i; l < j; ++l)
        if (int rc = issue(b, P.launches[l], st)) return rc;
    } else {
      MFQ_HIP(hipEventRecord(b->fork, st));
      for (int k = 1; k < S; ++k) MFQ_HIP(hipStreamWaitEvent(b->side[k - 1], b->fork, 0));
      for (size_t l = i; l < j; ++l) {
        const int g = P.launches[l].group % S;
        if (int rc = issue(b, P.launches[l], g == 0 ? st : b->side[g - 1])) return rc;
      }
      for (int k = 1; k < S; ++k) {
        MFQ_HIP(hipEventRecord(b->join[k - 1], b->side[k - 1]));
        MFQ_HIP(hipStreamWaitEvent(st, b->join[k - 1], 0));
      }
    }
    i = j;
  }
  return MFQ_OK;
}

}  // namespace

namespace mfq {

size_t cg_work_bytes(int64_t n) { return 3 * round_up((size_t)n * 8, 256) + round_up(sizeof(SolverState), 256); }

int cg_unpreconditioned(const Apply& apply, const double* b, double* x, int64_t n, double rtol, int max_iter,
                        void* work, hipStream_t st, mfq_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  const size_t vb = round_up((size_t)n * 8, 256);
  char* w = (char*)work;
  double* r = (double*)w;
  double* p = (double*)(w + vb);
  double* Ap = (double*)(w + 2 * vb);
  SolverState* state = (SolverState*)(w + 3 * vb);
  // the grid reductions need a zero counter; a fill kernel (no memset node) clears the scalars
  MFQ_HIP(launch_fill(MFQ_FP64, state, (int64_t)(offsetof(SolverState, partials) / sizeof(double)), 0.0, st));
  PcgResult res;
  if (int rc = pcg(apply, nullptr, b, x, r, p, Ap, nullptr, n, state, rtol, max_iter, 8, st, res)) return rc;
  // true residual of the returned x
  if (int rc = apply(x, Ap)) return rc;
  MFQ_HIP(launch_residual_norm(b, Ap, nullptr, n, state, &state->res2, st));
  SolverState h{};
  if (int rc = poll(state, h, st)) return rc;
  const double rel = h.bb > 0 ? std::sqrt(h.res2 / h.bb) : 0.0;
  if (info) {
    info->iterations = res.iters;
    info->outer_iterations = 1;
    info->rel_residual = rel;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->n_levels = 0;
  }
  if (res.nonfinite || !std::isfinite(rel)) return fail(MFQ_ENONFINITE, "CG produced a non-finite residual");
  if (rel > rtol) return fail(MFQ_ENOCONV, "CG: relative residual %.3e after %d iterations (rtol %.1e)", rel, res.iters, rtol);
  return MFQ_OK;
}

}  // namespace mfq

extern "C" {

void mfq_solver_default_params(mfq_solver_params* p) {
  if (!p) return;
  p->smoother_degree = 3;
  p->lanczos_iters = 12;
  p->lambda_factor = 1.2;
  p->lambda_ratio = 15.0;
  p->inner_rtol = 1e-4;
  p->check_every = 4;
  p->n_lambda_override = 0;
  p->lambda_override = nullptr;
  p->coarse_mode = 0;
  p->coarse_degree = 16;
  p->coarse_ratio = 30.0;
  p->coarse_dofs = (int)kDenseCoarseLimit;
  p->use_graphs = 1;
}

int mfq_solver_create(const mfq_op* op64, int kind, const mfq_solver_params* params, mfq_solver** out) {
  if (!op64 || !out) return fail(MFQ_EINVAL, "op or out is NULL");
  if (op64->precision != MFQ_FP64) return fail(MFQ_EINVAL, "solver needs an FP64 operator");
  if (kind < MFQ_SOLVER_CG || kind > MFQ_SOLVER_GMG_MIXED_IR) return fail(MFQ_EINVAL, "unknown solver kind %d", kind);
  const mfq_space* fs = op64->space;
  if (kind != MFQ_SOLVER_CG && fs->bc != MFQ_BC_DIRICHLET0)
    return fail(MFQ_EINVAL, "multigrid solvers need Dirichlet boundary conditions");
  mfq_solver_params prm;
  mfq_solver_default_params(&prm);
  if (params) prm = *params;
  if (prm.smoother_degree < 1 || prm.smoother_degree > 32) return fail(MFQ_EINVAL, "smoother degree out of range");
  if (prm.lanczos_iters < 1 || prm.lanczos_iters > 200) return fail(MFQ_EINVAL, "lanczos_iters out of range");
  if (prm.check_every < 1) prm.check_every = 1;
  if (!(prm.lambda_ratio > 1) || !(prm.lambda_factor > 0)) return fail(MFQ_EINVAL, "bad Chebyshev interval parameters");
  if (!(prm.inner_rtol > 0 && prm.inner_rtol < 1)) return fail(MFQ_EINVAL, "inner_rtol must be in (0,1)");
  if (prm.coarse_mode != 0 && prm.coarse_mode != 1) return fail(MFQ_EINVAL, "coarse_mode must be 0 or 1");
  if (prm.coarse_degree < 1 || prm.coarse_degree > 256) return fail(MFQ_EINVAL, "coarse_degree out of range");
  if (!(prm.coarse_ratio > 1)) return fail(MFQ_EINVAL, "coarse_ratio must exceed 1");
  if (prm.coarse_dofs < 1 || prm.coarse_dofs > kDenseCoarseLimit)
    return fail(MFQ_EINVAL, "coarse_dofs must be in [1, %d]", (int)kDenseCoarseLimit);
  mfq_solver* s = new (std::nothrow) mfq_solver();
  if (!s) return fail(MFQ_ENOMEM, "host allocation failed");
  s->op64 = op64;
  s->kind = kind;
  s->prm = prm;
  s->prec_v = (kind == MFQ_SOLVER_GMG_MIXED || kind == MFQ_SOLVER_GMG_MIXED_IR) ? MFQ_FP32 : MFQ_FP64;

  size_t off = 0;
  auto take = [&off](size_t bytes) {
    size_t o = off;
    off += round_up(bytes, 256);
    return o;
  };
  const int64_t N = fs->n_dofs;
  s->off_state = take(sizeof(SolverState));
  s->off_aux = take(sizeof(SolverState) + 64);
  s->off_kry = take(6 * round_up(N * 8, 256));
  s->trace_stride = 2 * prm.lanczos_iters + 1;

  if (kind != MFQ_SOLVER_CG) {
    // hierarchy: halve n while even and > 4096 free DoFs, then p -> ceil(p/2) while > 4096
    std::vector<std::pair<int, int>> spec;
    int p = fs->p, n = fs->mesh->n;
    spec.push_back({p, n});
    const int64_t limit = prm.coarse_dofs;
    while (n % 2 == 0 && n_free(p, n) > limit) {
      n /= 2;
      spec.push_back({p, n});
    }
    while (p > 1 && n_free(p, n) > limit) {
      p = (p + 1) / 2;
      spec.push_back({p, n});
    }
    std::reverse(spec.begin(), spec.end());
    s->lv.resize(spec.size());
    const int prec = s->prec_v;
    for (size_t l = 0; l < spec.size(); ++l) {
      Level& L = s->lv[l];
      int rc = MFQ_OK;
      if (l + 1 == spec.size()) {
        L.sp = fs;
      } else {
        const mfq_mesh* m0 = fs->mesh;
        rc = mfq_mesh_create(spec[l].second, m0->amplitude, &L.mesh);
        if (!rc) rc = mfq_space_create(L.mesh, spec[l].first, fs->bc, &L.space);
        L.sp = L.space;
      }
      if (rc) {
        delete s;
        return rc;
      }
      L.n = L.sp->n_dofs;
      if (l + 1 == spec.size() && prec == MFQ_FP64) {
        L.op = const_cast<mfq_op*>(op64);
        L.owns_op = false;
      } else if (l > 0 || prm.coarse_mode == 1 || (l + 1 == spec.size() && kind == MFQ_SOLVER_GMG_MIXED_IR)) {
        if (int rc2 = mfq_op_create(L.sp, op64->alpha, prec, &L.op)) {
          delete s;
          return rc2;
        }
        L.op->fuse = op64->fuse;
        size_t ob;
        mfq_op_device_bytes(L.op, &ob);
        L.off_op = take(ob);
      } else {
        L.op = nullptr;
        L.owns_op = false;
      }
      const size_t vb = round_up(L.n * rsize(prec), 256);
      L.off_b = take(vb);
      L.off_x = take(vb);
      L.off_r = take(3 * vb);  // r, d, t contiguous (Chebyshev work)
      L.off_dinv = take(vb);
      if (l > 0) {
        if (int rc2 = mfq_transfer_create(s->lv[l - 1].sp, L.sp, &s->lv[l - 1].to_fine)) {
          delete s;
          return rc2;
        }
      }
    }
    s->off_trace = take(s->lv.size() * s->trace_stride * sizeof(double));
    s->off_lz = take(s->lv.size() * round_up(sizeof(SolverState), 256));
    // coarse level
    Level& C = s->lv[0];
    s->nf = n_free(C.sp->p, C.sp->mesh->n);
    s->dense = s->nf <= limit;
    if (prm.coarse_mode == 1) {
      s->dense = false;
      s->bytes = off;
      *out = s;
      return MFQ_OK;
    }
    if (int rc = mfq_op_create(C.sp, op64->alpha, MFQ_FP64, &s->coarse64)) {
      delete s;
      return rc;
    }
    size_t cb;
    mfq_op_device_bytes(s->coarse64, &cb);
    s->off_coarse64 = take(cb);
    if (s->dense) {
      s->off_ainv = take((size_t)s->nf * s->nf * 8);
    } else {
      s->off_cvec = take(7 * round_up(C.n * 8, 256));
      s->off_cstate = take(sizeof(SolverState));
    }
  }
  s->bytes = off;
  *out = s;
  return MFQ_OK;
}

void mfq_solver_destroy(mfq_solver* s) { delete s; }

int mfq_solver_device_bytes(const mfq_solver* s, size_t* bytes) {
  if (!s || !bytes) return fail(MFQ_EINVAL, "solver or bytes is NULL");
  *bytes = s->bytes;
  return MFQ_OK;
}

}  // extern "C"

namespace {

int bind_solver(mfq_solver* s, void* dev_buf, size_t bytes, void* hip_stream, bool lazy) {
  if (!s) return fail(MFQ_EINVAL, "solver is NULL");
  if (!s->op64->buf) return fail(MFQ_EINVAL, "the solver's FP64 operator is not bound");
  if (!dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) % 256)) return fail(MFQ_EINVAL, "buffer NULL or misaligned");
  if (bytes < s->bytes) return fail(MFQ_ENOMEM, "buffer of %zu bytes, solver needs %zu", bytes, s->bytes);
  hipStream_t st = (hipStream_t)hip_stream;
  // captured iterations refer to the previous buffer's vectors and the operators' current data
  for (auto& g : s->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = mfq_solver::IterGraph{};
  }
  if (!s->hstat) {
    MFQ_HIP(hipHostMalloc((void**)&s->hstat, sizeof(mfq_solver::HostStatus), hipHostMallocDefault));
    std::memset(s->hstat, 0, sizeof(mfq_solver::HostStatus));
  }
  char* base = (char*)dev_buf;
  s->buf = dev_buf;
  s->state = (SolverState*)(base + s->off_state);
  s->aux = (SolverState*)(base + s->off_aux);
  s->scal = (double*)(base + s->off_aux + sizeof(SolverState));
  MFQ_HIP(launch_fill(MFQ_FP64, s->state, sizeof(SolverState) / 8, 0.0, st));
  MFQ_HIP(launch_fill(MFQ_FP64, s->aux, (sizeof(SolverState) + 64) / 8, 0.0, st));
  const int64_t N = s->op64->space->n_dofs;
  const size_t vb = round_up(N * 8, 256);
  double* k = (double*)(base + s->off_kry);
  s->r = k;
  s->p = (double*)((char*)k + vb);
  s->Ap = (double*)((char*)k + 2 * vb);
  s->z = (double*)((char*)k + 3 * vb);
  s->rout = (double*)((char*)k + 4 * vb);
  s->c = (double*)((char*)k + 5 * vb);
  if (s->kind == MFQ_SOLVER_CG) {
    // the state's reduction counter must be zero before a solve starts on any stream
    MFQ_HIP(hipStreamSynchronize(st));
    return MFQ_OK;
  }

  const int prec = s->prec_v;
  for (size_t l = 0; l < s->lv.size(); ++l) {
    Level& L = s->lv[l];
    const size_t lb = round_up(L.n * rsize(prec), 256);
    L.b = base + L.off_b;
    L.x = base + L.off_x;
    L.r = base + L.off_r;
    L.d = base + L.off_r + lb;
    L.t = base + L.off_r + 2 * lb;
    L.dinv = base + L.off_dinv;
    if (L.op && L.owns_op) {
      size_t ob;
      mfq_op_device_bytes(L.op, &ob);
      if (int rc = mfq_op_bind(L.op, base + L.off_op, ob, st)) return rc;
    }
  }
  if (s->coarse64) {
    size_t cb;
    mfq_op_device_bytes(s->coarse64, &cb);
    if (int rc = mfq_op_bind(s->coarse64, base + s->off_coarse64, cb, st)) return rc;
  }

  // diagonals and eigenvalue bounds of the smoothed levels (and of the Chebyshev coarse level):
  // all Lanczos runs are enqueued, then their traces come back in one copy (lazily bound: the
  // first step of the first solve estimates them, batched with other solves by mfq_batch_run)
  const size_t nlv = s->lv.size();
  s->trace = (double*)(base + s->off_trace);
  s->lz = (SolverState*)(base + s->off_lz);
  MFQ_HIP(launch_fill(MFQ_FP64, s->lz, nlv * round_up(sizeof(SolverState), 256) / 8, 0.0, st));
  if (!s->trace_host)
    MFQ_HIP(hipHostMalloc((void**)&s->trace_host, nlv * s->trace_stride * sizeof(double), hipHostMallocDefault));
  for (size_t l = first_estimated(s); l < nlv; ++l) {
    Level& L = s->lv[l];
    if (int rc = op_diagonal(L.op, L.dinv, st)) return rc;
    MFQ_HIP(launch_reciprocal(prec, L.dinv, L.n, st));
  }
  s->eig_pending = true;
  if (!lazy)
    if (int rc = estimate_eigenvalues(s, st)) return rc;
  if (s->prm.coarse_mode == 1) {
    MFQ_HIP(hipStreamSynchronize(st));
    return MFQ_OK;
  }
  // coarse level
  Level& C = s->lv[0];
  const int64_t nf = s->nf;
  if (s->dense) {
    s->ainv = (double*)(base + s->off_ainv);
    if (nf > 0) {
      MFQ_HIP(launch_fill(MFQ_FP64, s->ainv, nf * nf, 0.0, st));
      MFQ_HIP(launch_assemble_dense(view(s->coarse64), s->ainv, nf, st));
      std::vector<double> A((size_t)nf * nf);
      MFQ_HIP(hipMemcpyAsync(A.data(), s->ainv, A.size() * 8, hipMemcpyDeviceToHost, st));
      MFQ_HIP(hipStreamSynchronize(st));
      if (!spd_inverse(A, nf)) return fail(MFQ_ENONFINITE, "coarse matrix is not SPD");
      MFQ_HIP(hipMemcpyAsync(s->ainv, A.data(), A.size() * 8, hipMemcpyHostToDevice, st));
    }
  } else {
    const size_t cvb = round_up(C.n * 8, 256);
    char* cv = base + s->off_cvec;
    double** ptrs[7] = {&s->cb, &s->cx, &s->cr, &s->cp, &s->cAp, &s->cz, &s->cdinv};
    for (int i = 0; i < 7; ++i) *ptrs[i] = (double*)(cv + i * cvb);
    s->cstate = (SolverState*)(base + s->off_cstate);
    MFQ_HIP(launch_fill(MFQ_FP64, s->cstate, sizeof(SolverState) / 8, 0.0, st));
    if (int rc = op_diagonal(s->coarse64, s->cdinv, st)) return rc;
    MFQ_HIP(launch_reciprocal(MFQ_FP64, s->cdinv, C.n, st));
  }
  MFQ_HIP(hipStreamSynchronize(st));
  return MFQ_OK;
}

}  // namespace

extern "C" {

int mfq_solver_bind(mfq_solver* s, void* dev_buf, size_t bytes, void* hip_stream) {
  return bind_solver(s, dev_buf, bytes, hip_stream, false);
}

int mfq_solver_bind_lazy(mfq_solver* s, void* dev_buf, size_t bytes, void* hip_stream) {
  return bind_solver(s, dev_buf, bytes, hip_stream, true);
}

int mfq_solver_precondition(mfq_solver* s, const double* r, double* z, void* hip_stream) {
  if (!s) return fail(MFQ_EINVAL, "solver is NULL");
  if (!s->buf) return fail(MFQ_EINVAL, "solver is not bound");
  if (!r || !z || (reinterpret_cast<uintptr_t>(r) % 16) || (reinterpret_cast<uintptr_t>(z) % 16))
    return fail(MFQ_EINVAL, "r or z NULL or misaligned");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t N = s->op64->space->n_dofs;
  if (s->kind == MFQ_SOLVER_CG) {
    MFQ_HIP(hipMemcpyAsync(z, r, N * 8, hipMemcpyDeviceToDevice, st));
    return MFQ_OK;
  }
  if (s->eig_pending)
    if (int rc = estimate_eigenvalues(s, st)) return rc;
  return precondition(s, r, z, st);
}

int mfq_solver_lambdas(const mfq_solver* s, double* out, int n_out) {
  if (!s || !out) return fail(MFQ_EINVAL, "solver or out is NULL");
  const int m = s->lv.empty() ? 0 : (int)s->lv.size() - 1;
  if (n_out < m) return fail(MFQ_EINVAL, "need room for %d values", m);
  if (s->eig_pending) return fail(MFQ_EINVAL, "bound lazily: the estimates are made by the first solve step");
  for (int i = 0; i < m; ++i) out[i] = s->lv[i + 1].lhat;
  return MFQ_OK;
}

int mfq_solve(mfq_solver* s, const double* b, double* x, double rtol, int max_iter, void* hip_stream,
              mfq_solve_info* info) {
  if (int rc = begin_solve(s, b, x, rtol, max_iter, (hipStream_t)hip_stream)) return rc;
  mfq_solver* const one[1] = {s};
  int done = 0;
  while (!done)
    if (int rc = mfq_batch_step(one, 1, s->prm.check_every, &done)) {
      s->run.phase = Run::kIdle;
      return rc;
    }
  return mfq_solve_end(s, info);
}

int mfq_solve_begin(mfq_solver* s, const double* b, double* x, double rtol, int max_iter, void* hip_stream) {
  return begin_solve(s, b, x, rtol, max_iter, (hipStream_t)hip_stream);
}

int mfq_batch_step(mfq_solver* const* solvers, int count, int iters, int* done) {
  if (count < 0 || (count > 0 && (!solvers || !done))) return fail(MFQ_EINVAL, "bad solver list");
  if (iters < 1) return fail(MFQ_EINVAL, "iters must be >= 1");
  for (int i = 0; i < count; ++i) {
    mfq_solver* s = solvers[i];
    if (!s || s->run.phase == Run::kIdle) return fail(MFQ_EINVAL, "solver %d has no running solve", i);
    if (s->step_pending) return fail(MFQ_EBUSY, "solver %d has an asynchronous step in flight", i);
  }
  for (int i = 0; i < count; ++i) {
    mfq_solver* s = solvers[i];
    if (s->run.phase != Run::kDone)
      if (int rc = step_enqueue(s, iters)) return rc;
  }
  // one wait per distinct stream, then every solve's outcome is in pinned host memory
  std::vector<hipStream_t> seen;
  for (int i = 0; i < count; ++i) {
    mfq_solver* s = solvers[i];
    if (s->run.phase == Run::kDone) continue;
    if (std::find(seen.begin(), seen.end(), s->run.st) != seen.end()) continue;
    seen.push_back(s->run.st);
    MFQ_HIP(hipStreamSynchronize(s->run.st));
  }
  for (int i = 0; i < count; ++i) {
    mfq_solver* s = solvers[i];
    if (s->run.phase != Run::kDone)
      if (int rc = step_collect(s)) return rc;
    done[i] = s->run.phase == Run::kDone ? 1 : 0;
  }
  return MFQ_OK;
}

int mfq_batch_create(int max_solvers, mfq_batch** out) {
  if (!out) return fail(MFQ_EINVAL, "out is NULL");
  if (max_solvers < 1 || max_solvers > 4096) return fail(MFQ_EINVAL, "max_solvers %d outside [1,4096]", max_solvers);
  mfq_batch* b = new (std::nothrow) mfq_batch();
  if (!b) return fail(MFQ_ENOMEM, "host allocation failed");
  b->max_solvers = max_solvers;
  b->table_cap = round_up((size_t)max_solvers * kBatchTableBytesPerSolve, 256);
  b->state_off = b->table_cap;
  const size_t state_bytes = (size_t)max_solvers * (kStateDoubles + 1) * sizeof(double);
  const size_t trace_bytes = (size_t)max_solvers * kTraceDoubles * sizeof(double);
  b->trace_off = b->state_off + round_up(state_bytes, 256);
  b->bytes = b->trace_off + round_up(trace_bytes, 256);
  if (hipHostMalloc((void**)&b->host_tables, b->table_cap, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b->host_states, state_bytes, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b->host_traces, trace_bytes, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming) != hipSuccess) {
    delete b;
    return fail(MFQ_ENOMEM, "pinned host staging of the batch tables could not be allocated");
  }
  bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; k < mfq_batch::kSide && ok; ++k)
    ok = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    delete b;
    return fail(MFQ_EHIP, "side streams of the batch could not be created");
  }
  *out = b;
  return MFQ_OK;
}

void mfq_batch_destroy(mfq_batch* b) { delete b; }

int mfq_batch_device_bytes(const mfq_batch* b, size_t* bytes) {
  if (!b || !bytes) return fail(MFQ_EINVAL, "b or bytes is NULL");
  *bytes = b->bytes;
  return MFQ_OK;
}

int mfq_batch_bind(mfq_batch* b, void* dev_buf, size_t bytes, void* hip_stream) {
  (void)hip_stream;
  if (!b) return fail(MFQ_EINVAL, "b is NULL");
  if (!dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) % 256) != 0)
    return fail(MFQ_EINVAL, "buffer NULL or not 256-byte aligned");
  if (bytes < b->bytes) return fail(MFQ_ENOMEM, "buffer of %zu bytes, the batch needs %zu", bytes, b->bytes);
  b->buf = (char*)dev_buf;
  return MFQ_OK;
}

int mfq_batch_run(mfq_batch* b, mfq_solver* const* solvers, int count, int iters, void* hip_stream, int* done) {
  if (!b || !b->buf) return fail(MFQ_EINVAL, "batch is NULL or not bound");
  if (count < 0 || count > b->max_solvers) return fail(MFQ_EINVAL, "count %d outside [0,%d]", count, b->max_solvers);
  if (count > 0 && (!solvers || !done)) return fail(MFQ_EINVAL, "bad solver list");
  if (iters < 1) return fail(MFQ_EINVAL, "iters must be >= 1");
  hipStream_t st = (hipStream_t)hip_stream;
  const mfq_solver* lead = nullptr;  // the batched solves share its smoother and coarse degrees
  for (int i = 0; i < count; ++i) {
    mfq_solver* s = solvers[i];
    if (!s || s->run.phase == Run::kIdle) return fail(MFQ_EINVAL, "solver %d has no running solve", i);
    if (s->step_pending) return fail(MFQ_EBUSY, "solver %d has an asynchronous step in flight", i);
    if (s->run.phase != Run::kDone && s->run.st != st)
      return fail(MFQ_EINVAL, "solver %d runs on another stream than the batch step", i);
    for (int j = 0; j < i; ++j)
      if (solvers[j] == s) return fail(MFQ_EINVAL, "solver %d listed twice", i);
    if ((s->run.phase == Run::kStart || s->run.phase == Run::kInner) && batch_form(s)) {
      if (lead && (s->prm.smoother_degree != lead->prm.smoother_degree ||
                   s->prm.coarse_degree != lead->prm.coarse_degree))
        return fail(MFQ_EINVAL, "solver %d: smoother or coarse degree differs within the batch", i);
      if (!lead) lead = s;
    }
  }
  // (1) eigenvalue estimates of the lazily bound solves that start now: all their levels' Lanczos
  // runs in one set of launches, the traces gathered and read back in one copy
  std::vector<mfq_solver*> e;
  for (int i = 0; i < count; ++i) {
    mfq_solver* s = solvers[i];
    if (s->run.phase != Run::kStart || !s->eig_pending || !batch_form(s)) continue;
    if (s->lv.size() * s->trace_stride > (size_t)kTraceDoubles) continue;
    bool cube = true;  // the start vector's counter runs over the (p n + 1)^3 lattice of the level
    for (const Level& L : s->lv) {
      const int64_t N1 = (int64_t)L.sp->p * L.sp->mesh->n + 1;
      cube = cube && N1 * N1 * N1 == L.n;
    }
    if (!cube) continue;
    if (!e.empty() && s->prm.lanczos_iters != e.front()->prm.lanczos_iters) continue;
    e.push_back(s);
  }
  if (!e.empty()) {
    Plan L;
    plan_lanczos_start(L, e);
    const size_t n_start = L.launches.size();
    plan_lanczos_step(L, e);
    const size_t n_step = L.launches.size();
    double* dev_traces = (double*)(b->buf + b->trace_off);
    std::vector<VecItem> gather;
    for (size_t i = 0; i < e.size(); ++i) {
      VecItem it{};
      it.n = (int64_t)(e[i]->lv.size() * e[i]->trace_stride);
      it.a = e[i]->trace;
      it.d = dev_traces + i * kTraceDoubles;
      gather.push_back(it);
    }
    L.vec(kBatchCopy64, gather);
    if (L.tab.size() > b->table_cap)
      return fail(MFQ_EINVAL, "batch tables of %zu bytes exceed the %zu bytes for %d solvers", L.tab.size(),
                  b->table_cap, b->max_solvers);
    MFQ_HIP(hipEventSynchronize(b->uploaded));
    std::memcpy(b->host_tables, L.tab.data(), L.tab.size());
    MFQ_HIP(hipMemcpyAsync(b->buf, b->host_tables, L.tab.size(), hipMemcpyHostToDevice, st));
    MFQ_HIP(hipEventRecord(b->uploaded, st));
    Plan part;
    part.launches.assign(L.launches.begin(), L.launches.begin() + n_start);
    if (int rc = run_plan(b, part, st)) return rc;
    part.launches.assign(L.launches.begin() + n_start, L.launches.begin() + n_step);
    for (int k = 0; k < e.front()->prm.lanczos_iters; ++k)
      if (int rc = run_plan(b, part, st)) return rc;
    part.launches.assign(L.launches.begin() + n_step, L.launches.end());
    if (int rc = run_plan(b, part, st)) return rc;
    MFQ_HIP(hipMemcpyAsync(b->host_traces, dev_traces, e.size() * kTraceDoubles * sizeof(double),
                           hipMemcpyDeviceToHost, st));
    MFQ_HIP(hipStreamSynchronize(st));
    for (size_t i = 0; i < e.size(); ++i) {
      const int rc = lambdas_from_traces(e[i], b->host_traces + i * kTraceDoubles);
      if (rc == MFQ_ENONFINITE)
        finish(e[i], rc);
      else if (rc)
        return rc;
    }
  }

  // (2) one plan: the starts of pending CG passes and the residual checks ending passes (once
  // each), one CG iteration of every solve with room for `iters` (replayed), the gather of the
  // scalar states and residual norms; its tables go up in one copy
  std::vector<mfq_solver*> starting, checking, g;
  for (int i = 0; i < count; ++i) {
    mfq_solver* s = solvers[i];
    if (s->run.phase == Run::kStart && !s->eig_pending && batch_form(s)) starting.push_back(s);
    if (s->run.phase == Run::kCheck && batch_form(s)) checking.push_back(s);
  }
  Plan P;
  plan_start(P, starting);
  for (mfq_solver* s : starting) pass_started(s, s->run.start_sol);
  plan_check(P, checking);
  const size_t n_once = P.launches.size();
  for (int i = 0; i < count; ++i)
    if (batchable(solvers[i], iters)) g.push_back(solvers[i]);
  if (!g.empty()) plan_iteration(P, g);
  const size_t n_iter = P.launches.size();
  double* dev_states = (double*)(b->buf + b->state_off);
  double* dev_norms = dev_states + (size_t)b->max_solvers * kStateDoubles;
  std::vector<VecItem> gather;
  for (size_t i = 0; i < g.size(); ++i) {
    VecItem it{};
    it.n = kStateDoubles;
    it.a = g[i]->state;
    it.d = dev_states + i * kStateDoubles;
    gather.push_back(it);
  }
  for (size_t i = 0; i < checking.size(); ++i) {
    VecItem it{};
    it.n = 1;
    it.a = checking[i]->scal;
    it.d = dev_norms + i;
    gather.push_back(it);
  }
  P.vec(kBatchCopy64, gather);
  if (!P.launches.empty()) {
    if (P.tab.size() > b->table_cap)
      return fail(MFQ_EINVAL, "batch tables of %zu bytes exceed the %zu bytes for %d solvers", P.tab.size(),
                  b->table_cap, b->max_solvers);
    MFQ_HIP(hipEventSynchronize(b->uploaded));  // the staging buffer is free again
    std::memcpy(b->host_tables, P.tab.data(), P.tab.size());
    MFQ_HIP(hipMemcpyAsync(b->buf, b->host_tables, P.tab.size(), hipMemcpyHostToDevice, st));
    MFQ_HIP(hipEventRecord(b->uploaded, st));
    Plan part;
    part.launches.assign(P.launches.begin(), P.launches.begin() + n_once);
    if (int rc = run_plan(b, part, st)) return rc;
    part.launches.assign(P.launches.begin() + n_once, P.launches.begin() + n_iter);
    if (!part.launches.empty())
      for (int k = 0; k < iters; ++k)
        if (int rc = run_plan(b, part, st)) return rc;
    part.launches.assign(P.launches.begin() + n_iter, P.launches.end());
    if (int rc = run_plan(b, part, st)) return rc;
    if (!g.empty())
      MFQ_HIP(hipMemcpyAsync(b->host_states, dev_states, g.size() * kStateDoubles * sizeof(double),
                             hipMemcpyDeviceToHost, st));
    if (!checking.empty())
      MFQ_HIP(hipMemcpyAsync(b->host_states + (size_t)b->max_solvers * kStateDoubles, dev_norms,
                             checking.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    for (mfq_solver* s : g) s->run.enqueued += iters;
  }
  // (3) the other running solves (solves that cannot be batched, passes without room for `iters`)
  for (int i = 0; i < count; ++i) {
    mfq_solver* s = solvers[i];
    if (s->run.phase == Run::kDone || std::find(g.begin(), g.end(), s) != g.end() ||
        std::find(checking.begin(), checking.end(), s) != checking.end())
      continue;
    if (int rc = step_enqueue(s, iters)) return rc;
  }
  MFQ_HIP(hipStreamSynchronize(st));
  for (size_t i = 0; i < g.size(); ++i)
    std::memcpy(&g[i]->hstat->head, b->host_states + i * kStateDoubles, kStateDoubles * sizeof(double));
  for (size_t i = 0; i < checking.size(); ++i)
    checking[i]->hstat->cert = b->host_states[(size_t)b->max_solvers * kStateDoubles + i];
  for (int i = 0; i < count; ++i) {
    mfq_solver* s = solvers[i];
    if (s->run.phase != Run::kDone)
      if (int rc = step_collect(s)) return rc;
    done[i] = s->run.phase == Run::kDone ? 1 : 0;
  }
  return MFQ_OK;
}

int mfq_solve_step_async(mfq_solver* s, int iters) {
  if (!s) return fail(MFQ_EINVAL, "solver is NULL");
  if (iters < 1) return fail(MFQ_EINVAL, "iters must be >= 1");
  if (s->run.phase == Run::kIdle) return fail(MFQ_EINVAL, "no running solve");
  if (s->step_pending) return fail(MFQ_EBUSY, "the previous step has not been polled to completion");
  if (s->run.phase == Run::kDone) return MFQ_OK;
  if (!s->step_event) MFQ_HIP(hipEventCreateWithFlags(&s->step_event, hipEventDisableTiming));
  if (int rc = step_enqueue(s, iters)) return rc;
  MFQ_HIP(hipEventRecord(s->step_event, s->run.st));
  s->step_pending = true;
  return MFQ_OK;
}

int mfq_solve_step_poll(mfq_solver* s, int* ready, int* done) {
  if (!s || !ready || !done) return fail(MFQ_EINVAL, "solver, ready or done is NULL");
  *ready = 0;
  *done = s->run.phase == Run::kDone ? 1 : 0;
  if (s->run.phase == Run::kIdle) return fail(MFQ_EINVAL, "no running solve");
  if (!s->step_pending) {
    *ready = 1;
    return MFQ_OK;
  }
  const hipError_t e = hipEventQuery(s->step_event);
  if (e == hipErrorNotReady) return MFQ_OK;
  if (e != hipSuccess) return fail(MFQ_EHIP, "hipEventQuery failed: %s", hipGetErrorString(e));
  s->step_pending = false;
  if (int rc = step_collect(s)) return rc;
  *ready = 1;
  *done = s->run.phase == Run::kDone ? 1 : 0;
  return MFQ_OK;
}

int mfq_solve_end(mfq_solver* s, mfq_solve_info* info) {
  if (!s) return fail(MFQ_EINVAL, "solver is NULL");
  Run& R = s->run;
  if (R.phase != Run::kDone || s->step_pending) return fail(MFQ_EINVAL, "no finished solve");
  mfq_solve_info inf{};
  inf.iterations = R.iters;
  inf.outer_iterations = R.pass;
  inf.rel_residual = R.bb > 0 ? std::sqrt(R.rr / R.bb) : 0.0;
  inf.seconds = R.seconds;
  inf.n_levels = (int)s->lv.size();
  if (info) *info = inf;
  const int status = R.status;
  R.phase = Run::kIdle;
  if (status == MFQ_ENOCONV) return fail(MFQ_ENOCONV, "no convergence to %g within %d iterations", R.rtol, R.max_iter);
  if (status == MFQ_ENONFINITE) return fail(MFQ_ENONFINITE, "non-finite residual");
  return MFQ_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- DG-SIPG multigrid solver
// FP64 CG on the DG operator, preconditioned by an FP32 V-cycle whose finest level is the DG space
// and whose coarser levels are the continuous Q_p space on the same mesh and its hierarchy (the
// switch from the discontinuous to the continuous space inside the hierarchy of the paper's
// experiment, Sec. 6.1): Chebyshev smoothing on the DG level, the residual restricted to the
// continuous lattice (sum over the cells holding each node), the continuous GMG_MIXED V-cycle as
// the coarse correction, prolongation by copying lattice values into every cell.
struct mfq_dg_solver {
  const mfq_dg* op = nullptr;
  mfq_solver_params prm{};
  int64_t N = 0, Ncg = 0;
  mfq_mesh* mesh = nullptr;    // owned: the continuous levels' mesh (same cells)
  mfq_space* space = nullptr;  // owned: continuous Q_p with Dirichlet nodes
  mfq_op* cg_op = nullptr;     // owned FP64 continuous operator
  mfq_solver* cg = nullptr;    // owned GMG_MIXED solver on cg_op: its V-cycle is the coarse correction
  size_t off_cgop = 0, off_cgsol = 0, off_vec = 0, off_state = 0, off_trace = 0, bytes = 0;
  void* buf = nullptr;
  float *b = nullptr, *x = nullptr, *r = nullptr, *d = nullptr, *t = nullptr, *dinv = nullptr;
  double *kr = nullptr, *kp = nullptr, *kAp = nullptr, *kz = nullptr, *kc = nullptr, *kres = nullptr;
  SolverState* state = nullptr;
  SolverState* aux = nullptr;
  double* scal = nullptr;
  double* trace = nullptr;
  double* trace_host = nullptr;
  double lmin = 0, lmax = 0;
  // the V-cycle captured as a HIP graph per (stream, r, z); replayed instead of its several
  // hundred launches
  struct VcycleGraph {
    hipStream_t st = nullptr;
    const double* r = nullptr;
    double* z = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  VcycleGraph graphs[2];
  int next_graph = 0;
  ~mfq_dg_solver() {
    for (VcycleGraph& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (trace_host) (void)hipHostFree(trace_host);
    mfq_solver_destroy(cg);
    mfq_op_destroy(cg_op);
    mfq_space_destroy(space);
    mfq_mesh_destroy(mesh);
  }
};

namespace {

int dg_apply(const mfq_dg_solver* s, int prec, const void* in, void* out, hipStream_t st) {
  MFQ_HIP(launch_dg_vmult(s->op->p, s->op->n, prec, in, out, st));
  return MFQ_OK;
}

// `degree` Chebyshev updates of x for A x = b on [lmin, lmax] of D^{-1}A (FP32 DG level)
int dg_chebyshev(mfq_dg_solver* s, bool x_is_zero, hipStream_t st) {
  const int64_t n = s->N;
  const double theta = 0.5 * (s->lmax + s->lmin), delta = 0.5 * (s->lmax - s->lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  if (!x_is_zero)
    if (int rc = dg_apply(s, MFQ_FP32, s->x, s->t, st)) return rc;
  MFQ_HIP(launch_cheb_first(MFQ_FP32, s->b, s->t, s->dinv, s->x, s->r, s->d, n, 1.0 / theta, x_is_zero, st));
  // each further step is one launch: the DG product of d with the vector update in its epilogue;
  // d alternates between the d and t buffers (other cells still read the old d)
  float* dc = s->d;
  float* dn = s->t;
  for (int k = 1; k < s->prm.smoother_degree; ++k) {
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    MFQ_HIP(launch_dg_cheb_step(s->op->p, s->op->n, MFQ_FP32, dc, s->dinv, s->x, s->r, dn, rho_new * rho,
                                2.0 * rho_new / delta, st));
    std::swap(dc, dn);
    rho = rho_new;
  }
  return MFQ_OK;
}

int dg_vcycle(mfq_dg_solver* s, hipStream_t st) {
  const int p = s->op->p, n = s->op->n;
  if (int rc = dg_chebyshev(s, true, st)) return rc;
  MFQ_HIP(launch_dg_residual(p, n, MFQ_FP32, s->b, s->x, s->r, st));
  // the continuous hierarchy's finest level holds FP32 vectors of the same mesh and degree
  Level& F = s->cg->lv.back();
  MFQ_HIP(launch_dg_transfer(p, n, MFQ_FP32, false, s->r, F.b, st));
  if (int rc = vcycle(s->cg, (int)s->cg->lv.size() - 1, st)) return rc;
  MFQ_HIP(launch_dg_transfer(p, n, MFQ_FP32, true, F.x, s->t, st));
  MFQ_HIP(launch_add(MFQ_FP32, s->x, MFQ_FP32, s->t, s->N, st));
  return dg_chebyshev(s, false, st);
}

int dg_precondition_direct(mfq_dg_solver* s, const double* r, double* z, hipStream_t st) {
  MFQ_HIP(launch_cast(MFQ_FP64, r, MFQ_FP32, s->b, s->N, st));
  if (int rc = dg_vcycle(s, st)) return rc;
  MFQ_HIP(launch_cast(MFQ_FP32, s->x, MFQ_FP64, z, s->N, st));
  return MFQ_OK;
}

// Graph replay on a non-default stream when no step of the V-cycle waits on the host (dense or
// Chebyshev coarse solve of the continuous hierarchy).
int dg_precondition(mfq_dg_solver* s, const double* r, double* z, hipStream_t st) {
  if (!s->prm.use_graphs || st == nullptr || !(s->cg->dense || s->cg->prm.coarse_mode == 1))
    return dg_precondition_direct(s, r, z, st);
  hipGraphExec_t exec = nullptr;
  for (auto& g : s->graphs)
    if (g.exec && g.st == st && g.r == r && g.z == z) exec = g.exec;
  if (!exec) {
    hipGraph_t graph = nullptr;
    MFQ_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int rc = dg_precondition_direct(s, r, z, st);
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(MFQ_EHIP, "capture of the V-cycle failed: %s", hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) return fail(MFQ_EHIP, "graph instantiation failed: %s", hipGetErrorString(e2));
    auto& slot = s->graphs[s->next_graph];
    s->next_graph = (s->next_graph + 1) % 2;
    if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
    slot.st = st;
    slot.r = r;
    slot.z = z;
    slot.exec = exec;
  }
  MFQ_HIP(hipGraphLaunch(exec, st));
  return MFQ_OK;
}

}  // namespace

extern "C" {

int mfq_dg_solver_create(const mfq_dg* op, const mfq_solver_params* params, mfq_dg_solver** out) {
  if (!op || !out) return fail(MFQ_EINVAL, "op or out is NULL");
  mfq_dg_solver* s = new (std::nothrow) mfq_dg_solver();
  if (!s) return fail(MFQ_ENOMEM, "host allocation failed");
  s->op = op;
  if (params) {
    s->prm = *params;
  } else {
    mfq_solver_default_params(&s->prm);
    s->prm.smoother_degree = 6;
  }
  if (s->prm.smoother_degree < 1 || s->prm.lanczos_iters < 2) {
    delete s;
    return fail(MFQ_EINVAL, "smoother_degree must be >= 1 and lanczos_iters >= 2");
  }
  if (op->p * op->n < 2) {
    delete s;
    return fail(MFQ_EINVAL, "the continuous level has no interior node (p n = %d); need p n >= 2", op->p * op->n);
  }
  s->N = op->n_dofs;
  int rc = mfq_mesh_create(op->n, 0.0, &s->mesh);
  if (rc == MFQ_OK) rc = mfq_space_create(s->mesh, op->p, MFQ_BC_DIRICHLET0, &s->space);
  if (rc == MFQ_OK) rc = mfq_op_create(s->space, 0.0, MFQ_FP64, &s->cg_op);
  if (rc == MFQ_OK) rc = mfq_solver_create(s->cg_op, MFQ_SOLVER_GMG_MIXED, &s->prm, &s->cg);
  if (rc == MFQ_OK && s->cg->prec_v != MFQ_FP32) rc = fail(MFQ_EINVAL, "continuous hierarchy is not FP32");
  if (rc != MFQ_OK) {
    delete s;
    return rc;
  }
  s->Ncg = s->space->n_dofs;
  size_t ob = 0, sb = 0;
  mfq_op_device_bytes(s->cg_op, &ob);
  mfq_solver_device_bytes(s->cg, &sb);
  size_t off = 0;
  s->off_cgop = off;
  off += round_up(ob, 256);
  s->off_cgsol = off;
  off += round_up(sb, 256);
  s->off_vec = off;
  off += 6 * round_up(s->N * 4, 256) + 6 * round_up(s->N * 8, 256);
  s->off_state = off;
  off += round_up(2 * sizeof(SolverState) + 64, 256);
  s->off_trace = off;
  off += round_up((2 * s->prm.lanczos_iters + 1) * sizeof(double), 256);
  s->bytes = off;
  *out = s;
  return MFQ_OK;
}

void mfq_dg_solver_destroy(mfq_dg_solver* s) { delete s; }

int mfq_dg_solver_device_bytes(const mfq_dg_solver* s, size_t* bytes) {
  if (!s || !bytes) return fail(MFQ_EINVAL, "solver or bytes is NULL");
  *bytes = s->bytes;
  return MFQ_OK;
}

int mfq_dg_solver_bind(mfq_dg_solver* s, void* dev_buf, size_t bytes, void* hip_stream) {
  if (!s) return fail(MFQ_EINVAL, "solver is NULL");
  if (!dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) % 256)) return fail(MFQ_EINVAL, "buffer NULL or misaligned");
  if (bytes < s->bytes) return fail(MFQ_ENOMEM, "buffer of %zu bytes, solver needs %zu", bytes, s->bytes);
  hipStream_t st = (hipStream_t)hip_stream;
  // captured V-cycles refer to the previous buffer's vectors
  for (auto& g : s->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = mfq_dg_solver::VcycleGraph{};
  }
  char* base = (char*)dev_buf;
  size_t ob = 0, sb = 0;
  mfq_op_device_bytes(s->cg_op, &ob);
  mfq_solver_device_bytes(s->cg, &sb);
  if (int rc = mfq_op_bind(s->cg_op, base + s->off_cgop, ob, st)) return rc;
  if (int rc = mfq_solver_bind(s->cg, base + s->off_cgsol, sb, st)) return rc;
  char* v = base + s->off_vec;
  const size_t f4 = round_up(s->N * 4, 256), f8 = round_up(s->N * 8, 256);
  float** fv[6] = {&s->b, &s->x, &s->r, &s->d, &s->t, &s->dinv};
  for (int i = 0; i < 6; ++i) {
    *fv[i] = (float*)v;
    v += f4;
  }
  double** dv[6] = {&s->kr, &s->kp, &s->kAp, &s->kz, &s->kc, &s->kres};
  for (int i = 0; i < 6; ++i) {
    *dv[i] = (double*)v;
    v += f8;
  }
  s->state = (SolverState*)(base + s->off_state);
  s->aux = s->state + 1;
  s->scal = (double*)(s->aux + 1);
  s->trace = (double*)(base + s->off_trace);
  s->buf = dev_buf;
  MFQ_HIP(launch_fill(MFQ_FP64, s->state, (2 * sizeof(SolverState) + 64) / 8, 0.0, st));
  // Jacobi diagonal and the largest eigenvalue of D^{-1}A on the DG level (FP32 Lanczos)
  MFQ_HIP(launch_dg_diagonal(s->op->p, s->op->n, MFQ_FP32, s->dinv, st));
  MFQ_HIP(launch_reciprocal(MFQ_FP32, s->dinv, s->N, st));
  // lambda_override: the continuous levels' entries (levels 1.. of that hierarchy), then the DG
  // level's
  const int dg_idx = (int)s->cg->lv.size() - 1;
  if (s->prm.lambda_override && s->prm.n_lambda_override > dg_idx) {
    s->lmax = s->prm.lambda_override[dg_idx];
    s->lmin = s->lmax / s->prm.lambda_ratio;
    MFQ_HIP(hipStreamSynchronize(st));
    return MFQ_OK;
  }
  const int k = s->prm.lanczos_iters;
  MFQ_HIP(launch_splitmix(MFQ_FP32, s->r, (int64_t)s->op->n * (s->op->p + 1), 0, false, st));
  MFQ_HIP(launch_lz_init(MFQ_FP32, s->r, s->dinv, s->d, s->t, s->N, s->aux, s->trace, 2 * k, st));
  for (int it = 0; it < k; ++it) {
    if (int rc = dg_apply(s, MFQ_FP32, s->t, s->x, st)) return rc;
    MFQ_HIP(launch_lz_alpha(MFQ_FP32, s->t, s->x, s->N, s->aux, s->trace, st));
    MFQ_HIP(launch_lz_update(MFQ_FP32, s->r, s->d, s->x, s->dinv, s->N, s->aux, s->trace, 2 * k, st));
    MFQ_HIP(launch_lz_direction(MFQ_FP32, s->d, s->t, s->N, s->aux, st));
  }
  if (!s->trace_host) MFQ_HIP(hipHostMalloc((void**)&s->trace_host, (2 * k + 1) * sizeof(double), hipHostMallocDefault));
  MFQ_HIP(hipMemcpyAsync(s->trace_host, s->trace, (2 * k + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
  MFQ_HIP(hipStreamSynchronize(st));
  const double* tr = s->trace_host;
  const int m = std::min(k, std::max(0, (int)tr[2 * k]));
  if (m == 0) return fail(MFQ_ENONFINITE, "eigenvalue estimate failed on the DG level");
  std::vector<double> T((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) {
    const double ai = tr[2 * i], bi = tr[2 * i + 1];
    T[i * m + i] = 1.0 / ai + (i > 0 ? tr[2 * i - 1] / tr[2 * i - 2] : 0.0);
    if (i + 1 < m) T[i * m + i + 1] = T[(i + 1) * m + i] = std::sqrt(bi) / ai;
  }
  s->lmax = s->prm.lambda_factor * sym_max_eig(T, m);
  s->lmin = s->lmax / s->prm.lambda_ratio;
  return MFQ_OK;
}

int mfq_dg_precondition(mfq_dg_solver* s, const double* r, double* z, void* hip_stream) {
  if (!s) return fail(MFQ_EINVAL, "solver is NULL");
  if (!s->buf) return fail(MFQ_EINVAL, "solver is not bound");
  if (!r || !z) return fail(MFQ_EINVAL, "r or z is NULL");
  return dg_precondition(s, r, z, (hipStream_t)hip_stream);
}

int mfq_dg_solve(mfq_dg_solver* s, const double* b, double* x, double rtol, int max_iter, void* hip_stream,
                 mfq_solve_info* info) {
  if (!s) return fail(MFQ_EINVAL, "solver is NULL");
  if (!s->buf) return fail(MFQ_EINVAL, "solver is not bound");
  if (!b || !x || (reinterpret_cast<uintptr_t>(b) % 16) || (reinterpret_cast<uintptr_t>(x) % 16))
    return fail(MFQ_EINVAL, "b or x NULL or misaligned");
  if (!(rtol > 0 && rtol < 1)) return fail(MFQ_EINVAL, "rtol must be in (0,1)");
  if (max_iter < 1) return fail(MFQ_EINVAL, "max_iter must be >= 1");
  hipStream_t st = (hipStream_t)hip_stream;
  const auto t0 = std::chrono::steady_clock::now();
  Apply A = [s, st](const double* in, double* out) { return dg_apply(s, MFQ_FP64, in, out, st); };
  Apply M = [s, st](const double* in, double* out) { return dg_precondition(s, in, out, st); };
  PcgResult res;
  MFQ_HIP(launch_fill(MFQ_FP64, s->state, sizeof(SolverState) / 8, 0.0, st));
  if (int rc = pcg(A, &M, b, x, s->kr, s->kp, s->kAp, s->kz, s->N, s->state, rtol, max_iter, s->prm.check_every, st, res))
    return rc;
  const double bb = res.bb;
  int iters = res.iters, passes = 1;
  double rr = 0;
  int status = MFQ_OK;
  // FP64 true residual; correction passes on A c = b - A x while it is above rtol ||b||
  for (;;) {
    if (int rc = A(x, s->kAp)) return rc;
    MFQ_HIP(launch_residual_norm(b, s->kAp, s->kres, s->N, s->aux, s->scal, st));
    MFQ_HIP(hipMemcpyAsync(&rr, s->scal, sizeof(double), hipMemcpyDeviceToHost, st));
    MFQ_HIP(hipStreamSynchronize(st));
    if (!std::isfinite(rr)) {
      status = MFQ_ENONFINITE;
      break;
    }
    if (bb == 0 || rr <= rtol * rtol * bb) break;
    if (iters >= max_iter || passes >= 8) {
      status = MFQ_ENOCONV;
      break;
    }
    const double tol = std::sqrt(std::min(0.25, 0.25 * rtol * rtol * bb / rr));
    MFQ_HIP(launch_fill(MFQ_FP64, s->state, sizeof(SolverState) / 8, 0.0, st));
    PcgResult rc2;
    if (int rc = pcg(A, &M, s->kres, s->kc, s->kr, s->kp, s->kAp, s->kz, s->N, s->state, tol, max_iter - iters,
                     s->prm.check_every, st, rc2))
      return rc;
    MFQ_HIP(launch_add(MFQ_FP64, x, MFQ_FP64, s->kc, s->N, st));
    iters += rc2.iters;
    ++passes;
  }
  if (info) {
    mfq_solve_info inf{};
    inf.iterations = iters;
    inf.outer_iterations = passes;
    inf.rel_residual = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    inf.n_levels = (int)s->cg->lv.size() + 1;
    *info = inf;
  }
  if (status == MFQ_ENOCONV) return fail(MFQ_ENOCONV, "no convergence to %g within %d iterations", rtol, max_iter);
  if (status == MFQ_ENONFINITE) return fail(MFQ_ENONFINITE, "non-finite residual");
  return MFQ_OK;
}

}  // extern "C"
