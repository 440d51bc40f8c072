// Device-resident scalar state of one Krylov solve (CG / PCG / iterative refinement).
#pragma once

#include <cstdint>

namespace mfq {

constexpr int kStatePartials = 1024;

struct SolverState {
  double bb;          // ||b||^2
  double rr;          // ||r||^2 of the current (recurred) residual
  double rz;          // r.z (r.r when unpreconditioned)
  double pAp;
  double alpha, beta;
  double tol2;        // rtol^2: converged when rr <= tol2 * bb
  double res2;        // scratch: last true residual norm^2
  int iter;           // iterations done
  int done;           // 1 once converged or non-finite; later kernels become no-ops
  int converged_iter;
  int nonfinite;
  unsigned counter;   // last-block counter of the grid reductions (reset to 0 after use)
  unsigned pad_[3];
  double partials[kStatePartials];
};

}  // namespace mfq
