// 1D reference data of the tensor-product element (host, FP64).
//
// The paper (Sec. 3.4) defines elements on the reference cell [0,1]^d and evaluates them at
// quadrature points, with caching of the reference data; on hexahedra elements and quadrature
// are tensor products of 1D objects (Sec. 3.1).  Node family and rule are readings: GLL nodes
// for Q_p and (p+1)-point Gauss-Legendre quadrature.  Both are computed here by Newton's method
// on the three-term Legendre recurrence.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "mfq_internal.hpp"

namespace mfq {

namespace {
thread_local std::string g_error;

// Legendre P_k(s) and its first two derivatives at s in (-1,1), by the Bonnet recurrence
// (k+1) P_{k+1} = (2k+1) s P_k - k P_{k-1}, and P' from (1-s^2) P_k' = k (P_{k-1} - s P_k).
void legendre(int k, double s, double& P, double& dP, double& d2P) {
  double p0 = 1.0, p1 = s;
  if (k == 0) {
    P = 1.0; dP = 0.0; d2P = 0.0;
    return;
  }
  for (int j = 1; j < k; ++j) {
    double p2 = ((2.0 * j + 1.0) * s * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = k * (p0 - s * p1) / (1.0 - s * s);
  // Legendre ODE: (1-s^2) P'' - 2 s P' + k(k+1) P = 0
  d2P = (2.0 * s * dP - k * (k + 1.0) * P) / (1.0 - s * s);
}
}  // namespace

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
}

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

const char* last_error_cstr() { return g_error.c_str(); }

void gauss_points(int nq, std::vector<double>& x, std::vector<double>& w) {
  // roots of P_nq; Chebyshev-like initial guesses, Newton on P_nq, weights 2/((1-s^2) P'^2)
  x.assign(nq, 0.0);
  w.assign(nq, 0.0);
  for (int k = 0; k < nq; ++k) {
    double s = -std::cos(M_PI * (k + 0.75) / (nq + 0.5));
    double P, dP, d2P;
    for (int it = 0; it < 100; ++it) {
      legendre(nq, s, P, dP, d2P);
      double ds = P / dP;
      s -= ds;
      if (std::fabs(ds) < 1e-17) break;
    }
    legendre(nq, s, P, dP, d2P);
    x[k] = 0.5 * (s + 1.0);
    w[k] = 1.0 / ((1.0 - s * s) * dP * dP);  // 2/(...) on [-1,1], halved on [0,1]
  }
  // symmetrise (removes last-bit asymmetry of the Newton iterates)
  for (int k = 0; k < nq / 2; ++k) {
    double a = 0.5 * (x[k] + (1.0 - x[nq - 1 - k]));
    x[k] = a;
    x[nq - 1 - k] = 1.0 - a;
    double b = 0.5 * (w[k] + w[nq - 1 - k]);
    w[k] = w[nq - 1 - k] = b;
  }
  if (nq % 2 == 1) x[nq / 2] = 0.5;
}

std::vector<double> gll_points(int p) {
  // 0, 1 and the roots of P_p'(2t-1): Newton on P_p' using P_p'' from the Legendre ODE
  std::vector<double> x(p + 1);
  x[0] = 0.0;
  x[p] = 1.0;
  for (int k = 1; k < p; ++k) {
    double s = -std::cos(M_PI * k / p);
    double P, dP, d2P;
    for (int it = 0; it < 100; ++it) {
      legendre(p, s, P, dP, d2P);
      double ds = dP / d2P;
      s -= ds;
      if (std::fabs(ds) < 1e-17) break;
    }
    x[k] = 0.5 * (s + 1.0);
  }
  for (int k = 1; k <= (p - 1) / 2; ++k) {
    double a = 0.5 * (x[k] + (1.0 - x[p - k]));
    x[k] = a;
    x[p - k] = 1.0 - a;
  }
  if (p % 2 == 0) x[p / 2] = 0.5;
  return x;
}

double lagrange_value(const std::vector<double>& nodes, int a, double t) {
  double v = 1.0;
  for (size_t b = 0; b < nodes.size(); ++b)
    if ((int)b != a) v *= (t - nodes[b]) / (nodes[a] - nodes[b]);
  return v;
}

double lagrange_derivative(const std::vector<double>& nodes, int a, double t) {
  double sum = 0.0;
  for (size_t c = 0; c < nodes.size(); ++c) {
    if ((int)c == a) continue;
    double term = 1.0 / (nodes[a] - nodes[c]);
    for (size_t b = 0; b < nodes.size(); ++b)
      if ((int)b != a && b != c) term *= (t - nodes[b]) / (nodes[a] - nodes[b]);
    sum += term;
  }
  return sum;
}

const Tables1D& tables(int p) {
  static Tables1D cache[kMaxDegree + 1];
  static std::once_flag once[kMaxDegree + 1];
  std::call_once(once[p], [p] {
    Tables1D& t = cache[p];
    t.p = p;
    t.xi = gll_points(p);
    gauss_points(p + 1, t.zeta, t.omega);
    const int n1 = p + 1;
    t.S.resize(n1 * n1);
    t.D.resize(n1 * n1);
    for (int q = 0; q < n1; ++q)
      for (int a = 0; a < n1; ++a) {
        t.S[q * n1 + a] = lagrange_value(t.xi, a, t.zeta[q]);
        t.D[q * n1 + a] = lagrange_derivative(t.xi, a, t.zeta[q]);
      }
  });
  return cache[p];
}

std::vector<double> transfer_matrix_1d(int pc, int pf, bool h_transfer, int* nf1) {
  const std::vector<double> xc = gll_points(pc);
  std::vector<double> pos;
  if (h_transfer) {
    // fine nodes of the two halves [0,1/2] and [1/2,1] (the midpoint once)
    for (int i = 0; i <= pc; ++i) pos.push_back(0.5 * xc[i]);
    for (int i = 1; i <= pc; ++i) pos.push_back(0.5 + 0.5 * xc[i]);
  } else {
    pos = gll_points(pf);
  }
  *nf1 = (int)pos.size();
  std::vector<double> P((size_t)pos.size() * (pc + 1));
  for (size_t i = 0; i < pos.size(); ++i)
    for (int a = 0; a <= pc; ++a) P[i * (pc + 1) + a] = lagrange_value(xc, a, pos[i]);
  return P;
}

}  // namespace mfq
