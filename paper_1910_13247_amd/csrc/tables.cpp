// 1D reference data of the tensor-product element (host, FP64).
//
// The paper (Sec. 3.4) defines elements on the reference cell [0,1]^d and evaluates them at
// quadrature points, with caching of the reference data; on hexahedra elements and quadrature
// are tensor products of 1D objects (Sec. 3.1).  Node family and rule are readings: GLL nodes
// for Q_p and (p+1)-point Gauss-Legendre quadrature, computed at compile time (tables_ct.hpp);
// this file serves host copies and the level-transfer matrices.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "mfq_internal.hpp"
#include "tables_ct.hpp"

namespace mfq {

namespace {
thread_local std::string g_error;
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

namespace {
template <int P>
void copy_table(Tables1D& t) {
  constexpr const ct::Tab<P>& c = ct::kTab<P>;
  t.p = P;
  t.xi.assign(c.xi, c.xi + P + 1);
  t.zeta.assign(c.zeta, c.zeta + P + 1);
  t.omega.assign(c.omega, c.omega + P + 1);
  t.S.assign(c.S, c.S + (P + 1) * (P + 1));
  t.D.assign(c.D, c.D + (P + 1) * (P + 1));
}
}  // namespace

std::vector<double> gll_points(int p) { return tables(p).xi; }

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
    switch (p) {
      case 1: copy_table<1>(t); break;
      case 2: copy_table<2>(t); break;
      case 3: copy_table<3>(t); break;
      case 4: copy_table<4>(t); break;
      case 5: copy_table<5>(t); break;
      case 6: copy_table<6>(t); break;
      case 7: copy_table<7>(t); break;
      case 8: copy_table<8>(t); break;
      default: break;
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
