// Compile-time 1D reference data of Q_p (GLL nodes, Gauss rule, Lagrange values and derivatives
// at the Gauss points), shared by host code and kernels.
//
// The paper (Sec. 3.4) defines elements on the reference cell and notes that reference data at
// the quadrature points is computed once and cached; on hexahedra both element and quadrature
// are tensor products of 1D objects (Sec. 3.1).  Readings: Gauss-Lobatto-Legendre nodes and the
// (p+1)-point Gauss-Legendre rule on [0,1].  Computed here in constexpr arithmetic (IEEE
// round-to-nearest, the same operations at compile time as at run time) by Newton's method on
// the three-term Legendre recurrence, so kernels see the tables as immediate constants.
#pragma once

namespace mfq {
namespace ct {

constexpr double kPi = 3.14159265358979323846;

// cos on [0, pi] by its Taylor series (initial guesses for Newton only)
constexpr double cos_guess(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

constexpr double fabs_(double x) { return x < 0 ? -x : x; }

// Legendre P_k(s), P_k'(s), P_k''(s) for s in (-1,1): Bonnet recurrence
// (j+1) P_{j+1} = (2j+1) s P_j - j P_{j-1}; (1-s^2) P_k' = k (P_{k-1} - s P_k); Legendre ODE for P''.
struct Leg {
  double P, dP, d2P;
};
constexpr Leg legendre(int k, double s) {
  double p0 = 1.0, p1 = s;
  if (k == 0) return Leg{1.0, 0.0, 0.0};
  for (int j = 1; j < k; ++j) {
    const double p2 = ((2.0 * j + 1.0) * s * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
  }
  const double dP = k * (p0 - s * p1) / (1.0 - s * s);
  const double d2P = (2.0 * s * dP - k * (k + 1.0) * p1) / (1.0 - s * s);
  return Leg{p1, dP, d2P};
}

template <int P>
struct Tab {
  static constexpr int N1 = P + 1;
  double xi[N1]{};     // GLL nodes on [0,1]
  double zeta[N1]{};   // Gauss points on [0,1]
  double omega[N1]{};  // Gauss weights, sum 1
  double S[N1 * N1]{}; // S[q*N1+a] = l_a(zeta_q)
  double D[N1 * N1]{}; // D[q*N1+a] = l_a'(zeta_q)

  constexpr Tab() {
    // GLL: 0, 1, roots of P_P'(2t-1)
    xi[0] = 0.0;
    xi[P] = 1.0;
    for (int k = 1; k < P; ++k) {
      double s = -cos_guess(kPi * k / P);
      for (int it = 0; it < 100; ++it) {
        const Leg l = legendre(P, s);
        const double ds = l.dP / l.d2P;
        s -= ds;
        if (fabs_(ds) < 1e-17) break;
      }
      xi[k] = 0.5 * (s + 1.0);
    }
    for (int k = 1; k <= (P - 1) / 2; ++k) {
      const double a = 0.5 * (xi[k] + (1.0 - xi[P - k]));
      xi[k] = a;
      xi[P - k] = 1.0 - a;
    }
    if (P % 2 == 0) xi[P / 2] = 0.5;
    // Gauss: roots of P_N1(2t-1), weights 1/((1-s^2) P'(s)^2)
    for (int k = 0; k < N1; ++k) {
      const double x = kPi * (k + 0.75) / (N1 + 0.5);
      double s = -cos_guess(x);
      for (int it = 0; it < 100; ++it) {
        const Leg l = legendre(N1, s);
        const double ds = l.P / l.dP;
        s -= ds;
        if (fabs_(ds) < 1e-17) break;
      }
      const Leg l = legendre(N1, s);
      zeta[k] = 0.5 * (s + 1.0);
      omega[k] = 1.0 / ((1.0 - s * s) * l.dP * l.dP);
    }
    for (int k = 0; k < N1 / 2; ++k) {
      const double a = 0.5 * (zeta[k] + (1.0 - zeta[N1 - 1 - k]));
      zeta[k] = a;
      zeta[N1 - 1 - k] = 1.0 - a;
      const double b = 0.5 * (omega[k] + omega[N1 - 1 - k]);
      omega[k] = omega[N1 - 1 - k] = b;
    }
    if (N1 % 2 == 1) zeta[N1 / 2] = 0.5;
    // Lagrange values and derivatives (product rule over the dropped factor)
    for (int q = 0; q < N1; ++q)
      for (int a = 0; a < N1; ++a) {
        const double t = zeta[q];
        double v = 1.0;
        for (int b = 0; b < N1; ++b)
          if (b != a) v *= (t - xi[b]) / (xi[a] - xi[b]);
        double d = 0.0;
        for (int c = 0; c < N1; ++c) {
          if (c == a) continue;
          double term = 1.0 / (xi[a] - xi[c]);
          for (int b = 0; b < N1; ++b)
            if (b != a && b != c) term *= (t - xi[b]) / (xi[a] - xi[b]);
          d += term;
        }
        S[q * N1 + a] = v;
        D[q * N1 + a] = d;
      }
  }
};

template <int P>
inline constexpr Tab<P> kTab{};

}  // namespace ct
}  // namespace mfq
