// 1D rules and basis tables of the sum factorisation, as constexpr code.
//
// The same functions run at compile time, where they turn the weight-folded
// 1D matrices of each (p, q) instantiation into literal constants of the
// kernels (uniform operands: no loads, no registers spent on holding them),
// and at run time on the host (mf_basis_1d and the operator setup).
//
//  - Gauss-Legendre points: roots of P_q by Newton's method on the three-term
//    recurrence; weights 2 / ((1 - x^2) P_q'(x)^2).
//  - Gauss-Lobatto-Legendre nodes: -1, the roots of P_p', +1 (Sec. 2.2.2).
//  - N(a, i) = L_i(xq_a), D(a, i) = L_i'(xq_a): Lagrange basis on the GLL nodes.
//  - Dt(a, b) = l_b'(xq_a): collocation derivative on the Gauss points, in
//    barycentric form, so that D = Dt N (eq. DU) when q >= p + 1.
//  - Folding (Sec. 3.2.4): Nf(a, i) = N(a, i) sqrt(w_a),
//    Dtf(a, b) = Dt(a, b) sqrt(w_a / w_b); the quadrature weights then drop out
//    of the per-point scaling factors.
#pragma once

namespace mf {
namespace ct {

constexpr double kPi = 3.14159265358979323846;

constexpr double sqrt_(double x) {
  if (!(x > 0.0)) return 0.0;
  double g = x < 1.0 ? 1.0 : x;
  for (int i = 0; i < 300; ++i) {
    const double n = 0.5 * (g + x / g);
    if (n == g) break;
    g = n;
  }
  return g;
}

// cos on [0, pi] by its Taylor series: used only for Newton starting points.
constexpr double cos_(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

constexpr double abs_(double x) { return x < 0.0 ? -x : x; }

// P_n(x) and its first two derivatives.
constexpr void legendre(int n, double x, double& P, double& dP, double& ddP) {
  double pk = 1.0, pkm1 = 0.0, dk = 0.0, ddk = 0.0;
  for (int k = 1; k <= n; ++k) {
    const double pn = ((2.0 * k - 1.0) * x * pk - (k - 1.0) * pkm1) / k;
    const double dn = x * dk + k * pk;
    const double ddn = x * ddk + (k + 1.0) * dk;
    pkm1 = pk;
    pk = pn;
    dk = dn;
    ddk = ddn;
  }
  P = pk;
  dP = dk;
  ddP = ddk;
}

constexpr void gauss(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double t = -cos_(kPi * (i + 0.75) / (n + 0.5));
    double P = 0, dP = 0, ddP = 0;
    for (int it = 0; it < 100; ++it) {
      legendre(n, t, P, dP, ddP);
      const double dt = P / dP;
      t -= dt;
      if (abs_(dt) < 1e-17) break;
    }
    legendre(n, t, P, dP, ddP);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dP * dP);
  }
}

constexpr void gll(int p, double* x) {
  x[0] = -1.0;
  x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double t = -cos_(kPi * i / p);
    double P = 0, dP = 0, ddP = 0;
    for (int it = 0; it < 100; ++it) {
      legendre(p, t, P, dP, ddP);
      const double dt = dP / ddP;
      t -= dt;
      if (abs_(dt) < 1e-17) break;
    }
    x[i] = t;
  }
}

// All tables for np = p + 1 nodes and nq points; arrays row-major, point major.
constexpr void tables(int np, int nq, double* xq, double* wq, double* xn, double* N, double* D,
                      double* Dt, double* Nf, double* Dtf) {
  gauss(nq, xq, wq);
  gll(np - 1, xn);
  for (int a = 0; a < nq; ++a) {
    const double x = xq[a];
    for (int i = 0; i < np; ++i) {
      double L = 1.0;
      for (int m = 0; m < np; ++m)
        if (m != i) L *= (x - xn[m]) / (xn[i] - xn[m]);
      double dL = 0.0;
      for (int l = 0; l < np; ++l) {
        if (l == i) continue;
        double term = 1.0 / (xn[i] - xn[l]);
        for (int m = 0; m < np; ++m)
          if (m != i && m != l) term *= (x - xn[m]) / (xn[i] - xn[m]);
        dL += term;
      }
      N[a * np + i] = L;
      D[a * np + i] = dL;
      Nf[a * np + i] = L * sqrt_(wq[a]);
    }
  }
  // barycentric weights of the Gauss points (bounded size: nq <= 16)
  double lam[16] = {};
  for (int b = 0; b < nq; ++b) {
    lam[b] = 1.0;
    for (int m = 0; m < nq; ++m)
      if (m != b) lam[b] /= (xq[b] - xq[m]);
  }
  for (int a = 0; a < nq; ++a) {
    double diag = 0.0;
    for (int b = 0; b < nq; ++b) {
      if (a == b) continue;
      const double v = (lam[b] / lam[a]) / (xq[a] - xq[b]);
      Dt[a * nq + b] = v;
      diag -= v;
    }
    Dt[a * nq + a] = diag;
    for (int b = 0; b < nq; ++b) Dtf[a * nq + b] = Dt[a * nq + b] * sqrt_(wq[a] / wq[b]);
  }
}

}  // namespace ct

template <int NP, int NQ>
struct CtTables {
  double xq[NQ], wq[NQ], xn[NP];
  double N[NQ * NP], D[NQ * NP], Dt[NQ * NQ];
  double Nf[NQ * NP], Dtf[NQ * NQ];
  // Lf = Dtf^T Dtf: on an axis-aligned cell the 3x3 factor of eq. sjacobian is
  // diagonal and the two derivative stages of direction s collapse into one
  // symmetric NQ x NQ contraction g_ss Lf along s.
  double Lf[NQ * NQ];
};

template <int NP, int NQ>
constexpr CtTables<NP, NQ> make_ct_tables() {
  CtTables<NP, NQ> t{};
  ct::tables(NP, NQ, t.xq, t.wq, t.xn, t.N, t.D, t.Dt, t.Nf, t.Dtf);
  for (int a = 0; a < NQ; ++a)
    for (int b = 0; b < NQ; ++b) {
      double acc = 0.0;
      for (int k = 0; k < NQ; ++k) acc += t.Dtf[k * NQ + a] * t.Dtf[k * NQ + b];
      t.Lf[a * NQ + b] = acc;
    }
  return t;
}

// Compile-time folded tables of one (NP, NQ) instantiation.
template <int NP, int NQ>
struct Tab {
  static constexpr CtTables<NP, NQ> v = make_ct_tables<NP, NQ>();
};

}  // namespace mf
