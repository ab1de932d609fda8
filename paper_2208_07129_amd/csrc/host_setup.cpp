// Host-side setup of the matrix-free operator: 1D rules, 1D basis tables with
// the weight folding of Sec. 3.2.4, and the structured-mesh numbering.
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "mf_internal.h"

namespace mf {

namespace {

// Legendre P_n(x) with first and second derivatives (Bonnet recurrence).
void legendre(int n, double x, double& P, double& dP, double& ddP) {
  double p0 = 1.0, p1 = 0.0, d1 = 0.0, dd1 = 0.0;  // p0 = P_{k-1}, p1 = P_{k-2}
  double d0 = 0.0, dd0 = 0.0;
  for (int k = 1; k <= n; ++k) {
    const double pk = ((2.0 * k - 1.0) * x * p0 - (k - 1.0) * p1) / k;
    const double dk = x * d0 + k * p0;
    const double ddk = x * dd0 + (k + 1.0) * d0;
    p1 = p0;
    p0 = pk;
    d1 = d0;
    d0 = dk;
    dd1 = dd0;
    dd0 = ddk;
  }
  (void)d1;
  (void)dd1;
  P = p0;
  dP = d0;
  ddP = dd0;
}

}  // namespace

Rule1D gauss_rule(int n) {
  Rule1D r;
  r.x.resize(n);
  r.w.resize(n);
  for (int i = 0; i < n; ++i) {
    // Chebyshev-like initial guess, ascending order
    double x = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double P, dP, ddP;
    for (int it = 0; it < 100; ++it) {
      legendre(n, x, P, dP, ddP);
      const double dx = P / dP;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    legendre(n, x, P, dP, ddP);
    r.x[i] = x;
    r.w[i] = 2.0 / ((1.0 - x * x) * dP * dP);
  }
  return r;
}

std::vector<double> gll_points(int p) {
  std::vector<double> x(p + 1);
  x[0] = -1.0;
  x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double t = -std::cos(M_PI * i / p);
    double P, dP, ddP;
    for (int it = 0; it < 100; ++it) {
      legendre(p, t, P, dP, ddP);
      const double dt = dP / ddP;
      t -= dt;
      if (std::fabs(dt) < 1e-17) break;
    }
    x[i] = t;
  }
  return x;
}

Tables1D make_tables(int p, int q) {
  Tables1D t;
  t.np = p + 1;
  t.nq = q;
  Rule1D g = gauss_rule(q);
  t.xq = g.x;
  t.wq = g.w;
  t.xn = gll_points(p);
  const int np = t.np, nq = t.nq;
  t.N.assign(nq * np, 0.0);
  t.D.assign(nq * np, 0.0);
  for (int a = 0; a < nq; ++a) {
    const double x = t.xq[a];
    for (int i = 0; i < np; ++i) {
      double L = 1.0;
      for (int m = 0; m < np; ++m)
        if (m != i) L *= (x - t.xn[m]) / (t.xn[i] - t.xn[m]);
      double dL = 0.0;
      for (int l = 0; l < np; ++l) {
        if (l == i) continue;
        double term = 1.0 / (t.xn[i] - t.xn[l]);
        for (int m = 0; m < np; ++m)
          if (m != i && m != l) term *= (x - t.xn[m]) / (t.xn[i] - t.xn[m]);
        dL += term;
      }
      t.N[a * np + i] = L;
      t.D[a * np + i] = dL;
    }
  }
  // Collocation derivative on the Gauss points, barycentric form:
  // Dt(a,b) = (lam_b / lam_a) / (x_a - x_b) for a != b, rows sum to zero.
  std::vector<double> lam(nq, 1.0);
  for (int b = 0; b < nq; ++b)
    for (int m = 0; m < nq; ++m)
      if (m != b) lam[b] /= (t.xq[b] - t.xq[m]);
  t.Dt.assign(nq * nq, 0.0);
  for (int a = 0; a < nq; ++a) {
    double diag = 0.0;
    for (int b = 0; b < nq; ++b) {
      if (a == b) continue;
      const double v = (lam[b] / lam[a]) / (t.xq[a] - t.xq[b]);
      t.Dt[a * nq + b] = v;
      diag -= v;
    }
    t.Dt[a * nq + a] = diag;
  }
  // Weight folding (Sec. 3.2.4): quadrature weights move into the 1D matrices.
  t.Nf.resize(nq * np);
  t.Dtf.resize(nq * nq);
  for (int a = 0; a < nq; ++a) {
    for (int i = 0; i < np; ++i) t.Nf[a * np + i] = t.N[a * np + i] * std::sqrt(t.wq[a]);
    for (int b = 0; b < nq; ++b) t.Dtf[a * nq + b] = t.Dt[a * nq + b] * std::sqrt(t.wq[a] / t.wq[b]);
  }
  return t;
}

void lin_matrix(const mf_box_mesh& m, double L[9]) {
  bool zero = true;
  for (int k = 0; k < 9; ++k) zero = zero && m.lin[k] == 0.0;
  for (int k = 0; k < 9; ++k) L[k] = zero ? (k % 4 == 0 ? 1.0 : 0.0) : m.lin[k];
}

static double det3(const double A[9]) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

int validate_mesh(const mf_box_mesh* m) {
  if (!m) return fail(MF_ERR_ARG, "mesh is NULL");
  for (int d = 0; d < 3; ++d) {
    if (m->n[d] < 1) return fail(MF_ERR_ARG, "mesh: n[d] must be >= 1");
    if (!(std::isfinite(m->lo[d]) && std::isfinite(m->hi[d]) && m->hi[d] > m->lo[d]))
      return fail(MF_ERR_ARG, "mesh: need finite lo < hi");
  }
  if (m->bc != MF_BC_NONE && m->bc != MF_BC_DIRICHLET0 && m->bc != MF_BC_PERIODIC)
    return fail(MF_ERR_UNSUPPORTED, "mesh: unknown boundary condition");
  double L[9];
  lin_matrix(*m, L);
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(L[k])) return fail(MF_ERR_ARG, "mesh: non-finite linear map");
  if (!(det3(L) > 0.0)) return fail(MF_ERR_ARG, "mesh: linear map must have positive determinant");
  return MF_OK;
}

int64_t nodes_per_dir(const mf_box_mesh& m, int p, int d) {
  return (int64_t)m.n[d] * p + (m.bc == MF_BC_PERIODIC ? 0 : 1);
}

}  // namespace mf
