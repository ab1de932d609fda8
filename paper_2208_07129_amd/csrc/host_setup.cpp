// Host-side setup of the matrix-free operator: 1D rules and basis tables (the
// constexpr code of sf_tables.h, evaluated at run time) and mesh validation.
#include <cmath>
#include <cstring>
#include <algorithm>
#include <stdexcept>

#include "mf_internal.h"
#include "sf_tables.h"

namespace mf {

Rule1D gauss_rule(int n) {
  Rule1D r;
  r.x.resize(n);
  r.w.resize(n);
  ct::gauss(n, r.x.data(), r.w.data());
  return r;
}

std::vector<double> gll_points(int p) {
  std::vector<double> x(p + 1);
  ct::gll(p, x.data());
  return x;
}

Tables1D make_tables(int p, int q) {
  Tables1D t;
  t.np = p + 1;
  t.nq = q;
  t.xq.resize(q);
  t.wq.resize(q);
  t.xn.resize(p + 1);
  t.N.resize(q * (p + 1));
  t.D.resize(q * (p + 1));
  t.Dt.resize(q * q);
  t.Nf.resize(q * (p + 1));
  t.Dtf.resize(q * q);
  ct::tables(p + 1, q, t.xq.data(), t.wq.data(), t.xn.data(), t.N.data(), t.D.data(), t.Dt.data(),
             t.Nf.data(), t.Dtf.data());
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

double cell_factor(const double L[9], const double h[3], double mu, double G6[6]) {
  double J[9], Ji[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) J[3 * r + c] = L[3 * r + c] * 0.5 * h[c];
  const double detJ = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                      J[2] * (J[3] * J[7] - J[4] * J[6]);
  Ji[0] = (J[4] * J[8] - J[5] * J[7]) / detJ;
  Ji[1] = (J[2] * J[7] - J[1] * J[8]) / detJ;
  Ji[2] = (J[1] * J[5] - J[2] * J[4]) / detJ;
  Ji[3] = (J[5] * J[6] - J[3] * J[8]) / detJ;
  Ji[4] = (J[0] * J[8] - J[2] * J[6]) / detJ;
  Ji[5] = (J[2] * J[3] - J[0] * J[5]) / detJ;
  Ji[6] = (J[3] * J[7] - J[4] * J[6]) / detJ;
  Ji[7] = (J[1] * J[6] - J[0] * J[7]) / detJ;
  Ji[8] = (J[0] * J[4] - J[1] * J[3]) / detJ;
  double G[9];  // mu det J J^-1 J^-T
  for (int s = 0; s < 3; ++s)
    for (int d = 0; d < 3; ++d) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += Ji[3 * s + k] * Ji[3 * d + k];
      G[3 * s + d] = mu * detJ * acc;
    }
  G6[0] = G[0];
  G6[1] = G[1];
  G6[2] = G[2];
  G6[3] = G[4];
  G6[4] = G[5];
  G6[5] = G[8];
  return detJ;
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

std::vector<int> cell_colours(const int n[3], const bool periodic[3]) {
  for (int d = 0; d < 3; ++d)
    if (periodic[d] && n[d] == 1) return {};
  const int64_t ne = (int64_t)n[0] * n[1] * n[2];
  std::vector<int> col(ne);
  auto c1 = [&](int d, int c) { return (periodic[d] && n[d] % 2 == 1 && c == n[d] - 1) ? 2 : c % 2; };
  for (int64_t e = 0; e < ne; ++e) {
    const int cx = (int)(e % n[0]), cy = (int)((e / n[0]) % n[1]), cz = (int)(e / ((int64_t)n[0] * n[1]));
    col[e] = c1(0, cx) + 3 * (c1(1, cy) + 3 * c1(2, cz));
  }
  return col;
}

std::vector<int32_t> cell_order(const int n[3]) {
  struct Blk {
    int lo[3], hi[3];
  };
  std::vector<Blk> blocks{Blk{{0, 0, 0}, {n[0], n[1], n[2]}}};
  for (int level = 0; level < 3; ++level) {  // 8 blocks: one per XCD
    std::vector<Blk> next;
    for (const Blk& b : blocks) {
      int d = 0;
      for (int k = 1; k < 3; ++k)
        if (b.hi[k] - b.lo[k] > b.hi[d] - b.lo[d]) d = k;
      const int len = b.hi[d] - b.lo[d];
      if (len < 2) {
        next.push_back(b);
        continue;
      }
      Blk a = b, c = b;
      a.hi[d] = b.lo[d] + len / 2;
      c.lo[d] = a.hi[d];
      next.push_back(a);
      next.push_back(c);
    }
    blocks.swap(next);
  }
  auto morton = [](uint32_t x, uint32_t y, uint32_t z) {
    uint64_t code = 0;
    for (int bit = 0; bit < 21; ++bit) {
      code |= (uint64_t)((x >> bit) & 1) << (3 * bit);
      code |= (uint64_t)((y >> bit) & 1) << (3 * bit + 1);
      code |= (uint64_t)((z >> bit) & 1) << (3 * bit + 2);
    }
    return code;
  };
  std::vector<int32_t> order;
  order.reserve((size_t)n[0] * n[1] * n[2]);
  for (const Blk& b : blocks) {
    std::vector<std::pair<uint64_t, int32_t>> cells;
    for (int z = b.lo[2]; z < b.hi[2]; ++z)
      for (int y = b.lo[1]; y < b.hi[1]; ++y)
        for (int x = b.lo[0]; x < b.hi[0]; ++x)
          cells.emplace_back(morton(x - b.lo[0], y - b.lo[1], z - b.lo[2]),
                             (int32_t)(x + n[0] * (y + (int64_t)n[1] * z)));
    std::sort(cells.begin(), cells.end());
    for (auto& c : cells) order.push_back(c.second);
  }
  return order;
}

int64_t nodes_per_dir(const mf_box_mesh& m, int p, int d) {
  return (int64_t)m.n[d] * p + (m.bc == MF_BC_PERIODIC ? 0 : 1);
}

}  // namespace mf
