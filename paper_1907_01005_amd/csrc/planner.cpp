// Host planning: 1D basis, Hilbert order, row/column blocking, BCSR pattern,
// apply work list and the block-product list of the overlap.
//
// Built with -ffp-contract=off so that the geometric predicates below
// (which batch holds a centre, which batch centres lie within the support
// radius) round exactly as written.
#include "planner.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <iterator>
#include <numeric>

namespace mfb {

// ---------------------------------------------------------------- 1D basis
namespace {

// Legendre P_n(t) and P_n'(t) by the three-term recurrence.
void legendre(int n, double t, double& P, double& dP) {
  double p0 = 1.0, p1 = t;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = (std::fabs(t) < 1.0) ? n * (t * p1 - p0) / (t * t - 1.0) : 0.0;
}

double lagrange(const std::vector<double>& x, int k, double t) {
  double v = 1.0;
  for (size_t j = 0; j < x.size(); ++j)
    if ((int)j != k) v *= (t - x[j]) / (x[k] - x[j]);
  return v;
}

double lagrange_d(const std::vector<double>& x, int k, double t) {
  double s = 0.0;
  for (size_t j = 0; j < x.size(); ++j) {
    if ((int)j == k) continue;
    double term = 1.0 / (x[k] - x[j]);
    for (size_t l = 0; l < x.size(); ++l)
      if ((int)l != k && l != j) term *= (t - x[l]) / (x[k] - x[l]);
    s += term;
  }
  return s;
}

}  // namespace

Basis1D make_basis(int p) {
  Basis1D b;
  b.p = p;
  b.n = p + 1;
  const int n = b.n;
  // Gauss-Legendre: Newton on P_n from Chebyshev-like guesses.
  std::vector<double> t(n), w(n);
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, x, P, dP);
      double dx = P / dP;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    double P, dP;
    legendre(n, x, P, dP);
    t[i] = x;
    w[i] = 2.0 / ((1.0 - x * x) * dP * dP);
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int c) { return t[a] < t[c]; });
  b.xq.resize(n);
  b.wq.resize(n);
  for (int i = 0; i < n; ++i) {
    b.xq[i] = 0.5 * (1.0 + t[idx[i]]);
    b.wq[i] = 0.5 * w[idx[i]];
  }
  // Gauss-Lobatto-Legendre: end points and the roots of P_p'.
  std::vector<double> g;
  g.push_back(-1.0);
  for (int i = p - 1; i >= 1; --i) {
    double x = std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, x, P, dP);
      double d2P = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);
      double dx = dP / d2P;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    g.push_back(x);
  }
  g.push_back(1.0);
  std::sort(g.begin(), g.end());
  b.nodes.resize(n);
  for (int i = 0; i < n; ++i) b.nodes[i] = 0.5 * (1.0 + g[i]);
  if (p % 2 == 0) b.nodes[p / 2] = 0.5;  // exact midpoint for even degree
  b.S.resize(n * n);
  b.Dco.resize(n * n);
  for (int q = 0; q < n; ++q)
    for (int k = 0; k < n; ++k) {
      b.S[q * n + k] = lagrange(b.nodes, k, b.xq[q]);
      b.Dco[q * n + k] = lagrange_d(b.xq, k, b.xq[q]);
    }
  return b;
}

// ---------------------------------------------------------------- Hilbert
// Skilling (2004): transform the axes to the "transposed" Hilbert index by
// undoing excess work per bit plane, Gray encoding, then read the bits plane
// by plane (most significant first, axis x first within a plane).
uint64_t hilbert3(uint32_t x, uint32_t y, uint32_t z, int bits) {
  uint32_t a[3] = {x, y, z};
  const uint32_t top = 1u << (bits - 1);
  for (uint32_t q = top; q > 1; q >>= 1) {
    const uint32_t low = q - 1;
    for (int i = 0; i < 3; ++i) {
      if (a[i] & q) {
        a[0] ^= low;
      } else {
        uint32_t t = (a[0] ^ a[i]) & low;
        a[0] ^= t;
        a[i] ^= t;
      }
    }
  }
  a[1] ^= a[0];
  a[2] ^= a[1];
  uint32_t t = 0;
  for (uint32_t q = top; q > 1; q >>= 1)
    if (a[2] & q) t ^= q - 1;
  for (int i = 0; i < 3; ++i) a[i] ^= t;
  uint64_t h = 0;
  for (int b = bits - 1; b >= 0; --b)
    for (int i = 0; i < 3; ++i) h = (h << 1) | ((a[i] >> b) & 1u);
  return h;
}

int bits_for(int extent) {
  int b = 1;
  while ((1 << b) < extent) ++b;
  return b;
}

// ---------------------------------------------------------------- mesh
void plan_mesh(MeshPlan& m, const int nc[3], const double L[3], int degree, unsigned dirichlet,
               int order) {
  for (int d = 0; d < 3; ++d) {
    if (nc[d] <= 0 || nc[d] % 2 != 0)
      throw Error(-1, "cell counts must be positive and even (2x2x2 batches)");
    if (!(L[d] > 0.0) || !std::isfinite(L[d])) throw Error(-1, "box lengths must be positive");
  }
  if (degree < 1 || degree > kMaxDeg) throw Error(-2, "only degrees 1 to 6 are implemented");
  if (order != 0 && order != 1) throw Error(-1, "order must be 0 (Hilbert) or 1 (lexicographic)");
  if (dirichlet > 0x3F) throw Error(-1, "dirichlet_faces has bits beyond the 6 faces");
  m.p = degree;
  m.n = degree + 1;
  m.NB = 2 * degree + 1;
  m.dirichlet = dirichlet;
  m.order = order;
  for (int d = 0; d < 3; ++d) {
    m.nc[d] = nc[d];
    m.L[d] = L[d];
    m.h[d] = L[d] / nc[d];
    m.nb[d] = nc[d] / 2;
    m.na[d] = (int64_t)degree * nc[d] + 1;
  }
  const int64_t nbatch64 = (int64_t)m.nb[0] * m.nb[1] * m.nb[2];
  if (nbatch64 > (1 << 30)) throw Error(-1, "mesh too large");
  m.nbatch = (int)nbatch64;
  m.N = m.na[0] * m.na[1] * m.na[2];
  m.ncells = (int64_t)nc[0] * nc[1] * nc[2];
  m.basis = make_basis(degree);

  // batch order (Alg. 1 step 2)
  const int nbt = m.nbatch;
  std::vector<uint64_t> key(nbt);
  const int bits = bits_for(std::max(m.nb[0], std::max(m.nb[1], m.nb[2])));
  for (int b = 0; b < nbt; ++b) {
    int bx, by, bz;
    m.batch_coords(b, bx, by, bz);
    key[b] = (order == 0) ? hilbert3(bx, by, bz, bits) : (uint64_t)b;
  }
  m.batch_order.resize(nbt);
  std::iota(m.batch_order.begin(), m.batch_order.end(), 0);
  std::stable_sort(m.batch_order.begin(), m.batch_order.end(),
                   [&](int a, int c) { return key[a] < key[c]; });
  m.batch_rank.resize(nbt);
  for (int r = 0; r < nbt; ++r) m.batch_rank[m.batch_order[r]] = r;

  // Dirichlet nodes
  m.is_dirichlet.assign(m.N, 0);
  for (int64_t Z = 0; Z < m.na[2]; ++Z)
    for (int64_t Y = 0; Y < m.na[1]; ++Y)
      for (int64_t X = 0; X < m.na[0]; ++X) {
        const int64_t c[3] = {X, Y, Z};
        bool on = false;
        for (int d = 0; d < 3; ++d) {
          if ((dirichlet >> (2 * d)) & 1u) on |= (c[d] == 0);
          if ((dirichlet >> (2 * d + 1)) & 1u) on |= (c[d] == m.na[d] - 1);
        }
        m.is_dirichlet[m.node_id(X, Y, Z)] = on;
      }

  // first-encounter row numbering and row blocks (Alg. 1 steps 5-7)
  const int P2 = 2 * degree;
  m.node_rb.assign(m.N, -1);
  m.node_row.assign(m.N, -1);
  m.dof_perm.resize(m.N);
  m.rb_start.resize(nbt + 1);
  int64_t cnt = 0;
  for (int r = 0; r < nbt; ++r) {
    m.rb_start[r] = cnt;
    int bx, by, bz;
    m.batch_coords(m.batch_order[r], bx, by, bz);
    for (int k = 0; k <= P2; ++k)
      for (int j = 0; j <= P2; ++j)
        for (int i = 0; i <= P2; ++i) {
          const int64_t g = m.node_id((int64_t)P2 * bx + i, (int64_t)P2 * by + j, (int64_t)P2 * bz + k);
          if (m.node_rb[g] < 0) {
            m.node_rb[g] = r;
            m.node_row[g] = cnt;
            m.dof_perm[cnt++] = g;
          }
        }
  }
  m.rb_start[nbt] = cnt;
  if (cnt != m.N) throw Error(-1, "internal: row numbering does not cover the mesh");

  // per-batch gather tables: owner slot and row of every batch node
  const int NB = m.NB, NB3 = NB * NB * NB;
  m.gtab.assign((size_t)nbt * NB3, -1);
  for (int r = 0; r < nbt; ++r) {
    int bx, by, bz;
    m.batch_coords(m.batch_order[r], bx, by, bz);
    for (int k = 0; k < NB; ++k)
      for (int j = 0; j < NB; ++j)
        for (int i = 0; i < NB; ++i) {
          const int64_t g = m.node_id((int64_t)P2 * bx + i, (int64_t)P2 * by + j, (int64_t)P2 * bz + k);
          if (m.is_dirichlet[g]) continue;
          const int ro = m.node_rb[g];
          int ox, oy, oz;
          m.batch_coords(m.batch_order[ro], ox, oy, oz);
          const int dx = ox - bx, dy = oy - by, dz = oz - bz;
          if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1)
            throw Error(-1, "internal: node owner is not a neighbour batch");
          const int slot = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
          const int64_t row = m.node_row[g] - m.rb_start[ro];
          m.gtab[(size_t)r * NB3 + i + NB * (j + NB * k)] = (int32_t)((slot << 24) | row);
        }
  }
  m.cV.clear();
  m.has_potential = false;
}

void mesh_cells(const MeshPlan& m, int32_t* ijk) {
  for (int r = 0; r < m.nbatch; ++r) {
    int bx, by, bz;
    m.batch_coords(m.batch_order[r], bx, by, bz);
    for (int e = 0; e < 8; ++e) {
      const int64_t c = 8 * (int64_t)r + e;
      ijk[3 * c + 0] = 2 * bx + (e & 1);
      ijk[3 * c + 1] = 2 * by + ((e >> 1) & 1);
      ijk[3 * c + 2] = 2 * bz + (e >> 2);
    }
  }
}

namespace {
// Global node ids of cell (cx, cy, cz) in local order i + n j + n^2 k.
void cell_node_ids(const MeshPlan& m, const int32_t* ijk, int64_t* ids) {
  const int n = m.n, p = m.p;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        ids[i + n * (j + n * k)] =
            m.node_id((int64_t)p * ijk[0] + i, (int64_t)p * ijk[1] + j, (int64_t)p * ijk[2] + k);
}
}  // namespace

void mesh_node_points(const MeshPlan& m, double* xyz) {
  if (m.curved) {
    std::copy(m.nodes.begin(), m.nodes.end(), xyz);
    return;
  }
  std::vector<double> pos[3];
  for (int d = 0; d < 3; ++d) {
    pos[d].resize(m.na[d]);
    for (int64_t X = 0; X < m.na[d]; ++X) {
      const int64_t c = std::min<int64_t>(X / m.p, m.nc[d] - 1);
      pos[d][X] = (c + m.basis.nodes[X - m.p * c]) * m.h[d];
    }
  }
  for (int64_t Z = 0; Z < m.na[2]; ++Z)
    for (int64_t Y = 0; Y < m.na[1]; ++Y)
      for (int64_t X = 0; X < m.na[0]; ++X) {
        double* o = xyz + 3 * m.node_id(X, Y, Z);
        o[0] = pos[0][X];
        o[1] = pos[1][Y];
        o[2] = pos[2][Z];
      }
}

void mesh_set_nodes(MeshPlan& m, const double* xyz) {
  const int n = m.n, n3 = n * n * n;
  // phi_k and phi_k' of the GLL basis at the Gauss points
  std::vector<double> dphi(n * n);
  for (int q = 0; q < n; ++q)
    for (int k = 0; k < n; ++k) dphi[q * n + k] = lagrange_d(m.basis.nodes, k, m.basis.xq[q]);
  const std::vector<double>& phi = m.basis.S;
  m.nodes.assign(xyz, xyz + 3 * m.N);
  m.cG.assign((size_t)m.ncells * 6 * n3, 0.0);
  m.cJ.assign((size_t)m.ncells * n3, 0.0);
  std::vector<int32_t> ijk(3 * m.ncells);
  mesh_cells(m, ijk.data());
  std::vector<int64_t> ids(n3);
  for (int64_t c = 0; c < m.ncells; ++c) {
    cell_node_ids(m, ijk.data() + 3 * c, ids.data());
    for (int q3 = 0; q3 < n; ++q3)
      for (int q2 = 0; q2 < n; ++q2)
        for (int q1 = 0; q1 < n; ++q1) {
          const int q = q1 + n * (q2 + n * q3);
          // J[a][b] = dx_a / dxi_b = sum_k x_k,a dN_k/dxi_b
          double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
          for (int k3 = 0; k3 < n; ++k3)
            for (int k2 = 0; k2 < n; ++k2)
              for (int k1 = 0; k1 < n; ++k1) {
                const double* x = xyz + 3 * ids[k1 + n * (k2 + n * k3)];
                const double s1 = phi[q1 * n + k1], s2 = phi[q2 * n + k2], s3 = phi[q3 * n + k3];
                const double d[3] = {dphi[q1 * n + k1] * s2 * s3, s1 * dphi[q2 * n + k2] * s3,
                                     s1 * s2 * dphi[q3 * n + k3]};
                for (int a = 0; a < 3; ++a)
                  for (int b = 0; b < 3; ++b) J[a][b] += x[a] * d[b];
              }
          const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                             J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                             J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
          if (!std::isfinite(det) || det == 0.0)
            throw Error(-1, "a cell's Jacobian is singular at a quadrature point");
          // inverse by cofactors: Ji[a][b] = cof(J)[b][a] / det
          double Ji[3][3];
          Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
          Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
          Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
          Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
          Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
          Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
          Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
          Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
          Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
          const double jxw = m.basis.wq[q1] * m.basis.wq[q2] * m.basis.wq[q3] * std::fabs(det);
          auto g = [&](int a, int b) {
            return 0.5 * jxw * (Ji[a][0] * Ji[b][0] + Ji[a][1] * Ji[b][1] + Ji[a][2] * Ji[b][2]);
          };
          double* G = m.cG.data() + c * 6 * n3;
          G[0 * n3 + q] = g(0, 0);
          G[1 * n3 + q] = g(1, 1);
          G[2 * n3 + q] = g(2, 2);
          G[3 * n3 + q] = g(0, 1);
          G[4 * n3 + q] = g(0, 2);
          G[5 * n3 + q] = g(1, 2);
          m.cJ[c * n3 + q] = jxw;
        }
  }
  m.curved = true;
}

void mesh_qp_points(const MeshPlan& m, double* xyz) {
  const int n = m.n, n3 = n * n * n;
  std::vector<int32_t> ijk(3 * m.ncells);
  mesh_cells(m, ijk.data());
  if (m.curved) {
    // x(xi_q) = sum_k x_k N_k(xi_q) over the cell's own nodes
    const std::vector<double>& phi = m.basis.S;
    std::vector<int64_t> ids(n3);
    for (int64_t c = 0; c < m.ncells; ++c) {
      cell_node_ids(m, ijk.data() + 3 * c, ids.data());
      for (int q3 = 0; q3 < n; ++q3)
        for (int q2 = 0; q2 < n; ++q2)
          for (int q1 = 0; q1 < n; ++q1) {
            double* o = xyz + 3 * (c * n3 + q1 + n * (q2 + n * q3));
            o[0] = o[1] = o[2] = 0.0;
            for (int k3 = 0; k3 < n; ++k3)
              for (int k2 = 0; k2 < n; ++k2)
                for (int k1 = 0; k1 < n; ++k1) {
                  const double w = phi[q1 * n + k1] * phi[q2 * n + k2] * phi[q3 * n + k3];
                  const double* x = m.nodes.data() + 3 * ids[k1 + n * (k2 + n * k3)];
                  for (int a = 0; a < 3; ++a) o[a] += w * x[a];
                }
          }
    }
    return;
  }
  for (int64_t c = 0; c < m.ncells; ++c)
    for (int q3 = 0; q3 < n; ++q3)
      for (int q2 = 0; q2 < n; ++q2)
        for (int q1 = 0; q1 < n; ++q1) {
          double* o = xyz + 3 * (c * n3 + q1 + n * (q2 + n * q3));
          o[0] = (ijk[3 * c + 0] + m.basis.xq[q1]) * m.h[0];
          o[1] = (ijk[3 * c + 1] + m.basis.xq[q2]) * m.h[1];
          o[2] = (ijk[3 * c + 2] + m.basis.xq[q3]) * m.h[2];
        }
}

void mesh_set_potential(MeshPlan& m, const double* v) {
  const int n = m.n, n3 = n * n * n;
  const double det = m.h[0] * m.h[1] * m.h[2];
  m.cV.resize((size_t)m.ncells * n3);
  for (int64_t c = 0; c < m.ncells; ++c)
    for (int q3 = 0; q3 < n; ++q3)
      for (int q2 = 0; q2 < n; ++q2)
        for (int q1 = 0; q1 < n; ++q1) {
          const int64_t i = c * n3 + q1 + n * (q2 + n * q3);
          const double jxw =
              m.curved ? m.cJ[i] : m.basis.wq[q1] * m.basis.wq[q2] * m.basis.wq[q3] * det;
          m.cV[i] = jxw * v[i];
        }
  m.has_potential = true;
}

// ---------------------------------------------------------------- layouts
int64_t MvPlan::block_index(int r, int C) const {
  const int32_t* b = colidx.data() + rowptr[r];
  const int32_t* e = colidx.data() + rowptr[r + 1];
  const int32_t* it = std::lower_bound(b, e, C);
  if (it != e && *it == C) return rowptr[r] + (it - b);
  return -1;
}

// Overlap products of Alg. 8 for S = A^T B (A and B have the same rows and
// columns): every pair of a stored block of A and a stored block of B in the
// same row block.  Partial products are stored pair by pair (row-block order
// within a pair), so that the second stage streams one contiguous run per
// block of S.  The plan goes into `mv`.
void plan_overlap(MvPlan& mv, const MvPlan& A, const MvPlan& B, const MeshPlan& m) {
  const int nbt = m.nbatch, ncb = A.ncb;
  std::vector<int32_t> w(ncb);
  for (int C = 0; C < ncb; ++C) w[C] = A.cb_start[C + 1] - A.cb_start[C];
  mv.units.clear();
  mv.pair_tab.assign((size_t)ncb * ncb, -1);
  int npairs = 0;
  for (int r = 0; r < nbt; ++r)
    for (int64_t k1 = A.rowptr[r]; k1 < A.rowptr[r + 1]; ++k1)
      for (int64_t k2 = B.rowptr[r]; k2 < B.rowptr[r + 1]; ++k2) {
        int32_t& pid = mv.pair_tab[(size_t)A.colidx[k1] * ncb + B.colidx[k2]];
        if (pid < 0) pid = npairs++;
      }
  std::vector<int32_t> pair_c1(npairs), pair_c2(npairs);
  for (int C1 = 0; C1 < ncb; ++C1)
    for (int C2 = 0; C2 < ncb; ++C2) {
      const int32_t pid = mv.pair_tab[(size_t)C1 * ncb + C2];
      if (pid >= 0) { pair_c1[pid] = C1; pair_c2[pid] = C2; }
    }

  // Tasks: runs of up to kTaskMaxSeg consecutive densely populated row blocks
  // over the union of their column blocks.  A row block qualifies on its own
  // (pairs, widths, rows); a run grows while the union stays within the
  // task limits and costs at most kTaskMaxWaste times the members' products.
  auto rows_of = [&](int r) { return (int64_t)(m.rb_start[r + 1] - m.rb_start[r]); };
  auto width = [&](const std::vector<int32_t>& cs) {
    int64_t s = 0;
    for (int C : cs) s += w[C];
    return s;
  };
  auto blocks = [&](const MvPlan& L, int r) {
    return std::vector<int32_t>(L.colidx.begin() + L.rowptr[r], L.colidx.begin() + L.rowptr[r + 1]);
  };
  auto qualifies = [&](int r) {
    const int64_t ka = A.rowptr[r + 1] - A.rowptr[r], kb = B.rowptr[r + 1] - B.rowptr[r];
    return ka * kb >= kTaskMinPairs && ka * kb <= kTaskMaxPairs &&
           width(blocks(A, r)) <= kTaskMaxWidth && width(blocks(B, r)) <= kTaskMaxWidth &&
           rows_of(r) <= kTaskMaxRows;
  };
  // widths of the task kernel classes: a run stays in its widest member's
  auto task_width_cap = [](int64_t wmax) -> int64_t { return wmax <= 64 ? 64 : (wmax <= 96 ? 96 : 128); };
  auto merged = [](const std::vector<int32_t>& x, const std::vector<int32_t>& y) {
    std::vector<int32_t> u;
    std::set_union(x.begin(), x.end(), y.begin(), y.end(), std::back_inserter(u));
    return u;
  };
  std::vector<int32_t> run_len(nbt, 0);  // > 0 at the first row block of a run
  for (int r = 0; r < nbt;) {
    if (!qualifies(r)) { ++r; continue; }
    std::vector<int32_t> ua = blocks(A, r), ub = blocks(B, r);
    int64_t rows = rows_of(r);
    double own = (double)rows * width(ua) * width(ub);
    int64_t wcap = task_width_cap(std::max(width(ua), width(ub)));
    int len = 1;
    while (len < kTaskMaxSeg && r + len < nbt && qualifies(r + len)) {
      const int q = r + len;
      std::vector<int32_t> na = merged(ua, blocks(A, q)), nb = merged(ub, blocks(B, q));
      const int64_t nrows = rows + rows_of(q);
      const double nown = own + (double)rows_of(q) * width(blocks(A, q)) * width(blocks(B, q));
      const int64_t ncap =
          std::max(wcap, task_width_cap(std::max(width(blocks(A, q)), width(blocks(B, q)))));
      if (width(na) > ncap || width(nb) > ncap ||
          (int64_t)na.size() * (int64_t)nb.size() > kTaskMaxPairs || nrows > kTaskMaxRunRows ||
          (double)nrows * width(na) * width(nb) > kTaskMaxWaste * nown)
        break;
      ua.swap(na);
      ub.swap(nb);
      rows = nrows;
      own = nown;
      wcap = ncap;
      ++len;
    }
    run_len[r] = len;
    r += len;
  }
  // the union blocks of a run and which of their pairs meet in some member
  struct Run {
    std::vector<int32_t> ua, ub;
    std::vector<char> meet;  // [ua.size()][ub.size()]
  };
  auto run_of = [&](int r) {
    Run R;
    for (int q = r; q < r + run_len[r]; ++q) {
      R.ua = merged(R.ua, blocks(A, q));
      R.ub = merged(R.ub, blocks(B, q));
    }
    R.meet.assign(R.ua.size() * R.ub.size(), 0);
    for (int q = r; q < r + run_len[r]; ++q)
      for (int64_t k1 = A.rowptr[q]; k1 < A.rowptr[q + 1]; ++k1)
        for (int64_t k2 = B.rowptr[q]; k2 < B.rowptr[q + 1]; ++k2) {
          const size_t i = std::lower_bound(R.ua.begin(), R.ua.end(), A.colidx[k1]) - R.ua.begin();
          const size_t j = std::lower_bound(R.ub.begin(), R.ub.end(), B.colidx[k2]) - R.ub.begin();
          R.meet[i * R.ub.size() + j] = 1;
        }
    return R;
  };

  // one partial per (unit) and per (run, pair meeting in it)
  std::vector<int64_t> pair_count(npairs, 0);
  for (int r = 0; r < nbt;) {
    if (run_len[r] > 0) {
      const Run R = run_of(r);
      for (size_t i = 0; i < R.ua.size(); ++i)
        for (size_t j = 0; j < R.ub.size(); ++j)
          if (R.meet[i * R.ub.size() + j]) ++pair_count[mv.pair_tab[(size_t)R.ua[i] * ncb + R.ub[j]]];
      r += run_len[r];
      continue;
    }
    for (int64_t k1 = A.rowptr[r]; k1 < A.rowptr[r + 1]; ++k1)
      for (int64_t k2 = B.rowptr[r]; k2 < B.rowptr[r + 1]; ++k2)
        ++pair_count[mv.pair_tab[(size_t)A.colidx[k1] * ncb + B.colidx[k2]]];
    ++r;
  }
  // pair_ptr: first slot of each pair; pair_list[pid] = partial base
  mv.pair_ptr.assign(npairs + 1, 0);
  mv.pair_list.assign(npairs, 0);
  int64_t part = 0;
  for (int pid = 0; pid < npairs; ++pid) {
    mv.pair_ptr[pid + 1] = mv.pair_ptr[pid] + (int32_t)pair_count[pid];
    mv.pair_list[pid] = part;
    part += pair_count[pid] * (int64_t)w[pair_c1[pid]] * w[pair_c2[pid]];
  }
  mv.part_doubles = part;
  std::vector<int64_t> fill(npairs, 0);
  mv.tasks.clear();
  mv.task_blk.clear();
  mv.task_part.clear();
  for (int r = 0; r < nbt;) {
    if (run_len[r] > 0) {
      // the run as one task; task_blk holds [segment][union block] per side
      // (offset -1 where the member does not store the block)
      const Run R = run_of(r);
      const int ns = run_len[r];
      TmTask T{};
      T.ka = (int32_t)R.ua.size();
      T.kb = (int32_t)R.ub.size();
      T.nseg = ns;
      T.seg_start[0] = 0;
      for (int sgi = 0; sgi < ns; ++sgi)
        T.seg_start[sgi + 1] = T.seg_start[sgi] + (int32_t)rows_of(r + sgi);
      for (int sgi = ns + 1; sgi <= kTaskMaxSeg; ++sgi) T.seg_start[sgi] = T.seg_start[ns];
      T.rows = T.seg_start[ns];
      auto side = [&](const MvPlan& L, const std::vector<int32_t>& u, int32_t& wsum) {
        const int64_t first = (int64_t)mv.task_blk.size();
        for (int sgi = 0; sgi < ns; ++sgi) {
          const int q = r + sgi;
          int32_t col = 0;
          for (int C : u) {
            const int32_t* b = std::lower_bound(L.colidx.data() + L.rowptr[q],
                                                L.colidx.data() + L.rowptr[q + 1], C);
            const bool has = b != L.colidx.data() + L.rowptr[q + 1] && *b == C;
            const int64_t off = has ? L.block_offset[b - L.colidx.data()] : -1;
            mv.task_blk.push_back(TaskBlk{off, col, w[C]});
            col += w[C];
          }
          wsum = col;
        }
        return first;
      };
      T.a_first = side(A, R.ua, T.wa);
      T.b_first = side(B, R.ub, T.wb);
      T.p_first = (int64_t)mv.task_part.size();
      for (size_t i = 0; i < R.ua.size(); ++i)
        for (size_t j = 0; j < R.ub.size(); ++j) {
          if (!R.meet[i * R.ub.size() + j]) {
            mv.task_part.push_back(-1);
            continue;
          }
          const int32_t pid = mv.pair_tab[(size_t)R.ua[i] * ncb + R.ub[j]];
          mv.task_part.push_back(mv.pair_list[pid] + fill[pid]++ * (int64_t)w[R.ua[i]] * w[R.ub[j]]);
        }
      mv.tasks.push_back(T);
      r += ns;
      continue;
    }
    const int64_t rows = rows_of(r);
    for (int64_t k1 = A.rowptr[r]; k1 < A.rowptr[r + 1]; ++k1)
      for (int64_t k2 = B.rowptr[r]; k2 < B.rowptr[r + 1]; ++k2) {
        const int C1 = A.colidx[k1], C2 = B.colidx[k2];
        const int32_t pid = mv.pair_tab[(size_t)C1 * ncb + C2];
        const int64_t E = (int64_t)w[C1] * w[C2];
        TmUnit u;
        u.off1 = A.block_offset[k1];
        u.off2 = B.block_offset[k2];
        u.part = mv.pair_list[pid] + fill[pid]++ * E;
        u.rows = (int32_t)rows;
        u.w1 = w[C1];
        u.w2 = w[C2];
        u.tslot = C1 == C2 ? -2 : -1;  // a diagonal block of S: slot assigned below
        mv.units.push_back(u);
      }
    ++r;
  }
  mv.s2.assign((size_t)ncb * ncb, S2Desc{0, 0, 0, 0, 0, 0, 0});
  for (int C1 = 0; C1 < ncb; ++C1)
    for (int C2 = 0; C2 < ncb; ++C2) {
      S2Desc& d = mv.s2[(size_t)C1 * ncb + C2];
      const int32_t pid = mv.pair_tab[(size_t)C1 * ncb + C2];
      d.base = pid >= 0 ? mv.pair_list[pid] : 0;
      d.n = pid >= 0 ? mv.pair_ptr[pid + 1] - mv.pair_ptr[pid] : 0;
      d.c1 = A.cb_start[C1];
      d.c2 = A.cb_start[C2];
      d.w1 = w[C1];
      d.w2 = w[C2];
    }
  // longest sums first: the workgroups start in this order, so the blocks
  // with the most partials do not end up last on a busy CU
  std::stable_sort(mv.s2.begin(), mv.s2.end(),
                   [](const S2Desc& x, const S2Desc& y) { return x.n > y.n; });
  // one overlap kernel per class, each with its own thread count and
  // register budget
  auto tm_class = [](const TmUnit& u) {
    const bool shortb = u.rows <= 128;
    if (u.w1 == 8 && u.w2 == 8 && shortb) return 0;
    if (u.w1 <= 8 && u.w2 <= 8) return 1;
    return shortb ? 2 : 3;
  };
  std::stable_sort(mv.units.begin(), mv.units.end(),
                   [&](const TmUnit& x, const TmUnit& y) { return tm_class(x) < tm_class(y); });
  mv.tm_class_end.fill(0);
  for (const TmUnit& u : mv.units)
    for (int c = tm_class(u); c < 4; ++c) ++mv.tm_class_end[c];
  // the products with C1 = C2 (same column block on both sides: A and B
  // share the column blocks) carry the trace; one slot each, in unit order
  mv.ndiag = 0;
  for (TmUnit& u : mv.units) u.tslot = u.tslot == -2 ? (int32_t)mv.ndiag++ : -1;
  // tasks by register tile: 4, 6 or 8 columns of each block product per thread
  auto task_class = [](const TmTask& T) {
    const int wmax = T.wa > T.wb ? T.wa : T.wb;
    return wmax <= 64 ? 0 : (wmax <= 96 ? 1 : 2);
  };
  std::stable_sort(mv.tasks.begin(), mv.tasks.end(),
                   [&](const TmTask& x, const TmTask& y) { return task_class(x) < task_class(y); });
  mv.task_class_end.fill(0);
  for (const TmTask& T : mv.tasks)
    for (int c = task_class(T); c < 3; ++c) ++mv.task_class_end[c];
}

void plan_mv(MvPlan& mv, const MeshPlan& m, int M, const double* centers, const double* radius,
             int radius_count, int ncolblocks, const int32_t* sizes, int B, int col_order) {
  if (M <= 0) throw Error(-1, "M must be positive");
  if (!centers || !radius) throw Error(-1, "null centres or radius");
  if (radius_count != 1 && radius_count != M) throw Error(-1, "radius_count must be 1 or M");
  for (int a = 0; a < radius_count; ++a)
    if (!(radius[a] >= 0.0) || !std::isfinite(radius[a])) throw Error(-1, "bad radius");
  for (int a = 0; a < 3 * M; ++a)
    if (!std::isfinite(centers[a])) throw Error(-1, "non-finite centre");
  if (col_order != 0 && col_order != 1) throw Error(-1, "col_order must be 0 or 1");
  mv.mesh = &m;
  mv.M = M;

  // column blocks (Alg. 2 step 4)
  std::vector<int32_t> w;
  if (sizes) {
    if (ncolblocks <= 0) throw Error(-1, "ncolblocks must be positive");
    int64_t s = 0;
    for (int i = 0; i < ncolblocks; ++i) {
      if (sizes[i] <= 0) throw Error(-1, "column block sizes must be positive");
      s += sizes[i];
      w.push_back(sizes[i]);
    }
    if (s != M) throw Error(-1, "column block sizes must sum to M");
  } else {
    if (B <= 0) throw Error(-1, "block size B must be positive");
    const int nblk = std::max(1, M / B);
    w.assign(nblk, B);
    w.back() += M - B * nblk;
  }
  for (int x : w)
    if (x > 16) throw Error(-2, "column blocks wider than 16 are not supported");
  mv.ncb = (int)w.size();
  mv.cb_start.resize(mv.ncb + 1);
  mv.cb_start[0] = 0;
  for (int i = 0; i < mv.ncb; ++i) mv.cb_start[i + 1] = mv.cb_start[i] + w[i];
  mv.cb_of_col.resize(M);
  for (int C = 0; C < mv.ncb; ++C)
    for (int c = mv.cb_start[C]; c < mv.cb_start[C + 1]; ++c) mv.cb_of_col[c] = C;

  // column order (Alg. 2 steps 1-3): Hilbert index of the batch holding the centre
  const int bits = bits_for(std::max(m.nb[0], std::max(m.nb[1], m.nb[2])));
  std::vector<uint64_t> key(M);
  for (int a = 0; a < M; ++a) {
    int bc[3];
    for (int d = 0; d < 3; ++d) {
      const double f = std::floor((centers[3 * a + d] * m.nb[d]) / m.L[d]);
      int k = (f < 0.0) ? 0 : (f > m.nb[d] - 1 ? m.nb[d] - 1 : (int)f);
      bc[d] = k;
    }
    key[a] = (col_order == 0) ? hilbert3(bc[0], bc[1], bc[2], bits) : (uint64_t)a;
  }
  mv.col_perm.resize(M);
  std::iota(mv.col_perm.begin(), mv.col_perm.end(), 0);
  std::stable_sort(mv.col_perm.begin(), mv.col_perm.end(),
                   [&](int a, int c) { return key[a] < key[c]; });
  mv.col_pos.resize(M);
  for (int c = 0; c < M; ++c) mv.col_pos[mv.col_perm[c]] = c;

  // stored blocks: row block r's batch within the radius of an orbital of C
  const int nbt = m.nbatch, ncb = mv.ncb;
  std::vector<uint8_t> stored((size_t)nbt * ncb, 0);
  for (int a = 0; a < M; ++a) {
    const double* c = centers + 3 * a;
    const double r = radius[radius_count == 1 ? 0 : a];
    const int C = mv.cb_of_col[mv.col_pos[a]];
    int lo[3], hi[3];
    bool empty = false;
    for (int d = 0; d < 3; ++d) {
      lo[d] = m.nb[d];
      hi[d] = -1;
      for (int b = 0; b < m.nb[d]; ++b) {
        const double bcd = (2.0 * b + 1.0) * m.h[d];
        if (std::fabs(bcd - c[d]) <= r * (1.0 + 1e-12)) {
          lo[d] = std::min(lo[d], b);
          hi[d] = std::max(hi[d], b);
        }
      }
      if (hi[d] < lo[d]) empty = true;
    }
    if (empty) continue;
    for (int bz = lo[2]; bz <= hi[2]; ++bz)
      for (int by = lo[1]; by <= hi[1]; ++by)
        for (int bx = lo[0]; bx <= hi[0]; ++bx) {
          const double dx = (2.0 * bx + 1.0) * m.h[0] - c[0];
          const double dy = (2.0 * by + 1.0) * m.h[1] - c[1];
          const double dz = (2.0 * bz + 1.0) * m.h[2] - c[2];
          const double d2 = (dx * dx + dy * dy) + dz * dz;
          if (d2 <= r * r) {
            const int b = bx + m.nb[0] * (by + m.nb[1] * bz);
            stored[(size_t)m.batch_rank[b] * ncb + C] = 1;
          }
        }
  }
  mv.rowptr.assign(nbt + 1, 0);
  mv.colidx.clear();
  for (int r = 0; r < nbt; ++r) {
    for (int C = 0; C < ncb; ++C)
      if (stored[(size_t)r * ncb + C]) mv.colidx.push_back(C);
    mv.rowptr[r + 1] = (int64_t)mv.colidx.size();
  }
  const int64_t nblocks = (int64_t)mv.colidx.size();
  mv.block_offset.assign(nblocks + 1, 0);
  for (int r = 0; r < nbt; ++r) {
    const int64_t rows = m.rb_start[r + 1] - m.rb_start[r];
    for (int64_t k = mv.rowptr[r]; k < mv.rowptr[r + 1]; ++k)
      mv.block_offset[k + 1] = mv.block_offset[k] + rows * w[mv.colidx[k]];
  }

  // apply work list: (batch, C) for every C stored in a row block owning a
  // non-Dirichlet node of the batch; one item per 8-column chunk of C.
  const int NB = m.NB, NB3 = NB * NB * NB, n = m.n;
  mv.items.clear();
  mv.item_cb.clear();
  std::vector<ApplyItem> shell;  // batches whose own block is not stored for C
  std::vector<int32_t> shell_cb;
  mv.apply_pairs = mv.apply_pairs_own = 0;
  mv.cell_colblocks.assign(m.ncells, 0);
  std::vector<int> mark(ncb, 0), list;
  for (int r = 0; r < nbt; ++r) {
    int owner[27];
    for (int s = 0; s < 27; ++s) owner[s] = -1;
    const int32_t* g = m.gtab.data() + (size_t)r * NB3;
    int bx, by, bz;
    m.batch_coords(m.batch_order[r], bx, by, bz);
    for (int v = 0; v < NB3; ++v)
      if (g[v] >= 0) {
        const int s = g[v] >> 24;
        const int ox = bx + (s % 3) - 1, oy = by + ((s / 3) % 3) - 1, oz = bz + (s / 9) - 1;
        owner[s] = m.batch_rank[ox + m.nb[0] * (oy + m.nb[1] * oz)];
      }
    list.clear();
    for (int s = 0; s < 27; ++s) {
      if (owner[s] < 0) continue;
      for (int64_t k = mv.rowptr[owner[s]]; k < mv.rowptr[owner[s] + 1]; ++k) {
        const int C = mv.colidx[k];
        if (!mark[C]) { mark[C] = 1; list.push_back(C); }
      }
    }
    std::sort(list.begin(), list.end());
    std::vector<std::array<int64_t, 27>> offs(list.size());
    for (size_t li = 0; li < list.size(); ++li) {
      const int C = list[li];
      mark[C] = 0;
      ApplyItem it;
      it.rank = r;
      it.ld = w[C];
      for (int s = 0; s < 27; ++s) {
        const int64_t k = owner[s] >= 0 ? mv.block_index(owner[s], C) : -1;
        it.off[s] = k >= 0 ? mv.block_offset[k] : -1;
        offs[li][s] = it.off[s];
      }
      ++mv.apply_pairs;
      const bool own = mv.block_index(r, C) >= 0;
      if (own) ++mv.apply_pairs_own;
      for (int c0 = 0; c0 < w[C]; c0 += 8) {
        it.c0 = c0;
        it.nc = std::min(8, w[C] - c0);
        (own ? mv.items : shell).push_back(it);
        (own ? mv.item_cb : shell_cb).push_back(C);
      }
    }
    // non-empty column blocks per cell (Table 1, last row)
    for (int e = 0; e < 8; ++e) {
      uint32_t smask = 0;
      const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
      for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            const int v = (ex * m.p + i) + NB * ((ey * m.p + j) + NB * (ez * m.p + k));
            if (g[v] >= 0) smask |= 1u << (g[v] >> 24);
          }
      int cntc = 0;
      for (size_t li = 0; li < list.size(); ++li) {
        bool any = false;
        for (int s = 0; s < 27 && !any; ++s)
          if (((smask >> s) & 1u) && offs[li][s] >= 0) any = true;
        cntc += any;
      }
      mv.cell_colblocks[8 * (int64_t)r + e] = cntc;
    }
  }

  // own items first, then the shell items (processed by a separate kernel)
  mv.n_own_items = (int64_t)mv.items.size();
  mv.items.insert(mv.items.end(), shell.begin(), shell.end());
  mv.item_cb.insert(mv.item_cb.end(), shell_cb.begin(), shell_cb.end());

  // per item, the value offset of every batch node's row in its block of C,
  // at the item's first column (-1 when the node is on a Dirichlet face or
  // its block is not stored)
  if (mv.block_offset.back() >= ((int64_t)1 << 31))
    throw Error(-2, "multivectors of 2^31 or more stored values are not supported");
  mv.rowoff.assign(mv.items.size() * (size_t)NB3, -1);
  for (size_t q = 0; q < mv.items.size(); ++q) {
    const ApplyItem& it = mv.items[q];
    const int32_t* g = m.gtab.data() + (size_t)it.rank * NB3;
    int32_t* ro = mv.rowoff.data() + q * NB3;
    for (int v = 0; v < NB3; ++v) {
      if (g[v] < 0) continue;
      const int64_t o = it.off[g[v] >> 24];
      if (o < 0) continue;
      ro[v] = (int32_t)(o + (int64_t)(g[v] & 0xFFFFFF) * it.ld + it.c0);
    }
  }
  // compact lists of the present row offsets of the shell items
  mv.shell_ptr.assign(1, 0);
  mv.shell_ro.clear();
  for (size_t q = (size_t)mv.n_own_items; q < mv.items.size(); ++q) {
    const int32_t* ro = mv.rowoff.data() + q * NB3;
    for (int v = 0; v < NB3; ++v)
      if (ro[v] >= 0) mv.shell_ro.push_back(ro[v]);
    mv.shell_ptr.push_back((int32_t)mv.shell_ro.size());
  }

  plan_overlap(mv, mv, mv, m);
}

void plan_closure(MvPlan& y, const MvPlan& x, const MeshPlan& m) {
  if (x.source) throw Error(-1, "the closure of a closure layout is not supported");
  y = MvPlan();
  y.mesh = &m;
  y.source = &x;
  y.M = x.M;
  y.ncb = x.ncb;
  y.col_perm = x.col_perm;
  y.col_pos = x.col_pos;
  y.cb_start = x.cb_start;
  y.cb_of_col = x.cb_of_col;
  const int nbt = m.nbatch, ncb = x.ncb, NB = m.NB, NB3 = NB * NB * NB, n = m.n;
  std::vector<int32_t> w(ncb);
  for (int C = 0; C < ncb; ++C) w[C] = x.cb_start[C + 1] - x.cb_start[C];

  // owner rank of each neighbour slot of every batch
  std::vector<std::array<int, 27>> owners(nbt);
  for (int r = 0; r < nbt; ++r) {
    owners[r].fill(-1);
    const int32_t* g = m.gtab.data() + (size_t)r * NB3;
    int bx, by, bz;
    m.batch_coords(m.batch_order[r], bx, by, bz);
    for (int v = 0; v < NB3; ++v)
      if (g[v] >= 0) {
        const int s = g[v] >> 24;
        const int ox = bx + (s % 3) - 1, oy = by + ((s / 3) % 3) - 1, oz = bz + (s / 9) - 1;
        owners[r][s] = m.batch_rank[ox + m.nb[0] * (oy + m.nb[1] * oz)];
      }
  }
  // cell by cell: the column blocks stored for any free node of the cell
  // reach the row blocks of all free nodes of the cell
  std::vector<uint8_t> stored((size_t)nbt * ncb, 0);
  std::vector<int> mark(ncb, 0), list;
  for (int r = 0; r < nbt; ++r) {
    const int32_t* g = m.gtab.data() + (size_t)r * NB3;
    for (int e = 0; e < 8; ++e) {
      const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
      uint32_t slots = 0;
      for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            const int v = (ex * m.p + i) + NB * ((ey * m.p + j) + NB * (ez * m.p + k));
            if (g[v] >= 0) slots |= 1u << (g[v] >> 24);
          }
      list.clear();
      for (int s = 0; s < 27; ++s) {
        if (!((slots >> s) & 1u)) continue;
        const int o = owners[r][s];
        for (int64_t kb = x.rowptr[o]; kb < x.rowptr[o + 1]; ++kb) {
          const int C = x.colidx[kb];
          if (!mark[C]) { mark[C] = 1; list.push_back(C); }
        }
      }
      for (int C : list) {
        mark[C] = 0;
        for (int s = 0; s < 27; ++s)
          if ((slots >> s) & 1u) stored[(size_t)owners[r][s] * ncb + C] = 1;
      }
    }
  }
  y.rowptr.assign(nbt + 1, 0);
  for (int r = 0; r < nbt; ++r) {
    for (int C = 0; C < ncb; ++C)
      if (stored[(size_t)r * ncb + C]) y.colidx.push_back(C);
    y.rowptr[r + 1] = (int64_t)y.colidx.size();
  }
  const int64_t nblocks = (int64_t)y.colidx.size();
  y.block_offset.assign(nblocks + 1, 0);
  for (int r = 0; r < nbt; ++r) {
    const int64_t rows = m.rb_start[r + 1] - m.rb_start[r];
    for (int64_t k = y.rowptr[r]; k < y.rowptr[r + 1]; ++k)
      y.block_offset[k + 1] = y.block_offset[k] + rows * w[y.colidx[k]];
  }
  if (y.block_offset.back() >= ((int64_t)1 << 31))
    throw Error(-2, "multivectors of 2^31 or more stored values are not supported");

  // destination row offsets of x's apply items
  y.dest_rowoff.assign(x.items.size() * (size_t)NB3, -1);
  for (size_t q = 0; q < x.items.size(); ++q) {
    const ApplyItem& it = x.items[q];
    const int32_t* g = m.gtab.data() + (size_t)it.rank * NB3;
    const int CC = x.item_cb[q];
    int32_t* ro = y.dest_rowoff.data() + q * NB3;
    for (int v = 0; v < NB3; ++v) {
      if (g[v] < 0) continue;
      const int64_t k = y.block_index(owners[it.rank][g[v] >> 24], CC);
      if (k < 0) continue;
      ro[v] = (int32_t)(y.block_offset[k] + (int64_t)(g[v] & 0xFFFFFF) * it.ld + it.c0);
    }
  }
  plan_overlap(y, x, y, m);
}

}  // namespace mfb
