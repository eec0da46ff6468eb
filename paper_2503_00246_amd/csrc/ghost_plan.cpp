// Host plan of the ghost-penalty operator (pure C++17).
//
// * Cell classification by a ball level set (§2: phi > 0 inside) or caller classes.
// * Ghost-face set (§2.2, Fig. 1): interior faces between two active cells, one of
//   them cut.
// * Face ordering for the GPU: faces batched by normal axis (§2.7: faces with the
//   same normal share the Kronecker layout) and ordered along a Morton curve of the
//   lower cell, so that a workgroup, and the workgroups resident on one XCD, touch
//   a compact region of the lattice; optional colouring for a race-free scatter.
// * 1D tables (§2.4): jump vectors of the two-cell reference patch and the exact
//   reference mass matrix, in long double, rounded once to double.
//
// Classification arithmetic is kept free of contraction (cell bounds lo + c*h are
// rounded twice, as plain IEEE expressions) so that it matches any other IEEE
// implementation bit for bit.
#pragma clang fp contract(off)

#include "ghost_plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <functional>
#include <numeric>

namespace ghost {
namespace {

using ld = long double;

// Legendre P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, ld x, ld &p, ld &dp) {
  ld p0 = 1, p1 = x;
  if (n == 0) { p = 1; dp = 0; return; }
  for (int m = 1; m < n; ++m) {
    ld p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1);
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = n * (x * p1 - p0) / (x * x - 1);  // valid for |x| < 1
}

const ld kPi = 3.141592653589793238462643383279502884L;

// GLL nodes on [-1, 1]: endpoints and roots of P_k' (Newton with P_k'' from Legendre's ODE).
std::vector<ld> gll_nodes_pm1(int k) {
  std::vector<ld> x(k + 1);
  x[0] = -1;
  x[k] = 1;
  for (int i = 1; i < k; ++i) {
    ld t = -cosl(kPi * i / k);
    for (int it = 0; it < 100; ++it) {
      ld p, dp;
      legendre(k, t, p, dp);
      ld d2p = (2 * t * dp - k * (k + 1) * p) / (1 - t * t);
      ld step = dp / d2p;
      t -= step;
      if (fabsl(step) < 1e-21L) break;
    }
    x[i] = t;
  }
  return x;
}

// Gauss-Legendre rule with n points on [-1, 1].
void gauss_pm1(int n, std::vector<ld> &x, std::vector<ld> &w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    ld t = -cosl(kPi * (i + 0.75L) / (n + 0.5L));
    ld p = 0, dp = 1;
    for (int it = 0; it < 100; ++it) {
      legendre(n, t, p, dp);
      ld step = p / dp;
      t -= step;
      if (fabsl(step) < 1e-21L) break;
    }
    legendre(n, t, p, dp);
    x[i] = t;
    w[i] = 2 / ((1 - t * t) * dp * dp);
  }
}

ld lagrange_at(const std::vector<ld> &nodes, int i, ld x) {
  ld v = 1;
  for (size_t m = 0; m < nodes.size(); ++m)
    if ((int)m != i) v *= (x - nodes[m]) / (nodes[i] - nodes[m]);
  return v;
}

// j-th derivative of l_i at the node e (0 or 1), j = 0..k.  Expands l_i in the shifted
// variable t = x - e: l_i = c * prod_{m != i} (t - d_m), d_m = node_m - e.  All d_m share a
// sign, so each coefficient is a sum of same-signed products (no cancellation).
std::vector<ld> lagrange_derivs_at(const std::vector<ld> &nodes, int i, ld e) {
  int K = (int)nodes.size();
  std::vector<ld> poly(1, 1);
  ld c = 1;
  for (int m = 0; m < K; ++m) {
    if (m == i) continue;
    ld d = nodes[m] - e;
    std::vector<ld> nxt(poly.size() + 1, 0);
    for (size_t t = 0; t < poly.size(); ++t) {
      nxt[t + 1] += poly[t];
      nxt[t] -= d * poly[t];
    }
    poly.swap(nxt);
    c /= (nodes[i] - nodes[m]);
  }
  std::vector<ld> out(K, 0);
  ld fact = 1;
  for (int j = 0; j < K; ++j) {
    if (j > 0) fact *= j;
    out[j] = fact * c * poly[j];
  }
  return out;
}

uint64_t spread3(uint64_t v) {  // 21 bits -> every third bit
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}
uint64_t spread2(uint64_t v) {  // 32 bits -> every second bit
  v &= 0xffffffffULL;
  v = (v | v << 16) & 0x0000ffff0000ffffULL;
  v = (v | v << 8) & 0x00ff00ff00ff00ffULL;
  v = (v | v << 4) & 0x0f0f0f0f0f0f0f0fULL;
  v = (v | v << 2) & 0x3333333333333333ULL;
  v = (v | v << 1) & 0x5555555555555555ULL;
  return v;
}
uint64_t morton(int dim, const int32_t *c) {
  if (dim == 3) return spread3(c[0]) | spread3(c[1]) << 1 | spread3(c[2]) << 2;
  return spread2(c[0]) | spread2(c[1]) << 1;
}

struct Interval {
  int64_t line;
  int64_t start, end;  // [start, end) along x
  bool operator<(const Interval &o) const { return line != o.line ? line < o.line : start < o.start; }
};

void merge_runs(std::vector<Interval> &iv, int64_t L0, std::vector<Run> &runs, int64_t &total) {
  std::sort(iv.begin(), iv.end());
  runs.clear();
  total = 0;
  size_t i = 0;
  while (i < iv.size()) {
    int64_t line = iv[i].line, s = iv[i].start, e = iv[i].end;
    size_t j = i + 1;
    while (j < iv.size() && iv[j].line == line && iv[j].start <= e) {
      e = std::max(e, iv[j].end);
      ++j;
    }
    runs.push_back(Run{line * L0 + s, (int32_t)(e - s), 0});
    total += e - s;
    i = j;
  }
}

}  // namespace

void tables_1d(int k, std::vector<ld> &nodes, std::vector<ld> &weights, std::vector<ld> &jumps,
               std::vector<ld> &mass) {
  const int K = k + 1, NN = 2 * k + 1;
  std::vector<ld> x = gll_nodes_pm1(k);
  // make the node set exactly symmetric before mapping to [0, 1]
  for (int i = 0; i < K / 2; ++i) {
    ld a = 0.5L * (x[k - i] - x[i]);
    x[i] = -a;
    x[k - i] = a;
  }
  if (k % 2 == 0) x[k / 2] = 0;
  nodes.assign(K, 0);
  weights.assign(K, 0);
  for (int i = 0; i < K; ++i) {
    ld p, dp;
    legendre(k, x[i], p, dp);
    if (i == 0 || i == k) p = (i == 0 && k % 2 == 1) ? -1 : 1;  // P_k(+-1) = (+-1)^k
    weights[i] = 1 / (k * (k + 1) * p * p);                      // GLL weight on [-1,1], halved
    nodes[i] = (x[i] + 1) / 2;
  }
  nodes[0] = 0;
  nodes[k] = 1;

  // jumps of the j-th derivative (right minus left) of the 2k+1 patch functions
  std::vector<std::vector<ld>> at1(K), at0(K);
  for (int i = 0; i < K; ++i) {
    at1[i] = lagrange_derivs_at(nodes, i, 1);  // lower cell, face at its x = 1
    at0[i] = lagrange_derivs_at(nodes, i, 0);  // upper cell, face at its x = 0
  }
  jumps.assign((size_t)k * NN, 0);
  for (int j = 1; j <= k; ++j) {
    for (int i = 0; i < NN; ++i) {
      ld v = 0;
      if (i >= k) v += at0[i - k][j];
      if (i <= k) v -= at1[i][j];
      jumps[(j - 1) * NN + i] = v;
    }
    // reflection about the face maps entry i to 2k-i with sign (-1)^(j+1); enforce it exactly
    ld sgn = (j % 2 == 1) ? 1 : -1;
    for (int i = 0; i < k; ++i) {
      ld a = jumps[(j - 1) * NN + i], b = jumps[(j - 1) * NN + 2 * k - i];
      ld m = 0.5L * (a + sgn * b);
      jumps[(j - 1) * NN + i] = m;
      jumps[(j - 1) * NN + 2 * k - i] = sgn * m;
    }
    if (sgn < 0) jumps[(j - 1) * NN + k] = 0;
  }

  // exact mass matrix by (k+1)-point Gauss-Legendre on [0, 1]
  std::vector<ld> gx, gw;
  gauss_pm1(K, gx, gw);
  mass.assign((size_t)K * K, 0);
  for (int q = 0; q < K; ++q) {
    ld xq = (gx[q] + 1) / 2, wq = gw[q] / 2;
    for (int a = 0; a < K; ++a)
      for (int b = 0; b < K; ++b)
        mass[a * K + b] += wq * lagrange_at(nodes, a, xq) * lagrange_at(nodes, b, xq);
  }
  std::vector<ld> raw = mass;  // make it exactly symmetric and centro-symmetric
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b)
      mass[a * K + b] = 0.25L * (raw[a * K + b] + raw[b * K + a] + raw[(k - a) * K + (k - b)] +
                                 raw[(k - b) * K + (k - a)]);
}

void stiffness_1d(int k, std::vector<ld> &stiff) {
  const int K = k + 1;
  std::vector<ld> nodes, weights, jumps, mass;
  tables_1d(k, nodes, weights, jumps, mass);
  std::vector<ld> gx, gw;
  gauss_pm1(K, gx, gw);
  std::vector<ld> raw((size_t)K * K, 0);
  for (int q = 0; q < K; ++q) {
    const ld xq = (gx[q] + 1) / 2, wq = gw[q] / 2;
    std::vector<ld> d1(K);
    for (int a = 0; a < K; ++a) d1[a] = lagrange_derivs_at(nodes, a, xq)[1];
    for (int a = 0; a < K; ++a)
      for (int b = 0; b < K; ++b) raw[a * K + b] += wq * d1[a] * d1[b];
  }
  stiff.assign((size_t)K * K, 0);
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b)
      stiff[a * K + b] = 0.25L * (raw[a * K + b] + raw[b * K + a] + raw[(k - a) * K + (k - b)] +
                                  raw[(k - b) * K + (k - a)]);
}

void macro_mix_1d(int k, std::vector<ld> &mix) {
  std::vector<ld> fact(2 * k + 2, 1);
  for (int i = 1; i < (int)fact.size(); ++i) fact[i] = fact[i - 1] * i;
  mix.assign((size_t)k * k, 0);
  for (int i = 1; i <= k; ++i)
    for (int j = 1; j <= k; ++j)
      if ((i + j) % 2 == 0) mix[(i - 1) * k + (j - 1)] = 2.0L / ((i + j + 1) * fact[i] * fact[j]);
}

std::string build_plan(Plan &p, int dim, const int n[3], const double lo[3], double h, int k,
                       int ls_kind, const double centre[3], double radius,
                       const signed char *cell_class, int n_balls, const double *balls, bool coloured) {
  p = Plan();
  p.dim = dim;
  p.k = k;
  p.h = h;
  int64_t n_cells = 1;
  for (int a = 0; a < 3; ++a) {
    p.n[a] = a < dim ? n[a] : 1;
    p.lo[a] = a < dim ? lo[a] : 0.0;
    p.L[a] = a < dim ? (int64_t)k * n[a] + 1 : 1;
    n_cells *= p.n[a];
  }
  p.stride[0] = 1;
  p.stride[1] = p.L[0];
  p.stride[2] = p.L[0] * p.L[1];
  p.n_lattice = p.L[0] * p.L[1] * p.L[2];
  // in-patch offsets are 32-bit in the kernels
  if ((2 * k + 1) * p.stride[dim - 1] >= ((int64_t)1 << 31))
    return "lattice too large: a patch spans more than 2^31 linear indices";

  // ---- classification
  p.cls.assign(n_cells, GHOST_OUTSIDE);
  if (ls_kind == 1) {
    for (int64_t i = 0; i < n_cells; ++i) {
      int v = cell_class[i];
      if (v < 0 || v > 2) return "cell_class entries must be 0, 1 or 2";
      p.cls[i] = (int8_t)v;
    }
  } else {
    // ball, or union of balls: a cell is INSIDE when some closed ball contains it, CUT when it meets
    // some open ball without that, OUTSIDE otherwise (exact squared distances of the cell box to the
    // centre).  Each ball only visits the cells of its bounding box.
    std::vector<double> one;
    if (ls_kind == 0) one = {centre[0], centre[1], centre[2], radius};
    const double *bl = ls_kind == 0 ? one.data() : balls;
    const int nb = ls_kind == 0 ? 1 : n_balls;
    for (int i = 0; i < nb; ++i) {
      const double *b = bl + 4 * i;
      const double r2 = b[3] * b[3];
      int cmin[3] = {0, 0, 0}, cmax[3] = {0, 0, 0};
      for (int a = 0; a < 3; ++a) {
        if (a >= dim) continue;
        const double f0 = std::floor((b[a] - b[3] - p.lo[a]) / h) - 1.0, f1 = std::floor((b[a] + b[3] - p.lo[a]) / h) + 1.0;
        cmin[a] = (int)std::max(0.0, std::min(f0, (double)p.n[a]));
        cmax[a] = (int)std::max(-1.0, std::min(f1, (double)p.n[a] - 1.0));
      }
      for (int c2 = cmin[2]; c2 <= cmax[2]; ++c2)
        for (int c1 = cmin[1]; c1 <= cmax[1]; ++c1)
          for (int c0 = cmin[0]; c0 <= cmax[0]; ++c0) {
            int c[3] = {c0, c1, c2};
            double dmin2 = 0.0, dmax2 = 0.0;
            for (int a = 0; a < dim; ++a) {
              double cd = (double)c[a];
              double lo_a = p.lo[a] + cd * h;
              double hi_a = p.lo[a] + (cd + 1.0) * h;
              double below = std::max(lo_a - b[a], 0.0);
              double above = std::max(b[a] - hi_a, 0.0);
              double nearv = std::max(below, above);
              double farv = std::max(std::fabs(lo_a - b[a]), std::fabs(hi_a - b[a]));
              dmin2 = dmin2 + nearv * nearv;
              dmax2 = dmax2 + farv * farv;
            }
            int8_t &v = p.cls[c0 + (int64_t)p.n[0] * (c1 + (int64_t)p.n[1] * c2)];
            if (dmin2 < r2 && dmax2 <= r2) v = GHOST_INSIDE;
            else if (dmin2 < r2 && v == GHOST_OUTSIDE) v = GHOST_CUT;
          }
    }
  }
  for (int8_t v : p.cls) {
    p.n_active_cells += v != GHOST_OUTSIDE;
    p.n_cut_cells += v == GHOST_CUT;
  }
  auto cls_at = [&](int c0, int c1, int c2) {
    return p.cls[c0 + (int64_t)p.n[0] * (c1 + (int64_t)p.n[1] * c2)];
  };

  // ---- ghost faces, lexicographic (x fastest) per axis
  for (int a = 0; a < dim; ++a) {
    auto &fc = p.face_cell[a];
    for (int c2 = 0; c2 < p.n[2]; ++c2)
      for (int c1 = 0; c1 < p.n[1]; ++c1)
        for (int c0 = 0; c0 < p.n[0]; ++c0) {
          int c[3] = {c0, c1, c2};
          if (c[a] + 1 >= p.n[a]) continue;
          int d[3] = {c0, c1, c2};
          d[a] += 1;
          int8_t x = cls_at(c0, c1, c2), y = cls_at(d[0], d[1], d[2]);
          if (x != GHOST_OUTSIDE && y != GHOST_OUTSIDE &&
              (x == GHOST_CUT || y == GHOST_CUT)) {
            fc.push_back(c0);
            fc.push_back(c1);
            fc.push_back(c2);
          }
        }
  }

  // ---- colours: (axis) x (normal position mod 3) x (tangential positions mod 2)
  const int per_axis = 3 << (dim - 1);
  p.coloured = coloured;
  p.n_colours = coloured ? dim * per_axis : 0;
  for (int a = 0; a < dim; ++a) {
    size_t nf = p.face_cell[a].size() / 3;
    p.face_colour[a].assign(nf, -1);
    if (!coloured) continue;
    for (size_t f = 0; f < nf; ++f) {
      const int32_t *c = &p.face_cell[a][3 * f];
      int col = (c[a] % 3) << (dim - 1), bit = 0;
      for (int t = 0; t < dim; ++t)
        if (t != a) col |= (c[t] & 1) << bit++;
      p.face_colour[a][f] = (int8_t)(a * per_axis + col);
    }
  }

  // ---- batches
  const int fpb = faces_per_block(dim, k);
  struct Pending { uint64_t key; int axis; int colour; std::vector<int> faces; };
  std::vector<Pending> pend;
  for (int a = 0; a < dim; ++a) {
    size_t nf = p.face_cell[a].size() / 3;
    int groups = coloured ? per_axis : 1;
    for (int g = 0; g < groups; ++g) {
      std::vector<std::pair<uint64_t, int>> order;
      for (size_t f = 0; f < nf; ++f)
        if (!coloured || p.face_colour[a][f] == a * per_axis + g)
          order.push_back({morton(dim, &p.face_cell[a][3 * f]), (int)f});
      std::sort(order.begin(), order.end());
      for (size_t s = 0; s < order.size(); s += fpb) {
        Pending b;
        b.key = order[s].first;
        b.axis = a;
        b.colour = coloured ? a * per_axis + g : -1;
        for (size_t t = s; t < std::min(order.size(), s + fpb); ++t) b.faces.push_back(order[t].second);
        pend.push_back(std::move(b));
      }
    }
  }
  if (coloured)
    std::stable_sort(pend.begin(), pend.end(), [](const Pending &x, const Pending &y) {
      return x.colour != y.colour ? x.colour < y.colour : x.key < y.key;
    });
  else
    std::stable_sort(pend.begin(), pend.end(),
                     [](const Pending &x, const Pending &y) { return x.key < y.key; });
  if ((int64_t)p.face_cell[0].size() / 3 + (int64_t)p.face_cell[1].size() / 3 +
          (int64_t)p.face_cell[2].size() / 3 >= ((int64_t)1 << 31))
    return "too many faces";
  for (auto &b : pend) {
    Batch bt;
    bt.first = (int32_t)p.face_base.size();
    bt.count = (int16_t)b.faces.size();
    bt.axis = (int8_t)b.axis;
    bt.colour = (int8_t)b.colour;
    for (int f : b.faces) {
      const int32_t *c = &p.face_cell[b.axis][3 * f];
      int64_t base = 0;
      for (int t = 0; t < 3; ++t) base += (int64_t)k * c[t] * p.stride[t];
      p.face_base.push_back(base);
    }
    p.batches.push_back(bt);
  }
  if (coloured) {
    p.colour_begin.assign(p.n_colours + 1, 0);
    size_t bi = 0;
    for (int c = 0; c < p.n_colours; ++c) {
      p.colour_begin[c] = (int)bi;
      while (bi < p.batches.size() && p.batches[bi].colour == c) ++bi;
    }
    p.colour_begin[p.n_colours] = (int)bi;
  }

  // ---- support: union of patch node boxes, as x-runs
  {
    std::vector<Interval> iv;
    for (int a = 0; a < dim; ++a) {
      size_t nf = p.face_cell[a].size() / 3;
      for (size_t f = 0; f < nf; ++f) {
        const int32_t *c = &p.face_cell[a][3 * f];
        int64_t ext[3], base[3];
        for (int t = 0; t < 3; ++t) {
          ext[t] = t >= dim ? 1 : (t == a ? 2 * k + 1 : k + 1);
          base[t] = (int64_t)k * c[t];
        }
        for (int64_t i2 = 0; i2 < ext[2]; ++i2)
          for (int64_t i1 = 0; i1 < ext[1]; ++i1)
            iv.push_back({(base[1] + i1) + p.L[1] * (base[2] + i2), base[0], base[0] + ext[0]});
      }
    }
    merge_runs(iv, p.L[0], p.support_runs, p.n_support);
  }
  // ---- active nodes: nodes of active cells, as x-runs
  {
    std::vector<Interval> iv;
    for (int c2 = 0; c2 < p.n[2]; ++c2)
      for (int c1 = 0; c1 < p.n[1]; ++c1) {
        int c0 = 0;
        while (c0 < p.n[0]) {  // one interval per maximal run of active cells in this cell row
          if (cls_at(c0, c1, c2) == GHOST_OUTSIDE) { ++c0; continue; }
          int e0 = c0;
          while (e0 < p.n[0] && cls_at(e0, c1, c2) != GHOST_OUTSIDE) ++e0;
          int64_t e1 = dim >= 2 ? k + 1 : 1, e2 = dim >= 3 ? k + 1 : 1;
          for (int64_t i2 = 0; i2 < e2; ++i2)
            for (int64_t i1 = 0; i1 < e1; ++i1)
              iv.push_back({((int64_t)k * c1 + i1) + p.L[1] * ((int64_t)k * c2 + i2),
                            (int64_t)k * c0, (int64_t)k * e0 + 1});
          c0 = e0;
        }
      }
    merge_runs(iv, p.L[0], p.active_runs, p.n_active);
  }
  // ---- inside cells in chunks along x, by colour
  {
    const int chunk = cell_chunk(dim, k + 1);
    std::vector<std::vector<CellChunk>> byc(1 << dim);
    for (int c2 = 0; c2 < p.n[2]; ++c2)
      for (int c1 = 0; c1 < p.n[1]; ++c1)
        for (int c0 = 0; c0 < p.n[0];) {
          if (cls_at(c0, c1, c2) != GHOST_INSIDE) {
            ++c0;
            continue;
          }
          int e0 = c0;
          while (e0 < p.n[0] && cls_at(e0, c1, c2) == GHOST_INSIDE) ++e0;
          // the run [c0, e0), cut into chunks; neighbouring chunks of a run share one node and get
          // different colours, runs of one row are at least a cell apart
          for (int j = 0, a = c0; a < e0; ++j, a += chunk) {
            const int col = (j & 1) + (dim >= 2 ? 2 * (c1 & 1) : 0) + (dim >= 3 ? 4 * (c2 & 1) : 0);
            const int64_t base = (int64_t)k * a + p.stride[1] * ((int64_t)k * c1) + p.stride[2] * ((int64_t)k * c2);
            byc[col].push_back({base, std::min(chunk, e0 - a), 0});
          }
          c0 = e0;
        }
    p.inside_chunks.clear();
    for (int col = 0; col <= 8; ++col) p.inside_colour_begin[col] = 0;
    for (int col = 0; col < (1 << dim); ++col) {
      p.inside_colour_begin[col] = (int64_t)p.inside_chunks.size();
      p.inside_chunks.insert(p.inside_chunks.end(), byc[col].begin(), byc[col].end());
    }
    for (int col = 1 << dim; col <= 8; ++col) p.inside_colour_begin[col] = (int64_t)p.inside_chunks.size();
    // their distinct nodes, counted through x-runs as for the active nodes
    std::vector<Interval> iv;
    for (int c2 = 0; c2 < p.n[2]; ++c2)
      for (int c1 = 0; c1 < p.n[1]; ++c1) {
        int c0 = 0;
        while (c0 < p.n[0]) {
          if (cls_at(c0, c1, c2) != GHOST_INSIDE) { ++c0; continue; }
          int e0 = c0;
          while (e0 < p.n[0] && cls_at(e0, c1, c2) == GHOST_INSIDE) ++e0;
          int64_t e1 = dim >= 2 ? k + 1 : 1, e2 = dim >= 3 ? k + 1 : 1;
          for (int64_t i2 = 0; i2 < e2; ++i2)
            for (int64_t i1 = 0; i1 < e1; ++i1)
              iv.push_back({((int64_t)k * c1 + i1) + p.L[1] * ((int64_t)k * c2 + i2),
                            (int64_t)k * c0, (int64_t)k * e0 + 1});
          c0 = e0;
        }
      }
    std::vector<Run> runs;
    merge_runs(iv, p.L[0], runs, p.n_inside);
  }

  // ---- box layout for the default scatter
  {
    std::string err = build_box_layout(p);
    if (!err.empty()) return err;
  }

  // ---- tables
  std::vector<ld> nd, wt, jp, ms;
  tables_1d(k, nd, wt, jp, ms);
  p.nodes.assign(nd.begin(), nd.end());
  p.weights.assign(wt.begin(), wt.end());
  p.jumps.assign(jp.begin(), jp.end());
  p.mass.assign(ms.begin(), ms.end());
  std::vector<ld> mx;
  macro_mix_1d(k, mx);
  p.mix.assign(mx.begin(), mx.end());
  return "";
}

std::string build_box_layout(Plan &p) {
  const int d = p.dim, k = p.k;
  const int B = box_cells(d, k), NB = box_nodes(d, k), E = box_extent(d), P = box_pitch(d);
  const int64_t kB = (int64_t)k * B;
  int nbr[3] = {1, 1, 1};
  for (int a = 0; a < d; ++a) nbr[a] = (p.n[a] + B - 1) / B;
  const int64_t nbricks = (int64_t)nbr[0] * nbr[1] * nbr[2];
  auto bid = [&](const int b[3]) { return b[0] + (int64_t)nbr[0] * (b[1] + (int64_t)nbr[1] * b[2]); };

  // visits per brick
  std::vector<std::vector<Visit>> bv(nbricks);
  for (int a = 0; a < d; ++a) {
    const size_t nf = p.face_cell[a].size() / 3;
    for (size_t f = 0; f < nf; ++f) {
      const int32_t *c = &p.face_cell[a][3 * f];
      int bl[3] = {0, 0, 0}, bu[3] = {0, 0, 0};
      for (int t = 0; t < d; ++t) {
        bl[t] = c[t] / B;
        bu[t] = (c[t] + (t == a ? 1 : 0)) / B;
      }
      const Visit base = (Visit)c[0] | (Visit)c[1] << 20 | (Visit)c[2] << 40 | (Visit)a << 60;
      if (bl[a] == bu[a]) {
        bv[bid(bl)].push_back(base);
      } else {
        bv[bid(bl)].push_back(base | (Visit)1 << 62);
        bv[bid(bu)].push_back(base | (Visit)2 << 62);
      }
    }
  }

  // launch order: Morton order of the brick
  std::vector<std::pair<uint64_t, int64_t>> order;
  for (int64_t b = 0; b < nbricks; ++b) {
    if (bv[b].empty()) continue;
    int32_t bc[3] = {(int32_t)(b % nbr[0]), (int32_t)((b / nbr[0]) % nbr[1]), (int32_t)(b / ((int64_t)nbr[0] * nbr[1]))};
    order.push_back({morton(d, bc), b});
  }
  std::sort(order.begin(), order.end());

  p.brick = B;
  p.box_nodes = NB;
  p.boxes.clear();
  p.visits.clear();
  p.box_runs.clear();
  p.box_lines.clear();
  if (NB > E) return "box node extent exceeds the accumulator extent";
  {
    // the kernel addresses u and y around a box with 32-bit byte offsets: nodes within E + k of the
    // box origin along each axis (k below it for the lower cells of split faces)
    const int64_t s1 = p.L[0], s2 = d == 3 ? p.L[0] * p.L[1] : 0;
    if ((int64_t)8 * (E + 2 * k) * (1 + s1 + s2) >= ((int64_t)1 << 31))
      return "lattice planes too large for the box scatter (use the atomic scatter)";
  }
  // Boxes: one per brick with visits, in brick order; a brick with more visits than one box holds is
  // split into several boxes over the same node box.  Within a box the visits are interleaved so that
  // the faces of one batch (consecutive visits) come from different parts of the brick and rarely add
  // into the same accumulator nodes.
  struct BoxTmp {
    int64_t brick;
    std::vector<Visit> v;
    std::vector<Run> runs;  // nodes the box contributes to
  };
  std::vector<BoxTmp> tmp;
  for (const auto &o : order) {
    const std::vector<Visit> &all = bv[o.second];
    const size_t nparts = (all.size() + kMaxBoxVisits - 1) / kMaxBoxVisits;
    for (size_t part = 0; part < nparts; ++part) {
      BoxTmp t;
      t.brick = o.second;
      for (size_t i = part; i < all.size(); i += nparts) t.v.push_back(all[i]);
      tmp.push_back(std::move(t));
    }
  }
  // Touched nodes of each box (union over its visits of the expanded part of the patch).  The first box
  // (in box order) that touches a support node writes it to y; every later box touching it sends its
  // contribution through a halo slot, which the halo pass adds to y.
  std::vector<int64_t> sup_start(p.support_runs.size()), sup_off(p.support_runs.size());
  {
    int64_t acc = 0;
    for (size_t r = 0; r < p.support_runs.size(); ++r) {
      sup_start[r] = p.support_runs[r].start;
      sup_off[r] = acc;
      acc += p.support_runs[r].len;
    }
  }
  auto sup_index = [&](int64_t node) -> int64_t {
    const size_t r = (size_t)(std::upper_bound(sup_start.begin(), sup_start.end(), node) - sup_start.begin()) - 1;
    return sup_off[r] + (node - sup_start[r]);
  };
  for (BoxTmp &t : tmp) {
    std::vector<Interval> iv;
    for (Visit v : t.v) {
      const int c[3] = {(int)(v & 0xFFFFF), (int)((v >> 20) & 0xFFFFF), (int)((v >> 40) & 0xFFFFF)};
      const int a = (int)((v >> 60) & 3), half = (int)((v >> 62) & 3);
      int64_t lo[3], hi[3];  // node ranges, inclusive
      for (int q = 0; q < 3; ++q) {
        lo[q] = q < d ? (int64_t)k * c[q] : 0;
        hi[q] = q < d ? lo[q] + k : 0;
      }
      if (half == 0) hi[a] = lo[a] + 2 * k;
      if (half == 2) { lo[a] = (int64_t)k * c[a] + k + 1; hi[a] = (int64_t)k * c[a] + 2 * k; }
      for (int64_t z = lo[2]; z <= hi[2]; ++z)
        for (int64_t y = lo[1]; y <= hi[1]; ++y) iv.push_back({y + p.L[1] * z, lo[0], hi[0] + 1});
    }
    int64_t tot = 0;
    merge_runs(iv, p.L[0], t.runs, tot);
  }
  std::vector<uint8_t> claimed((size_t)p.n_support, 0);  // a box already writes the node to y

  struct HaloRef { int64_t node; int32_t slot; };
  std::vector<HaloRef> halo;
  int64_t slots = 0;
  const size_t fpb = (size_t)box_faces_per_batch(d, k);
  for (const BoxTmp &t : tmp) {
    const int64_t b = t.brick;
    const int bb[3] = {(int)(b % nbr[0]), (int)((b / nbr[0]) % nbr[1]), (int)(b / ((int64_t)nbr[0] * nbr[1]))};
    Box bx{};
    for (int a = 0; a < 3; ++a) bx.org[a] = a < d ? (int32_t)(kB * bb[a]) : 0;
    bx.visit_first = (int32_t)p.visits.size();
    bx.visit_count = (int32_t)t.v.size();
    // visits grouped by normal axis (x first: a wave whose faces all have their normal along x gathers
    // contiguous lines with 16-byte loads), each group interleaved as described above
    for (int a = 0; a < d; ++a) {
      std::vector<Visit> g;
      for (Visit v : t.v)
        if ((int)((v >> 60) & 3) == a) g.push_back(v);
      const size_t nv = g.size(), nbatch = (nv + fpb - 1) / fpb;
      for (size_t q = 0; q < nbatch; ++q)
        for (size_t r = 0; r < fpb; ++r)
          if (q + r * nbatch < nv) p.visits.push_back(g[q + r * nbatch]);
    }
    bx.run_first = (int32_t)p.box_runs.size();
    bx.line_first = (int32_t)p.box_lines.size();
    bx.halo_first = (int32_t)slots;
    for (const Run &r : t.runs) {
      const int64_t line = r.start / p.L[0], x0 = r.start % p.L[0];
      const int64_t Y = line % p.L[1], Z = line / p.L[1];
      const int64_t ry = d >= 2 ? Y - bx.org[1] : 0, rz = d >= 3 ? Z - bx.org[2] : 0;
      const int64_t sbase = sup_index(r.start);
      // split the run where the status changes: written to y by this box, or through a halo slot
      int64_t q0 = 0;
      while (q0 < r.len) {
        const bool node_shared = claimed[sbase + q0] != 0;
        int64_t q1 = q0 + 1;
        while (q1 < r.len && (claimed[sbase + q1] != 0) == node_shared) ++q1;
        for (int64_t q = q0; q < q1; ++q) claimed[sbase + q] = 1;
        const int64_t rx = x0 + q0 - bx.org[0];
        BoxRun br{};
        br.start = r.start + q0;
        br.acc = (int32_t)(rx + P * (ry + (int64_t)E * rz));  // accumulator index
        br.len = (int32_t)(q1 - q0);
        br.slot = -1;
        if (node_shared) {
          br.slot = (int32_t)slots;
          for (int64_t q = 0; q < br.len; ++q) halo.push_back({br.start + q, (int32_t)(slots + q)});
          slots += br.len;
        }
        p.box_runs.push_back(br);
        // device line record (runs of one line are consecutive: start a record at a new line)
        const int32_t lrel = (int32_t)(ry + (int64_t)E * rz);
        if (p.box_lines.size() == (size_t)bx.line_first || p.box_lines.back().line != lrel)
          p.box_lines.push_back(BoxLine{0, 0, lrel, (int32_t)(node_shared ? br.slot : slots)});
        BoxLine &bl = p.box_lines.back();
        for (int64_t q = 0; q < br.len; ++q) {
          bl.touched |= (uint64_t)1 << (rx + q);
          if (node_shared) bl.shared |= (uint64_t)1 << (rx + q);
        }
        q0 = q1;
      }
    }
    bx.run_count = (int32_t)(p.box_runs.size() - bx.run_first);
    bx.line_count = (int32_t)(p.box_lines.size() - bx.line_first);
    // the kernel reads the first visit and line of every box unconditionally, one visit per thread
    // and one lane group per box line: a box has at least one of each, at most kMaxBoxVisits visits
    // and at most one line per (y, z) of its node box
    if (bx.visit_count < 1 || bx.visit_count > kMaxBoxVisits || bx.line_count < 1 ||
        bx.line_count > (d == 3 ? E * E : E) || slots - bx.halo_first > kMaxBoxHalo)
      return "box layout: a box without visits or lines, or with more visits, lines or halo slots than it holds";
    p.boxes.push_back(bx);
  }
  if (slots >= ((int64_t)1 << 31) || (int64_t)p.visits.size() >= ((int64_t)1 << 31))
    return "box layout too large";
  p.n_visits = (int64_t)p.visits.size();
  p.n_slots = slots;
  std::sort(halo.begin(), halo.end(), [](const HaloRef &x, const HaloRef &y) {
    return x.node != y.node ? x.node < y.node : x.slot < y.slot;
  });
  // Halo CSR: the nodes with exactly one slot first (most shared nodes lie on one face between two
  // boxes; the pass reads their slot at h without the pointer), then the others, each group in
  // ascending node order.
  p.halo_node.clear();
  p.halo_ptr.clear();
  p.halo_slot.clear();
  std::vector<std::pair<size_t, size_t>> groups;  // [begin, end) in `halo` per node
  for (size_t i = 0; i < halo.size(); ++i)
    if (i == 0 || halo[i].node != halo[i - 1].node) groups.push_back({i, i});
  for (size_t g = 0; g < groups.size(); ++g) groups[g].second = g + 1 < groups.size() ? groups[g + 1].first : halo.size();
  for (int pass = 0; pass < 2; ++pass)
    for (const auto &g : groups) {
      if ((g.second - g.first == 1) != (pass == 0)) continue;
      p.halo_node.push_back(halo[g.first].node);
      p.halo_ptr.push_back((int32_t)p.halo_slot.size());
      for (size_t i = g.first; i < g.second; ++i) p.halo_slot.push_back(halo[i].slot);
    }
  p.halo_ptr.push_back((int32_t)p.halo_slot.size());
  p.n_halo_single = 0;
  for (const auto &g : groups) p.n_halo_single += g.second - g.first == 1 ? 1 : 0;
  return "";
}

}  // namespace ghost
