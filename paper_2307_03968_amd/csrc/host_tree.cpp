// Entries, cluster tree and block partition of the H-matrix (Sec. II eq. 5,
// Sec. III eq. 6-7).  Host code.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "hm_internal.h"

namespace hm {

static inline double dist3(const Problem& p, int64_t i, int64_t j) {
  const double dx = p.xyz[3 * i] - p.xyz[3 * j];
  const double dy = p.xyz[3 * i + 1] - p.xyz[3 * j + 1];
  const double dz = p.xyz[3 * i + 2] - p.xyz[3 * j + 2];
  return std::sqrt(dx * dx + dy * dy + dz * dz);
}

// Free-space Green's function e^{-jkR} / (4 pi R) times the kernel scale:
// h^2 for the surface stand-in, k^2 h^3 for the volume one.
cplx kernel(const Problem& p, int64_t i, int64_t j) {
  const double r = dist3(p, i, j);
  double s, c;
  sincos(p.k * r, &s, &c);
  const double scale = (p.kind == HM_SURFACE) ? p.h * p.h : p.k * p.k * p.h * p.h * p.h;
  const double a = scale / (4.0 * M_PI * r);
  return cplx(a * c, -a * s);
}

cplx entry(const Problem& p, int64_t i, int64_t j) {
  if (i == j) {
    if (p.kind == HM_SURFACE) return cplx(2.0 * p.h, 0.2 * p.h);
    return cplx(1.0 / p.chi[i] + 0.5, 0.0);
  }
  const cplx g = kernel(p, i, j);
  return (p.kind == HM_SURFACE) ? g : g * p.chi[j];
}

// Binary tree division: split a cluster with more than leaf_max points along
// the longest axis of its bounding box (first axis on equal extents); order
// by that coordinate with ties broken by original index; left child takes
// floor(n/2).
Tree build_tree(const Problem& p, int leaf_max) {
  Tree tr;
  tr.perm.resize(p.n);
  std::iota(tr.perm.begin(), tr.perm.end(), int64_t(0));
  tr.leaf_of.assign(p.n, -1);
  struct Item { int32_t node; };
  tr.nodes.push_back(Cluster{0, (int32_t)p.n, 0, {-1, -1}, {0, 0, 0}, {0, 0, 0}});
  // depth-first, left child first, so leaves come out in tree order
  std::vector<int32_t> stack{0};
  while (!stack.empty()) {
    const int32_t id = stack.back();
    stack.pop_back();
    Cluster c = tr.nodes[id];
    for (int d = 0; d < 3; ++d) { c.lo[d] = INFINITY; c.hi[d] = -INFINITY; }
    for (int32_t q = c.off; q < c.off + c.size; ++q) {
      const int64_t i = tr.perm[q];
      for (int d = 0; d < 3; ++d) {
        c.lo[d] = std::min(c.lo[d], p.xyz[3 * i + d]);
        c.hi[d] = std::max(c.hi[d], p.xyz[3 * i + d]);
      }
    }
    if (c.size > leaf_max) {
      int ax = 0;
      for (int d = 1; d < 3; ++d)
        if (c.hi[d] - c.lo[d] > c.hi[ax] - c.lo[ax]) ax = d;
      auto b = tr.perm.begin() + c.off;
      std::sort(b, b + c.size, [&](int64_t u, int64_t v) {
        const double cu = p.xyz[3 * u + ax], cv = p.xyz[3 * v + ax];
        return cu < cv || (cu == cv && u < v);
      });
      const int32_t h = c.size / 2;
      const int32_t l = (int32_t)tr.nodes.size();
      tr.nodes.push_back(Cluster{c.off, h, c.depth + 1, {-1, -1}, {0, 0, 0}, {0, 0, 0}});
      tr.nodes.push_back(Cluster{c.off + h, c.size - h, c.depth + 1, {-1, -1}, {0, 0, 0}, {0, 0, 0}});
      c.child[0] = l;
      c.child[1] = l + 1;
      tr.nodes[id] = c;
      stack.push_back(l + 1);
      stack.push_back(l);
    } else {
      tr.nodes[id] = c;
      tr.depth = std::max(tr.depth, c.depth);
    }
  }
  // leaves in tree order
  for (int32_t id = 0; id < (int32_t)tr.nodes.size(); ++id)
    if (tr.nodes[id].leaf()) tr.leaves.push_back(id);
  std::sort(tr.leaves.begin(), tr.leaves.end(),
            [&](int32_t a, int32_t b) { return tr.nodes[a].off < tr.nodes[b].off; });
  for (int32_t a = 0; a < (int32_t)tr.leaves.size(); ++a) {
    const Cluster& c = tr.nodes[tr.leaves[a]];
    for (int32_t q = c.off; q < c.off + c.size; ++q) tr.leaf_of[q] = a;
  }
  return tr;
}

static double diam(const Cluster& c) {
  double s = 0;
  for (int d = 0; d < 3; ++d) s += (c.hi[d] - c.lo[d]) * (c.hi[d] - c.lo[d]);
  return std::sqrt(s);
}

static double gap(const Cluster& t, const Cluster& s) {
  double q = 0;
  for (int d = 0; d < 3; ++d) {
    const double g = std::max(0.0, std::max(s.lo[d] - t.hi[d], t.lo[d] - s.hi[d]));
    q += g * g;
  }
  return std::sqrt(q);
}

// eq. 7, inclusive: eta * dist(t, s) >= min(diam(t), diam(s)).
static bool admissible(const Cluster& t, const Cluster& s, double eta) {
  return eta * gap(t, s) >= std::min(diam(t), diam(s));
}

static void partition_rec(const Tree& tr, int32_t t, int32_t s, double eta,
                          std::vector<BlockPair>& near, std::vector<BlockPair>& far) {
  const Cluster& ct = tr.nodes[t];
  const Cluster& cs = tr.nodes[s];
  const int32_t level = std::max(ct.depth, cs.depth);
  // a cluster with itself holds the diagonal: never far (eq. 7 holds
  // trivially for a one-point cluster)
  if (t != s && admissible(ct, cs, eta)) {
    far.push_back({t, s, level});
    return;
  }
  if (ct.leaf() && cs.leaf()) {
    near.push_back({t, s, level});
    return;
  }
  const int32_t tc[2] = {ct.leaf() ? t : ct.child[0], ct.leaf() ? -1 : ct.child[1]};
  const int32_t sc[2] = {cs.leaf() ? s : cs.child[0], cs.leaf() ? -1 : cs.child[1]};
  for (int a = 0; a < 2; ++a) {
    if (tc[a] < 0) continue;
    for (int b = 0; b < 2; ++b) {
      if (sc[b] < 0) continue;
      partition_rec(tr, tc[a], sc[b], eta, near, far);
    }
  }
}

void build_partition(const Tree& tr, double eta, std::vector<BlockPair>& near,
                     std::vector<BlockPair>& far) {
  near.clear();
  far.clear();
  partition_rec(tr, 0, 0, eta, near, far);
}

}  // namespace hm
