// Host construction of the H-matrix (Sec. III): tree, partition, exact near
// blocks, compressed far blocks with the half (symmetric) computation.
#include <omp.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "hm_internal.h"

namespace hm {

int build_host(const Problem& p, const hm_build_opts& o, HostH& H) {
  H.prob = p;
  H.leaf_max = o.leaf_max;
  H.eta = o.eta;
  H.tol = o.aca_tol;
  H.tree = build_tree(p, o.leaf_max);
  const Tree& tr = H.tree;
  const int nl = (int)tr.leaves.size();
  H.leaf_off.resize(nl);
  H.leaf_size.resize(nl);
  std::vector<int32_t> leaf_index(tr.nodes.size(), -1);
  H.max_leaf = 0;
  for (int a = 0; a < nl; ++a) {
    const Cluster& c = tr.nodes[tr.leaves[a]];
    H.leaf_off[a] = c.off;
    H.leaf_size[a] = c.size;
    leaf_index[tr.leaves[a]] = a;
    H.max_leaf = std::max(H.max_leaf, c.size);
  }
  if (p.kind == HM_VOLUME) {
    H.chi_tree.resize(p.n);
    for (int64_t q = 0; q < p.n; ++q) H.chi_tree[q] = p.chi[tr.perm[q]];
  }
  H.xyz_tree.resize(3 * (size_t)p.n);
  for (int64_t q = 0; q < p.n; ++q)
    for (int c = 0; c < 3; ++c) H.xyz_tree[3 * q + c] = p.xyz[3 * tr.perm[q] + c];
  H.inst.assign(1, EntryParams{p.kind, 0, p.k, p.h});
  H.leaf_inst.assign(nl, 0);
  // a handle that keeps no host blocks has its near entries computed by the
  // device build straight into the panels
  H.near_on_device = (o.flags & (HM_BUILD_HOST_ONLY | HM_BUILD_KEEP_HOST)) == 0;

  std::vector<BlockPair> near, far;
  build_partition(tr, o.eta, near, far);

  // ---- near blocks: exact entries, sorted by (row leaf, column leaf)
  H.near.clear();
  for (const auto& bp : near) H.near.push_back({leaf_index[bp.t], leaf_index[bp.s], 0});
  std::sort(H.near.begin(), H.near.end(), [](const NearBlock& a, const NearBlock& b) {
    return a.t_leaf < b.t_leaf || (a.t_leaf == b.t_leaf && a.s_leaf < b.s_leaf);
  });
  int64_t tot = 0;
  for (auto& nb : H.near) {
    nb.data = tot;
    tot += (int64_t)H.leaf_size[nb.t_leaf] * H.leaf_size[nb.s_leaf];
  }
  std::atomic<int> bad{0};
  const int nthreads = o.num_threads > 0 ? o.num_threads : omp_get_max_threads();
  // host entries (every block is written below), or none when the device
  // build computes them (it also rejects coincident points there)
  const int64_t nfill = H.near_on_device ? 0 : (int64_t)H.near.size();
  if (nfill) H.near_data = bigvec<cplx>((size_t)tot);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
  for (int64_t q = 0; q < nfill; ++q) {
    const NearBlock& nb = H.near[q];
    const int m = H.leaf_size[nb.t_leaf], n = H.leaf_size[nb.s_leaf];
    const int t0 = H.leaf_off[nb.t_leaf], s0 = H.leaf_off[nb.s_leaf];
    cplx* dst = H.near_data.data() + nb.data;
    for (int j = 0; j < n; ++j) {
      const int64_t gj = tr.perm[s0 + j];
      for (int i = 0; i < m; ++i) {
        const int64_t gi = tr.perm[t0 + i];
        if (gi != gj) {
          const double dx = p.xyz[3 * gi] - p.xyz[3 * gj], dy = p.xyz[3 * gi + 1] - p.xyz[3 * gj + 1],
                       dz = p.xyz[3 * gi + 2] - p.xyz[3 * gj + 2];
          if (dx * dx + dy * dy + dz * dz < 1e-24) bad.store(1);
        }
        dst[i + (size_t)j * m] = entry(p, gi, gj);
      }
    }
  }
  if (bad.load()) {
    set_error("coincident points off the diagonal (R < 1e-12)");
    return HM_EINVAL;
  }

  // ---- far blocks: compress (t, s) with t before s; (s, t) is its transpose
  std::vector<int32_t> primary;
  for (int32_t q = 0; q < (int32_t)far.size(); ++q)
    if (tr.nodes[far[q].t].off < tr.nodes[far[q].s].off) primary.push_back(q);
  std::sort(primary.begin(), primary.end(), [&](int32_t a, int32_t b) {
    const auto& A = far[a];
    const auto& B = far[b];
    const int32_t ta = tr.nodes[A.t].off, tb = tr.nodes[B.t].off;
    return ta < tb || (ta == tb && tr.nodes[A.s].off < tr.nodes[B.s].off);
  });
  H.lowrank.assign(primary.size(), LowRank());
  // with the near entries, the compression is left to the device build
  H.aca_pending = H.near_on_device;
  H.aca.clear();
  if (H.aca_pending)
    for (const int32_t q : primary) {
      const Cluster& ct = tr.nodes[far[q].t];
      const Cluster& cs = tr.nodes[far[q].s];
      H.aca.push_back({ct.off, ct.size, cs.off, cs.size, 0});
    }
  const int64_t ncomp = H.aca_pending ? 0 : (int64_t)primary.size();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t q = 0; q < ncomp; ++q) {
    const auto& bp = far[primary[q]];
    const Cluster& ct = tr.nodes[bp.t];
    const Cluster& cs = tr.nodes[bp.s];
    H.lowrank[q] = compress_block(p, tr.perm.data() + ct.off, ct.size, tr.perm.data() + cs.off,
                                  cs.size, o.aca_tol, o.max_rank);
  }
  // map (t_off, s_off) of a primary block -> index
  H.far.clear();
  std::vector<std::pair<std::pair<int32_t, int32_t>, int32_t>> key;
  for (int32_t q = 0; q < (int32_t)primary.size(); ++q) {
    const auto& bp = far[primary[q]];
    key.push_back({{tr.nodes[bp.t].off, tr.nodes[bp.s].off}, q});
  }
  std::sort(key.begin(), key.end());
  H.min_far_level = -1;
  for (const auto& bp : far) {
    const Cluster& ct = tr.nodes[bp.t];
    const Cluster& cs = tr.nodes[bp.s];
    FarBlock fb{ct.off, ct.size, cs.off, cs.size, bp.level, -1, false};
    std::pair<int32_t, int32_t> k = (ct.off < cs.off) ? std::make_pair(ct.off, cs.off)
                                                       : std::make_pair(cs.off, ct.off);
    auto it = std::lower_bound(key.begin(), key.end(), std::make_pair(k, int32_t(-1)));
    if (it == key.end() || it->first != k) {
      set_error("internal: partition is not symmetric");
      return HM_EINVAL;
    }
    fb.src = it->second;
    fb.transposed = !(ct.off < cs.off);
    H.far.push_back(fb);
    H.min_far_level = (H.min_far_level < 0) ? bp.level : std::min(H.min_far_level, bp.level);
  }
  // finest level first, then by row and column offset
  std::sort(H.far.begin(), H.far.end(), [](const FarBlock& a, const FarBlock& b) {
    if (a.level != b.level) return a.level > b.level;
    if (a.t_off != b.t_off) return a.t_off < b.t_off;
    return a.s_off < b.s_off;
  });
  return HM_OK;
}

// ---------------------------------------------------------------- batching
void merge_hosts(std::vector<HostH>& parts, HostH& H, std::vector<int64_t>& inst_off) {
  H = HostH();
  int64_t n = 0, nd = 0;
  int32_t nleaf = 0, nlr = 0;
  bool any_volume = false;
  for (auto& P : parts) any_volume = any_volume || P.prob.kind == HM_VOLUME;
  inst_off.assign(parts.size() + 1, 0);
  H.prob.kind = parts.empty() ? HM_SURFACE : parts[0].prob.kind;
  H.near_on_device = !parts.empty();
  H.aca_pending = !parts.empty();
  for (auto& P : parts) {
    H.near_on_device = H.near_on_device && P.near_on_device;
    H.aca_pending = H.aca_pending && P.aca_pending;
  }
  H.tree.depth = kTopLevel;
  H.min_far_level = -1;
  size_t near_total = 0;
  for (auto& P : parts) near_total += P.near_data.size();
  H.near_data.reserve(near_total);
  for (size_t i = 0; i < parts.size(); ++i) {
    HostH& P = parts[i];
    inst_off[i] = n;
    const int32_t L = P.tree.depth;
    for (int64_t q = 0; q < P.prob.n; ++q) {
      H.tree.perm.push_back(P.tree.perm[q] + n);
      H.tree.leaf_of.push_back(P.tree.leaf_of[q] + nleaf);
    }
    const int32_t ibase = (int32_t)H.inst.size();
    for (size_t a = 0; a < P.leaf_off.size(); ++a) {
      H.leaf_off.push_back((int32_t)(P.leaf_off[a] + n));
      H.leaf_size.push_back(P.leaf_size[a]);
      H.leaf_inst.push_back(P.leaf_inst[a] + ibase);
    }
    H.inst.insert(H.inst.end(), P.inst.begin(), P.inst.end());
    H.xyz_tree.insert(H.xyz_tree.end(), P.xyz_tree.begin(), P.xyz_tree.end());
    for (const NearBlock& b : P.near) H.near.push_back({b.t_leaf + nleaf, b.s_leaf + nleaf, b.data + nd});
    H.near_data.insert(H.near_data.end(), P.near_data.begin(), P.near_data.end());
    for (const FarBlock& f : P.far) {
      FarBlock g = f;
      g.t_off += (int32_t)n;
      g.s_off += (int32_t)n;
      g.level = kTopLevel - (L - f.level);
      g.src += nlr;
      H.far.push_back(g);
      H.min_far_level = (H.min_far_level < 0) ? g.level : std::min(H.min_far_level, g.level);
    }
    for (auto& lr : P.lowrank) H.lowrank.push_back(std::move(lr));
    for (HostH::AcaBlock d : P.aca) {
      d.t_off += (int32_t)n;
      d.s_off += (int32_t)n;
      d.inst += ibase;
      H.aca.push_back(d);
    }
    if (any_volume) {
      if (P.prob.kind == HM_VOLUME)
        H.chi_tree.insert(H.chi_tree.end(), P.chi_tree.begin(), P.chi_tree.end());
      else
        H.chi_tree.insert(H.chi_tree.end(), (size_t)P.prob.n, 1.0);
    }
    H.max_leaf = std::max(H.max_leaf, P.max_leaf);
    n += P.prob.n;
    nd += (int64_t)P.near_data.size();
    nleaf += (int32_t)P.leaf_off.size();
    nlr += (int32_t)P.lowrank.size();
    P = HostH();  // release the part
  }
  inst_off[parts.size()] = n;
  H.prob.n = n;
  std::sort(H.far.begin(), H.far.end(), [](const FarBlock& a, const FarBlock& b) {
    if (a.level != b.level) return a.level > b.level;
    if (a.t_off != b.t_off) return a.t_off < b.t_off;
    return a.s_off < b.s_off;
  });
}

// ---------------------------------------------------------------- export
namespace {
struct Writer {
  FILE* f;
  bool ok = true;
  void arr(const char* name, uint32_t dtype, const std::vector<uint64_t>& shape, const void* data,
           size_t bytes) {
    const uint32_t nl = (uint32_t)std::strlen(name);
    const uint32_t nd = (uint32_t)shape.size();
    ok = ok && fwrite(&nl, 4, 1, f) == 1 && fwrite(name, 1, nl, f) == nl &&
         fwrite(&dtype, 4, 1, f) == 1 && fwrite(&nd, 4, 1, f) == 1 &&
         (nd == 0 || fwrite(shape.data(), 8, nd, f) == nd) &&
         (bytes == 0 || fwrite(data, 1, bytes, f) == bytes);
  }
};
}  // namespace

int export_host(const HostH& H, const char* path, const std::vector<cplx>* lu,
                const std::vector<int32_t>* piv) {
  FILE* f = std::fopen(path, "wb");
  if (!f) {
    set_error(std::string("cannot open ") + path);
    return HM_EINVAL;
  }
  Writer w{f};
  const int64_t n = H.prob.n;
  w.arr("perm", 2, {(uint64_t)n}, H.tree.perm.data(), n * 8);
  w.arr("leaf_off", 1, {H.leaf_off.size()}, H.leaf_off.data(), H.leaf_off.size() * 4);
  w.arr("leaf_size", 1, {H.leaf_size.size()}, H.leaf_size.data(), H.leaf_size.size() * 4);
  std::vector<int64_t> nb;
  for (const auto& b : H.near) { nb.push_back(b.t_leaf); nb.push_back(b.s_leaf); nb.push_back(b.data); }
  w.arr("near", 2, {H.near.size(), 3}, nb.data(), nb.size() * 8);
  w.arr("near_data", 4, {H.near_data.size()}, H.near_data.data(), H.near_data.size() * 16);
  std::vector<int64_t> fb;
  std::vector<cplx> uv;  // per block: U (m x r) then V (n x r) of the stored orientation
  for (const auto& b : H.far) {
    const LowRank& lr = H.lowrank[b.src];
    fb.push_back(b.t_off); fb.push_back(b.m); fb.push_back(b.s_off); fb.push_back(b.n);
    fb.push_back(b.level); fb.push_back(lr.r); fb.push_back((int64_t)uv.size());
    const auto& U = b.transposed ? lr.V : lr.U;
    const auto& V = b.transposed ? lr.U : lr.V;
    uv.insert(uv.end(), U.begin(), U.end());
    uv.insert(uv.end(), V.begin(), V.end());
  }
  w.arr("far", 2, {H.far.size(), 7}, fb.data(), fb.size() * 8);
  w.arr("far_uv", 4, {uv.size()}, uv.data(), uv.size() * 16);
  if (!H.chi_tree.empty()) w.arr("chi_tree", 3, {H.chi_tree.size()}, H.chi_tree.data(), H.chi_tree.size() * 8);
  if (lu) w.arr("diag_lu", 4, {lu->size()}, lu->data(), lu->size() * 16);
  if (piv) w.arr("diag_piv", 1, {piv->size()}, piv->data(), piv->size() * 4);
  const bool ok = w.ok;
  if (std::fclose(f) != 0 || !ok) {
    set_error(std::string("write failed: ") + path);
    return HM_EINVAL;
  }
  return HM_OK;
}

}  // namespace hm
