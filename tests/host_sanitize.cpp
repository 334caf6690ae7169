// The host part of the library's build (cluster tree, eq. 7 partition, ACA
// with recompression, batching of instances, export) run under
// AddressSanitizer and UndefinedBehaviorSanitizer.  tests/test_host_sanitize.py
// compiles this file with the host sources and runs it; any sanitizer
// report, failed build or broken invariant ends it with a non-zero status.
// Inputs: seeded point sets (sphere surfaces and a cube volume) drawn here
// with a small linear congruential generator; no solver arithmetic.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "hm_internal.h"

namespace hm {
void set_error(const std::string& msg) { std::fprintf(stderr, "library error: %s\n", msg.c_str()); }
}  // namespace hm

using namespace hm;

namespace {

struct Lcg {
  uint64_t s;
  double uniform() {  // [0, 1)
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(s >> 11) * (1.0 / 9007199254740992.0);
  }
};

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      std::exit(2);                                                       \
    }                                                                     \
  } while (0)

Problem sphere(int n, double radius, uint64_t seed) {
  Problem p;
  p.n = n;
  p.kind = HM_SURFACE;
  p.k = 2.0 * M_PI;
  p.h = std::sqrt(4.0 * M_PI * radius * radius / n);
  Lcg g{seed};
  for (int i = 0; i < n; ++i) {
    const double z = 1.0 - (2.0 * i + 1.0) / n, r = std::sqrt(std::max(0.0, 1.0 - z * z));
    const double phi = i * M_PI * (3.0 - std::sqrt(5.0));
    double x[3] = {r * std::cos(phi), r * std::sin(phi), z};
    for (double& c : x) c = radius * c + 0.01 * (2.0 * g.uniform() - 1.0);
    const double nn = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    for (double& c : x) p.xyz.push_back(radius * c / nn);
  }
  return p;
}

Problem cube(int side, uint64_t seed) {
  Problem p;
  p.n = (int64_t)side * side * side;
  p.kind = HM_VOLUME;
  p.k = 2.0 * M_PI;
  p.h = 1.0 / 16.0;
  Lcg g{seed};
  for (int i = 0; i < side; ++i)
    for (int j = 0; j < side; ++j)
      for (int l = 0; l < side; ++l) {
        const int idx[3] = {i, j, l};
        for (int c = 0; c < 3; ++c) p.xyz.push_back((idx[c] + 0.5) * p.h + 0.01 * (2.0 * g.uniform() - 1.0));
        p.chi.push_back(0.5 + 1.5 * g.uniform());
      }
  return p;
}

// Invariants of a built host H-matrix: the permutation, the leaves, and the
// blocks covering `cover` entries (n^2 for one instance: every (i, j) once;
// the sum of n_i^2 for a block-diagonal batch).
void check(const HostH& H, int64_t n, int leaf_max, double cover) {
  std::vector<char> seen((size_t)n, 0);
  for (int64_t v : H.tree.perm) {
    CHECK(v >= 0 && v < n && !seen[(size_t)v]);
    seen[(size_t)v] = 1;
  }
  int64_t rows = 0;
  for (size_t a = 0; a < H.leaf_size.size(); ++a) {
    CHECK(H.leaf_off[a] == rows && H.leaf_size[a] >= 1 && H.leaf_size[a] <= leaf_max);
    rows += H.leaf_size[a];
  }
  CHECK(rows == n);
  double covered = 0.0;
  for (const NearBlock& nb : H.near) covered += (double)H.leaf_size[nb.t_leaf] * H.leaf_size[nb.s_leaf];
  for (const FarBlock& fb : H.far) {
    covered += (double)fb.m * fb.n;
    const LowRank& lr = H.lowrank[fb.src];
    CHECK(lr.r >= 1 && lr.r <= std::min(lr.m, lr.n));
    CHECK((int64_t)lr.U.size() == (int64_t)lr.m * lr.r && (int64_t)lr.V.size() == (int64_t)lr.n * lr.r);
    for (const cplx& u : lr.U) CHECK(std::isfinite(u.real()) && std::isfinite(u.imag()));
  }
  CHECK(covered == cover);
}

}  // namespace

int main(int argc, char** argv) {
  const std::string tmp = argc > 1 ? argv[1] : "host_sanitize_export.bin";
  struct Case {
    Problem p;
    int leaf;
    double tol;
  };
  std::vector<Case> cases;
  cases.push_back({sphere(1536, 1.0, 1), 64, 1e-4});
  cases.push_back({sphere(1000, std::sqrt(1000.0 / 1536.0), 7), 40, 1e-4});   // ragged leaves
  cases.push_back({sphere(2200, std::sqrt(2200.0 / 1536.0), 9), 68, 1e-4});   // ragged depths
  cases.push_back({cube(10, 2), 32, 1e-5});
  std::vector<HostH> parts;
  for (Case& c : cases) {
    hm_build_opts o{};
    o.leaf_max = c.leaf;
    o.eta = 1.0;
    o.aca_tol = c.tol;
    o.max_rank = 0;
    o.num_threads = 4;
    o.flags = HM_BUILD_KEEP_HOST;  // the host computes the near entries
    HostH H;
    CHECK(build_host(c.p, o, H) == HM_OK);
    check(H, c.p.n, c.leaf, (double)c.p.n * (double)c.p.n);
    CHECK(!H.near_on_device && !H.near_data.empty());
    // the same build leaving the near entries to the device
    o.flags = 0;
    HostH Hd;
    CHECK(build_host(c.p, o, Hd) == HM_OK);
    CHECK(Hd.near_on_device && Hd.near_data.empty() && Hd.near.size() == H.near.size());
    CHECK((int64_t)Hd.xyz_tree.size() == 3 * c.p.n && Hd.leaf_inst.size() == Hd.leaf_size.size());
    CHECK(Hd.aca_pending && Hd.aca.size() == Hd.lowrank.size() && Hd.aca.size() == H.lowrank.size());
    std::printf("built n=%lld leaf=%d: %zu near, %zu far blocks\n", (long long)c.p.n, c.leaf,
                H.near.size(), H.far.size());
    parts.push_back(std::move(H));
  }
  // a batch of three instances, merged, then exported
  std::vector<HostH> three;
  for (int i = 0; i < 3; ++i) three.push_back(parts[(size_t)i]);
  HostH M;
  std::vector<int64_t> inst_off;
  merge_hosts(three, M, inst_off);
  CHECK(inst_off.size() == 4 && inst_off[3] == 1536 + 1000 + 2200);
  check(M, inst_off[3], 68, 1536.0 * 1536.0 + 1000.0 * 1000.0 + 2200.0 * 2200.0);
  CHECK(export_host(M, tmp.c_str(), nullptr, nullptr) == HM_OK);
  std::remove(tmp.c_str());
  std::printf("ok\n");
  return 0;
}
