// Internal types of libhmps shared by the host build, the device packer and
// the solver driver.  Not part of the C-ABI.
#pragma once

#include <sys/mman.h>

#include <complex>
#include <cstdint>
#include <cstdlib>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "hmps.h"

namespace hm {

using cplx = std::complex<double>;

// Allocator for large host arrays (blocks, panels): zeroed storage (calloc,
// or 2 MiB-aligned anonymous mappings from 8 MiB on) whose elements are not
// stored to on value initialisation, so that the parallel fills are the
// first touch of the pages (a serial zero fill of tens of GB would dominate
// the build of large batches).
template <typename T>
struct BigAlloc {
  using value_type = T;
  static constexpr size_t kBig = (size_t)8 << 20, kHuge = (size_t)2 << 20, kPage = 4096;
  BigAlloc() = default;
  template <typename U>
  BigAlloc(const BigAlloc<U>&) {}
  static size_t mapped(size_t bytes) { return (bytes + kPage - 1) / kPage * kPage; }
  T* allocate(size_t n) {
    const size_t bytes = n * sizeof(T);
    if (bytes < kBig) {
      void* p = std::calloc(bytes ? bytes : 1, 1);
      if (!p) throw std::bad_alloc();
      return static_cast<T*>(p);
    }
    const size_t len = mapped(bytes);
    void* raw = mmap(nullptr, len + kHuge, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    if (raw == MAP_FAILED) throw std::bad_alloc();
    const uintptr_t r = reinterpret_cast<uintptr_t>(raw);
    const uintptr_t a = (r + kHuge - 1) / kHuge * kHuge;
    if (a > r) munmap(raw, a - r);
    if (r + len + kHuge > a + len) munmap(reinterpret_cast<void*>(a + len), r + len + kHuge - (a + len));
    return reinterpret_cast<T*>(a);
  }
  void deallocate(T* p, size_t n) {
    const size_t bytes = n * sizeof(T);
    if (bytes < kBig)
      std::free(p);
    else
      munmap(p, mapped(bytes));
  }
  // Storage comes zeroed (calloc or fresh anonymous pages), so value
  // initialisation (zero for the arithmetic and complex types stored here)
  // needs no store: large arrays are first touched by the parallel fills.
  template <typename U>
  void construct(U* p) noexcept {
    static_assert(std::is_trivially_copyable<U>::value, "BigAlloc holds plain values");
    (void)p;
  }
  template <typename U, typename... Args>
  void construct(U* p, Args&&... args) {
    ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
  }
  template <typename U>
  bool operator==(const BigAlloc<U>&) const { return true; }
  template <typename U>
  bool operator!=(const BigAlloc<U>&) const { return false; }
};
template <typename T>
using bigvec = std::vector<T, BigAlloc<T>>;

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
struct Error {
  int code;
  std::string msg;
};

// ---------------------------------------------------------------- problem
struct Problem {
  int64_t n = 0;
  int kind = HM_SURFACE;
  double k = 0, h = 0;
  std::vector<double> xyz;  // n x 3
  std::vector<double> chi;  // n (volume)
};

// Entries of Z in original indices (see include/hmps.h for the formulas).
cplx entry(const Problem& p, int64_t i, int64_t j);
// Symmetric kernel part for i != j: Z_ij (surface) or G_ij (volume).
cplx kernel(const Problem& p, int64_t i, int64_t j);

// ---------------------------------------------------------------- tree
struct Cluster {
  int32_t off, size, depth;
  int32_t child[2];  // -1 for a leaf
  double lo[3], hi[3];
  bool leaf() const { return child[0] < 0; }
};

struct Tree {
  std::vector<int64_t> perm;      // tree position -> original index
  std::vector<Cluster> nodes;     // nodes[0] = root
  std::vector<int32_t> leaves;    // node ids in tree order
  std::vector<int32_t> leaf_of;   // tree position -> leaf index
  int32_t depth = 0;              // deepest leaf depth
};

Tree build_tree(const Problem& p, int leaf_max);

struct BlockPair {
  int32_t t, s;    // node ids
  int32_t level;   // max(depth t, depth s)
};

void build_partition(const Tree& tr, double eta, std::vector<BlockPair>& near,
                     std::vector<BlockPair>& far);

// ---------------------------------------------------------------- blocks
// Far block with A ~ U V^T (U m x r, V n x r, both column-major) on the
// symmetric kernel part.  For the volume case the contrast of the source
// points multiplies V's rows when the block is packed for the device.
struct LowRank {
  int32_t m = 0, n = 0, r = 0;
  std::vector<cplx> U, V;
};

// ACA with partial pivoting followed by recompression (rules in aca.cpp).
LowRank compress_block(const Problem& p, const int64_t* rows, int32_t m, const int64_t* cols,
                       int32_t n, double eps, int32_t max_rank);

struct FarBlock {
  int32_t t_off, m, s_off, n, level;
  int32_t src;       // index into the compressed list
  bool transposed;   // block (s,t) stored as the transpose of (t,s)
};

struct NearBlock {
  int32_t t_leaf, s_leaf;
  int64_t data;      // offset into HostH::near_data (column-major m x n)
};

// Kernel parameters of one instance (the entry formulas of include/hmps.h).
struct EntryParams {
  int32_t kind = HM_SURFACE, pad = 0;
  double k = 0, h = 0;
};

// Host-side H-matrix in tree order.
struct HostH {
  Problem prob;
  Tree tree;
  int leaf_max = 0;
  double eta = 1, tol = 1e-4;
  std::vector<int32_t> leaf_off, leaf_size;      // per leaf
  std::vector<NearBlock> near;                   // incl. diagonal, sorted by (t, s)
  bigvec<cplx> near_data;
  std::vector<LowRank> lowrank;                  // compressed (t before s) blocks
  std::vector<FarBlock> far;                     // both orientations
  std::vector<double> chi_tree;                  // volume: chi in tree order
  std::vector<double> xyz_tree;                  // points in tree order (3 per point)
  std::vector<EntryParams> inst;                 // kernel parameters per instance
  std::vector<int32_t> leaf_inst;                // instance of each leaf
  bool near_on_device = false;                   // near entries are left to the device build
  // far blocks left to the device compression (one per lowrank entry):
  // rows t_off .. t_off + m - 1, columns s_off .. s_off + n - 1, tree order
  struct AcaBlock {
    int32_t t_off, m, s_off, n, inst;
  };
  std::vector<AcaBlock> aca;
  bool aca_pending = false;
  int32_t min_far_level = -1;
  int32_t max_leaf = 0;
};

int build_host(const Problem& p, const hm_build_opts& o, HostH& out);

// Level of a far block in a merged (batched) H-matrix: kTopLevel minus its
// distance above the leaf level of its own instance, so that "leaf level"
// (level -1) selects every instance's leaf-level blocks.
constexpr int32_t kTopLevel = HM_MAX_LEVELS - 1;

// Concatenate independent H-matrices into one block-diagonal H-matrix
// (instances keep their own points, leaves and blocks, offset in tree
// order).  parts are consumed.
void merge_hosts(std::vector<HostH>& parts, HostH& out, std::vector<int64_t>& inst_off);

// Two-phase build for the request server: the host part (tree, partition,
// blocks) into a handle without device data, an estimate of the device bytes
// the device part will allocate (workspace for nrhs right-hand sides
// included), then the device part on a stream.
int build_host_phase(const hm_problem* prob, const hm_build_opts* opts, hm_matrix_t* out);
int64_t device_bytes_estimate(hm_matrix_t h, int nrhs);
int build_device_phase(hm_matrix_t h, const hm_build_opts* opts, void* hip_stream);
int64_t workspace_bytes(hm_matrix_t h, int nrhs, int64_t T);
int workspace_rhs(hm_matrix_t h);        // right-hand sides the workspace holds
int64_t resident_bytes(hm_matrix_t h);  // device blocks + workspace
constexpr int kMmMinRhsDefault = 8;  // default right-hand sides from which MFMA kernels run
// GMRES (PS_GMRES): the cycle length a call with these options uses, and the
// device bytes its workspace would add for m and nrhs (0 when it fits)
int gmres_restart(const ps_opts& o);
int64_t gmres_growth_bytes(hm_matrix_t h, int m, int nrhs);
int gmres_rhs(hm_matrix_t h, int m);   // right-hand sides the GMRES basis holds at restart m
int64_t matrix_n(hm_matrix_t h);

// Export helper (binary named arrays).
int export_host(const HostH& H, const char* path, const std::vector<cplx>* lu_host,
                const std::vector<int32_t>* piv_host);

}  // namespace hm
