// libhmps C-ABI: device packing of the H-matrix, batched leaf LU, the
// power-series solve and the H-matvec (Sec. III-IV).  The host only builds,
// packs and enqueues; every step of the solve runs in the kernels of
// device.hip on the caller's stream.
#include <hip/hip_runtime.h>
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "build_dev.h"
#include "dev.h"
#include "hm_internal.h"
#include "krylov.h"

namespace hm {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

#define HIPCHK(x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      set_error(std::string(#x) + ": " + hipGetErrorString(e_));                    \
      return e_ == hipErrorOutOfMemory ? HM_ENOMEM : HM_EHIP;                       \
    }                                                                               \
  } while (0)

#define STCHK(x)                 \
  do {                           \
    int s_ = (x);                \
    if (s_ != HM_OK) return s_;  \
  } while (0)

struct TermList {
  TermItem* items = nullptr;   // device: pieces grouped by workgroup
  int32_t* wptr = nullptr;     // device: nwg + 1
  int32_t* lptr = nullptr;     // device: nleaves + 1
  int32_t* lprow = nullptr;    // device: partial rows of each leaf's pieces
  int nwg = 0;                 // persistent workgroups
  int npieces = 0;
  int64_t rows = 0;            // partial rows
  int64_t vrow = 0;            // half lists: first partial row of the v slots
  int64_t frow = 0;            // half lists: first partial row of the far-pair slots
  std::vector<TermItem> host;  // the pieces, in list order (before grouping)
};

struct GroupList {
  GroupItem* items = nullptr;  // device
  int n = 0;
};

}  // namespace hm

struct hm_matrix {
  hm::HostH H;
  bool host_only = false;
  bool has_f32 = false;
  bool want_half = true;  // build the half-storage data where the problem allows it
  bool host_kept = true;
  int device = -1;
  int64_t N = 0, T = 0;
  int nl = 0, max_m = 0, L = 0, lmin = -1, nlev = 1;
  int ninst = 1;
  std::vector<int64_t> inst_off;
  double build_ms = 0;
  int64_t bytes = 0;
  std::vector<void*> allocs;

  // per leaf
  int64_t* perm = nullptr;
  int32_t* leaf_off = nullptr;
  int32_t* leaf_m = nullptr;
  // apply panels [D | near | far], series panels D^{-1}[near | far], D^{-1}
  double2* R64 = nullptr;
  float2* R32 = nullptr;
  int64_t* R_off = nullptr;
  int32_t* src = nullptr;
  int64_t* R_col = nullptr;
  double2* M64 = nullptr;
  float2* M32 = nullptr;
  int64_t* M_off = nullptr;
  int64_t* M_col = nullptr;
  double2* LU = nullptr;      // m x m per leaf (ld m)
  int64_t* LU_off = nullptr;
  double2* Dinv = nullptr;    // ld even(m) per leaf
  int64_t* Dinv_off = nullptr;
  int32_t* piv = nullptr;
  int64_t* piv_off = nullptr;
  // stage A groups (global far blocks)
  double2* W64 = nullptr;
  float2* W32 = nullptr;
  hm::Group* groups = nullptr;
  // in-row W stacks
  double2* IR64 = nullptr;
  float2* IR32 = nullptr;
  int64_t* ir_off = nullptr;
  int32_t *ir_ld = nullptr, *ir_ncol = nullptr, *ir_row0 = nullptr, *ir_soff = nullptr,
          *ir_n = nullptr;
  // per level index
  std::vector<hm::TermList> tl_apply, tl_series;
  std::vector<hm::GroupList> sa;
  std::vector<int64_t> ent_R, ent_M, ent_W, ncoef;
  hm::TermList tl_dinv;
  // many right-hand sides (matrix-core kernels): every far block goes
  // through stage A (groups over all far blocks by source cluster), so the
  // panels' in-row U columns read their t from xin like the global ones
  int32_t* src_mm = nullptr;
  double2* Wmm64 = nullptr;
  float2* Wmm32 = nullptr;
  hm::Group* groups_mm = nullptr;
  std::vector<hm::TermList> tl_apply_mm, tl_series_mm;
  hm::TermList tl_dinv_mm;  // D^{-1} panels on the matrix-core kernels
  // half-storage product (symmetric problems, one right-hand side): per
  // row leaf t its near blocks (t, s > t) side by side (half panels), the
  // source row and v slot of every half-panel column, and per-level lists
  // whose pieces are half-panel column ranges plus the far pieces of the
  // apply panels
  double2* H64 = nullptr;
  float2* H32 = nullptr;
  double2 *HF64 = nullptr, *IRT64 = nullptr, *WT64 = nullptr;  // scaled far data
  float2 *HF32 = nullptr, *IRT32 = nullptr, *WT32 = nullptr;
  int64_t *hf_off = nullptr, *hf_col = nullptr;
  double2 *CH = nullptr, *CHT = nullptr;  // C_a^{-1}, C_a^{-T} panels (ld even m)
  double2 *CF = nullptr, *CFT = nullptr;  // C_a, C_a^T panels (ld even m)
  double2* hwork = nullptr;               // half-storage H-matvec: (I + S) C^T x (N)
  int64_t* ch_off = nullptr;
  int64_t* hp_off = nullptr;
  int32_t *hp_col = nullptr, *hsrc = nullptr;
  int64_t hp_cols = 0;            // half-panel columns in all (v slots)
  std::vector<int32_t> vptr_h, vstart_h;  // per leaf: v slots of its blocks (t, leaf), t < leaf
  double2* zbuf = nullptr;        // sum of the scaled terms (tree order, N)
  int32_t* hq = nullptr;          // piece queue of the half-storage kernel (2 ints)
  bool half_ok = false;
  std::vector<int64_t> hp_ncol;   // per leaf: half-panel columns
  std::vector<std::vector<int32_t>> hp_bcol, hp_bleaf;  // per leaf: block starts, leaves
  struct HalfList {
    hm::TermList tl;
    int32_t *lcnt = nullptr, *vleaf = nullptr;
    bool multi = false;  // every far block of the level is a pair: all K terms in one launch
  };
  std::vector<HalfList> half;
  // far blocks between two leaves in the scaled basis, stored once per pair
  // (t < s): U' then W' per pair; the remaining far blocks keep in-row
  // stacks (hir_*) and far-panel columns [in-row U' | global U'] (HF*)
  double2* FP64 = nullptr;
  float2* FP32 = nullptr;
  int64_t* fp_off = nullptr;
  int32_t *fp_rank = nullptr, *fp_slot = nullptr;
  std::vector<int32_t> fp_first_h;              // per leaf (+ end): first pair
  std::vector<int32_t> fp_rank_h, fp_tgt_h, fp_slot_h;  // per pair
  std::vector<std::vector<int32_t>> fp_end;     // per level, per leaf: pairs of level >= l
  int64_t fp_rows = 0;                          // partial rows of all pairs' z_s
  int64_t* hir_off = nullptr;
  int32_t *hir_ld = nullptr, *hir_ncol = nullptr, *hir_row0 = nullptr, *hir_soff = nullptr,
          *hir_n = nullptr;
  std::vector<int64_t> hir_cols;                // per leaf: in-row stack rows
  std::vector<int32_t> hir_ncol_h;
  std::vector<std::vector<int64_t>> hir_end;    // per level, per leaf
  std::vector<int64_t> ent_half;  // entries read per half-storage product, per level
  int use_half = 1;               // 1: half storage where available (K terms per launch
                                  // where the level allows), 3: one launch per term, 2: panels
  int32_t* hdone = nullptr;       // multi-term launch: per leaf, last finished term
  int32_t* herr = nullptr;        // multi-term launch: a dependency wait gave up
  int half_pct = 100;             // cost weight (%) of half-panel columns in the work split
  std::vector<hm::GroupList> sa_mm;
  std::vector<std::vector<hm::GroupItem>> sa_mm_host;  // the same tiles on the host
  std::vector<int32_t> group_mm_inst;                  // instance of each many-RHS group
  // multi-term matrix-core series, per level (see MMSeriesArgs)
  struct MMMulti {
    hm::MMItem* items = nullptr;
    int n_a = 0, n_b = 0;
    int32_t* need_a = nullptr;
    int32_t* need_b = nullptr;
    bool ok = false;
  };
  std::vector<MMMulti> mm_multi;
  int32_t* mm_cnt = nullptr;    // instances x kMmSeriesMaxTerms x 2, zero between launches
  int32_t* mm_queue = nullptr;  // 2
  int32_t* mm_err = nullptr;    // a wait of the multi-term launch gave up
  int mm_multi_mode = 2;        // 1: one launch for the K terms where it applies; 2: per term
  int mm_series_wgs[2][2] = {{0, 0}, {0, 0}};  // resident round by [f32][nrhs > 16]
  int mm_min_rhs = hm::kMmMinRhsDefault;  // right-hand sides from which the MFMA kernels run
  int rhs_tile = 0;             // MFMA right-hand-side tile (0: by nrhs)
  int inrow_pct = 100;          // cost weight (%) of in-row rows in the work split
  // per-leaf column layout of the panels, kept to rebuild the work lists
  std::vector<int64_t> near_cols, ir_cols;
  std::vector<int32_t> ir_ncol_h;
  std::vector<std::vector<int64_t>> ir_end, gl_end;
  std::vector<void*> list_allocs;  // device work lists (rebuilt by hmat_tune)
  int64_t list_bytes = 0;
  int64_t partial_rows = 0;
  int term_wgs = 1024;          // persistent workgroups of a term kernel
  int term_wgs_auto = 1024;
  int num_cus = 256;            // compute units of the device
  int half_wgs_auto = 512;      // resident round of the half-storage kernel
  int half_wgs_multi = 512;     // the same for its multi-term form
  int32_t* counters = nullptr;  // workspace
  // workspace
  int ws_nrhs = 0;
  int64_t ws_bytes = 0;
  double2 *xin0 = nullptr, *xin1 = nullptr, *xt = nullptr, *bt = nullptr, *rt = nullptr,
          *dt = nullptr, *partial = nullptr;
  // [y | t] in row layout for the matrix-core kernels (ld ws_ldr): FP64 and
  // FP32 copies, two of each (term input and output)
  double2 *xr64_0 = nullptr, *xr64_1 = nullptr;
  float2 *xr32_0 = nullptr, *xr32_1 = nullptr;
  int64_t ws_ldr = 0;
  double *nscratch = nullptr, *norms = nullptr;
  double* norms_host = nullptr;  // pinned
  // norm segments (one per instance) and their row items
  hm::NormItem* norm_items = nullptr;
  int32_t* norm_seg = nullptr;
  int n_norm_items = 0, nseg = 1;
  std::vector<void*> ws_allocs;
  // restarted GMRES: basis and preconditioned blocks, small per-column state
  std::vector<void*> gm_allocs;
  int gm_m = 0, gm_nrhs = 0;
  double2 *gm_V = nullptr, *gm_Z = nullptr, *gm_part = nullptr, *gm_h1 = nullptr,
          *gm_h2 = nullptr, *gm_hn = nullptr, *gm_bn = nullptr, *gm_y = nullptr;
  hm::KrylovState gm_S{};
  double* gm_host = nullptr;  // pinned: residual estimates, then flags
  // nested multi-level solve: a LIFO pool of N x nrhs work vectors
  double2* nest_pool = nullptr;
  int nest_cap = 0, nest_nrhs = 0;
  // per-kernel timing
  bool prof = false;
  struct ProfRec { int cls; hipEvent_t e0, e1; };
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> ev_pool;

  ~hm_matrix() {
    for (auto& r : prof_recs) { (void)hipEventDestroy(r.e0); (void)hipEventDestroy(r.e1); }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (void* p : ws_allocs) (void)hipFree(p);
    for (void* p : gm_allocs) (void)hipFree(p);
    if (gm_host) (void)hipHostFree(gm_host);
    if (nest_pool) (void)hipFree(nest_pool);
    for (void* p : list_allocs) (void)hipFree(p);
    for (void* p : allocs) (void)hipFree(p);
    if (norms_host) (void)hipHostFree(norms_host);
  }
};

namespace hm {

namespace {

// Device allocation owned by the handle (freed with it), or by the work
// lists when `lists` is set (freed when they are rebuilt).
int dalloc(hm_matrix* h, void** p, size_t bytes, bool lists = false) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    return HM_ENOMEM;
  }
  (lists ? h->list_allocs : h->allocs).push_back(*p);
  h->bytes += (int64_t)bytes;
  if (lists) h->list_bytes += (int64_t)bytes;
  return HM_OK;
}

// pad: zeroed bytes after the data (panels the matrix-core kernels read
// past their last column, kPanelPad)
template <typename T, typename A>
int upload(hm_matrix* h, T** dst, const std::vector<T, A>& v, hipStream_t st, bool lists = false,
           size_t pad = 0) {
  STCHK(dalloc(h, (void**)dst, v.size() * sizeof(T) + pad, lists));
  if (!v.empty()) HIPCHK(hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  if (pad) HIPCHK(hipMemsetAsync(reinterpret_cast<char*>(*dst) + v.size() * sizeof(T), 0, pad, st));
  HIPCHK(hipStreamSynchronize(st));  // host vectors may be freed after return
  return HM_OK;
}

int level_index(const hm_matrix* h, int level, int* li) {
  if (h->lmin < 0) {
    if (level > h->L) { set_error("level beyond the leaf level"); return HM_EINVAL; }
    *li = 0;
    return HM_OK;
  }
  int l = level < 0 ? h->L : level;
  if (l > h->L) { set_error("level beyond the leaf level"); return HM_EINVAL; }
  l = std::max(l, h->lmin);
  *li = l - h->lmin;
  return HM_OK;
}

// Pieces of one term kernel, split evenly over h->term_wgs persistent
// workgroups.  Per leaf a, in order: dense column ranges dense[a] (pairs
// [begin, end), cost m per column), then in-row stack rows [0, inrow_rows[a])
// (cost W row + U column per row) whose panel columns start at inrow_col[a].
// Each unit of work goes to the workgroup whose share its cost start falls
// in; runs of units of one segment within one workgroup form a piece (in-row
// pieces at most kInRowTile rows).
int make_termlist(hm_matrix* h, const std::vector<std::vector<std::pair<int64_t, int64_t>>>& dense,
                  const std::vector<int64_t>& inrow_rows, const std::vector<int64_t>& inrow_col,
                  const std::vector<int32_t>& inrow_ncol, TermList& tl, hipStream_t st,
                  hm_matrix::HalfList* hl = nullptr, int units = 0, bool whole = false,
                  const std::vector<int32_t>* npairs = nullptr) {
  struct Seg { int leaf, kind; int64_t u0, u1, col0, cost; };
  std::vector<Seg> segs;
  int64_t total = 0;
  for (int a = 0; a < h->nl; ++a) {
    const int64_t m = h->H.leaf_size[a];
    const size_t first = segs.size();
    if (hl && h->hp_ncol[a] > 0) segs.push_back({a, 2, 0, h->hp_ncol[a], 0, m * h->half_pct / 100});
    for (auto& r : dense[a])
      if (r.second > r.first) segs.push_back({a, 0, r.first, r.second, 0, m});
    if (inrow_rows[a] > 0)
      segs.push_back({a, 1, 0, inrow_rows[a], inrow_col[a],
                      ((int64_t)inrow_ncol[a] + m) * h->inrow_pct / 100});
    if (hl && npairs && (*npairs)[a] > 0) {  // far pairs: cost of the leaf's average pair
      const int32_t p0 = h->fp_first_h[a], np = (*npairs)[a];
      int64_t c = 0;
      for (int32_t p = p0; p < p0 + np; ++p)
        c += (int64_t)h->fp_rank_h[p] * (m + h->H.leaf_size[h->fp_tgt_h[p]]);
      segs.push_back({a, 3, 0, np, 0, std::max<int64_t>(1, c / np)});
    }
    if (segs.size() == first) segs.push_back({a, 0, 0, 0, 0, 0});  // epilogue only
    for (size_t k = first; k < segs.size(); ++k) total += (segs[k].u1 - segs[k].u0) * segs[k].cost;
  }
  // the half-storage kernel's own resident round unless a count was set
  const int G = units > 0 ? units
                          : std::max(1, hl && h->term_wgs == h->term_wgs_auto ? h->half_wgs_auto
                                                                               : h->term_wgs);
  std::vector<TermItem> items;
  std::vector<int32_t> wg_of, vleaf, lcnt(hl ? h->nl : 0, 0);
  int64_t rows = 0, done = 0;
  if (hl) {
    // Half lists are consumed dynamically (each workgroup takes the next
    // piece from a queue): pieces of bounded size, largest estimated cost
    // first so that the last pieces taken are small.
    std::vector<std::pair<int64_t, TermItem>> pcs;
    for (const Seg& sg : segs) {
      const int m = h->H.leaf_size[sg.leaf];
      int64_t u = sg.u0;
      do {
        int64_t k = sg.u1 - u;
        if (sg.kind == 1) k = std::min<int64_t>(k, kHalfInRowTile);  // starts stay even
        if (sg.kind == 0) k = std::min<int64_t>(k, kHalfChunk);
        std::vector<int32_t>::const_iterator b0, b1;
        if (sg.kind == 2) {
          k = std::min<int64_t>(k, kHalfPieceCols);
          const std::vector<int32_t>& bc = h->hp_bcol[sg.leaf];
          b0 = std::upper_bound(bc.begin(), bc.end(), (int32_t)u) - 1;
          const int64_t nb = (int64_t)bc.size() - 1;
          const int64_t lim = std::min<int64_t>(b0 - bc.begin() + kMaxVLeaves, nb);
          k = std::min<int64_t>(k, bc[lim] - u);
          b1 = std::upper_bound(bc.begin(), bc.end(), (int32_t)(u + k - 1));
        }
        if (sg.kind == 3) k = std::min<int64_t>(k, kMaxVLeaves);
        TermItem it{sg.leaf, sg.kind, 0, 0, 0, 0, (int32_t)rows, 0};
        int64_t cost = k * sg.cost;
        if (sg.kind == 1) {
          it.r0 = (int32_t)u;
          it.r1 = (int32_t)(u + k);
          it.c0 = (int32_t)(sg.col0 + u);
          it.c1 = (int32_t)(sg.col0 + u + k);
        } else if (sg.kind == 3) {
          it.c0 = (int32_t)(h->fp_first_h[sg.leaf] + u);
          it.c1 = (int32_t)(it.c0 + k);
          it.r0 = (int32_t)vleaf.size();
          cost = 0;
          for (int32_t p = it.c0; p < it.c1; ++p) {
            const int s = h->fp_tgt_h[p];
            vleaf.push_back(s);
            lcnt[s]++;
            cost += (int64_t)h->fp_rank_h[p] * (m + h->H.leaf_size[s]);
          }
          it.r1 = (int32_t)vleaf.size();
        } else {
          it.c0 = (int32_t)u;
          it.c1 = (int32_t)(u + k);
        }
        if (sg.kind == 2) {
          const std::vector<int32_t>& bl = h->hp_bleaf[sg.leaf];
          const int64_t q0 = b0 - h->hp_bcol[sg.leaf].begin(), q1 = b1 - h->hp_bcol[sg.leaf].begin();
          it.r0 = (int32_t)vleaf.size();
          for (int64_t q = q0; q < q1; ++q) {
            vleaf.push_back(bl[q]);
            lcnt[bl[q]]++;
          }
          it.r1 = (int32_t)vleaf.size();
        }
        pcs.push_back({cost, it});
        rows += m;
        u += k;
      } while (u < sg.u1);
    }
    // Queue order.  Pieces whose leaves (its own and those its columns or
    // pairs read) all lie in the first part of the tree order come first,
    // those whose leaves all lie in the last part come last, the rest in
    // between, each part about a third of the pieces.  When the K terms
    // run as one launch, the pieces still running at the end of a term then
    // touch only the last leaves, and the first pieces of the next term
    // read only the first ones, which are done: the terms overlap instead
    // of waiting for each other.  Within a part, far pairs (the slowest per
    // byte) first, then the largest estimated cost first, so that the last
    // pieces taken are small.
    std::vector<int32_t> lo(pcs.size()), hi(pcs.size());
    for (size_t q = 0; q < pcs.size(); ++q) {
      const TermItem& it = pcs[q].second;
      lo[q] = hi[q] = it.leaf;
      if (it.kind >= 2)
        for (int32_t r = it.r0; r < it.r1; ++r) {
          lo[q] = std::min(lo[q], vleaf[r]);
          hi[q] = std::max(hi[q], vleaf[r]);
        }
    }
    // first leaf bound h1 with a third of the pieces below it, last bound h2
    // with a third at or above it
    const int64_t third = (int64_t)pcs.size() / 3;
    std::vector<int32_t> sh(hi), sl(lo);
    std::sort(sh.begin(), sh.end());
    std::sort(sl.begin(), sl.end());
    const int32_t h1 = sh.empty() ? 0 : sh[(size_t)third];
    const int32_t h2 = sl.empty() ? 0 : sl[sl.size() - 1 - (size_t)third];
    std::vector<int> part(pcs.size());
    for (size_t q = 0; q < pcs.size(); ++q)
      part[q] = hi[q] < h1 ? 0 : (lo[q] > h2 ? 2 : 1);
    std::vector<size_t> ord(pcs.size());
    for (size_t q = 0; q < ord.size(); ++q) ord[q] = q;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
      if (part[x] != part[y]) return part[x] < part[y];
      const bool px = pcs[x].second.kind == 3, py = pcs[y].second.kind == 3;
      if (px != py) return px;
      return pcs[x].first > pcs[y].first;
    });
    std::vector<std::pair<int64_t, TermItem>> sorted;
    for (size_t q : ord) sorted.push_back(pcs[q]);
    pcs.swap(sorted);
    for (auto& pc : pcs) {
      items.push_back(pc.second);
      wg_of.push_back(0);
    }
  }
  auto wg_at = [&](int64_t cost) {
    return total > 0 ? (int)std::min<int64_t>(G - 1, (cost * G) / total) : 0;
  };
  if (whole && !hl) {
    // whole leaves: every segment of a leaf is one piece of the same unit
    // (no partial sums for a single-segment leaf); leaves go to the least
    // loaded unit, largest first (LPT), and each unit runs its pieces in
    // tree order
    std::vector<int64_t> lcost(h->nl, 0);
    for (const Seg& sg : segs) lcost[sg.leaf] += (sg.u1 - sg.u0) * sg.cost + 1;
    std::vector<int> order(h->nl);
    for (int a = 0; a < h->nl; ++a) order[a] = a;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return lcost[x] > lcost[y]; });
    std::vector<std::pair<int64_t, int>> heap;  // (load, unit), min-heap
    for (int g = 0; g < G; ++g) heap.push_back({0, g});
    auto gt = [](const std::pair<int64_t, int>& x, const std::pair<int64_t, int>& y) { return x > y; };
    std::make_heap(heap.begin(), heap.end(), gt);
    std::vector<int> unit_of(h->nl, 0);
    for (int a : order) {
      std::pop_heap(heap.begin(), heap.end(), gt);
      unit_of[a] = heap.back().second;
      heap.back().first += lcost[a];
      std::push_heap(heap.begin(), heap.end(), gt);
    }
    for (const Seg& sg : segs) {
      const int m = h->H.leaf_size[sg.leaf];
      TermItem it{sg.leaf, 0, (int32_t)sg.u0, (int32_t)sg.u1, 0, 0, (int32_t)rows, 0};
      items.push_back(it);
      wg_of.push_back(unit_of[sg.leaf]);
      rows += m;
    }
  }
  // other lists: pieces split evenly over the G workgroups by cost, each
  // workgroup taking a contiguous run
  for (size_t si = 0; si < (hl || whole ? 0 : segs.size()); ++si) {
    const Seg& sg = segs[si];
    const int m = h->H.leaf_size[sg.leaf];
    int64_t u = sg.u0;
    do {
      const int g = wg_at(done);
      // units of this segment that start before the next workgroup boundary
      int64_t k = sg.u1 - u;
      if (g < G - 1 && sg.cost > 0) {
        const int64_t bound = ((int64_t)(g + 1) * total + G - 1) / G;
        k = std::min(k, std::max<int64_t>(1, (bound - done + sg.cost - 1) / sg.cost));
      }
      if (sg.kind == 1) {
        // FP32 stacks are read two rows per load from an even row: keep
        // every in-row piece start even (kInRowTile is even)
        k = std::min<int64_t>(k, kInRowTile);
        if ((k & 1) && u + k < sg.u1) ++k;
      }
      TermItem it{sg.leaf, sg.kind, 0, 0, 0, 0, (int32_t)rows, 0};
      if (sg.kind == 0) {
        it.c0 = (int32_t)u;
        it.c1 = (int32_t)(u + k);
      } else {
        it.r0 = (int32_t)u;
        it.r1 = (int32_t)(u + k);
        it.c0 = (int32_t)(sg.col0 + u);
        it.c1 = (int32_t)(sg.col0 + u + k);
      }
      items.push_back(it);
      wg_of.push_back(g);
      rows += m;
      done += k * sg.cost;
      u += k;
    } while (u < sg.u1);
  }
  for (const TermItem& it : items)
    if ((it.kind == 1 && ((it.r0 & 1) || it.r1 - it.r0 > (hl ? kHalfInRowTile : kInRowTile))) ||
        ((it.kind == 2 || it.kind == 3) && (it.r1 - it.r0 < 1 || it.r1 - it.r0 > kMaxVLeaves)) ||
        (it.kind == 3 && (!hl || it.c1 - it.c0 != it.r1 - it.r0)) ||
        (hl && it.c1 - it.c0 > kHalfChunk && it.kind != 1)) {
      set_error("internal: bad term piece");
      return HM_EINVAL;
    }
  if (rows >= ((int64_t)1 << 31)) { set_error("term partial rows exceed 2^31"); return HM_EINVAL; }
  // group pieces by workgroup (stable: pieces of one workgroup keep their order)
  std::vector<int32_t> wptr(G + 1, 0);
  for (int g : wg_of) wptr[g + 1]++;
  for (int g = 0; g < G; ++g) wptr[g + 1] += wptr[g];
  std::vector<TermItem> by_wg(items.size());
  std::vector<int32_t> fill(wptr.begin(), wptr.end() - 1);
  for (size_t q = 0; q < items.size(); ++q) by_wg[fill[wg_of[q]]++] = items[q];
  // per leaf: the partial rows of its pieces, in piece order (half lists:
  // then the v slots of the blocks (t, leaf), t < leaf, which follow the
  // pieces' rows in the partial buffer, then the z rows of the far pairs
  // (t, leaf) of the list, in pair order)
  std::vector<int32_t> lptr(h->nl + 1, 0), lprow, own(h->nl, 0);
  std::vector<std::vector<int32_t>> pair_in(hl ? h->nl : 0);
  for (auto& it : items) {
    lptr[it.leaf + 1]++;
    own[it.leaf]++;
    if (it.kind == 3)
      for (int32_t p = it.c0; p < it.c1; ++p) pair_in[h->fp_tgt_h[p]].push_back(p);
  }
  if (hl)
    for (int a = 0; a < h->nl; ++a) {
      std::sort(pair_in[a].begin(), pair_in[a].end());
      lptr[a + 1] += h->vptr_h[a + 1] - h->vptr_h[a] + (int32_t)pair_in[a].size();
    }
  for (int a = 0; a < h->nl; ++a) lptr[a + 1] += lptr[a];
  lprow.assign(lptr[h->nl], 0);
  std::vector<int32_t> lf(lptr.begin(), lptr.end() - 1);
  for (auto& it : items) lprow[lf[it.leaf]++] = it.prow;
  tl.vrow = rows;
  if (hl && rows + h->hp_cols >= ((int64_t)1 << 31)) {
    set_error("term partial rows exceed 2^31");
    return HM_EINVAL;
  }
  if (hl) {
    for (int a = 0; a < h->nl; ++a)
      for (int q = h->vptr_h[a]; q < h->vptr_h[a + 1]; ++q)
        lprow[lf[a]++] = (int32_t)(rows + h->vstart_h[q]);
    rows += h->hp_cols;
    tl.frow = rows;
    if (rows + h->fp_rows >= ((int64_t)1 << 31)) {
      set_error("term partial rows exceed 2^31");
      return HM_EINVAL;
    }
    for (int a = 0; a < h->nl; ++a)
      for (int32_t p : pair_in[a]) lprow[lf[a]++] = (int32_t)(rows + h->fp_slot_h[p]);
    rows += h->fp_rows;
  }
  tl.nwg = G;
  tl.npieces = (int)items.size();
  tl.rows = rows;
  tl.host = items;
  STCHK(upload(h, &tl.items, by_wg, st, true));
  STCHK(upload(h, &tl.wptr, wptr, st, true));
  STCHK(upload(h, &tl.lptr, lptr, st, true));
  STCHK(upload(h, &tl.lprow, lprow, st, true));
  if (hl) {
    hl->multi = true;
    for (const TermItem& it : items)
      if (it.kind == 1 || (it.kind == 0 && it.c1 > it.c0)) hl->multi = false;
    for (int a = 0; a < h->nl; ++a) lcnt[a] += own[a];
    STCHK(upload(h, &hl->lcnt, lcnt, st, true));
    STCHK(upload(h, &hl->vleaf, vleaf, st, true));
  }
  h->partial_rows = std::max(h->partial_rows, rows);
  return HM_OK;
}

int upload_groups(hm_matrix* h, const std::vector<GroupItem>& v, GroupList& gl, hipStream_t st) {
  gl.n = (int)v.size();
  return upload(h, &gl.items, v, st);
}

// Split-K counters: per (leaf, right-hand-side tile) for the streaming
// kernels, per (leaf, block of rows < 4, 16-RHS tile) for the matrix cores.
int64_t counter_count(const hm_matrix* h, int nrhs) {
  return (int64_t)h->nl * std::max<int64_t>(nrhs, 4 * ((nrhs + 15) / 16));
}

__global__ void k_zero_i32(int32_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// n 32-bit words at p set to zero on stream st: a fill kernel, ordered with
// the stream's later work (a memset on the null stream is not ordered with
// a non-blocking stream), and no memset node when the caller captures
hipError_t zero_words(void* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256),
                     0, st, (int32_t*)p, n);
  return hipGetLastError();
}

// The row-layout and counter workspace for nrhs right-hand sides; the
// counters and the zero rows are cleared on st, ahead of the solve's work.
int ensure_workspace(hm_matrix* h, int nrhs, hipStream_t st) {
  if (nrhs <= h->ws_nrhs) return HM_OK;
  for (void* p : h->ws_allocs) (void)hipFree(p);
  h->ws_allocs.clear();
  h->ws_nrhs = 0;
  h->ws_bytes = 0;
  const int64_t ldin = h->N + h->T;
  auto al = [&](void** p, size_t bytes) -> int {
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("workspace hipMalloc failed: " + std::string(hipGetErrorString(e)));
      return HM_ENOMEM;
    }
    h->ws_allocs.push_back(*p);
    h->ws_bytes += (int64_t)std::max<size_t>(bytes, 16);
    return HM_OK;
  };
  const int64_t ldr = row_ld(nrhs);
  STCHK(al((void**)&h->xin0, sizeof(double2) * ldin * nrhs));
  STCHK(al((void**)&h->xin1, sizeof(double2) * ldin * nrhs));
  // row-layout vectors: rows [y | t] plus one row of zeros (zrow = N + T)
  STCHK(al((void**)&h->xr64_0, sizeof(double2) * (ldin + 1) * ldr));
  STCHK(al((void**)&h->xr64_1, sizeof(double2) * (ldin + 1) * ldr));
  STCHK(al((void**)&h->xr32_0, sizeof(float2) * (ldin + 1) * ldr));
  STCHK(al((void**)&h->xr32_1, sizeof(float2) * (ldin + 1) * ldr));
  HIPCHK(zero_words(h->xr64_0 + ldin * ldr, 4 * ldr, st));
  HIPCHK(zero_words(h->xr64_1 + ldin * ldr, 4 * ldr, st));
  HIPCHK(zero_words(h->xr32_0 + ldin * ldr, 2 * ldr, st));
  HIPCHK(zero_words(h->xr32_1 + ldin * ldr, 2 * ldr, st));
  STCHK(al((void**)&h->xt, sizeof(double2) * h->N * nrhs));
  STCHK(al((void**)&h->bt, sizeof(double2) * h->N * nrhs));
  STCHK(al((void**)&h->rt, sizeof(double2) * h->N * nrhs));
  STCHK(al((void**)&h->dt, sizeof(double2) * h->N * nrhs));
  STCHK(al((void**)&h->partial, sizeof(double2) * h->partial_rows * ldr));
  STCHK(al((void**)&h->nscratch, sizeof(double) * h->n_norm_items * nrhs * 2));
  STCHK(al((void**)&h->norms, sizeof(double) * h->nseg * nrhs * 2));
  STCHK(al((void**)&h->counters, sizeof(int32_t) * counter_count(h, nrhs)));
  HIPCHK(zero_words(h->counters, counter_count(h, nrhs), st));
  h->ws_ldr = ldr;
  if (h->norms_host) (void)hipHostFree(h->norms_host);
  h->norms_host = nullptr;
  HIPCHK(hipHostMalloc((void**)&h->norms_host, sizeof(double) * h->nseg * nrhs * 2,
                       hipHostMallocDefault));
  h->ws_nrhs = nrhs;
  return HM_OK;
}

PanelSet apply_set(const hm_matrix* h, bool f32, const int32_t* src) {
  return PanelSet{f32 ? (const void*)h->R32 : (const void*)h->R64, h->R_off, src, h->R_col,
                  h->leaf_m};
}
PanelSet series_set(const hm_matrix* h, bool f32, const int32_t* src) {
  return PanelSet{f32 ? (const void*)h->M32 : (const void*)h->M64, h->M_off, src, h->M_col,
                  h->leaf_m};
}
PanelSet dinv_set(const hm_matrix* h) {
  return PanelSet{(const void*)h->Dinv, h->Dinv_off, h->src, h->R_col, h->leaf_m};
}

TermArgs term_args(const hm_matrix* h, const PanelSet& ps, const TermList& tl, bool f32,
                   const double2* xin, int64_t ldx) {
  TermArgs t{};
  t.ps = ps;
  t.ir = InRow{f32 ? (const void*)h->IR32 : (const void*)h->IR64, h->ir_off, h->ir_ld,
               h->ir_ncol, h->ir_row0, h->ir_soff, h->ir_n};
  t.items = tl.items;
  t.wptr = tl.wptr;
  t.lptr = tl.lptr;
  t.lprow = tl.lprow;
  t.leaf_off = h->leaf_off;
  t.xin = xin;
  t.ldx = ldx;
  t.partial = h->partial;
  t.ldp = h->partial_rows;
  t.counters = h->counters;
  t.ldr = h->ws_ldr;
  t.zrow = (int32_t)(h->N + h->T);
  t.alpha = 1.0;
  t.beta = 0.0;
  return t;
}

hipEvent_t pool_event(hm_matrix* h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  // timing-only events: no system-scope fence when they are recorded
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Brackets one kernel launch with events when profiling is on.
struct ProfScope {
  hm_matrix* h;
  int cls;
  hipStream_t st;
  hipEvent_t e0 = nullptr;
  ProfScope(hm_matrix* h_, int cls_, hipStream_t st_) : h(h_), cls(cls_), st(st_) {
    if (h->prof && (e0 = pool_event(h)) != nullptr) (void)hipEventRecord(e0, st);
  }
  void done() {
    if (!e0) return;
    hipEvent_t e1 = pool_event(h);
    if (!e1) { h->ev_pool.push_back(e0); e0 = nullptr; return; }
    (void)hipEventRecord(e1, st);
    h->prof_recs.push_back({cls, e0, e1});
    e0 = nullptr;
  }
  ~ProfScope() { if (e0) h->ev_pool.push_back(e0); }
};

#define TIMED(cls, call)                 \
  do {                                   \
    ProfScope ps_(h, cls, st);           \
    HIPCHK(call);                        \
    ps_.done();                          \
  } while (0)

// Power series of Sec. IV: y_0 = D^{-1} rhs, y_k = -(D^{-1} R_l) y_{k-1},
// x = sum y_k, accumulated in tree order in x_tree (ld N).  rhs is read in
// tree order (ld N), or in original order through the permutation when
// rhs_perm is set (ld ldr).  When out is set the final x is also written
// there in original order (ld ldo).
// Squared norms of v per (instance, column) into slot 0 or 1 of h->norms
// (slot * nseg * nrhs + c * nseg + instance).
hipError_t norms_into(hm_matrix* h, const double2* v, int64_t ld, int nrhs, int slot,
                      hipStream_t st) {
  return launch_norm2(v, ld, h->norm_items, h->n_norm_items, h->norm_seg, h->nseg, nrhs,
                      h->nscratch + (int64_t)slot * h->n_norm_items * nrhs,
                      h->norms + (int64_t)slot * h->nseg * nrhs, st);
}

// From h->mm_min_rhs right-hand sides on, the term and stage-A products run
// on the matrix cores (MM kernels, their own lists and stage-A groups).
struct Path {
  bool mm;
  const void* W;
  const Group* groups;
  const std::vector<GroupList>* sa;
  const std::vector<TermList>* tl_series;
  const std::vector<TermList>* tl_apply;
  const int32_t* src;
};

Path pick_path(const hm_matrix* h, bool f32, int nrhs) {
  // the matrix-core kernels index the row-layout vectors with 32-bit offsets
  const bool fits = (h->N + h->T + 1) * row_ld(nrhs) * (int64_t)sizeof(double2) < ((int64_t)1 << 32);
  if (nrhs >= h->mm_min_rhs && fits)
    return Path{true, f32 ? (const void*)h->Wmm32 : (const void*)h->Wmm64, h->groups_mm,
                &h->sa_mm, &h->tl_series_mm, &h->tl_apply_mm, h->src_mm};
  return Path{false, f32 ? (const void*)h->W32 : (const void*)h->W64, h->groups, &h->sa,
              &h->tl_series, &h->tl_apply, h->src};
}

hipError_t run_term(const hm_matrix* h, const Path& P, bool f32, const TermArgs& t,
                    const TermList& tl, int nrhs, hipStream_t st) {
  return P.mm ? launch_term_mm(f32, h->max_m, t, tl.nwg, nrhs, h->rhs_tile, st)
              : launch_term(f32, h->max_m, t, tl.nwg, nrhs, st);
}

// Stage A: streaming kernels on [y | t] in column layout (xin, ld ldx), the
// matrix-core ones on the row-layout vectors (xr64 or xr32, ld ws_ldr).
hipError_t run_stageA(const hm_matrix* h, const Path& P, bool f32, const GroupList& sa,
                      double2* xin, int64_t ldx, double2* xr64, float2* xr32, int nrhs,
                      hipStream_t st) {
  return P.mm ? launch_stageA_mm(f32, P.W, P.groups, sa.items, sa.n, xr64, xr32, h->ws_ldr, h->N,
                                 (int)(h->N + h->T), nrhs, h->rhs_tile, st)
              : launch_stageA(f32, P.W, P.groups, sa.items, sa.n, xin, ldx, h->N, nrhs, st);
}

// The half-storage series serves one right-hand side of a symmetric
// problem, when the tuning allows it.
bool use_half(const hm_matrix* h, int li, int nrhs) {
  return nrhs == 1 && nrhs < h->mm_min_rhs && (h->use_half == 1 || h->use_half == 3) && h->half_ok &&
         li < (int)h->half.size();
}

// One scaled term product at level li: input yhat = [y | t] (tree order).
HalfArgs half_args(const hm_matrix* h, int li, bool f32, const double2* xin, int64_t ldx) {
  const hm_matrix::HalfList& L = h->half[li];
  HalfArgs a{};
  a.t = term_args(h, PanelSet{f32 ? (const void*)h->HF32 : (const void*)h->HF64, h->hf_off, h->src,
                              h->hf_col, h->leaf_m},
                  L.tl, f32, xin, ldx);
  a.t.ir = InRow{f32 ? (const void*)h->IRT32 : (const void*)h->IRT64, h->hir_off, h->hir_ld,
                 h->hir_ncol, h->hir_row0, h->hir_soff, h->hir_n};
  a.hp = f32 ? (const void*)h->H32 : (const void*)h->H64;
  a.hp_off = h->hp_off;
  a.hp_col = h->hp_col;
  a.hsrc = h->hsrc;
  a.vrow = L.tl.vrow;
  a.lcnt = L.lcnt;
  a.vleaf = L.vleaf;
  a.npieces = L.tl.npieces;
  a.queue = h->hq;
  a.fp = f32 ? (const void*)h->FP32 : (const void*)h->FP64;
  a.fp_off = h->fp_off;
  a.fp_rank = h->fp_rank;
  a.fp_slot = h->fp_slot;
  a.frow = L.tl.frow;
  return a;
}

// Block-diagonal product with the C_a^{-1} (or C_a^{-T}) panels.
PanelSet chat_set(const hm_matrix* h, bool transposed) {
  return PanelSet{transposed ? (const void*)h->CHT : (const void*)h->CH, h->ch_off, h->src,
                  h->R_col, h->leaf_m};
}

// Block-diagonal product with the C_a (or C_a^T) panels.
PanelSet cf_set(const hm_matrix* h, bool transposed) {
  return PanelSet{transposed ? (const void*)h->CFT : (const void*)h->CF, h->ch_off, h->src,
                  h->R_col, h->leaf_m};
}

// One right-hand side through block-diagonal panels: one workgroup per leaf
// where the leaves fit it, else the term kernel on the D^{-1} work list.
hipError_t block_launch(const hm_matrix* h, const TermArgs& t, hipStream_t st) {
  if (h->max_m <= kBlockDiagMaxLeaf) return launch_block_diag(t, h->nl, h->max_m, st);
  return launch_term(false, h->max_m, t, h->tl_dinv.nwg, 1, st);
}

// Block-diagonal launch (C^{-1}, C^{-T} or D^{-1} panels, one right-hand
// side): y = M in per leaf, then the TermArgs stores (yout, xacc, out).
hipError_t block_pass(hm_matrix* h, const PanelSet& ps, const double2* in, int64_t ldi,
                      bool perm_in, double2* yout, int64_t ldy, double2* xacc, int accumulate,
                      double2* out, int64_t ldo, hipStream_t st) {
  TermArgs t = term_args(h, ps, h->tl_dinv, false, in, ldi);
  t.in_perm = perm_in ? h->perm : nullptr;
  t.yout = yout;
  t.ldy = ldy;
  t.xacc = xacc;
  t.ldxa = h->N;
  t.accumulate = accumulate;
  if (out) { t.out = out; t.ldo = ldo; t.out_perm = h->perm; }
  return block_launch(h, t, st);
}

// K terms of the scaled series from yhat_0 in xin0 ([y | t], tree order):
// yhat_k = -S yhat_{k-1}, each added to xh (tree order); *last receives the
// buffer holding yhat_K.
int scaled_terms(hm_matrix* h, int li, bool f32, int K, double2* xh, double2** last,
                 hipStream_t st) {
  const int64_t N = h->N, ldin = h->N + h->T;
  double2* y_cur = h->xin0;
  double2* y_nxt = h->xin1;
  if (K > 0 && h->use_half == 1 && h->half[li].multi) {
    // all K terms in one launch (pieces gated by per-leaf term marks)
    HalfArgs ha = half_args(h, li, f32, y_cur, ldin);
    ha.t.alpha = -1.0;
    const MultiArgs m{K, h->nl, {y_cur, y_nxt}, xh, h->hdone, h->herr};
    // a resident round of the multi-term kernel (pieces come from its queue,
    // so the count need not match the list's)
    const int nwg = h->half[li].tl.nwg == h->half_wgs_auto ? h->half_wgs_multi : h->half[li].tl.nwg;
    TIMED(HM_K_TERM_SERIES, launch_half_multi(f32, h->max_m, ha, m, nwg, st));
    *last = (K & 1) ? y_nxt : y_cur;
    return HM_OK;
  }
  const GroupList& sa1 = h->sa[li];  // the one-RHS stage-A groups (global far only)
  const void* W1 = f32 ? (const void*)h->WT32 : (const void*)h->WT64;
  for (int k = 1; k <= K; ++k) {
    if (sa1.n > 0)
      TIMED(HM_K_STAGEA, launch_stageA(f32, W1, h->groups, sa1.items, sa1.n, y_cur, ldin, N, 1, st));
    HalfArgs ha = half_args(h, li, f32, y_cur, ldin);
    ha.t.alpha = -1.0;
    ha.t.yout = y_nxt;
    ha.t.ldy = ldin;
    ha.t.xacc = xh;
    ha.t.ldxa = N;
    ha.t.accumulate = 1;
    TIMED(HM_K_TERM_SERIES, launch_half(f32, h->max_m, ha, h->half[li].tl.nwg, st));
    std::swap(y_cur, y_nxt);
  }
  *last = y_cur;
  return HM_OK;
}

// Refinement in the scaled basis (one right-hand side of a symmetric
// problem): with xhat = C^T x and bhat = C^{-1} b the residual is
// rhat = C^{-1} (b - Z x) = (bhat - xhat) - S xhat, which is yhat_0 of the
// correction's series, so a pass is one FP64 product with S (w = bhat - xhat
// kept up to date) and K terms, and no H-matvec or block-diagonal step.
// Work vectors: xhat in zbuf, w in bt, dhat in dt.
int scaled_refine_init(hm_matrix* h, int li, bool f32, int K, bool want_norms, hipStream_t st) {
  const int64_t N = h->N, ldin = h->N + h->T;
  // yhat_0 = bhat (xin0), and a copy in rt
  HIPCHK(block_pass(h, chat_set(h, false), h->bt, N, false, h->xin0, ldin, h->rt, 0, nullptr, 0, st));
  if (want_norms) {  // ||y_0||, y_0 = D^{-1} b
    HIPCHK(block_pass(h, dinv_set(h), h->bt, N, false, h->xin1, ldin, nullptr, 0, nullptr, 0, st));
    HIPCHK(norms_into(h, h->xin1, ldin, 1, 0, st));
  }
  HIPCHK(launch_axpy(1.0, h->rt, N, h->zbuf, N, N, 1, 0, st));
  double2* last = nullptr;
  STCHK(scaled_terms(h, li, f32, K, h->zbuf, &last, st));
  if (want_norms) {  // ||y_K||, y_K = C^{-T} yhat_K
    double2* tmp = last == h->xin0 ? h->xin1 : h->xin0;
    HIPCHK(block_pass(h, chat_set(h, true), last, ldin, false, tmp, ldin, nullptr, 0, nullptr, 0, st));
    HIPCHK(norms_into(h, tmp, ldin, 1, 1, st));
  }
  // w = bhat - xhat
  HIPCHK(launch_axpy(1.0, h->rt, N, h->bt, N, N, 1, 0, st));
  HIPCHK(launch_axpy(-1.0, h->zbuf, N, h->bt, N, N, 1, 1, st));
  return HM_OK;
}

// One refinement pass; with `check`, x = C^{-T} xhat lands in xt and the
// correction d = C^{-T} dhat in rt for the norms.
int scaled_refine_pass(hm_matrix* h, int li, bool f32, int K, bool check, hipStream_t st) {
  const int64_t N = h->N, ldin = h->N + h->T;
  // rhat = w - S xhat in FP64, written as yhat_0 (xin0) and as dhat's first term
  HIPCHK(launch_axpy(1.0, h->zbuf, N, h->xin1, ldin, N, 1, 0, st));
  const GroupList& sa1 = h->sa[li];
  if (sa1.n > 0)
    TIMED(HM_K_STAGEA, launch_stageA(false, h->WT64, h->groups, sa1.items, sa1.n, h->xin1, ldin, N, 1, st));
  HalfArgs ha = half_args(h, li, false, h->xin1, ldin);
  ha.t.alpha = -1.0;
  ha.t.beta = 1.0;
  ha.t.v = h->bt;
  ha.t.ldv = N;
  ha.t.yout = h->xin0;
  ha.t.ldy = ldin;
  ha.t.xacc = h->dt;
  ha.t.ldxa = N;
  ha.t.accumulate = 0;
  TIMED(HM_K_TERM_APPLY, launch_half(false, h->max_m, ha, h->half[li].tl.nwg, st));
  double2* last = nullptr;
  STCHK(scaled_terms(h, li, f32, K, h->dt, &last, st));
  // xhat += dhat, w -= dhat
  HIPCHK(launch_axpy(1.0, h->dt, N, h->zbuf, N, N, 1, 1, st));
  HIPCHK(launch_axpy(-1.0, h->dt, N, h->bt, N, N, 1, 1, st));
  if (check) {
    HIPCHK(block_pass(h, chat_set(h, true), h->zbuf, N, false, nullptr, 0, h->xt, 0, nullptr, 0, st));
    HIPCHK(block_pass(h, chat_set(h, true), h->dt, N, false, nullptr, 0, h->rt, 0, nullptr, 0, st));
  }
  return HM_OK;
}

// whether the many-RHS series at level li runs as one multi-term launch
bool mm_multi_ok(const hm_matrix* h, int li, int K, int nrhs) {
  return h->mm_multi_mode == 1 && h->mm_cnt && li < (int)h->mm_multi.size() && h->mm_multi[li].ok &&
         K <= kMmSeriesMaxTerms && nrhs <= 32 && mm_wave_mode(h->max_m);
}

int series_core(hm_matrix* h, int li, bool f32, int K, const double2* rhs, int64_t ldr,
                bool rhs_perm, double2* x_tree, double2* out, int64_t ldo, int nrhs,
                bool want_norms, hipStream_t st, bool allow_half = true) {
  const int64_t N = h->N, ldin = h->N + h->T;
  double2* y_cur = h->xin0;
  double2* y_nxt = h->xin1;
  if (allow_half && use_half(h, li, nrhs)) {
    // scaled series (see build_half): yhat_0 = C^{-1} b, yhat_k =
    // -S yhat_{k-1} with the half-storage product, x = C^{-T} sum_k yhat_k
    double2* xh = h->zbuf;
    auto block_diag = [&](const PanelSet& ps, const double2* in, int64_t ldi, bool perm_in,
                          double2* yout, int64_t ldy, double2* xacc, double2* o) -> hipError_t {
      TermArgs t = term_args(h, ps, h->tl_dinv, false, in, ldi);
      t.in_perm = perm_in ? h->perm : nullptr;
      t.yout = yout;
      t.ldy = ldy;
      t.xacc = xacc;
      t.ldxa = N;
      t.accumulate = 0;
      if (o) { t.out = o; t.ldo = ldo; t.out_perm = h->perm; }
      return block_launch(h, t, st);
    };
    TIMED(HM_K_TERM_DINV, block_diag(chat_set(h, false), rhs, ldr, rhs_perm, y_cur, ldin, xh, nullptr));
    if (want_norms) {  // ||y_0||, y_0 = D^{-1} b
      HIPCHK(block_diag(dinv_set(h), rhs, ldr, rhs_perm, y_nxt, ldin, nullptr, nullptr));
      HIPCHK(norms_into(h, y_nxt, ldin, nrhs, 0, st));
    }
    STCHK(scaled_terms(h, li, f32, K, xh, &y_cur, st));
    y_nxt = y_cur == h->xin0 ? h->xin1 : h->xin0;
    if (want_norms) {  // ||y_K||, y_K = C^{-T} yhat_K
      HIPCHK(block_diag(chat_set(h, true), y_cur, ldin, false, y_nxt, ldin, nullptr, nullptr));
      HIPCHK(norms_into(h, y_nxt, ldin, nrhs, 1, st));
    }
    TIMED(HM_K_TERM_DINV, block_diag(chat_set(h, true), xh, N, false, nullptr, 0, x_tree, out));
    return HM_OK;
  }
  const Path P = pick_path(h, f32, nrhs);
  const TermList& tl = (*P.tl_series)[li];
  const GroupList& sa = (*P.sa)[li];
  if (P.mm) {
    // matrix cores: [y | t] in row layout, FP64 (r64) or FP32 (r32) by the
    // block precision; the column-layout y is written only for the norms
    double2* r64[2] = {h->xr64_0, h->xr64_1};
    float2* r32[2] = {h->xr32_0, h->xr32_1};
    HIPCHK(launch_rows(rhs, ldr, rhs_perm ? h->perm : nullptr, N, nrhs, r64[1], nullptr, h->ws_ldr,
                       st));
    {
      TermArgs t = term_args(h, dinv_set(h), h->tl_dinv_mm, false, nullptr, 0);
      t.xr = r64[1];
      t.yrow = f32 ? nullptr : r64[0];
      t.yrow32 = f32 ? r32[0] : nullptr;
      t.yout = want_norms ? y_cur : nullptr;
      t.ldy = ldin;
      t.xacc = x_tree;
      t.ldxa = N;
      t.accumulate = 0;
      if (K == 0 && out) { t.out = out; t.ldo = ldo; t.out_perm = h->perm; }
      TIMED(HM_K_TERM_DINV, run_term(h, P, false, t, h->tl_dinv_mm, nrhs, st));
    }
    if (want_norms) HIPCHK(norms_into(h, y_cur, ldin, nrhs, 0, st));
    if (K >= 1 && mm_multi_ok(h, li, K, nrhs)) {
      // the K terms in one launch (stage A included)
      const hm_matrix::MMMulti& mmm = h->mm_multi[li];
      TermArgs t = term_args(h, series_set(h, f32, P.src), tl, f32, nullptr, 0);
      t.xr = r64[0];
      t.xr32 = r32[0];
      t.alpha = -1.0;
      t.xacc = x_tree;
      t.ldxa = N;
      t.accumulate = 1;
      MMSeriesArgs s{};
      s.K = K;
      s.n_a = mmm.n_a;
      s.n_b = mmm.n_b;
      s.items = mmm.items;
      s.groups = P.groups;
      s.W = P.W;
      s.r64[0] = r64[0];
      s.r64[1] = r64[1];
      s.r32[0] = r32[0];
      s.r32[1] = r32[1];
      s.N = N;
      s.cnt = h->mm_cnt;
      s.kmax = kMmSeriesMaxTerms;
      s.need_a = mmm.need_a;
      s.need_b = mmm.need_b;
      s.ninst = (int)h->inst_off.size() - 1;
      s.queue = h->mm_queue;
      s.err = h->mm_err;
      s.yout = want_norms ? y_nxt : nullptr;
      s.ldy = ldin;
      s.out = out;
      s.ldo = ldo;
      s.out_perm = h->perm;
      TIMED(HM_K_TERM_SERIES, launch_series_mm(f32, t, s, h->mm_series_wgs[f32][nrhs > 16], nrhs, st));
      std::swap(y_cur, y_nxt);
      if (want_norms) HIPCHK(norms_into(h, y_cur, ldin, nrhs, 1, st));
      return HM_OK;
    }
    int cur = 0;
    for (int k = 1; k <= K; ++k) {
      if (sa.n > 0)
        TIMED(HM_K_STAGEA, run_stageA(h, P, f32, sa, nullptr, 0, r64[cur], r32[cur], nrhs, st));
      TermArgs t = term_args(h, series_set(h, f32, P.src), tl, f32, nullptr, 0);
      t.xr = r64[cur];
      t.xr32 = r32[cur];
      t.alpha = -1.0;
      t.yrow = f32 ? nullptr : r64[cur ^ 1];
      t.yrow32 = f32 ? r32[cur ^ 1] : nullptr;
      t.yout = (want_norms && k == K) ? y_nxt : nullptr;
      t.ldy = ldin;
      t.xacc = x_tree;
      t.ldxa = N;
      t.accumulate = 1;
      if (k == K && out) { t.out = out; t.ldo = ldo; t.out_perm = h->perm; }
      TIMED(HM_K_TERM_SERIES, run_term(h, P, f32, t, tl, nrhs, st));
      cur ^= 1;
      if (k == K) std::swap(y_cur, y_nxt);
    }
    if (want_norms) HIPCHK(norms_into(h, y_cur, ldin, nrhs, 1, st));
    return HM_OK;
  }
  {
    TermArgs t = term_args(h, dinv_set(h), h->tl_dinv, false, rhs, ldr);
    t.in_perm = rhs_perm ? h->perm : nullptr;
    t.yout = y_cur;
    t.ldy = ldin;
    t.xacc = x_tree;
    t.ldxa = N;
    t.accumulate = 0;
    if (K == 0 && out) { t.out = out; t.ldo = ldo; t.out_perm = h->perm; }
    TIMED(HM_K_TERM_DINV, run_term(h, P, false, t, h->tl_dinv, nrhs, st));
  }
  if (want_norms) HIPCHK(norms_into(h, y_cur, ldin, nrhs, 0, st));
  for (int k = 1; k <= K; ++k) {
    if (sa.n > 0)
      TIMED(HM_K_STAGEA, run_stageA(h, P, f32, sa, y_cur, ldin, nullptr, nullptr, nrhs, st));
    TermArgs t = term_args(h, series_set(h, f32, P.src), tl, f32, y_cur, ldin);
    t.alpha = -1.0;
    t.yout = y_nxt;
    t.ldy = ldin;
    t.xacc = x_tree;
    t.ldxa = N;
    t.accumulate = 1;
    if (k == K && out) { t.out = out; t.ldo = ldo; t.out_perm = h->perm; }
    TIMED(HM_K_TERM_SERIES, run_term(h, P, f32, t, tl, nrhs, st));
    std::swap(y_cur, y_nxt);
  }
  if (want_norms) HIPCHK(norms_into(h, y_cur, ldin, nrhs, 1, st));
  return HM_OK;
}

// alpha * Z_l x + beta * v (v tree order, ld N) from x in xin0 (tree order),
// into out_tree (tree order, ld N) and/or out (original order, ld ldo).
int apply_core(hm_matrix* h, int li, bool f32, int nrhs, double alpha, double beta,
               const double2* v, double2* out_tree, double2* out, int64_t ldo, hipStream_t st) {
  const int64_t N = h->N, ldin = h->N + h->T;
  if (use_half(h, li, nrhs)) {
    // half storage (symmetric problems, one right-hand side): with
    // D = C C^T and S = C^{-1} R C^{-T}, Z x = C (xhat + S xhat) for
    // xhat = C^T x, so the product reads S once (near blocks s > t and far
    // pairs once) plus the two block-diagonal factors
    TermArgs t0 = term_args(h, cf_set(h, true), h->tl_dinv, false, h->xin0, ldin);
    t0.yout = h->xin1;  // xhat (tree order, with the t rows of stage A after N)
    t0.ldy = ldin;
    HIPCHK(block_launch(h, t0, st));
    const GroupList& sa1 = h->sa[li];
    if (sa1.n > 0)
      TIMED(HM_K_STAGEA, launch_stageA(f32, f32 ? (const void*)h->WT32 : (const void*)h->WT64,
                                       h->groups, sa1.items, sa1.n, h->xin1, ldin, N, 1, st));
    HalfArgs ha = half_args(h, li, f32, h->xin1, ldin);
    ha.t.alpha = 1.0;
    ha.t.beta = 1.0;
    ha.t.v = h->xin1;
    ha.t.ldv = ldin;
    ha.t.yout = h->hwork;
    ha.t.ldy = N;
    TIMED(HM_K_TERM_APPLY, launch_half(f32, h->max_m, ha, h->half[li].tl.nwg, st));
    TermArgs t1 = term_args(h, cf_set(h, false), h->tl_dinv, false, h->hwork, N);
    t1.alpha = alpha;
    t1.beta = beta;
    t1.v = v;
    t1.ldv = N;
    t1.yout = out_tree;
    t1.ldy = N;
    if (out) { t1.out = out; t1.ldo = ldo; t1.out_perm = h->perm; }
    HIPCHK(block_launch(h, t1, st));
    return HM_OK;
  }
  const Path P = pick_path(h, f32, nrhs);
  // matrix cores: x into row layout, FP64 or FP32 by the block precision
  double2* r64 = (P.mm && !f32) ? h->xr64_0 : nullptr;
  float2* r32 = (P.mm && f32) ? h->xr32_0 : nullptr;
  if (P.mm) HIPCHK(launch_rows(h->xin0, ldin, nullptr, N, nrhs, r64, r32, h->ws_ldr, st));
  const GroupList& sa = (*P.sa)[li];
  if (sa.n > 0) TIMED(HM_K_STAGEA, run_stageA(h, P, f32, sa, h->xin0, ldin, r64, r32, nrhs, st));
  const TermList& tl = (*P.tl_apply)[li];
  TermArgs t = term_args(h, apply_set(h, f32, P.src), tl, f32, h->xin0, ldin);
  t.xr = r64;
  t.xr32 = r32;
  t.alpha = alpha;
  t.beta = beta;
  t.v = v;
  t.ldv = N;
  t.yout = out_tree;
  t.ldy = N;
  if (out) { t.out = out; t.ldo = ldo; t.out_perm = h->perm; }
  TIMED(HM_K_TERM_APPLY, run_term(h, P, f32, t, tl, nrhs, st));
  return HM_OK;
}

// GMRES workspace for restart length m and nrhs columns (kept on the
// handle, grown when a call needs more).
constexpr int kDefaultRestart = 30;  // GMRES basis vectors per cycle unless given

// bytes of the GMRES workspace for m and nrhs (as ensure_gmres allocates it)
int64_t gmres_bytes(int64_t N, int m, int nrhs) {
  if (m <= 0 || nrhs <= 0) return 0;
  const int64_t c2 = sizeof(double2), vs = N * nrhs;
  return c2 * (vs * (2 * m + 1) + kdots_partials(N, m + 1, nrhs) + 2 * (m + 1) * nrhs + 2 * nrhs +
               m * nrhs + (int64_t)(m + 1) * m * nrhs + m * nrhs + (m + 1) * nrhs) +
         (int64_t)sizeof(double) * (m * nrhs + 3 * nrhs) + 2 * sizeof(int32_t) * nrhs;
}

int ensure_gmres(hm_matrix* h, int m, int nrhs) {
  if (m <= h->gm_m && nrhs <= h->gm_nrhs) return HM_OK;
  m = std::max(m, h->gm_m);
  nrhs = std::max(nrhs, h->gm_nrhs);
  for (void* p : h->gm_allocs) (void)hipFree(p);
  h->gm_allocs.clear();
  if (h->gm_host) (void)hipHostFree(h->gm_host);
  h->gm_host = nullptr;
  h->gm_m = h->gm_nrhs = 0;
  const int64_t N = h->N, vs = N * nrhs;
  auto al = [&](void** p, size_t bytes) -> int {
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("GMRES workspace hipMalloc failed: " + std::string(hipGetErrorString(e)));
      return HM_ENOMEM;
    }
    h->gm_allocs.push_back(*p);
    return HM_OK;
  };
  const size_t c2 = sizeof(double2);
  STCHK(al((void**)&h->gm_V, c2 * vs * (m + 1)));
  STCHK(al((void**)&h->gm_Z, c2 * vs * m));
  STCHK(al((void**)&h->gm_part, c2 * kdots_partials(N, m + 1, nrhs)));
  STCHK(al((void**)&h->gm_h1, c2 * (m + 1) * nrhs));
  STCHK(al((void**)&h->gm_h2, c2 * (m + 1) * nrhs));
  STCHK(al((void**)&h->gm_hn, c2 * nrhs));
  STCHK(al((void**)&h->gm_bn, c2 * nrhs));
  STCHK(al((void**)&h->gm_y, c2 * m * nrhs));
  KrylovState& S = h->gm_S;
  STCHK(al((void**)&S.R, c2 * (int64_t)(m + 1) * m * nrhs));
  STCHK(al((void**)&S.cs, sizeof(double) * m * nrhs));
  STCHK(al((void**)&S.sn, c2 * m * nrhs));
  STCHK(al((void**)&S.g, c2 * (m + 1) * nrhs));
  STCHK(al((void**)&S.act, sizeof(int32_t) * nrhs));
  STCHK(al((void**)&S.kc, sizeof(int32_t) * nrhs));
  STCHK(al((void**)&S.resid, sizeof(double) * nrhs));
  STCHK(al((void**)&S.bnorm, sizeof(double) * nrhs));
  STCHK(al((void**)&S.inv, sizeof(double) * nrhs));
  HIPCHK(hipHostMalloc((void**)&h->gm_host, sizeof(double) * 2 * nrhs, hipHostMallocDefault));
  h->gm_m = m;
  h->gm_nrhs = nrhs;
  return HM_OK;
}

// Restarted GMRES on Z_l x = b with the series as right preconditioner
// (flexible form: x = x_0 + sum_j (P_K v_j) y_j), FP64 products with Z_l,
// Gram-Schmidt with one reorthogonalisation pass.  b is read in original
// order (ld ldb), x written in original order (ld ldx).  Each column runs
// until its residual estimate is below tol and the true residual of the
// cycle's end confirms it, or the iteration budget is spent.  iters[c] =
// Arnoldi steps in which column c was active; rel[c] = true final
// ||b - Z_l x|| / ||b||.  On a batched handle each column is one Krylov
// space over every instance and ||b|| is the smallest nonzero ||b_i|| of
// the column (every instance then meets the tolerance on its own b).
//
// One right-hand side of a symmetric single-instance problem iterates in the
// scaled basis
// of the half-storage series instead: (I + S) xhat = bhat with
// bhat = C^{-1} b and x = C^{-T} xhat, preconditioned by sum_k (-S)^k (the
// same series, K terms), so every product is one half-storage launch and
// no block-diagonal step runs inside a cycle.  Its Arnoldi estimates are
// scaled residuals, checked against tol / 4; the stopping test is the true
// ||b - Z_l x|| at each cycle's end (the scaled target tightens if the two
// disagree).
int gmres_solve(hm_matrix* h, int li, bool f32, int K, int m, int max_iter, double tol,
                const double2* b_dev, int64_t ldb, double2* x_dev, int64_t ldx, int nrhs,
                std::vector<int>& iters, std::vector<double>& rel, hipStream_t st) {
  const int64_t N = h->N, ldin = h->N + h->T, vs = N * nrhs;
  STCHK(ensure_gmres(h, m, nrhs));
  KrylovState S = h->gm_S;
  S.m = m;
  double2* V = h->gm_V;
  double2* Zb = h->gm_Z;
  double* hres = h->gm_host;               // nrhs residuals
  double* hact = h->gm_host + nrhs;         // nrhs flags (as doubles)
  const bool scaled = use_half(h, li, nrhs) && h->nseg == 1;
  const GroupList& sa1 = h->sa[li];
  auto dots = [&](const double2* Vb, int nvec, const double2* w, double2* out, int ldo) {
    return launch_kdots(Vb, vs, N, w, N, nvec, nrhs, h->gm_part, out, ldo, st);
  };
  // scaled basis: out = alpha S in + beta v (FP64 half-storage product)
  auto s_apply = [&](const double2* in, double alpha, double beta, const double2* v,
                     double2* out) -> int {
    HIPCHK(launch_axpy(1.0, in, N, h->xin1, ldin, N, 1, 0, st));
    if (sa1.n > 0)
      TIMED(HM_K_STAGEA, launch_stageA(false, h->WT64, h->groups, sa1.items, sa1.n, h->xin1, ldin, N, 1, st));
    HalfArgs ha = half_args(h, li, false, h->xin1, ldin);
    ha.t.alpha = alpha;
    ha.t.beta = beta;
    ha.t.v = v;
    ha.t.ldv = N;
    ha.t.xacc = out;
    ha.t.ldxa = N;
    ha.t.accumulate = 0;
    TIMED(HM_K_TERM_APPLY, launch_half(false, h->max_m, ha, h->half[li].tl.nwg, st));
    return HM_OK;
  };
  // z = P v
  auto precond = [&](const double2* v, double2* z) -> int {
    if (!scaled) return series_core(h, li, f32, K, v, N, false, z, nullptr, 0, nrhs, false, st);
    HIPCHK(launch_axpy(1.0, v, N, h->xin0, ldin, N, 1, 0, st));
    HIPCHK(launch_axpy(1.0, v, N, z, N, N, 1, 0, st));
    double2* last = nullptr;
    return scaled_terms(h, li, f32, K, z, &last, st);
  };
  // w = A z (A = Z_l, or I + S in the scaled basis)
  auto oper = [&](const double2* z, double2* w) -> int {
    if (scaled) return s_apply(z, 1.0, 1.0, z, w);
    HIPCHK(launch_axpy(1.0, z, N, h->xin0, ldin, N, nrhs, 0, st));
    return apply_core(h, li, false, nrhs, 1.0, 0.0, nullptr, w, nullptr, 0, st);
  };
  iters.assign(nrhs, 0);
  rel.assign(nrhs, 0.0);
  std::vector<int> active(nrhs, 0);
  std::vector<double> rel_true(nrhs, 1.0);
  double bn_true = 0.0;
  auto read_state = [&](bool flags) -> int {
    HIPCHK(hipMemcpyAsync(hres, S.resid, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    if (flags) {
      // the int flags land in the second half of the pinned buffer
      HIPCHK(hipMemcpyAsync(hact, S.act, sizeof(int32_t) * nrhs, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    if (flags) {
      const int32_t* f = reinterpret_cast<const int32_t*>(hact);
      for (int c = 0; c < nrhs; ++c) active[c] = f[c];
    }
    return HM_OK;
  };
  // ||v||^2 of the single column of v, read to the host
  auto host_norm2 = [&](const double2* v, double* out) -> int {
    HIPCHK(dots(v, 1, v, h->gm_hn, 1));
    HIPCHK(hipMemcpyAsync(hres, h->gm_hn, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *out = hres[0];
    return HM_OK;
  };
  if (scaled) {
    // b in tree order (dt), bhat = C^{-1} b (bt); xhat = 0 in xt
    HIPCHK(launch_permute_in(b_dev, ldb, h->perm, h->dt, N, N, 1, st));
    HIPCHK(block_pass(h, chat_set(h, false), h->dt, N, false, nullptr, 0, h->bt, 0, nullptr, 0, st));
    double bn2 = 0.0;
    STCHK(host_norm2(h->dt, &bn2));
    bn_true = bn2 > 0.0 ? std::sqrt(bn2) : (bn2 <= 0.0 ? 0.0 : bn2);  // NaN stays NaN
    rel_true[0] = bn_true > 0 ? 1.0 : (bn_true == 0.0 ? 0.0 : NAN);
    HIPCHK(dots(h->bt, 1, h->bt, h->gm_bn, 1));  // ||bhat||^2 for the scaled estimates
  } else {
    // b in tree order, ||b||^2; x = 0; the first residual is b
    HIPCHK(launch_permute_in(b_dev, ldb, h->perm, h->bt, N, N, nrhs, st));
    HIPCHK(dots(h->bt, 1, h->bt, h->gm_bn, 1));
    HIPCHK(launch_axpy(1.0, h->bt, N, V, N, N, nrhs, 0, st));
    if (h->nseg > 1) {
      // batched instances: one Krylov space per column over all of them,
      // measured against the smallest nonzero ||b_i|| of the column, so that
      // every instance's residual (at most the column's) meets the tolerance
      // relative to its own right-hand side.  A NaN norm stays NaN.
      HIPCHK(norms_into(h, h->bt, N, nrhs, 0, st));
      HIPCHK(hipMemcpyAsync(h->norms_host, h->norms, sizeof(double) * h->nseg * nrhs,
                            hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      std::vector<double2> bmin(nrhs);
      for (int c = 0; c < nrhs; ++c) {
        double mn = INFINITY;
        for (int g = 0; g < h->nseg; ++g) {
          const double v = h->norms_host[(int64_t)c * h->nseg + g];
          if (std::isnan(v) || std::isnan(mn)) mn = NAN;
          else if (v > 0.0 && v < mn) mn = v;
        }
        bmin[c] = make_double2(std::isinf(mn) ? 0.0 : mn, 0.0);  // all zero: b = 0
      }
      HIPCHK(hipMemcpyAsync(h->gm_bn, bmin.data(), sizeof(double2) * nrhs, hipMemcpyHostToDevice,
                            st));
      HIPCHK(hipStreamSynchronize(st));  // bmin is pageable host memory
    }
  }
  HIPCHK(hipMemsetAsync(h->xt, 0, sizeof(double2) * vs, st));
  double tol_s = scaled ? 0.25 * tol : tol;
  int tighten = 0, done_iters = 0;
  while (true) {
    if (scaled) {
      if (rel_true[0] <= tol) break;
      // rhat = (bhat - xhat) - S xhat into V_0
      HIPCHK(launch_axpy(1.0, h->bt, N, h->rt, N, N, 1, 0, st));
      HIPCHK(launch_axpy(-1.0, h->xt, N, h->rt, N, N, 1, 1, st));
      STCHK(s_apply(h->xt, -1.0, 1.0, h->rt, V));
    }
    // V_0 holds the residual r: ||r||, g = ||r|| e_1, V_0 = r / ||r||
    HIPCHK(dots(V, 1, V, h->gm_hn, 1));
    HIPCHK(launch_kstart(S, h->gm_hn, h->gm_bn, tol_s, nrhs, st));
    HIPCHK(launch_kscale(V, N, S.inv, N, nrhs, st));
    STCHK(read_state(true));
    if (!scaled)
      for (int c = 0; c < nrhs; ++c) rel[c] = hres[c];
    bool any = false;
    for (int c = 0; c < nrhs; ++c) any = any || active[c];
    if (scaled && !any && done_iters < max_iter && tighten < 3) {
      // the scaled residual is below its target but the true one is not
      tol_s *= 0.1;
      ++tighten;
      continue;
    }
    if (!any || done_iters >= max_iter) break;
    int j = 0;
    for (; j < m && done_iters < max_iter; ++j) {
      double2* vj = V + (int64_t)j * vs;
      double2* w = V + (int64_t)(j + 1) * vs;
      double2* zj = Zb + (int64_t)j * vs;
      // z_j = P v_j; w = A z_j
      STCHK(precond(vj, zj));
      STCHK(oper(zj, w));
      // two classical Gram-Schmidt passes against v_0 .. v_j
      HIPCHK(dots(V, j + 1, w, h->gm_h1, m + 1));
      HIPCHK(launch_kupdate(-1.0, V, vs, N, h->gm_h1, m + 1, j + 1, w, N, nrhs, st));
      HIPCHK(dots(V, j + 1, w, h->gm_h2, m + 1));
      HIPCHK(launch_kupdate(-1.0, V, vs, N, h->gm_h2, m + 1, j + 1, w, N, nrhs, st));
      HIPCHK(dots(w, 1, w, h->gm_hn, 1));
      HIPCHK(launch_kstep(S, j, h->gm_h1, h->gm_h2, m + 1, h->gm_hn, tol_s, nrhs, st));
      HIPCHK(launch_kscale(w, N, S.inv, N, nrhs, st));
      for (int c = 0; c < nrhs; ++c) iters[c] += active[c];
      ++done_iters;
      STCHK(read_state(true));
      bool more = false;
      for (int c = 0; c < nrhs; ++c) more = more || active[c];
      if (!more) {
        ++j;
        break;
      }
    }
    // x += sum_i z_i y_i over the steps of this cycle
    HIPCHK(launch_ksolve(S, h->gm_y, nrhs, st));
    HIPCHK(launch_kupdate(1.0, Zb, vs, N, h->gm_y, m, j, h->xt, N, nrhs, st));
    if (scaled) {
      // true residual: x = C^{-T} xhat (zbuf), r = b - Z_l x (rt)
      HIPCHK(block_pass(h, chat_set(h, true), h->xt, N, false, nullptr, 0, h->zbuf, 0, nullptr, 0, st));
      HIPCHK(launch_axpy(1.0, h->zbuf, N, h->xin0, ldin, N, 1, 0, st));
      STCHK(apply_core(h, li, false, 1, -1.0, 1.0, h->dt, h->rt, nullptr, 0, st));
      double rn2 = 0.0;
      STCHK(host_norm2(h->rt, &rn2));
      rel_true[0] = bn_true > 0 ? (rn2 >= 0.0 ? std::sqrt(rn2) : NAN) / bn_true : 0.0;
      if (!(rel_true[0] == rel_true[0])) break;  // not finite: stop, reported as such
    } else {
      // true residual r = b - Z x into V_0 (it starts the next cycle)
      HIPCHK(launch_axpy(1.0, h->xt, N, h->xin0, ldin, N, nrhs, 0, st));
      STCHK(apply_core(h, li, false, nrhs, -1.0, 1.0, h->bt, V, nullptr, 0, st));
    }
  }
  if (scaled) {
    rel[0] = rel_true[0];
    HIPCHK(block_pass(h, chat_set(h, true), h->xt, N, false, nullptr, 0, h->zbuf, 0, x_dev, ldx,
                      st));
  } else {
    HIPCHK(launch_permute_out(h->xt, N, h->perm, x_dev, ldx, N, nrhs, st));
  }
  return HM_OK;
}

// out = D^{-1} in + beta v (tree order, ld N; v may be null when beta = 0)
hipError_t dinv_pass(hm_matrix* h, const double2* in, const double2* v, double beta, double2* out,
                     int nrhs, hipStream_t st) {
  const Path P = pick_path(h, false, nrhs);
  const TermList& tl = P.mm ? h->tl_dinv_mm : h->tl_dinv;
  TermArgs t = term_args(h, dinv_set(h), tl, false, in, h->N);
  if (P.mm) {
    const hipError_t e = launch_rows(in, h->N, nullptr, h->N, nrhs, h->xr64_0, nullptr, h->ws_ldr, st);
    if (e != hipSuccess) return e;
    t.xr = h->xr64_0;
  }
  t.beta = beta;
  t.v = v;
  t.ldv = h->N;
  t.xacc = out;
  t.ldxa = h->N;
  t.accumulate = 0;
  return run_term(h, P, false, t, tl, nrhs, st);
}

constexpr int64_t kMaxNestedProducts = 100000;  // level products per nested solve, at most

// The nested multi-level form of eq. 14-22 with factors from the leaf level
// up: x = S_n(... S_1(D^{-1} b)), S_j v = sum_{k<=K} (-X_j)^k v with
// X_j w = S_{j-1}(... S_1(U_j w)) (the paper's V_2, W_3: each X_j applies the
// truncated inverses of the factors before it), U_1 = D^{-1} (R_L) (near
// off-diagonal blocks and leaf-level far blocks), U_j = D^{-1} F_{L-j+1} for
// the far blocks of exactly one coarser level, obtained as Z_l y - Z_{l+1} y
// from the level products of the apply panels.  Levels with no far blocks
// give X_j = 0 and are skipped.  All arithmetic is in the term, stage-A and
// axpy kernels; the host only walks the recursion.  b and x in original
// order.
struct Nested {
  hm_matrix* h;
  bool f32;
  int K, nrhs;
  hipStream_t st;
  std::vector<int> lev;  // level of each factor (index 0: the leaf level)
  int top = 0;
  int64_t N, ldin;
  double2* get() { return h->nest_pool + (int64_t)(top++) * N * nrhs; }
  void put() { --top; }
  int li(int l) const { return h->lmin < 0 ? 0 : l - h->lmin; }
  // out = U_j y
  int U(int j, const double2* y, double2* out) {
    HIPCHK(launch_axpy(1.0, y, N, h->xin0, ldin, N, nrhs, 0, st));
    double2* t1 = get();
    const int l = lev[j];
    STCHK(apply_core(h, li(l), f32, nrhs, 1.0, 0.0, nullptr, t1, nullptr, 0, st));
    if (j == 0) {
      HIPCHK(dinv_pass(h, t1, y, -1.0, out, nrhs, st));  // D^{-1} Z_L y - y
    } else {
      double2* t2 = get();
      STCHK(apply_core(h, li(l + 1), f32, nrhs, -1.0, 1.0, t1, t2, nullptr, 0, st));
      HIPCHK(dinv_pass(h, t2, nullptr, 0.0, out, nrhs, st));
      put();
    }
    put();
    return HM_OK;
  }
  // v <- S_{j-1}(... S_0(v)) (the first j truncated inverses, in place)
  int Q(int j, double2* v) {
    for (int i = 0; i < j; ++i) STCHK(S(i, v));
    return HM_OK;
  }
  // u <- sum_{k<=K} (-X_i)^k u, X_i w = Q(i, U_i w)
  int S(int i, double2* u) {
    if (K == 0) return HM_OK;
    double2* y = get();
    HIPCHK(launch_axpy(1.0, u, N, y, N, N, nrhs, 0, st));
    for (int k = 1; k <= K; ++k) {
      double2* w = get();
      STCHK(U(i, y, w));
      STCHK(Q(i, w));
      HIPCHK(launch_axpy(-1.0, w, N, y, N, N, nrhs, 0, st));  // y = -X_i y
      put();
      HIPCHK(launch_axpy(1.0, y, N, u, N, N, nrhs, 1, st));
    }
    put();
    return HM_OK;
  }
};

int nested_solve(hm_matrix* h, int level, bool f32, int K, const double2* b_dev, int64_t ldb,
                 double2* x_dev, int64_t ldx, int nrhs, hipStream_t st) {
  Nested ns{h, f32, K, nrhs, st};
  ns.N = h->N;
  ns.ldin = h->N + h->T;
  // factor levels: the leaf level, then each coarser level down to the
  // requested one that holds far blocks
  const int L = h->L;
  int lt = level < 0 ? L : level;
  if (lt > L) { set_error("level beyond the leaf level"); return HM_EINVAL; }
  lt = h->lmin < 0 ? L : std::max(lt, h->lmin);
  std::vector<int> nfar(L + 1, 0);
  for (const auto& fb : h->H.far)
    if (fb.level >= 0 && fb.level <= L) nfar[fb.level] += 1;
  ns.lev.push_back(L);
  for (int l = L - 1; l >= lt; --l)
    if (nfar[l] > 0) ns.lev.push_back(l);
  const int n = (int)ns.lev.size();
  // level products: c_j = c_{j-1} + K (1 + c_{j-1})
  double c = 0;
  for (int j = 0; j < n; ++j) c = c + K * (1.0 + c);
  if (c > kMaxNestedProducts) {
    set_error("nested solve: too many level products for this K and level count");
    return HM_EINVAL;
  }
  const int cap = 2 * n + 4;
  if (cap > h->nest_cap || nrhs > h->nest_nrhs) {
    if (h->nest_pool) (void)hipFree(h->nest_pool);
    h->nest_pool = nullptr;
    h->nest_cap = h->nest_nrhs = 0;
    const int ncap = std::max(cap, 0), nr = std::max(nrhs, 1);
    const hipError_t e = hipMalloc((void**)&h->nest_pool, sizeof(double2) * h->N * nr * ncap);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("nested workspace hipMalloc failed");
      return HM_ENOMEM;
    }
    h->nest_cap = ncap;
    h->nest_nrhs = nr;
  }
  double2* x = ns.get();
  HIPCHK(launch_permute_in(b_dev, ldb, h->perm, h->bt, h->N, h->N, nrhs, st));
  HIPCHK(dinv_pass(h, h->bt, nullptr, 0.0, x, nrhs, st));
  STCHK(ns.Q(n, x));
  HIPCHK(launch_permute_out(x, h->N, h->perm, x_dev, ldx, h->N, nrhs, st));
  ns.put();
  return HM_OK;
}

bool check_arch(std::string* arch) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  *arch = prop.gcnArchName;
  return std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
}

// Work units of the matrix-core term lists: waves when one wave takes a
// whole leaf, else workgroups.
int mm_units(const hm_matrix* h) {
  return mm_wave_mode(h->max_m) ? 4 * h->term_wgs : h->term_wgs;
}

// One wave per whole leaf (no partial sums) when there are enough leaves
// for the waves to even out: small leaves and at least two per unit.
bool mm_whole(const hm_matrix* h) {
  return mm_wave_mode(h->max_m) && h->nl >= 2 * mm_units(h);
}

// Term-kernel work lists for every level (one resident round of h->term_wgs
// persistent workgroups): one-RHS lists (dense column ranges + in-row stack
// rows), many-RHS lists (dense column ranges only: in-row U columns read t
// like the global ones), and the D^{-1} list.  Replaces earlier lists.
// Queue items of the multi-term matrix-core series at level li (wave mode):
// the stage-A tiles (64 rows of a group each), then the term pieces of the
// level's many-RHS series list; per instance the tiles and the leaves
// (one epilogue each per term).
int build_mm_multi(hm_matrix* h, int li, hipStream_t st) {
  const HostH& H = h->H;
  const int ninst = (int)h->inst_off.size() - 1;
  std::vector<MMItem> items;
  std::vector<int32_t> need_a(ninst, 0), need_b(ninst, 0);
  for (const GroupItem& gi : h->sa_mm_host[li]) {  // one item per 64-row tile of a group
    const int inst = h->group_mm_inst[gi.group];
    items.push_back({0, inst, gi.group, 0, 0, 0, gi.row0, gi.rows});
    need_a[inst]++;
  }
  const int n_a = (int)items.size();
  std::vector<char> seen(h->nl, 0);
  for (const TermItem& it : h->tl_series_mm[li].host) {
    if (it.kind != 0) return HM_OK;  // not a list this launch runs
    const int inst = H.leaf_inst[it.leaf];
    items.push_back({1, inst, it.leaf, it.c0, it.c1, it.prow, 0, 0});
    if (!seen[it.leaf]) {
      seen[it.leaf] = 1;
      need_b[inst]++;
    }
  }
  for (int a = 0; a < h->nl; ++a)
    if (!seen[a]) return HM_OK;  // a leaf without an epilogue: keep the per-term launches
  // each part of a term in instance order: the first instances finish their
  // term first, and their next-term tiles, first in the next part, find
  // their waits already met (every wait stays on an earlier part)
  auto by_inst = [](const MMItem& x, const MMItem& y) { return x.inst < y.inst; };
  std::stable_sort(items.begin(), items.begin() + n_a, by_inst);
  std::stable_sort(items.begin() + n_a, items.end(), by_inst);
  hm_matrix::MMMulti& mm = h->mm_multi[li];
  STCHK(upload(h, &mm.items, items, st, true));
  STCHK(upload(h, &mm.need_a, need_a, st, true));
  STCHK(upload(h, &mm.need_b, need_b, st, true));
  mm.n_a = n_a;
  mm.n_b = (int)items.size() - n_a;
  mm.ok = true;
  return HM_OK;
}

int build_lists(hm_matrix* h, hipStream_t st) {
  HIPCHK(hipStreamSynchronize(st));
  for (void* p : h->list_allocs) (void)hipFree(p);
  h->list_allocs.clear();
  h->bytes -= h->list_bytes;
  h->list_bytes = 0;
  const int64_t old_rows = h->partial_rows;
  h->partial_rows = 0;
  const HostH& H = h->H;
  const int nl = h->nl;
  h->tl_apply.assign(h->nlev, TermList());
  h->tl_series.assign(h->nlev, TermList());
  h->tl_apply_mm.assign(h->nlev, TermList());
  h->tl_series_mm.assign(h->nlev, TermList());
  h->half.assign(h->half_ok ? h->nlev : 0, hm_matrix::HalfList());
  std::vector<std::vector<std::pair<int64_t, int64_t>>> dense(nl);
  std::vector<int64_t> irr(nl), irc(nl), zero(nl, 0);
  for (int li = 0; li < h->nlev && h->half_ok; ++li) {
    // half storage: half-panel columns, the scaled far panels
    // [in-row U' | global U'] of the far blocks not stored as pairs, and
    // the far pairs
    for (int a = 0; a < nl; ++a) {
      const int64_t gstart = h->hir_cols[a];
      dense[a].clear();
      if (h->gl_end[li][a] > 0) dense[a].push_back({gstart, gstart + h->gl_end[li][a]});
      irr[a] = h->hir_end[li][a];
      irc[a] = 0;
    }
    STCHK(make_termlist(h, dense, irr, irc, h->hir_ncol_h, h->half[li].tl, st, &h->half[li], 0,
                        false, &h->fp_end[li]));
  }
  for (int li = 0; li < h->nlev; ++li) {
    for (int pass = 0; pass < 4; ++pass) {  // apply, series, apply MM, series MM
      const bool series = pass & 1, mm = pass >= 2;
      for (int a = 0; a < nl; ++a) {
        const int64_t m = H.leaf_size[a];
        const int64_t head = (series ? 0 : m) + h->near_cols[a];  // [D |] near
        const int64_t gstart = head + h->ir_cols[a];
        dense[a].clear();
        dense[a].push_back({0, head + (mm ? h->ir_end[li][a] : 0)});
        if (h->gl_end[li][a] > 0) dense[a].push_back({gstart, gstart + h->gl_end[li][a]});
        irr[a] = h->ir_end[li][a];
        irc[a] = head;
      }
      TermList& tl = mm ? (series ? h->tl_series_mm[li] : h->tl_apply_mm[li])
                        : (series ? h->tl_series[li] : h->tl_apply[li]);
      STCHK(make_termlist(h, dense, mm ? zero : irr, irc, h->ir_ncol_h, tl, st, nullptr,
                          mm ? mm_units(h) : 0, mm && mm_whole(h)));
    }
  }
  for (int a = 0; a < nl; ++a) {
    dense[a].clear();
    dense[a].push_back({0, H.leaf_size[a]});
  }
  STCHK(make_termlist(h, dense, zero, zero, h->ir_ncol_h, h->tl_dinv, st));
  STCHK(make_termlist(h, dense, zero, zero, h->ir_ncol_h, h->tl_dinv_mm, st, nullptr, mm_units(h),
                      true));
  h->mm_multi.assign(h->nlev, hm_matrix::MMMulti());
  if (h->mm_cnt) {
    for (int li = 0; li < h->nlev; ++li) STCHK(build_mm_multi(h, li, st));
    for (int f = 0; f < 2; ++f)
      for (int big = 0; big < 2; ++big)
        h->mm_series_wgs[f][big] = h->num_cus * series_mm_occupancy(f != 0, big ? 32 : 16);
  }
  HIPCHK(hipStreamSynchronize(st));
  if (h->partial_rows > old_rows) h->ws_nrhs = 0;  // workspace is sized by partial_rows
  return HM_OK;
}

// Host layout of the far-field device arrays the half-storage data is
// derived from (the device arrays themselves are on the handle: apply
// panels R64, in-row stacks IR64, one-RHS stage-A groups W64).
struct HalfSrc {
  const std::vector<int64_t>* R_off;
  const std::vector<int64_t>* ncols;
  const std::vector<int64_t>* ir_off;
  const std::vector<int32_t>* ir_ld;
  const std::vector<int64_t>* ir_cols;
  const std::vector<Group>* groups;
  const std::vector<std::vector<int>>* inrow;  // per leaf: in-row far blocks, in order
};

// A temporary device buffer of the build (freed with the object).
template <typename T>
struct DevTmp {
  T* p = nullptr;
  DevTmp() = default;
  DevTmp(const DevTmp&) = delete;
  DevTmp& operator=(const DevTmp&) = delete;
  ~DevTmp() {
    if (p) (void)hipFree(p);
  }
  int alloc(size_t n) {
    if (hipMalloc((void**)&p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      set_error("hipMalloc of a build buffer failed");
      return HM_ENOMEM;
    }
    return HM_OK;
  }
};

// Runs a batch of complex products C = op(A) op(B) (one launch over the
// items' 64 x 64 output tiles) and waits for it.
int run_gemms(const double2* A, const double2* B, double2* C, const std::vector<GemmItem>& items,
              hipStream_t st) {
  if (items.empty()) return HM_OK;
  std::vector<GemmTile> tiles;
  for (int32_t q = 0; q < (int32_t)items.size(); ++q)
    for (int32_t i0 = 0; i0 < items[q].m; i0 += kGemmTile)
      for (int32_t j0 = 0; j0 < items[q].n; j0 += kGemmTile) tiles.push_back({q, i0, j0, 0});
  DevTmp<GemmItem> di;
  DevTmp<GemmTile> dt;
  STCHK(di.alloc(items.size()));
  STCHK(dt.alloc(tiles.size()));
  HIPCHK(hipMemcpyAsync(di.p, items.data(), sizeof(GemmItem) * items.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(dt.p, tiles.data(), sizeof(GemmTile) * tiles.size(), hipMemcpyHostToDevice, st));
  for (size_t t0 = 0; t0 < tiles.size(); t0 += (size_t)1 << 30)
    HIPCHK(launch_cgemm(A, B, C, di.p, dt.p + t0,
                        (int)std::min<size_t>(tiles.size() - t0, (size_t)1 << 30), st));
  HIPCHK(hipStreamSynchronize(st));  // the item and tile buffers are freed on return
  return HM_OK;
}

// The apply panels and the LU blocks with the near entries computed on the
// device: R64 (rtot elements and the zeroed pad) gets the near blocks of
// every leaf (fills, as the panel assembly listed them) and the packed
// far-factor columns (upack, leaf a at u_off[a], placed after the leaf's
// diagonal and near columns); LU (lutot) gets each leaf's diagonal block
// with leading dimension m_a.  Two distinct points closer than 1e-12 in a
// near block are refused as on the host.
int fill_near_device(hm_matrix* h, const std::vector<std::vector<FillItem>>& fills,
                     const bigvec<double2>& upack, const std::vector<int64_t>& u_off,
                     const std::vector<int64_t>& near_cols, const std::vector<int64_t>& R_off,
                     int64_t rtot, const std::vector<int64_t>& LU_off, int64_t lutot,
                     hipStream_t st) {
  const HostH& H = h->H;
  const int nl = (int)H.leaf_size.size();
  const size_t rbytes = sizeof(double2) * std::max<int64_t>(rtot, 1) + kPanelPad;
  STCHK(dalloc(h, (void**)&h->R64, rbytes));
  HIPCHK(hipMemsetAsync(h->R64, 0, rbytes, st));
  STCHK(dalloc(h, (void**)&h->LU, sizeof(double2) * std::max<int64_t>(lutot, 1)));
  // far-factor columns: one upload, then one segment per leaf
  std::vector<int64_t> seg;
  for (int a = 0; a < nl; ++a) {
    const int64_t end = a + 1 < nl ? u_off[a + 1] : (int64_t)upack.size();
    const int64_t ld = even_ld(H.leaf_size[a]);
    if (end > u_off[a]) {
      seg.push_back(u_off[a]);
      seg.push_back(R_off[a] + (H.leaf_size[a] + near_cols[a]) * ld);
      seg.push_back(end - u_off[a]);
    }
  }
  std::vector<FillItem> items, lu_items;
  for (int a = 0; a < nl; ++a) {
    items.insert(items.end(), fills[a].begin(), fills[a].end());
    lu_items.push_back({LU_off[a], H.leaf_size[a], a, a, 0});
  }
  std::vector<EntryInst> inst;
  for (const EntryParams& e : H.inst) inst.push_back({e.kind, 0, e.k, e.h});
  std::vector<int32_t> loff(H.leaf_off), lm(H.leaf_size);
  DevTmp<double2> du;
  DevTmp<int64_t> dseg;
  DevTmp<FillItem> ditems, dlu;
  DevTmp<double> dxyz, dchi;
  DevTmp<int32_t> dloff, dlm, dli, dbad;
  DevTmp<EntryInst> dinst;
  STCHK(du.alloc(upack.size()));
  STCHK(dseg.alloc(seg.size()));
  STCHK(ditems.alloc(items.size()));
  STCHK(dlu.alloc(lu_items.size()));
  STCHK(dxyz.alloc(H.xyz_tree.size()));
  STCHK(dchi.alloc(H.chi_tree.size()));
  STCHK(dloff.alloc(loff.size()));
  STCHK(dlm.alloc(lm.size()));
  STCHK(dli.alloc(H.leaf_inst.size()));
  STCHK(dbad.alloc(1));
  STCHK(dinst.alloc(inst.size()));
  auto put = [&](void* d, const void* s_, size_t bytes) {
    return bytes ? hipMemcpyAsync(d, s_, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  HIPCHK(put(du.p, upack.data(), sizeof(double2) * upack.size()));
  HIPCHK(put(dseg.p, seg.data(), sizeof(int64_t) * seg.size()));
  HIPCHK(put(ditems.p, items.data(), sizeof(FillItem) * items.size()));
  HIPCHK(put(dlu.p, lu_items.data(), sizeof(FillItem) * lu_items.size()));
  HIPCHK(put(dxyz.p, H.xyz_tree.data(), sizeof(double) * H.xyz_tree.size()));
  HIPCHK(put(dchi.p, H.chi_tree.data(), sizeof(double) * H.chi_tree.size()));
  HIPCHK(put(dloff.p, loff.data(), sizeof(int32_t) * loff.size()));
  HIPCHK(put(dlm.p, lm.data(), sizeof(int32_t) * lm.size()));
  HIPCHK(put(dli.p, H.leaf_inst.data(), sizeof(int32_t) * H.leaf_inst.size()));
  HIPCHK(put(dinst.p, inst.data(), sizeof(EntryInst) * inst.size()));
  HIPCHK(hipMemsetAsync(dbad.p, 0, sizeof(int32_t), st));
  HIPCHK(launch_seg_copy(du.p, h->R64, dseg.p, (int)(seg.size() / 3), st));
  const double* chi = H.chi_tree.empty() ? nullptr : dchi.p;
  for (size_t i0 = 0; i0 < items.size(); i0 += (size_t)1 << 30)
    HIPCHK(launch_fill_near(ditems.p + i0, (int)std::min<size_t>(items.size() - i0, (size_t)1 << 30),
                            dxyz.p, chi, dloff.p, dlm.p, dli.p, dinst.p, h->R64, dbad.p, st));
  HIPCHK(launch_fill_near(dlu.p, (int)lu_items.size(), dxyz.p, chi, dloff.p, dlm.p, dli.p, dinst.p,
                          h->LU, dbad.p, st));
  int32_t bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, dbad.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));  // the temporaries are freed on return
  if (bad) {
    set_error("coincident points off the diagonal (R < 1e-12)");
    return HM_EINVAL;
  }
  return HM_OK;
}

// Compression of the far blocks the host build left to the device
// (H.aca): cross approximation and recompression on the GPU in chunks of at
// most kAcaChunkBytes of scratch, first with 32 columns per block, then with
// kAcaMaxCols for the blocks that needed more; a block still short of
// columns is compressed on the host by the same rules.
constexpr int64_t kAcaChunkBytes = (int64_t)1 << 30;

int device_aca(HostH& H, const hm_build_opts& o, hipStream_t st) {
  if (!H.aca_pending) return HM_OK;
  const int nb = (int)H.aca.size();
  std::vector<EntryInst> inst;
  for (const EntryParams& e : H.inst) inst.push_back({e.kind, 0, e.k, e.h});
  DevTmp<double> dxyz;
  DevTmp<EntryInst> dinst;
  STCHK(dxyz.alloc(H.xyz_tree.size()));
  STCHK(dinst.alloc(inst.size()));
  HIPCHK(hipMemcpyAsync(dxyz.p, H.xyz_tree.data(), sizeof(double) * H.xyz_tree.size(),
                        hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(dinst.p, inst.data(), sizeof(EntryInst) * inst.size(), hipMemcpyHostToDevice, st));
  std::vector<int> todo(nb);
  std::iota(todo.begin(), todo.end(), 0);
  for (int pass = 0; pass < 2 && !todo.empty(); ++pass) {
    const int cols = pass == 0 ? 32 : kAcaMaxCols;
    // scratch of every block of the pass (elements), then the chunks
    auto need_of = [&](const HostH::AcaBlock& d, int* r_max, int* rc) {
      *r_max = o.max_rank <= 0 ? std::min(d.m, d.n) : std::min({o.max_rank, d.m, d.n});
      *rc = std::min(cols, *r_max);
      return 2 * ((int64_t)d.m + d.n) * *rc + 4 * (int64_t)*rc * *rc;
    };
    int64_t total = 0;
    for (int q : todo) {
      int r_max, rc;
      total += need_of(H.aca[q], &r_max, &rc);
    }
    const int64_t cap = std::min<int64_t>(total, kAcaChunkBytes / (int64_t)sizeof(double2));
    // buffers of the pass, reused by its chunks (grown when a chunk needs more)
    DevTmp<double2> ws, packed;
    DevTmp<AcaItem> ditems;
    DevTmp<AcaOut> dout;
    DevTmp<int64_t> dseg;
    int64_t ws_cap = 0, packed_cap = 0, items_cap = 0, out_cap = 0, seg_cap = 0;
    auto grow = [&](auto& buf, int64_t& have, int64_t want) -> int {
      if (want <= have) return HM_OK;
      if (buf.p) HIPCHK(hipFree(buf.p));
      buf.p = nullptr;
      have = 0;
      STCHK(buf.alloc((size_t)want));
      have = want;
      return HM_OK;
    };
    std::unique_ptr<char[]> host;
    int64_t host_cap = 0;
    std::vector<int> retry;
    size_t b0 = 0;
    while (b0 < todo.size()) {
      std::vector<AcaItem> items;
      int64_t off = 0;
      int max_m = 1;
      size_t b1 = b0;
      for (; b1 < todo.size(); ++b1) {
        const HostH::AcaBlock& d = H.aca[todo[b1]];
        int r_max, rc;
        const int64_t need = need_of(d, &r_max, &rc);
        if (!items.empty() && off + need > cap) break;
        const int64_t mn = (int64_t)d.m + d.n;
        items.push_back({d.t_off, d.m, d.s_off, d.n, d.inst, r_max, rc, 0, off, off + (int64_t)d.m * rc,
                         off + mn * rc, off + mn * rc + 4 * (int64_t)rc * rc});
        off += need;
        max_m = std::max(max_m, d.m);
      }
      const int ni = (int)items.size();
      STCHK(grow(ws, ws_cap, off));
      STCHK(grow(ditems, items_cap, ni));
      STCHK(grow(dout, out_cap, ni));
      HIPCHK(hipMemcpyAsync(ditems.p, items.data(), sizeof(AcaItem) * ni, hipMemcpyHostToDevice, st));
      HIPCHK(launch_aca(ditems.p, ni, max_m, dxyz.p, dinst.p, o.aca_tol, ws.p, dout.p, st));
      HIPCHK(launch_recompress(ditems.p, ni, o.aca_tol, ws.p, dout.p, st));
      std::vector<AcaOut> res(ni);
      HIPCHK(hipMemcpyAsync(res.data(), dout.p, sizeof(AcaOut) * ni, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      // the kept factors, packed U' then V' per block, in one download
      std::vector<int64_t> seg, pos(ni, -1);
      int64_t ptot = 0;
      for (int q = 0; q < ni; ++q) {
        if (res[q].status != 0) {
          retry.push_back(todo[b0 + q]);
          continue;
        }
        if (res[q].k < 1) continue;
        const AcaItem& a = items[q];
        const int r = res[q].rank;
        if (r < 1 || r > a.rcap) {
          set_error("internal: device compression returned rank " + std::to_string(r));
          return HM_EINVAL;
        }
        pos[q] = ptot;
        seg.insert(seg.end(), {a.o_off, ptot, (int64_t)a.m * r});
        seg.insert(seg.end(), {a.o_off + (int64_t)a.m * a.rcap, ptot + (int64_t)a.m * r, (int64_t)a.n * r});
        ptot += (int64_t)(a.m + a.n) * r;
      }
      if (ptot > 0) {
        STCHK(grow(packed, packed_cap, ptot));
        STCHK(grow(dseg, seg_cap, (int64_t)seg.size()));
        if (ptot > host_cap) {  // staging of the download, left uninitialised
          host.reset(new char[(size_t)ptot * sizeof(double2)]);
          host_cap = ptot;
        }
        HIPCHK(hipMemcpyAsync(dseg.p, seg.data(), sizeof(int64_t) * seg.size(), hipMemcpyHostToDevice, st));
        HIPCHK(launch_seg_copy(ws.p, packed.p, dseg.p, (int)(seg.size() / 3), st));
        HIPCHK(hipMemcpyAsync(host.get(), packed.p, sizeof(double2) * ptot, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
      }
      const cplx* hp = reinterpret_cast<const cplx*>(host.get());
      for (int q = 0; q < ni; ++q) {
        if (res[q].status != 0) continue;
        const AcaItem& a = items[q];
        LowRank& lr = H.lowrank[todo[b0 + q]];
        lr.m = a.m;
        lr.n = a.n;
        if (res[q].k < 1) {  // no pivot anywhere: a zero block of rank 1
          lr.r = 1;
          lr.U.assign(a.m, cplx(0));
          lr.V.assign(a.n, cplx(0));
          continue;
        }
        lr.r = res[q].rank;
        const cplx* src = hp + pos[q];
        lr.U.assign(src, src + (size_t)a.m * lr.r);
        lr.V.assign(src + (size_t)a.m * lr.r, src + (size_t)(a.m + a.n) * lr.r);
      }
      b0 = b1;
    }
    todo.swap(retry);
  }
  // blocks beyond the device's column limit
  for (const int q : todo) {
    const HostH::AcaBlock& d = H.aca[q];
    Problem pt;
    pt.n = (int64_t)H.xyz_tree.size() / 3;
    pt.kind = H.inst[d.inst].kind;
    pt.k = H.inst[d.inst].k;
    pt.h = H.inst[d.inst].h;
    pt.xyz = H.xyz_tree;
    std::vector<int64_t> rows(d.m), cols(d.n);
    std::iota(rows.begin(), rows.end(), (int64_t)d.t_off);
    std::iota(cols.begin(), cols.end(), (int64_t)d.s_off);
    H.lowrank[q] = compress_block(pt, rows.data(), d.m, cols.data(), d.n, o.aca_tol, o.max_rank);
  }
  H.aca_pending = false;
  std::vector<HostH::AcaBlock>().swap(H.aca);
  return HM_OK;
}

// Device buffer of the handle, zeroed.
int dzero(hm_matrix* h, double2** p, int64_t n, hipStream_t st) {
  STCHK(dalloc(h, (void**)p, sizeof(double2) * std::max<int64_t>(n, 1)));
  HIPCHK(hipMemsetAsync(*p, 0, sizeof(double2) * std::max<int64_t>(n, 1), st));
  return HM_OK;
}

// Half-storage data (leaves of at most kHalfMaxLeaf rows), computed on the
// device.  Surface problems are symmetric; a volume problem Z = A diag(chi)
// runs on its symmetric A (x = diag(1/chi) x_A term by term).
//
// Symmetric scaling: each leaf block factors as D_a = C_a C_a^T (complex
// symmetric, C_a lower triangular, Chat_a = C_a^{-1}).  With yhat = C^T y
// the series y_{k+1} = -D^{-1} R y_k reads yhat_{k+1} = -S yhat_k, where
// S = Chat R Chat^T is symmetric like R; yhat_0 = Chat b and
// x = Chat^T sum_k yhat_k.  So a term is one product with S and no
// block-diagonal step.  The half panels hold S_ts = Chat_t Z_ts Chat_s^T for
// the near blocks s > t of row leaf t, side by side (ld = even m_t); the far
// part of S is U' = Chat_t U (from the apply panels' far columns) and
// W' = W Chat_s^T (the in-row stacks and the one-RHS stage-A groups, row
// segments per source leaf).  Column j of the half panel of t is row jj of
// its block's leaf s: it reads yhat[off_s + jj] (hsrc) and its v value goes
// to vb slot hp_col[t] + j, which the epilogue of s adds (vstart, blocks
// ordered by t).  The factors (launch_csym) and every scaled block
// (launch_cgemm) are formed on the device from the handle's apply panels,
// in-row stacks and stage-A groups; the host lays out the arrays.
int build_half(hm_matrix* h, const HalfSrc& hs, hipStream_t st) {
  const HostH& H = h->H;
  const int nl = h->nl;
  h->half_ok = false;
  h->hp_ncol.assign(nl, 0);
  h->hp_bcol.assign(nl, std::vector<int32_t>());
  h->hp_bleaf.assign(nl, std::vector<int32_t>());
  h->ent_half.assign(h->nlev, 0);
  if (!h->want_half || H.near.empty() || h->max_m > kHalfMaxLeaf || h->max_m > kCsymMaxLeaf)
    return HM_OK;
  std::vector<int> diag(nl, -1);
  std::vector<std::vector<int>> blk(nl);
  std::vector<std::vector<std::pair<int, int64_t>>> near_col(nl);  // (s, apply-panel column)
  {
    std::vector<int64_t> c(nl);
    for (int a = 0; a < nl; ++a) c[a] = H.leaf_size[a];  // after D
    for (int q = 0; q < (int)H.near.size(); ++q) {  // H.near is sorted by (t, s)
      const NearBlock& nb = H.near[q];
      if (nb.t_leaf == nb.s_leaf) {
        diag[nb.t_leaf] = q;
        continue;
      }
      if (nb.t_leaf < nb.s_leaf) {
        blk[nb.t_leaf].push_back(q);
        near_col[nb.t_leaf].push_back({nb.s_leaf, c[nb.t_leaf]});
      }
      c[nb.t_leaf] += H.leaf_size[nb.s_leaf];
    }
  }
  for (int a = 0; a < nl; ++a)
    if (diag[a] < 0) return HM_OK;
  const std::vector<int64_t>& R_off = *hs.R_off;
  // ---- C_a, C_a^T, C_a^{-1}, C_a^{-T} as block-diagonal panels (ld even m)
  std::vector<int64_t> ch_off(nl);
  int64_t chtot = 0;
  for (int a = 0; a < nl; ++a) {
    ch_off[a] = chtot;
    chtot += (int64_t)even_ld(H.leaf_size[a]) * H.leaf_size[a];
  }
  DevTmp<int64_t> d_choff;
  DevTmp<int32_t> d_ok;
  STCHK(d_choff.alloc(nl));
  STCHK(d_ok.alloc(nl));
  HIPCHK(hipMemcpyAsync(d_choff.p, ch_off.data(), sizeof(int64_t) * nl, hipMemcpyHostToDevice, st));
  DevTmp<double2> cf, cft, ch, cht;
  for (DevTmp<double2>* b : {&cf, &cft, &ch, &cht}) {
    STCHK(b->alloc(chtot));
    HIPCHK(hipMemsetAsync(b->p, 0, sizeof(double2) * std::max<int64_t>(chtot, 1), st));
  }
  // volume: Z = A diag(chi) with A symmetric (the kernel part G and the
  // diagonal terms), so the scaled series runs on A: its blocks are the
  // panels' blocks with column j divided by chi_j (W' folds 1/chi into the
  // C^{-1} or C^{-T} factor it meets), and x = diag(1/chi) x_A
  DevTmp<double> d_chi;
  const bool vol = !H.chi_tree.empty();
  if (vol) {
    STCHK(d_chi.alloc(h->N));
    HIPCHK(hipMemcpyAsync(d_chi.p, H.chi_tree.data(), sizeof(double) * h->N,
                          hipMemcpyHostToDevice, st));
  }
  HIPCHK(launch_csym(h->R64, h->R_off, h->leaf_m, h->leaf_off, d_chi.p, nl, h->max_m, cf.p, cft.p,
                     ch.p, cht.p, d_choff.p, d_ok.p, st));
  {
    std::vector<int32_t> ok(nl, 0);
    HIPCHK(hipMemcpyAsync(ok.data(), d_ok.p, sizeof(int32_t) * nl, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int a = 0; a < nl; ++a)
      if (!ok[a]) return HM_OK;  // not safely factorable: the panels serve
  }
  // volume: C^{-T} with rows divided by chi (every use maps back to the
  // unknowns x = diag(1/chi) x_A, or meets a column divided by chi in the
  // scaled blocks), C^{-1} with columns divided by chi (the pairs' W'), and
  // C^T with columns multiplied by chi (the H-matvec's C^T diag(chi) x)
  DevTmp<double2> chx;
  if (vol) {
    STCHK(chx.alloc(chtot));
    HIPCHK(launch_panel_scale(cht.p, cht.p, d_choff.p, h->leaf_m, h->leaf_off, d_chi.p, nl, 0, st));
    HIPCHK(launch_panel_scale(ch.p, chx.p, d_choff.p, h->leaf_m, h->leaf_off, d_chi.p, nl, 1, st));
    HIPCHK(launch_panel_scale(cft.p, cft.p, d_choff.p, h->leaf_m, h->leaf_off, d_chi.p, nl, 2, st));
  }
  const double2* ch_w = vol ? chx.p : ch.p;  // C^{-1} the pairs' W' meet
  // ---- half-panel layout
  std::vector<int64_t> hp_off(nl + 1, 0);
  std::vector<int32_t> hp_col(nl + 1, 0);
  int64_t cols = 0, tot = 0;
  for (int t = 0; t < nl; ++t) {
    std::vector<int32_t>& bc = h->hp_bcol[t];
    std::vector<int32_t>& bl = h->hp_bleaf[t];
    int64_t c = 0;
    for (int q : blk[t]) {  // increasing s
      bc.push_back((int32_t)c);
      bl.push_back(H.near[q].s_leaf);
      c += H.leaf_size[H.near[q].s_leaf];
    }
    bc.push_back((int32_t)c);
    const int64_t ld = even_ld(H.leaf_size[t]);
    // 32-bit byte offsets within one half panel (FP64 elements)
    if (ld * c * 16 >= ((int64_t)1 << 31)) { set_error("half panel too large"); return HM_EINVAL; }
    h->hp_ncol[t] = c;
    hp_off[t] = tot;
    hp_col[t] = (int32_t)cols;
    tot += ld * c;
    cols += c;
    if (cols >= ((int64_t)1 << 31)) { set_error("half-panel columns exceed 2^31"); return HM_EINVAL; }
  }
  hp_off[nl] = tot;
  hp_col[nl] = (int32_t)cols;
  std::vector<int32_t> hsrc((size_t)cols);
  std::vector<std::vector<int32_t>> vs(nl);
  for (int t = 0; t < nl; ++t)
    for (size_t b = 0; b < h->hp_bleaf[t].size(); ++b) {
      const int s = h->hp_bleaf[t][b];
      const int64_t c0 = hp_col[t] + h->hp_bcol[t][b];
      for (int jj = 0; jj < H.leaf_size[s]; ++jj) hsrc[c0 + jj] = H.leaf_off[s] + jj;
      vs[s].push_back((int32_t)c0);
    }
  std::vector<int32_t> vptr(nl + 1, 0), vstart;
  for (int s = 0; s < nl; ++s) {
    vptr[s + 1] = vptr[s] + (int32_t)vs[s].size();
    vstart.insert(vstart.end(), vs[s].begin(), vs[s].end());
  }
  // ---- half panels S_ts = Chat_t Z_ts Chat_s^T: T = Chat_t Z_ts (Z_ts the
  // block's columns of the apply panel of t), then S = T Chat_s^T
  {
    DevTmp<double2> tmp;
    STCHK(tmp.alloc(tot));
    STCHK(dzero(h, &h->H64, tot, st));
    std::vector<GemmItem> g1, g2;
    for (int t = 0; t < nl; ++t) {
      const int mt = H.leaf_size[t];
      const int32_t ldt = even_ld(mt);
      for (size_t b = 0; b < near_col[t].size(); ++b) {
        const int s = near_col[t][b].first;
        const int ms = H.leaf_size[s];
        const int64_t c_off = hp_off[t] + (int64_t)h->hp_bcol[t][b] * ldt;
        g1.push_back({ch_off[t], R_off[t] + near_col[t][b].second * ldt, c_off, ldt, ldt, ldt, mt,
                      ms, mt, 0, 0});
        g2.push_back({c_off, ch_off[s], c_off, ldt, even_ld(ms), ldt, mt, ms, ms, 0, 0});
      }
    }
    STCHK(run_gemms(ch.p, h->R64, tmp.p, g1, st));
    STCHK(run_gemms(tmp.p, cht.p, h->H64, g2, st));
  }
  // ---- far part.  A far block whose row and column clusters are both
  // leaves (t, s) is a pair, stored once by its lower leaf t < s: U' =
  // Chat_t U (even(m_t) x r) and W' = Chat_s W (even(m_s) x r) with
  // S_ts = U' W'^T and S_st = W' U'^T.  Every other far block keeps U' =
  // Chat_t U as far-panel columns ([in-row U' | global U'] per leaf) and
  // W' = W Chat_s^T as rows of the in-row stacks or the one-RHS stage-A
  // groups (row segments per source leaf).  Blocks stay finest level first.
  auto lev_of = [&](int li) { return (h->lmin < 0) ? h->L + 1 : h->lmin + li; };
  auto rank = [&](int b) { return H.lowrank[H.far[b].src].r; };
  auto col_leaf = [&](int b) -> int {  // column leaf of a block onto one leaf, else -1
    const FarBlock& fb = H.far[b];
    const int s = H.tree.leaf_of[fb.s_off];
    return (H.leaf_off[s] == fb.s_off && H.leaf_size[s] == fb.n) ? s : -1;
  };
  struct Blk { int b; int64_t ucol, srow; };  // in-row block, its U' column and stack row
  std::vector<std::vector<Blk>> own_pairs(nl), rest(nl);
  for (int a = 0; a < nl; ++a) {
    int64_t ucol = 0;
    for (int b : (*hs.inrow)[a]) {
      const int s = col_leaf(b);
      if (s < 0) rest[a].push_back({b, ucol, ucol});
      else if (a < s) own_pairs[a].push_back({b, ucol, ucol});
      ucol += rank(b);  // in-row U' columns and stack rows share the order
    }
  }
  // pair index, data offsets and z_s slots
  std::vector<int32_t> fp_first(nl + 1, 0), fp_rank, fp_tgt, fp_slot;
  std::vector<int64_t> fp_off;
  int64_t fptot = 0, fprows = 0;
  for (int a = 0; a < nl; ++a) {
    fp_first[a] = (int32_t)fp_rank.size();
    for (const Blk& k : own_pairs[a]) {
      const int s = col_leaf(k.b), r = rank(k.b);
      fp_off.push_back(fptot);
      fp_rank.push_back(r);
      fp_tgt.push_back(s);
      fp_slot.push_back((int32_t)fprows);
      fptot += (int64_t)(even_ld(H.leaf_size[a]) + even_ld(H.leaf_size[s])) * r;
      fprows += H.leaf_size[s];
    }
  }
  const int npair = (int)fp_rank.size();
  fp_first[nl] = npair;
  // in-row stacks and far panels of the remaining blocks
  std::vector<int64_t> hir_off(nl), hir_cols(nl, 0), hf_off(nl);
  std::vector<int32_t> hir_ld(nl), hir_ncol(nl, 0), hir_row0(nl), hir_soff, hir_n;
  std::vector<int64_t> gl_cols(nl), hf_col(nl);
  int64_t irtot = 0, ftot = 0;
  for (int a = 0; a < nl; ++a) {
    const int m = H.leaf_size[a];
    for (const Blk& k : rest[a]) {
      hir_cols[a] += rank(k.b);
      hir_ncol[a] = std::max(hir_ncol[a], H.far[k.b].n);
      for (int q = 0; q < rank(k.b); ++q) {
        hir_soff.push_back(H.far[k.b].s_off);
        hir_n.push_back(H.far[k.b].n);
      }
    }
    hir_row0[a] = (int32_t)(hir_soff.size() - hir_cols[a]);
    hir_ld[a] = even_ld((int)hir_cols[a]);
    hir_off[a] = irtot;
    irtot += (int64_t)hir_ld[a] * hir_ncol[a];
    gl_cols[a] = (*hs.ncols)[a] - m - h->near_cols[a] - (*hs.ir_cols)[a];
    hf_off[a] = ftot;
    ftot += (int64_t)even_ld(m) * (hir_cols[a] + gl_cols[a]);
    if ((int64_t)hir_ld[a] * hir_ncol[a] >= ((int64_t)1 << 31) ||
        (int64_t)even_ld(m) * (hir_cols[a] + gl_cols[a]) >= ((int64_t)1 << 31)) {
      set_error("a leaf's far data exceeds 2^31 elements");
      return HM_EINVAL;
    }
  }
  // src index of far-panel column c of leaf a: global columns keep the
  // sources of the apply panel's global columns
  {
    int64_t ctot = 0;
    for (int a = 0; a < nl; ++a) {
      const int64_t far0 = ctot + H.leaf_size[a] + h->near_cols[a];
      hf_col[a] = far0 + (*hs.ir_cols)[a] - hir_cols[a];
      ctot += (*hs.ncols)[a];
    }
  }
  if (hir_soff.empty()) { hir_soff.push_back(0); hir_n.push_back(0); }
  // ---- scaled far data on the device: U' = Chat_a U for the far-panel
  // columns and the pairs, W' = Chat_s W for the pairs (W the block's rows
  // of the stack, transposed), W' = W Chat_s^T per source-leaf segment for
  // the remaining in-row stack rows and the one-RHS stage-A groups
  STCHK(dzero(h, &h->HF64, ftot, st));
  STCHK(dzero(h, &h->IRT64, irtot, st));
  STCHK(dzero(h, &h->FP64, fptot, st));
  int64_t wtot = 0;
  for (const Group& G : *hs.groups) wtot = std::max<int64_t>(wtot, G.w_off + (int64_t)G.ld * G.n);
  STCHK(dzero(h, &h->WT64, wtot, st));
  {
    std::vector<GemmItem> uf, up, wp, wi, wg;
    // segments of a source range [s0, s0 + n) by leaf: (leaf, column in range)
    auto segs = [&](int64_t s0, int64_t n, const std::function<void(int, int64_t)>& f) {
      for (int s = H.tree.leaf_of[s0]; s < nl && H.leaf_off[s] < s0 + n; ++s) f(s, H.leaf_off[s] - s0);
    };
    for (int a = 0; a < nl; ++a) {
      const int m = H.leaf_size[a];
      const int32_t ld = even_ld(m);
      const int64_t far0 = m + h->near_cols[a];  // first far column of the apply panel
      const int64_t rb = R_off[a] + far0 * ld;
      const int64_t irb = (*hs.ir_off)[a];
      const int32_t irld = (*hs.ir_ld)[a];
      int64_t c = 0;
      for (const Blk& k : rest[a]) {
        const FarBlock& fb = H.far[k.b];
        const int r = rank(k.b);
        uf.push_back({ch_off[a], rb + k.ucol * ld, hf_off[a] + c * ld, ld, ld, ld, m, r, m, 0, 0});
        segs(fb.s_off, fb.n, [&](int s, int64_t j0) {
          const int ms = H.leaf_size[s];
          wi.push_back({irb + k.srow + j0 * irld, ch_off[s], hir_off[a] + c + j0 * hir_ld[a], irld,
                        even_ld(ms), hir_ld[a], r, ms, ms, 0, 0});
        });
        c += r;
      }
      if (gl_cols[a] > 0)
        uf.push_back({ch_off[a], rb + (*hs.ir_cols)[a] * ld, hf_off[a] + c * ld, ld, ld, ld, m,
                      (int32_t)gl_cols[a], m, 0, 0});
      for (size_t kk = 0; kk < own_pairs[a].size(); ++kk) {
        const Blk& k = own_pairs[a][kk];
        const int p = fp_first[a] + (int)kk;
        const int s = fp_tgt[p], r = fp_rank[p], ms = H.leaf_size[s];
        up.push_back({ch_off[a], rb + k.ucol * ld, fp_off[p], ld, ld, ld, m, r, m, 0, 0});
        wp.push_back({ch_off[s], irb + k.srow, fp_off[p] + (int64_t)ld * r, even_ld(ms), irld,
                      even_ld(ms), ms, r, ms, 0, 1});
      }
    }
    for (const Group& G : *hs.groups)
      segs(G.s_off, G.n, [&](int s, int64_t j0) {
        const int ms = H.leaf_size[s];
        wg.push_back({G.w_off + j0 * G.ld, ch_off[s], G.w_off + j0 * G.ld, G.ld, even_ld(ms), G.ld,
                      G.ld, ms, ms, 0, 0});
      });
    STCHK(run_gemms(ch.p, h->R64, h->HF64, uf, st));
    STCHK(run_gemms(ch.p, h->R64, h->FP64, up, st));
    STCHK(run_gemms(ch_w, h->IR64, h->FP64, wp, st));
    STCHK(run_gemms(h->IR64, cht.p, h->IRT64, wi, st));
    STCHK(run_gemms(h->W64, cht.p, h->WT64, wg, st));
  }
  // per level: pairs and in-row rows of the far blocks of level >= l, and
  // the entries one half-storage term reads (near blocks s > t, pairs once,
  // U' and W' of the other far blocks)
  h->fp_end.assign(h->nlev, std::vector<int32_t>(nl, 0));
  h->hir_end.assign(h->nlev, std::vector<int64_t>(nl, 0));
  for (int li = 0; li < h->nlev; ++li) {
    int64_t e = 0;
    for (int a = 0; a < nl; ++a) {
      const int m = H.leaf_size[a];
      e += (int64_t)m * h->hp_ncol[a];
      for (const Blk& k : own_pairs[a]) {
        if (H.far[k.b].level < lev_of(li)) break;
        h->fp_end[li][a]++;
        e += (int64_t)rank(k.b) * (m + H.far[k.b].n);
      }
      for (const Blk& k : rest[a]) {
        if (H.far[k.b].level < lev_of(li)) break;
        h->hir_end[li][a] += rank(k.b);
        e += (int64_t)rank(k.b) * (m + H.far[k.b].n);
      }
    }
    for (const FarBlock& fb : H.far)  // global blocks: U' slices and stage-A W'
      if (fb.level >= lev_of(li) && !(H.leaf_off[H.tree.leaf_of[fb.t_off]] == fb.t_off &&
                                      H.leaf_size[H.tree.leaf_of[fb.t_off]] == fb.m))
        e += (int64_t)H.lowrank[fb.src].r * (fb.m + fb.n);
    h->ent_half[li] = e;
  }
  // ---- the factor panels move to the handle
  for (auto pr : {std::make_pair(&ch, &h->CH), std::make_pair(&cht, &h->CHT),
                  std::make_pair(&cf, &h->CF), std::make_pair(&cft, &h->CFT)}) {
    *pr.second = pr.first->p;
    pr.first->p = nullptr;
    h->allocs.push_back(*pr.second);
    h->bytes += (int64_t)sizeof(double2) * std::max<int64_t>(chtot, 1);
  }
  STCHK(dalloc(h, (void**)&h->hwork, sizeof(double2) * h->N));
  if (h->has_f32) {
    const int64_t n_ir = std::max<int64_t>(irtot, 1), n_w = std::max<int64_t>(wtot, 1);
    const int64_t n_fp = std::max<int64_t>(fptot, 1);
    STCHK(dalloc(h, (void**)&h->H32, sizeof(float2) * std::max<int64_t>(tot, 1)));
    STCHK(dalloc(h, (void**)&h->HF32, sizeof(float2) * std::max<int64_t>(ftot, 1)));
    STCHK(dalloc(h, (void**)&h->IRT32, sizeof(float2) * n_ir));
    STCHK(dalloc(h, (void**)&h->FP32, sizeof(float2) * n_fp));
    STCHK(dalloc(h, (void**)&h->WT32, sizeof(float2) * std::max<int64_t>(n_w, 1)));
    HIPCHK(launch_cast(h->H64, h->H32, tot, st));
    HIPCHK(launch_cast(h->HF64, h->HF32, ftot, st));
    HIPCHK(launch_cast(h->IRT64, h->IRT32, n_ir, st));
    HIPCHK(launch_cast(h->FP64, h->FP32, n_fp, st));
    HIPCHK(launch_cast(h->WT64, h->WT32, n_w, st));
  }
  hp_off.pop_back();
  STCHK(upload(h, &h->hp_off, hp_off, st));
  STCHK(upload(h, &h->hp_col, hp_col, st));
  STCHK(upload(h, &h->hsrc, hsrc, st));
  h->vptr_h = vptr;
  h->vstart_h = vstart;
  h->hp_cols = cols;
  STCHK(upload(h, &h->hf_off, hf_off, st));
  STCHK(upload(h, &h->hf_col, hf_col, st));
  STCHK(upload(h, &h->ch_off, ch_off, st));
  STCHK(upload(h, &h->hir_off, hir_off, st));
  STCHK(upload(h, &h->hir_ld, hir_ld, st));
  STCHK(upload(h, &h->hir_ncol, hir_ncol, st));
  STCHK(upload(h, &h->hir_row0, hir_row0, st));
  STCHK(upload(h, &h->hir_soff, hir_soff, st));
  STCHK(upload(h, &h->hir_n, hir_n, st));
  h->hir_cols = hir_cols;
  h->hir_ncol_h = hir_ncol;
  if (fp_off.empty()) {  // device arrays of at least one entry
    fp_off.push_back(0);
    fp_rank.push_back(0);
    fp_slot.push_back(0);
  }
  STCHK(upload(h, &h->fp_off, fp_off, st));
  STCHK(upload(h, &h->fp_rank, fp_rank, st));
  STCHK(upload(h, &h->fp_slot, fp_slot, st));
  fp_rank.resize(npair);
  fp_slot.resize(npair);
  h->fp_first_h = fp_first;
  h->fp_rank_h = fp_rank;
  h->fp_tgt_h = fp_tgt;
  h->fp_slot_h = fp_slot;
  h->fp_rows = fprows;
  STCHK(dalloc(h, (void**)&h->zbuf, sizeof(double2) * h->N));
  STCHK(dalloc(h, (void**)&h->hq, 2 * sizeof(int32_t)));
  HIPCHK(hipMemsetAsync(h->hq, 0, 2 * sizeof(int32_t), st));
  STCHK(dalloc(h, (void**)&h->hdone, sizeof(int32_t) * (nl + 1)));
  HIPCHK(hipMemsetAsync(h->hdone, 0, sizeof(int32_t) * (nl + 1), st));
  h->herr = h->hdone + nl;
  h->half_ok = true;
  return HM_OK;
}

// ------------------------------------------------------------ device build
// Progress message of a build phase; with a progress callback attached the
// stream is drained first, so that the message marks the phase's end.
void build_mark(const hm_build_opts* o, hipStream_t st, const char* what) {
  if (!o || !o->progress) return;
  (void)hipStreamSynchronize(st);
  o->progress(what, o->progress_user);
}

int build_device(hm_matrix* h, const hm_build_opts* opts, hipStream_t st) {
  const HostH& H = h->H;
  const int nl = h->nl;
  const int64_t N = h->N;
  const int nfar = (int)H.far.size();
  h->nlev = (h->lmin < 0) ? 1 : (h->L - h->lmin + 1);
  auto lev_of = [&](int li) { return (h->lmin < 0) ? h->L + 1 : h->lmin + li; };
  auto rank = [&](int b) { return H.lowrank[H.far[b].src].r; };
  const double* chi = H.chi_tree.empty() ? nullptr : H.chi_tree.data();
  // W_b[q, j] = V[j, q] chi_s[j] of the stored orientation (n x r)
  auto wval = [&](int b, int q, int j) -> double2 {
    const FarBlock& fb = H.far[b];
    const LowRank& lr = H.lowrank[fb.src];
    const std::vector<cplx>& V = fb.transposed ? lr.U : lr.V;
    cplx v = V[j + (size_t)q * fb.n];
    if (chi) v *= chi[fb.s_off + j];
    return make_double2(v.real(), v.imag());
  };

  // ---- classify far blocks: in-row (row cluster = one leaf) or global
  std::vector<int> row_leaf(nfar, -1);
  for (int b = 0; b < nfar; ++b) {
    const int a = H.tree.leaf_of[H.far[b].t_off];
    if (H.leaf_off[a] == H.far[b].t_off && H.leaf_size[a] == H.far[b].m) row_leaf[b] = a;
  }

  // ---- stage-A groups: far blocks by source cluster, finest level first;
  // rows = (block, q), t slot of block b at tb[b].  The one-RHS kernels
  // group only the global blocks (in-row ones are folded into the term
  // kernel); the many-RHS kernels group every far block.
  struct GroupSet {
    std::vector<Group> groups;
    std::vector<std::vector<int>> blocks;
    std::vector<std::vector<int32_t>> rows;  // rows of group g at level li
    std::vector<int32_t> tb;
    int64_t T = 0, wtot = 0;
  };
  auto make_groups = [&](bool all, GroupSet& gs) {
    std::map<std::pair<int32_t, int32_t>, int> key;  // (s_off, n) -> group
    for (int b = 0; b < nfar; ++b)
      if (all || row_leaf[b] < 0) key.emplace(std::make_pair(H.far[b].s_off, H.far[b].n), 0);
    int ng = 0;
    for (auto& kv : key) kv.second = ng++;
    gs.blocks.assign(ng, {});
    for (int b = 0; b < nfar; ++b)
      if (all || row_leaf[b] < 0) gs.blocks[key[{H.far[b].s_off, H.far[b].n}]].push_back(b);
    gs.groups.assign(ng, Group{});
    gs.tb.assign(nfar, -1);
    gs.rows.assign(ng, std::vector<int32_t>(h->nlev, 0));
    for (auto& kv : key) {
      const int g = kv.second;
      auto& bl = gs.blocks[g];
      std::sort(bl.begin(), bl.end(), [&](int x, int y) {
        if (H.far[x].level != H.far[y].level) return H.far[x].level > H.far[y].level;
        return H.far[x].t_off < H.far[y].t_off;
      });
      int32_t R = 0;
      for (int b : bl) {
        gs.tb[b] = (int32_t)(gs.T + R);
        R += rank(b);
      }
      gs.groups[g] = Group{kv.first.first, kv.first.second, (int32_t)gs.T, even_ld(R), gs.wtot};
      gs.T += R;
      gs.wtot += (int64_t)even_ld(R) * kv.first.second;
      for (int li = 0; li < h->nlev; ++li) {
        int32_t rr = 0;
        for (int b : bl) {
          if (H.far[b].level < lev_of(li)) break;
          rr += rank(b);
        }
        gs.rows[g][li] = rr;
      }
    }
  };
  auto fill_W = [&](const GroupSet& gs, bigvec<double2>& W) {
    W = bigvec<double2>((size_t)std::max<int64_t>(gs.wtot, 1));  // zeroed (pad rows stay 0)
    const int ng = (int)gs.groups.size();
#pragma omp parallel for schedule(dynamic, 1)
    for (int g = 0; g < ng; ++g) {
      const Group& G = gs.groups[g];
      int32_t row = 0;
      for (int b : gs.blocks[g])
        for (int q = 0; q < rank(b); ++q, ++row)
          for (int j = 0; j < G.n; ++j) W[G.w_off + row + (int64_t)j * G.ld] = wval(b, q, j);
    }
  };
  GroupSet gs1, gsm;
  make_groups(false, gs1);
  make_groups(true, gsm);
  const std::vector<int32_t>& tb = gs1.tb;
  const int ng = (int)gs1.groups.size();
  const int64_t wtot = gs1.wtot, wtot_mm = gsm.wtot;
  // one t region after the N tree-order rows serves both layouts
  h->T = std::max(gs1.T, gsm.T);
  bigvec<double2> W;
  fill_W(gs1, W);

  // ---- per leaf: in-row blocks (finest first) and global slices (finest first)
  std::vector<std::vector<int>> inrow(nl);
  std::vector<std::vector<std::pair<int, int>>> gslices(nl);  // (block, row offset in block)
  for (int b = 0; b < nfar; ++b) {  // H.far is sorted finest level first
    const FarBlock& fb = H.far[b];
    if (row_leaf[b] >= 0) {
      inrow[row_leaf[b]].push_back(b);
      continue;
    }
    for (int a = H.tree.leaf_of[fb.t_off]; a < nl && H.leaf_off[a] < fb.t_off + fb.m; ++a)
      gslices[a].push_back({b, H.leaf_off[a] - fb.t_off});
  }
  std::vector<int64_t> near_cols(nl, 0), ir_cols(nl, 0), gl_cols(nl, 0), ncols(nl, 0);
  std::vector<std::vector<int64_t>> ir_end(h->nlev, std::vector<int64_t>(nl, 0));
  std::vector<std::vector<int64_t>> gl_end(h->nlev, std::vector<int64_t>(nl, 0));
  std::vector<std::vector<int>> near_of(nl);
  std::vector<int> diag_of(nl, -1);
  for (int q = 0; q < (int)H.near.size(); ++q) {
    const NearBlock& nb = H.near[q];
    if (nb.t_leaf != nb.s_leaf) {
      near_of[nb.t_leaf].push_back(q);
      near_cols[nb.t_leaf] += H.leaf_size[nb.s_leaf];
    } else {
      diag_of[nb.t_leaf] = q;
    }
  }
  for (int a = 0; a < nl; ++a) {
    if (diag_of[a] < 0) { set_error("internal: missing diagonal block"); return HM_EINVAL; }
    for (int b : inrow[a]) ir_cols[a] += rank(b);
    for (auto& sl : gslices[a]) gl_cols[a] += rank(sl.first);
    ncols[a] = H.leaf_size[a] + near_cols[a] + ir_cols[a] + gl_cols[a];
    for (int li = 0; li < h->nlev; ++li) {
      int64_t e = 0;
      for (int b : inrow[a]) {
        if (H.far[b].level < lev_of(li)) break;
        e += rank(b);
      }
      ir_end[li][a] = e;
      e = 0;
      for (auto& sl : gslices[a]) {
        if (H.far[sl.first].level < lev_of(li)) break;
        e += rank(sl.first);
      }
      gl_end[li][a] = e;
    }
  }

  // ---- in-row W stacks: rows = (block, q) in in-row order, columns = source
  std::vector<int64_t> ir_off(nl);
  std::vector<int32_t> ir_ld(nl), ir_ncol(nl), ir_row0(nl);
  int64_t irtot = 0, irrows = 0;
  for (int a = 0; a < nl; ++a) {
    int nmax = 0;
    for (int b : inrow[a]) nmax = std::max(nmax, H.far[b].n);
    ir_off[a] = irtot;
    ir_ld[a] = even_ld((int)ir_cols[a]);
    ir_ncol[a] = nmax;
    ir_row0[a] = (int32_t)irrows;
    irtot += (int64_t)ir_ld[a] * nmax;
    irrows += ir_cols[a];
  }
  bigvec<double2> IR((size_t)std::max<int64_t>(irtot, 1));  // zeroed
  std::vector<int32_t> ir_soff((size_t)std::max<int64_t>(irrows, 1)), ir_n((size_t)std::max<int64_t>(irrows, 1));
#pragma omp parallel for schedule(dynamic, 1)
  for (int a = 0; a < nl; ++a) {
    int32_t row = 0;
    for (int b : inrow[a]) {
      const FarBlock& fb = H.far[b];
      for (int q = 0; q < rank(b); ++q, ++row) {
        ir_soff[ir_row0[a] + row] = fb.s_off;
        ir_n[ir_row0[a] + row] = fb.n;
        for (int j = 0; j < fb.n; ++j) IR[ir_off[a] + row + (int64_t)j * ir_ld[a]] = wval(b, q, j);
      }
    }
  }

  // ---- panels (ld = even(m)): [D | near | in-row U | global U slices]
  std::vector<int64_t> R_off(nl), R_col(nl), M_off(nl), M_col(nl), LU_off(nl), Dinv_off(nl),
      piv_off(nl);
  int64_t rtot = 0, ctot = 0, mtot = 0, lutot = 0, ditot = 0, ptot = 0;
  for (int a = 0; a < nl; ++a) {
    const int m = H.leaf_size[a], ld = even_ld(m);
    R_off[a] = rtot;
    rtot += (int64_t)ld * ncols[a];
    R_col[a] = ctot;
    M_col[a] = ctot + m;
    ctot += ncols[a];
    M_off[a] = mtot;
    mtot += (int64_t)ld * (ncols[a] - m);
    LU_off[a] = lutot;
    lutot += (int64_t)m * m;
    Dinv_off[a] = ditot;
    ditot += (int64_t)ld * m;
    piv_off[a] = ptot;
    ptot += m;
  }
  // Near entries computed on the device (the handle keeps no host blocks):
  // the host packs only the far-factor columns of each panel, contiguous per
  // leaf (u_off), and lists the near blocks for the device fill.
  const bool dev_near = H.near_on_device;
  std::vector<int64_t> u_off(nl, 0);
  int64_t utot = 0;
  for (int a = 0; a < nl; ++a) {
    u_off[a] = utot;
    utot += (int64_t)even_ld(H.leaf_size[a]) * (ir_cols[a] + gl_cols[a]);
  }
  bigvec<double2> R((size_t)std::max<int64_t>(dev_near ? utot : rtot, 1));  // zeroed (pad rows stay 0)
  std::vector<int32_t> src((size_t)std::max<int64_t>(ctot, 1)), src_mm(src.size());
  bigvec<double2> D((size_t)(dev_near ? 0 : lutot));
  std::vector<std::vector<FillItem>> fills(nl);
#pragma omp parallel for schedule(dynamic, 1)
  for (int a = 0; a < nl; ++a) {
    const int m = H.leaf_size[a];
    const int64_t ld = even_ld(m), c_u = m + near_cols[a];
    // column c of the panel (near columns are not packed on the device path)
    auto col = [&](int64_t c) {
      return dev_near ? R.data() + u_off[a] + (c - c_u) * ld : R.data() + R_off[a] + c * ld;
    };
    int32_t* S = src.data() + R_col[a];
    int32_t* S2 = src_mm.data() + R_col[a];
    int64_t c = 0;
    auto put_block = [&](const NearBlock& nb) {
      const int n = H.leaf_size[nb.s_leaf];
      if (dev_near) fills[a].push_back({R_off[a] + c * ld, (int32_t)ld, a, nb.s_leaf, 0});
      for (int j = 0; j < n; ++j, ++c) {
        S[c] = S2[c] = H.leaf_off[nb.s_leaf] + j;
        if (dev_near) continue;
        const cplx* z = H.near_data.data() + nb.data + (size_t)j * m;
        double2* P = col(c);
        for (int i = 0; i < m; ++i) P[i] = make_double2(z[i].real(), z[i].imag());
      }
    };
    auto put_u = [&](int b, int row_in_block, int32_t src_base) {
      const int32_t src_mm_base = (int32_t)(N + gsm.tb[b]);
      const FarBlock& fb = H.far[b];
      const LowRank& lr = H.lowrank[fb.src];
      const std::vector<cplx>& U = fb.transposed ? lr.V : lr.U;  // m_b x r
      for (int q = 0; q < lr.r; ++q, ++c) {
        S[c] = src_base < 0 ? 0 : (int32_t)(src_base + q);
        S2[c] = src_mm_base + q;
        double2* P = col(c);
        for (int i = 0; i < m; ++i) {
          const cplx v = U[row_in_block + i + (size_t)q * fb.m];
          P[i] = make_double2(v.real(), v.imag());
        }
      }
    };
    put_block(H.near[diag_of[a]]);
    if (!dev_near) {
      const cplx* z = H.near_data.data() + H.near[diag_of[a]].data;
      for (int64_t e = 0; e < (int64_t)m * m; ++e) D[LU_off[a] + e] = make_double2(z[e].real(), z[e].imag());
    }
    for (int q : near_of[a]) put_block(H.near[q]);
    for (int b : inrow[a]) put_u(b, 0, -1);          // read from LDS, no source
    for (auto& sl : gslices[a]) put_u(sl.first, sl.second, (int32_t)(N + tb[sl.first]));
  }

  // kernels address one panel, W stack or group with 32-bit element offsets
  for (int a = 0; a < nl; ++a)
    if ((int64_t)even_ld(H.leaf_size[a]) * ncols[a] >= ((int64_t)1 << 31) ||
        (int64_t)ir_ld[a] * ir_ncol[a] >= ((int64_t)1 << 31)) {
      set_error("a leaf panel exceeds 2^31 elements");
      return HM_EINVAL;
    }
  for (const GroupSet* gs : {&gs1, &gsm})
    for (const Group& G : gs->groups)
      if ((int64_t)G.ld * G.n >= ((int64_t)1 << 31)) {
        set_error("a stage-A group exceeds 2^31 elements");
        return HM_EINVAL;
      }
  if (N + h->T >= ((int64_t)1 << 31)) {  // panel sources are 32-bit rows of [x | t]
    set_error("n plus the far-block coefficient count exceeds 2^31");
    return HM_EINVAL;
  }

  h->near_cols = near_cols;
  h->ir_cols = ir_cols;
  h->ir_ncol_h = ir_ncol;
  h->ir_end = ir_end;
  h->gl_end = gl_end;

  // ---- upload
  std::vector<int32_t> loff(H.leaf_off), lm(H.leaf_size);
  STCHK(upload(h, &h->perm, H.tree.perm, st));
  STCHK(upload(h, &h->leaf_off, loff, st));
  STCHK(upload(h, &h->leaf_m, lm, st));
  if (dev_near) {
    STCHK(fill_near_device(h, fills, R, u_off, near_cols, R_off, rtot, LU_off, lutot, st));
  } else {
    STCHK(upload(h, &h->R64, R, st, false, kPanelPad));
  }
  bigvec<double2>().swap(R);
  STCHK(upload(h, &h->src, src, st));
  STCHK(upload(h, &h->R_off, R_off, st));
  STCHK(upload(h, &h->R_col, R_col, st));
  STCHK(upload(h, &h->M_off, M_off, st));
  STCHK(upload(h, &h->M_col, M_col, st));
  STCHK(upload(h, &h->LU_off, LU_off, st));
  STCHK(upload(h, &h->Dinv_off, Dinv_off, st));
  STCHK(upload(h, &h->piv_off, piv_off, st));
  if (!dev_near) STCHK(upload(h, &h->LU, D, st));
  bigvec<double2>().swap(D);
  STCHK(upload(h, &h->W64, W, st));
  bigvec<double2>().swap(W);
  STCHK(upload(h, &h->groups, gs1.groups, st));
  STCHK(upload(h, &h->groups_mm, gsm.groups, st));
  STCHK(upload(h, &h->src_mm, src_mm, st));
  fill_W(gsm, W);
  STCHK(upload(h, &h->Wmm64, W, st, false, kPanelPad));
  bigvec<double2>().swap(W);
  STCHK(upload(h, &h->IR64, IR, st));
  bigvec<double2>().swap(IR);
  STCHK(upload(h, &h->ir_off, ir_off, st));
  STCHK(upload(h, &h->ir_ld, ir_ld, st));
  STCHK(upload(h, &h->ir_ncol, ir_ncol, st));
  STCHK(upload(h, &h->ir_row0, ir_row0, st));
  STCHK(upload(h, &h->ir_soff, ir_soff, st));
  STCHK(upload(h, &h->ir_n, ir_n, st));
  STCHK(dalloc(h, (void**)&h->Dinv, sizeof(double2) * std::max<int64_t>(ditot, 1) + kPanelPad));
  HIPCHK(hipMemsetAsync(h->Dinv, 0, sizeof(double2) * std::max<int64_t>(ditot, 1) + kPanelPad, st));
  STCHK(dalloc(h, (void**)&h->piv, sizeof(int32_t) * ptot));
  STCHK(dalloc(h, (void**)&h->M64, sizeof(double2) * std::max<int64_t>(mtot, 1) + kPanelPad));
  HIPCHK(hipMemsetAsync(h->M64, 0, sizeof(double2) * std::max<int64_t>(mtot, 1) + kPanelPad, st));

  build_mark(opts, st, "panels packed and uploaded");
  // ---- leaf LU with partial pivoting, then D^{-1} (eq. 12's near inverse)
  int* info = nullptr;
  STCHK(dalloc(h, (void**)&info, sizeof(int) * nl));
  HIPCHK(hipMemsetAsync(info, 0, sizeof(int) * nl, st));
  HIPCHK(launch_getrf(h->LU, h->LU_off, h->leaf_m, h->piv, h->piv_off, nl, info, st));
  HIPCHK(launch_getri(h->LU, h->LU_off, h->leaf_m, h->piv, h->piv_off, h->Dinv, h->Dinv_off, nl, st));
  std::vector<int> info_h(nl);
  HIPCHK(hipMemcpyAsync(info_h.data(), info, sizeof(int) * nl, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int a = 0; a < nl; ++a)
    if (info_h[a] != 0) {
      set_error("leaf block " + std::to_string(a) + " is singular");
      return HM_EINVAL;
    }

  build_mark(opts, st, "leaf LU and D^{-1} done");
  // ---- series panels M_a = D_a^{-1} [near | in-row U | global U] columns
  std::vector<int32_t> tiles, ncm(nl);
  for (int a = 0; a < nl; ++a) {
    ncm[a] = (int32_t)(ncols[a] - H.leaf_size[a]);
    for (int c = 0; c < ncm[a]; c += kPremulCols) { tiles.push_back(a); tiles.push_back(c); }
  }
  int32_t *d_tiles = nullptr, *d_ncm = nullptr;
  STCHK(upload(h, &d_tiles, tiles, st));
  STCHK(upload(h, &d_ncm, ncm, st));
  HIPCHK(launch_premul(h->Dinv, h->Dinv_off, h->R64, h->R_off, h->leaf_m, d_ncm, h->M64, h->M_off,
                       d_tiles, (int)(tiles.size() / 2), h->max_m, st));

  build_mark(opts, st, "premultiplied panels done");
  // ---- FP32 copies (same layout, pad rows stay zero)
  if (h->has_f32) {
    STCHK(dalloc(h, (void**)&h->R32, sizeof(float2) * std::max<int64_t>(rtot, 1) + kPanelPad));
    STCHK(dalloc(h, (void**)&h->M32, sizeof(float2) * std::max<int64_t>(mtot, 1) + kPanelPad));
    STCHK(dalloc(h, (void**)&h->W32, sizeof(float2) * std::max<int64_t>(wtot, 1)));
    STCHK(dalloc(h, (void**)&h->IR32, sizeof(float2) * std::max<int64_t>(irtot, 1)));
    STCHK(dalloc(h, (void**)&h->Wmm32, sizeof(float2) * std::max<int64_t>(wtot_mm, 1) + kPanelPad));
    HIPCHK(hipMemsetAsync(reinterpret_cast<char*>(h->R32) + sizeof(float2) * rtot, 0, kPanelPad, st));
    HIPCHK(hipMemsetAsync(reinterpret_cast<char*>(h->M32) + sizeof(float2) * mtot, 0, kPanelPad, st));
    HIPCHK(hipMemsetAsync(reinterpret_cast<char*>(h->Wmm32) + sizeof(float2) * wtot_mm, 0, kPanelPad,
                          st));
    HIPCHK(launch_cast(h->R64, h->R32, rtot, st));
    HIPCHK(launch_cast(h->M64, h->M32, mtot, st));
    HIPCHK(launch_cast(h->W64, h->W32, wtot, st));
    HIPCHK(launch_cast(h->IR64, h->IR32, irtot, st));
    HIPCHK(launch_cast(h->Wmm64, h->Wmm32, wtot_mm, st));
  }

  build_mark(opts, st, "FP32 copies done");
  // ---- stage-A items and entry counts per level
  h->sa.assign(h->nlev, GroupList());
  h->sa_mm.assign(h->nlev, GroupList());
  h->sa_mm_host.assign(h->nlev, std::vector<GroupItem>());
  h->group_mm_inst.assign(gsm.groups.size(), 0);
  for (size_t g = 0; g < gsm.groups.size(); ++g)
    h->group_mm_inst[g] = H.leaf_inst[H.tree.leaf_of[gsm.groups[g].s_off]];
  h->ent_R.assign(h->nlev, 0);
  h->ent_M.assign(h->nlev, 0);
  h->ent_W.assign(h->nlev, 0);
  h->ncoef.assign(h->nlev, 0);
  for (int li = 0; li < h->nlev; ++li) {
    int64_t eR = 0, eM = 0, eW = 0, nc = 0;
    for (int a = 0; a < nl; ++a) {
      const int64_t m = H.leaf_size[a];
      const int64_t cols = near_cols[a] + ir_end[li][a] + gl_end[li][a];
      eR += m * (m + cols);
      eM += m * cols;
    }
    std::vector<GroupItem> items, items_mm;
    for (int g = 0; g < ng; ++g) {
      const int rows = gs1.rows[g][li];
      for (int r0 = 0; r0 < rows; r0 += kGroupTile) items.push_back({g, r0, rows, 0});
    }
    for (int g = 0; g < (int)gsm.groups.size(); ++g) {
      const int rows = gsm.rows[g][li];
      eW += (int64_t)rows * gsm.groups[g].n;
      nc += rows;
      for (int r0 = 0; r0 < rows; r0 += kGroupTileMM) items_mm.push_back({g, r0, rows, 0});
    }
    STCHK(upload_groups(h, items, h->sa[li], st));
    STCHK(upload_groups(h, items_mm, h->sa_mm[li], st));
    h->sa_mm_host[li] = items_mm;
    h->ent_R[li] = eR;
    h->ent_M[li] = eM;
    h->ent_W[li] = eW;
    h->ncoef[li] = nc;
  }
  // counters and queue of the multi-term matrix-core launch (zero between launches)
  if (mm_wave_mode(h->max_m)) {
    const int64_t ncnt = (int64_t)(h->inst_off.size() - 1) * kMmSeriesMaxTerms * 2 + 3;
    STCHK(dalloc(h, (void**)&h->mm_cnt, sizeof(int32_t) * ncnt));
    HIPCHK(hipMemsetAsync(h->mm_cnt, 0, sizeof(int32_t) * ncnt, st));
    h->mm_queue = h->mm_cnt + ncnt - 3;
    h->mm_err = h->mm_cnt + ncnt - 1;
  }
  {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, h->device));
    const int occ = std::min(term_occupancy(false, h->max_m), term_occupancy(true, h->max_m));
    h->term_wgs_auto = std::max(1, prop.multiProcessorCount * occ);
    h->num_cus = std::max(1, prop.multiProcessorCount);
    h->term_wgs = h->term_wgs_auto;
    if (h->max_m <= kHalfMaxLeaf) {
      const int hocc = std::min(half_occupancy(false, h->max_m), half_occupancy(true, h->max_m));
      h->half_wgs_auto = std::max(1, prop.multiProcessorCount * hocc);
      const int mocc = std::min(half_occupancy(false, h->max_m, true), half_occupancy(true, h->max_m, true));
      h->half_wgs_multi = std::max(1, prop.multiProcessorCount * mocc);
    }
  }
  // ---- norm items: per instance (tree-order rows stay contiguous per
  // instance), rows in chunks of kNormRows
  {
    std::vector<NormItem> items;
    std::vector<int32_t> seg(1, 0);
    const int ns = (int)h->inst_off.size() - 1;
    if (ns < 1) { set_error("internal: no instance offsets"); return HM_EINVAL; }
    for (int g = 0; g < ns; ++g) {
      for (int64_t r = h->inst_off[g]; r < h->inst_off[g + 1]; r += kNormRows)
        items.push_back({r, std::min(r + kNormRows, h->inst_off[g + 1])});
      seg.push_back((int32_t)items.size());
    }
    h->nseg = ns;
    h->n_norm_items = (int)items.size();
    STCHK(upload(h, &h->norm_items, items, st));
    STCHK(upload(h, &h->norm_seg, seg, st));
  }
  {
    // half storage from the uploaded apply panels, stacks and groups
    const HalfSrc hs{&R_off, &ncols, &ir_off, &ir_ld, &ir_cols, &gs1.groups, &inrow};
    build_mark(opts, st, "work lists prepared");
    STCHK(build_half(h, hs, st));
    build_mark(opts, st, "half-storage data done");
  }
  STCHK(build_lists(h, st));
  HIPCHK(hipStreamSynchronize(st));
  return HM_OK;
}

int validate_problem(const hm_problem* p, const hm_build_opts* o) {
  if (!p || !o) { set_error("null problem or options"); return HM_EINVAL; }
  if (p->n < 1 || !p->xyz) { set_error("n must be >= 1 and xyz non-null"); return HM_EINVAL; }
  if (p->n > (int64_t)1 << 28) { set_error("n too large"); return HM_EINVAL; }
  if (p->kind != HM_SURFACE && p->kind != HM_VOLUME) { set_error("bad kind"); return HM_EINVAL; }
  if (p->kind == HM_VOLUME && !p->chi) { set_error("volume problem needs chi"); return HM_EINVAL; }
  if (!(p->k > 0) || !(p->h > 0)) { set_error("k and h must be > 0"); return HM_EINVAL; }
  if (o->leaf_max < 1 || o->leaf_max > 256) { set_error("leaf_max must be in [1, 256]"); return HM_EINVAL; }
  if (!(o->eta > 0) || !(o->aca_tol > 0) || o->aca_tol >= 1) {
    set_error("eta must be > 0 and aca_tol in (0, 1)");
    return HM_EINVAL;
  }
  if (o->max_rank < 0) { set_error("max_rank must be >= 0"); return HM_EINVAL; }
  for (int64_t i = 0; i < 3 * p->n; ++i)
    if (!std::isfinite(p->xyz[i])) { set_error("non-finite coordinate"); return HM_EINVAL; }
  if (p->kind == HM_VOLUME)
    for (int64_t i = 0; i < p->n; ++i)
      if (!(p->chi[i] != 0.0) || !std::isfinite(p->chi[i])) { set_error("chi must be finite and non-zero"); return HM_EINVAL; }
  return HM_OK;
}

void fill_info(const hm_matrix* h, hm_info* out) {
  std::memset(out, 0, sizeof(*out));
  const HostH& H = h->H;
  out->n = h->N;
  out->leaf_level = H.tree.depth;
  out->num_leaves = (int32_t)H.leaf_size.size();
  out->max_leaf = H.max_leaf;
  out->min_far_level = H.min_far_level;
  out->near_blocks = (int64_t)H.near.size();
  for (const auto& nb : H.near) {
    const int64_t e = (int64_t)H.leaf_size[nb.t_leaf] * H.leaf_size[nb.s_leaf];
    if (nb.t_leaf == nb.s_leaf) out->diag_entries += e; else out->near_offdiag_entries += e;
  }
  for (const auto& fb : H.far) {
    if (fb.level < 0 || fb.level >= HM_MAX_LEVELS) continue;
    const int r = H.lowrank[fb.src].r;
    out->far_blocks[fb.level] += 1;
    out->far_rank_sum[fb.level] += r;
    out->far_entries[fb.level] += (int64_t)r * (fb.m + fb.n);
  }
  out->device_bytes = h->bytes;
  out->build_ms = h->build_ms;
  out->num_instances = h->ninst;
  for (int li = 0; li < (int)h->ent_M.size(); ++li) {
    const int lev = (h->lmin < 0) ? h->L : h->lmin + li;
    if (lev < 0 || lev >= HM_MAX_LEVELS) continue;
    out->series_entries[lev] = h->ent_M[li];
    out->apply_entries[lev] = h->ent_R[li];
    out->stageA_entries[lev] = h->ent_W[li];
    out->coeffs[lev] = h->ncoef[li];
    if (li < (int)h->ent_half.size()) out->half_entries[lev] = h->ent_half[li];
  }
}

}  // namespace
}  // namespace hm

using namespace hm;

// ====================================================================== C-ABI
namespace hm {
// Host allocation failures inside a build surface as HM_ENOMEM.
template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    set_error("host memory exhausted during the build");
    return HM_ENOMEM;
  }
}
}  // namespace hm

// ====================================================================== no allocation
// Workspace of ps_solve_noalloc, for callers that cannot allocate device
// memory: a file-scope device array (static data of the code object, one
// copy per device, HM_NOALLOC_SCRATCH_BYTES bytes, held until the process
// ends).  In host code `scratch` names only a host-side stand-in; the
// array's device address on each device comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address
// reaches kernels.
static __device__ __align__(256) unsigned char scratch[HM_NOALLOC_SCRATCH_BYTES];

namespace hm {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device dev (the current device).
int scratch_address(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) { set_error("device index out of range"); return HM_EINVAL; }
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return HM_EHIP;
    }
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[dev];
  return HM_OK;
}

// The workspace buffers a series or fixed-pass refinement reads and writes.
struct WsView {
  double2 *xin0, *xin1, *xt, *bt, *rt, *dt, *partial, *xr64_0, *xr64_1;
  float2 *xr32_0, *xr32_1;
  int32_t* counters;
  int64_t ldr;
};

// Lays the workspace for nrhs right-hand sides out from base in 256-byte
// aligned pieces (base null: measures only); returns its size in bytes.
int64_t carve_workspace(const hm_matrix* h, int nrhs, unsigned char* base, WsView* v) {
  int64_t off = 0;
  auto take = [&](int64_t bytes) -> unsigned char* {
    unsigned char* q = base ? base + off : nullptr;
    off += (std::max<int64_t>(bytes, 16) + 255) / 256 * 256;
    return q;
  };
  const int64_t ldin = h->N + h->T, ldr = row_ld(nrhs);
  WsView w{};
  w.xin0 = (double2*)take(16 * ldin * nrhs);
  w.xin1 = (double2*)take(16 * ldin * nrhs);
  w.xr64_0 = (double2*)take(16 * (ldin + 1) * ldr);
  w.xr64_1 = (double2*)take(16 * (ldin + 1) * ldr);
  w.xr32_0 = (float2*)take(8 * (ldin + 1) * ldr);
  w.xr32_1 = (float2*)take(8 * (ldin + 1) * ldr);
  w.xt = (double2*)take(16 * h->N * nrhs);
  w.bt = (double2*)take(16 * h->N * nrhs);
  w.rt = (double2*)take(16 * h->N * nrhs);
  w.dt = (double2*)take(16 * h->N * nrhs);
  w.partial = (double2*)take(16 * h->partial_rows * ldr);
  w.counters = (int32_t*)take(4 * counter_count(h, nrhs));
  w.ldr = ldr;
  if (v) *v = w;
  return off;
}

// Points the handle's workspace fields at a WsView for the length of a
// call, then restores them.
struct WsSwap {
  hm_matrix* h;
  WsView saved;
  WsSwap(hm_matrix* h_, const WsView& w) : h(h_) {
    saved = WsView{h->xin0, h->xin1, h->xt, h->bt, h->rt, h->dt, h->partial, h->xr64_0,
                   h->xr64_1, h->xr32_0, h->xr32_1, h->counters, h->ws_ldr};
    set(w);
  }
  void set(const WsView& w) {
    h->xin0 = w.xin0; h->xin1 = w.xin1; h->xt = w.xt; h->bt = w.bt; h->rt = w.rt; h->dt = w.dt;
    h->partial = w.partial; h->xr64_0 = w.xr64_0; h->xr64_1 = w.xr64_1; h->xr32_0 = w.xr32_0;
    h->xr32_1 = w.xr32_1; h->counters = w.counters; h->ws_ldr = w.ldr;
  }
  ~WsSwap() { set(saved); }
};

}  // namespace
}  // namespace hm

extern "C" {

const char* hm_last_error(void) { return g_err.c_str(); }

const char* hm_strerror(int s) {
  switch (s) {
    case HM_OK: return "ok";
    case HM_ENOTREADY: return "not ready";
    case HM_EDIVERGED: return "series diverged";
    case HM_EINVAL: return "invalid argument";
    case HM_ENOMEM: return "out of device memory";
    case HM_EHIP: return "HIP runtime error";
    case HM_EBUSY: return "busy";
    case HM_ESTATE: return "invalid handle state";
    default: return "unknown status";
  }
}

static void report(const hm_build_opts* o, const std::string& msg) {
  if (o->progress) o->progress(msg.c_str(), o->progress_user);
}

static Problem copy_problem(const hm_problem* prob) {
  Problem p;
  p.n = prob->n;
  p.kind = prob->kind;
  p.k = prob->k;
  p.h = prob->h;
  p.xyz.assign(prob->xyz, prob->xyz + 3 * prob->n);
  if (prob->kind == HM_VOLUME) p.chi.assign(prob->chi, prob->chi + prob->n);
  return p;
}

// Device part of a build, shared by the single and batched builds.
// Fields derived from the host part, then the device part of a build.
static void prepare_fields(hm_matrix* h, const hm_build_opts* opts) {
  h->N = h->H.prob.n;
  h->nl = (int)h->H.leaf_size.size();
  h->max_m = h->H.max_leaf;
  h->L = h->H.tree.depth;
  h->lmin = h->H.min_far_level;
  h->host_only = (opts->flags & HM_BUILD_HOST_ONLY) != 0;
  h->has_f32 = (opts->flags & HM_BUILD_NO_F32) == 0;
  h->want_half = (opts->flags & HM_BUILD_NO_HALF) == 0;
}

static int device_part(hm_matrix* h, const hm_build_opts* opts, void* hip_stream) {
  std::string arch;
  if (!check_arch(&arch)) {
    set_error("no usable gfx950 device (found '" + arch + "')");
    return HM_EHIP;
  }
  HIPCHK(hipGetDevice(&h->device));
  if (h->H.aca_pending) {
    report(opts, "host build done, compressing far blocks on the device");
    STCHK(device_aca(h->H, *opts, (hipStream_t)hip_stream));
  }
  report(opts, "packing and uploading blocks");
  STCHK(build_device(h, opts, (hipStream_t)hip_stream));
  report(opts, "device build done");
  if (!(opts->flags & HM_BUILD_KEEP_HOST)) {
    bigvec<cplx>().swap(h->H.near_data);
    for (auto& lr : h->H.lowrank) {
      std::vector<cplx>().swap(lr.U);
      std::vector<cplx>().swap(lr.V);
    }
    h->host_kept = false;
  }
  return HM_OK;
}

static int finish_build(std::unique_ptr<hm_matrix>& h, const hm_build_opts* opts, void* hip_stream,
                        std::chrono::steady_clock::time_point t0, hm_matrix_t* out) {
  prepare_fields(h.get(), opts);
  if (!h->host_only) STCHK(device_part(h.get(), opts, hip_stream));
  h->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h.release();
  return HM_OK;
}

static int hmat_build_impl(const hm_problem* prob, const hm_build_opts* opts, void* hip_stream,
                           hm_matrix_t* out) {
  if (!out) { set_error("null output handle"); return HM_EINVAL; }
  *out = nullptr;
  STCHK(validate_problem(prob, opts));
  const auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<hm_matrix> h(new hm_matrix());
  STCHK(build_host(copy_problem(prob), *opts, h->H));
  h->inst_off = {0, prob->n};
  return finish_build(h, opts, hip_stream, t0, out);
}

static int hmat_build_batched_impl(const hm_problem* probs, int32_t count,
                                   const hm_build_opts* opts, void* hip_stream,
                                   hm_matrix_t* out) {
  if (!out) { set_error("null output handle"); return HM_EINVAL; }
  *out = nullptr;
  if (!probs || count < 1) { set_error("need count >= 1 problems"); return HM_EINVAL; }
  int64_t total = 0;
  for (int32_t i = 0; i < count; ++i) {
    STCHK(validate_problem(&probs[i], opts));
    total += probs[i].n;
  }
  if (total > (int64_t)1 << 28) { set_error("total n too large"); return HM_EINVAL; }
  const auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<hm_matrix> h(new hm_matrix());
  // instances one after another, each with the build's threads (the block
  // loops inside an instance parallelise well; instances in parallel
  // contend on the allocator and page faults)
  std::vector<HostH> parts(count);
  int64_t done_n = 0;
  for (int32_t i = 0; i < count; ++i) {
    const int st = build_host(copy_problem(&probs[i]), *opts, parts[i]);
    if (st != HM_OK) {
      set_error("instance " + std::to_string(i) + ": " + hm_last_error());
      return st;
    }
    done_n += probs[i].n;
    if (i + 1 == count || (i + 1) % 32 == 0)
      report(opts, "host blocks of " + std::to_string(i + 1) + " of " + std::to_string(count) +
                       " instances (" + std::to_string(done_n) + " of " + std::to_string(total) +
                       " points)");
  }
  merge_hosts(parts, h->H, h->inst_off);
  report(opts, "instances merged");
  h->ninst = count;
  return finish_build(h, opts, hip_stream, t0, out);
}

int hmat_build(const hm_problem* prob, const hm_build_opts* opts, void* hip_stream,
               hm_matrix_t* out) {
  return guarded([&] { return hmat_build_impl(prob, opts, hip_stream, out); });
}

int hmat_build_batched(const hm_problem* probs, int32_t count, const hm_build_opts* opts,
                       void* hip_stream, hm_matrix_t* out) {
  return guarded([&] { return hmat_build_batched_impl(probs, count, opts, hip_stream, out); });
}

int hmat_info(hm_matrix_t h, hm_info* out) {
  if (!h || !out) { set_error("null argument"); return HM_EINVAL; }
  fill_info(h, out);
  return HM_OK;
}

int hmat_apply(hm_matrix_t h, int32_t level, int32_t precision, const void* x_dev, int64_t ldx,
               void* y_dev, int64_t ldy, int32_t nrhs, void* hip_stream) {
  if (!h) { set_error("null handle"); return HM_EINVAL; }
  if (h->host_only) { set_error("handle was built host-only"); return HM_ESTATE; }
  if (nrhs < 0 || (nrhs > 0 && (!x_dev || !y_dev)) || ldx < h->N || ldy < h->N) {
    set_error("bad vector arguments");
    return HM_EINVAL;
  }
  if (precision != HM_F64 && precision != HM_F32_APPLY) { set_error("bad precision"); return HM_EINVAL; }
  const bool f32 = precision == HM_F32_APPLY;
  if (f32 && !h->has_f32) { set_error("FP32 copies were not kept"); return HM_ESTATE; }
  if (nrhs == 0) return HM_OK;
  int li = 0;
  STCHK(level_index(h, level, &li));
  HIPCHK(hipSetDevice(h->device));
  hipStream_t st = (hipStream_t)hip_stream;
  STCHK(ensure_workspace(h, nrhs, st));
  const int64_t ldin = h->N + h->T;
  HIPCHK(launch_permute_in((const double2*)x_dev, ldx, h->perm, h->xin0, ldin, h->N, nrhs, st));
  STCHK(apply_core(h, li, f32, nrhs, 1.0, 0.0, nullptr, nullptr, (double2*)y_dev, ldy, st));
  return HM_OK;
}

// ps_solve's body; own_ws: size the handle's own workspace (otherwise the
// caller has pointed the workspace fields at memory it provides).
static int ps_solve_impl(hm_matrix_t h, const ps_opts* o, const void* b_dev, int64_t ldb,
                         void* x_dev, int64_t ldx, int32_t nrhs, ps_stats* per_rhs,
                         void* hip_stream, bool own_ws) {
  if (!h || !o) { set_error("null argument"); return HM_EINVAL; }
  if (h->host_only) { set_error("handle was built host-only"); return HM_ESTATE; }
  if (nrhs < 0 || (nrhs > 0 && (!b_dev || !x_dev)) || ldb < h->N || ldx < h->N) {
    set_error("bad vector arguments");
    return HM_EINVAL;
  }
  if (o->K < 0 || o->K > 10000) { set_error("K must be in [0, 10000]"); return HM_EINVAL; }
  if (o->precision != HM_F64 && o->precision != HM_F32_APPLY) { set_error("bad precision"); return HM_EINVAL; }
  if (o->kind != PS_SERIES && o->kind != PS_REFINE && o->kind != PS_REFINE_FIXED &&
      o->kind != PS_GMRES && o->kind != PS_NESTED) {
    set_error("bad kind");
    return HM_EINVAL;
  }
  if (o->kind == PS_NESTED && h->nseg != 1) {
    set_error("the nested solve takes single-instance handles only");
    return HM_EINVAL;
  }
  if (o->kind == PS_GMRES) {
    if (o->max_passes < 1 || !(o->refine_tol > 0) || o->restart < 0 || o->restart > kMaxKrylov) {
      set_error("GMRES needs max_passes >= 1, refine_tol > 0 and restart in [0, 64]");
      return HM_EINVAL;
    }
  }
  const bool refine = o->kind == PS_REFINE || o->kind == PS_REFINE_FIXED,
             adaptive = o->kind == PS_REFINE;
  if (refine && (o->max_passes < 0 || !(o->refine_tol > 0))) {
    set_error("refinement needs max_passes >= 0 and refine_tol > 0");
    return HM_EINVAL;
  }
  const bool f32 = o->precision == HM_F32_APPLY;
  if (f32 && !h->has_f32) { set_error("FP32 copies were not kept"); return HM_ESTATE; }
  if (nrhs == 0) return HM_OK;
  int li = 0;
  STCHK(level_index(h, o->level, &li));
  HIPCHK(hipSetDevice(h->device));
  hipStream_t st = (hipStream_t)hip_stream;
  if (own_ws) STCHK(ensure_workspace(h, nrhs, st));
  const int64_t N = h->N, ldin = h->N + h->T;
  const int ns = h->nseg;
  // host reads of norms happen only with stats or adaptive refinement;
  // otherwise the call only enqueues work (a stream capture can record it)
  const bool want = per_rhs != nullptr || adaptive;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (per_rhs) {
    HIPCHK(hipEventCreate(&ev0));
    HIPCHK(hipEventCreate(&ev1));
    HIPCHK(hipEventRecord(ev0, st));
  }
  // a multi-term launch (half storage or matrix cores) that gave up a
  // dependency wait (a list inconsistent with its data; never expected) is
  // reported by the calls that synchronise
  auto multi_ok = [&]() -> int {
    for (int32_t* flag : {h->herr, h->mm_err}) {
      if (!flag) continue;
      int32_t e = 0;
      HIPCHK(hipMemcpyAsync(&e, flag, sizeof(e), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (e == 0) continue;
      HIPCHK(hipMemsetAsync(flag, 0, sizeof(e), st));
      set_error("multi-term launch: a dependency wait gave up");
      return HM_EHIP;
    }
    return HM_OK;
  };
  if (o->kind == PS_NESTED) {
    STCHK(nested_solve(h, o->level, f32, o->K, (const double2*)b_dev, ldb, (double2*)x_dev, ldx,
                       nrhs, st));
    if (per_rhs) {
      float ms = 0;
      HIPCHK(hipEventRecord(ev1, st));
      HIPCHK(hipEventSynchronize(ev1));
      HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
      (void)hipEventDestroy(ev0);
      (void)hipEventDestroy(ev1);
      for (int c = 0; c < nrhs; ++c) per_rhs[c] = ps_stats{0, 0, 0.0, 0.0, ms, 0, 0};
    }
    return HM_OK;
  }
  if (o->kind == PS_GMRES) {
    const int m = gmres_restart(*o);
    std::vector<int> it;
    std::vector<double> rr;
    STCHK(gmres_solve(h, li, f32, o->K, m, o->max_passes, o->refine_tol, (const double2*)b_dev,
                      ldb, (double2*)x_dev, ldx, nrhs, it, rr, st));
    STCHK(multi_ok());
    int status = HM_OK;
    float ms = 0;
    if (per_rhs) {
      HIPCHK(hipEventRecord(ev1, st));
      HIPCHK(hipEventSynchronize(ev1));
      HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
      (void)hipEventDestroy(ev0);
      (void)hipEventDestroy(ev1);
    }
    for (int c = 0; c < nrhs; ++c) {
      const bool bad = !(rr[c] <= o->refine_tol);
      if (bad) status = HM_EDIVERGED;
      if (!per_rhs) continue;
      ps_stats& s = per_rhs[c];
      s.passes = it[c];
      s.growth = 0.0;
      s.resid_rel = rr[c];
      s.t_ms = ms;
      s.diverged = bad ? 1 : 0;
    }
    return status;
  }
  // one right-hand side of a symmetric problem refines in the scaled basis
  const bool scaled = refine && use_half(h, li, nrhs);
  if (refine) {
    HIPCHK(launch_permute_in((const double2*)b_dev, ldb, h->perm, h->bt, N, N, nrhs, st));
    if (scaled)
      STCHK(scaled_refine_init(h, li, f32, o->K, want, st));
    else
      STCHK(series_core(h, li, f32, o->K, h->bt, N, false, h->xt, nullptr, 0, nrhs, want, st));
  } else {
    STCHK(series_core(h, li, f32, o->K, (const double2*)b_dev, ldb, true, h->xt, (double2*)x_dev,
                      ldx, nrhs, want, st));
  }
  std::vector<double> growth(nrhs, 0.0), resid(nrhs, 0.0);
  std::vector<int> passes(nrhs, 0), done(nrhs, 0), rising(nrhs, 0);
  std::vector<double> prev_d((size_t)ns * nrhs, INFINITY);  // ||d|| per (column, instance)
  auto read_norms = [&]() -> int {
    HIPCHK(hipMemcpyAsync(h->norms_host, h->norms, sizeof(double) * 2 * ns * nrhs,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return HM_OK;
  };
  // max over instances of sqrt(slot 1 / slot 0) for column c
  auto ratio = [&](int c) {
    double r = 0.0;
    for (int g = 0; g < ns; ++g) {
      const double a = std::sqrt(h->norms_host[(int64_t)c * ns + g]);
      const double b = std::sqrt(h->norms_host[(int64_t)(nrhs + c) * ns + g]);
      // a non-finite norm (NaN or inf in the column) makes the ratio NaN
      const double q = !(std::isfinite(a) && std::isfinite(b)) ? NAN
                       : (a > 0) ? b / a : (b > 0 ? INFINITY : 0.0);
      if (!(q <= r)) r = q;  // keeps NaN / inf
    }
    return r;
  };
  if (want) {
    STCHK(read_norms());
    for (int c = 0; c < nrhs; ++c) growth[c] = ratio(c);
  }
  for (int pass = 1; refine && pass <= o->max_passes; ++pass) {
    const bool check = adaptive || (per_rhs && pass == o->max_passes);
    if (scaled) {
      STCHK(scaled_refine_pass(h, li, f32, o->K, check, st));
    } else {
      // r = b - Z_l x in FP64 (all blocks including D)
      HIPCHK(launch_axpy(1.0, h->xt, N, h->xin0, ldin, N, nrhs, 0, st));
      STCHK(apply_core(h, li, false, nrhs, -1.0, 1.0, h->bt, h->rt, nullptr, 0, st));
      // d = P_K r, x += d
      STCHK(series_core(h, li, f32, o->K, h->rt, N, false, h->dt, nullptr, 0, nrhs, false, st));
      HIPCHK(launch_axpy(1.0, h->dt, N, h->xt, N, N, nrhs, 1, st));
    }
    if (!check) continue;
    HIPCHK(norms_into(h, h->xt, N, nrhs, 0, st));
    HIPCHK(norms_into(h, scaled ? h->rt : h->dt, N, nrhs, 1, st));
    STCHK(read_norms());
    bool all = true;
    for (int c = 0; c < nrhs; ++c) {
      const double rel = ratio(c);  // max over instances of |d| / |x|
      // a correction whose norm grew (for some instance not yet within the
      // tolerance) five passes in a row means the series does not contract
      // (rho^(K+1) >= 1): stop, reported as diverged
      bool grew = false;
      for (int g = 0; g < ns; ++g) {
        const double xn = std::sqrt(h->norms_host[(int64_t)c * ns + g]);
        const double dn = std::sqrt(h->norms_host[(int64_t)(nrhs + c) * ns + g]);
        double& pd = prev_d[(size_t)c * ns + g];
        // instances already within the tolerance sit at their rounding
        // floor, where the correction no longer shrinks: they do not count
        const bool open = !(dn <= o->refine_tol * xn);
        if (open && !(dn < pd)) grew = true;
        pd = dn;
      }
      if (!done[c]) {
        rising[c] = grew ? rising[c] + 1 : 0;
        resid[c] = rel;
        passes[c] = pass;
        if (rel <= o->refine_tol || (adaptive && rising[c] >= 5)) done[c] = 1;
      }
      all = all && done[c];
    }
    if (adaptive && all) break;
  }
  if (scaled) {  // x = C^{-T} xhat, in original order
    HIPCHK(block_pass(h, chat_set(h, true), h->zbuf, N, false, nullptr, 0, h->xt, 0,
                      (double2*)x_dev, ldx, st));
    if (want) {
      // check of the scaled basis from the unscaled operator: the next
      // correction P_K (b - Z_l x) with the FP64 H-matvec and the pivoted
      // LU's panels; its size relative to x joins the reported correction
      HIPCHK(launch_permute_in((const double2*)b_dev, ldb, h->perm, h->rt, N, N, nrhs, st));
      HIPCHK(launch_axpy(1.0, h->xt, N, h->xin0, ldin, N, nrhs, 0, st));
      STCHK(apply_core(h, li, false, nrhs, -1.0, 1.0, h->rt, h->bt, nullptr, 0, st));
      STCHK(series_core(h, li, f32, o->K, h->bt, N, false, h->dt, nullptr, 0, nrhs, false, st,
                        false));
      HIPCHK(norms_into(h, h->xt, N, nrhs, 0, st));
      HIPCHK(norms_into(h, h->dt, N, nrhs, 1, st));
      STCHK(read_norms());
      for (int c = 0; c < nrhs; ++c) {
        const double rel = ratio(c);
        if (!(rel <= resid[c])) resid[c] = rel;
      }
    }
  } else if (refine)
    HIPCHK(launch_permute_out(h->xt, N, h->perm, (double2*)x_dev, ldx, N, nrhs, st));
  int status = HM_OK;
  if (want) STCHK(multi_ok());
  if (per_rhs) {
    HIPCHK(hipEventRecord(ev1, st));
    HIPCHK(hipEventSynchronize(ev1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    for (int c = 0; c < nrhs; ++c) {
      ps_stats& s = per_rhs[c];
      s.passes = passes[c];
      s.growth = growth[c];
      s.resid_rel = resid[c];
      s.t_ms = ms;
      const bool bad = !(growth[c] <= 1.0) || (refine && !(resid[c] <= o->refine_tol));
      s.diverged = bad ? 1 : 0;
      if (bad) status = HM_EDIVERGED;
    }
  }
  return status;
}

int ps_solve(hm_matrix_t h, const ps_opts* o, const void* b_dev, int64_t ldb, void* x_dev,
             int64_t ldx, int32_t nrhs, ps_stats* per_rhs, void* hip_stream) {
  return ps_solve_impl(h, o, b_dev, ldb, x_dev, ldx, nrhs, per_rhs, hip_stream, true);
}

int hmat_export(hm_matrix_t h, const char* path) {
  if (!h || !path) { set_error("null argument"); return HM_EINVAL; }
  if (!h->host_kept) { set_error("host blocks were released (build with HM_BUILD_KEEP_HOST)"); return HM_ESTATE; }
  if (h->host_only) return export_host(h->H, path, nullptr, nullptr);
  HIPCHK(hipSetDevice(h->device));
  int64_t dtot = 0;
  for (int a = 0; a < h->nl; ++a) dtot += (int64_t)h->H.leaf_size[a] * h->H.leaf_size[a];
  std::vector<cplx> lu((size_t)dtot);
  std::vector<int32_t> piv((size_t)h->N);
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(lu.data(), h->LU, sizeof(cplx) * dtot, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(piv.data(), h->piv, sizeof(int32_t) * h->N, hipMemcpyDeviceToHost));
  return export_host(h->H, path, &lu, &piv);
}

int hmat_tune(hm_matrix_t h, const hm_tuning* t, void* hip_stream) {
  if (!h || !t) { set_error("null argument"); return HM_EINVAL; }
  if (h->host_only) { set_error("handle was built host-only"); return HM_ESTATE; }
  if (t->mm_min_rhs < -1 || t->term_wgs < -1 || t->term_wgs > (1 << 20) ||
      !(t->rhs_tile == -1 || t->rhs_tile == 0 || t->rhs_tile == 16 || t->rhs_tile == 32 ||
        t->rhs_tile == 64)) {
    set_error("bad tuning values");
    return HM_EINVAL;
  }
  if (t->half_storage < -1 || t->half_storage > 3) {
    set_error("bad tuning values");
    return HM_EINVAL;
  }
  if (t->half_storage > 0) h->use_half = t->half_storage;
  if (t->half_storage == -1) h->use_half = 1;
  if (t->mm_multi < -1 || t->mm_multi > 2) {
    set_error("bad tuning values");
    return HM_EINVAL;
  }
  if (t->mm_multi > 0) h->mm_multi_mode = t->mm_multi;
  if (t->mm_multi == -1) h->mm_multi_mode = 2;
  if (t->inrow_pct < -1 || t->inrow_pct > 1000) {
    set_error("bad tuning values");
    return HM_EINVAL;
  }
  if (t->mm_min_rhs > 0) h->mm_min_rhs = t->mm_min_rhs;
  if (t->mm_min_rhs == -1) h->mm_min_rhs = kMmMinRhsDefault;
  if (t->rhs_tile > 0) h->rhs_tile = t->rhs_tile;
  if (t->rhs_tile == -1) h->rhs_tile = 0;
  int wgs = h->term_wgs;
  if (t->term_wgs > 0) wgs = t->term_wgs;
  if (t->term_wgs == -1) wgs = h->term_wgs_auto;
  int pct = h->inrow_pct;
  if (t->inrow_pct > 0) pct = t->inrow_pct;
  if (t->inrow_pct == -1) pct = 100;
  if (wgs != h->term_wgs || pct != h->inrow_pct) {
    HIPCHK(hipSetDevice(h->device));
    h->term_wgs = wgs;
    h->inrow_pct = pct;
    STCHK(build_lists(h, (hipStream_t)hip_stream));
  }
  return HM_OK;
}

int hmat_get_tuning(hm_matrix_t h, hm_tuning* out) {
  if (!h || !out) { set_error("null argument"); return HM_EINVAL; }
  out->mm_min_rhs = h->mm_min_rhs;
  out->term_wgs = h->term_wgs;
  out->rhs_tile = h->rhs_tile;
  out->inrow_pct = h->inrow_pct;
  out->half_storage = h->use_half;
  out->mm_multi = h->mm_multi_mode;
  return HM_OK;
}

// Times ps_solve (series kind) for every candidate tuning on zero vectors
// of nrhs columns and keeps the fastest (median of 5 timed calls after 2).
int hmat_autotune(hm_matrix_t h, const ps_opts* opts, int32_t nrhs, void* hip_stream,
                  hm_tuning* best, double* best_ms) {
  if (!h || !opts || nrhs < 1) { set_error("null argument or nrhs < 1"); return HM_EINVAL; }
  if (h->host_only) { set_error("handle was built host-only"); return HM_ESTATE; }
  HIPCHK(hipSetDevice(h->device));
  hipStream_t st = (hipStream_t)hip_stream;
  ps_opts o = *opts;
  o.kind = PS_SERIES;
  void *b = nullptr, *x = nullptr;
  const size_t bytes = sizeof(double2) * (size_t)h->N * nrhs;
  HIPCHK(hipMalloc(&b, bytes));
  if (hipMalloc(&x, bytes) != hipSuccess) { (void)hipFree(b); set_error("hipMalloc failed"); return HM_ENOMEM; }
  struct Buf { void *b, *x; ~Buf() { (void)hipFree(b); (void)hipFree(x); } } bufs{b, x};
  HIPCHK(hipMemsetAsync(b, 0, bytes, st));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  struct Ev { hipEvent_t a, b; ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } evs{e0, e1};
  auto time_one = [&](double* ms) -> int {
    for (int r = 0; r < 2; ++r) STCHK(ps_solve(h, &o, b, h->N, x, h->N, nrhs, nullptr, st));
    std::vector<double> t;
    for (int r = 0; r < 5; ++r) {
      HIPCHK(hipEventRecord(e0, st));
      STCHK(ps_solve(h, &o, b, h->N, x, h->N, nrhs, nullptr, st));
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      float f = 0;
      HIPCHK(hipEventElapsedTime(&f, e0, e1));
      t.push_back(f);
    }
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return HM_OK;
  };
  const int autow = h->term_wgs_auto;
  std::vector<int> wgs = {autow, std::max(1, autow / 2), 2 * autow, 4 * autow};
  // the matrix-core kernels hold one or two workgroups per compute unit
  if (nrhs >= 2)
    for (int w : {h->num_cus, 2 * h->num_cus})
      if (std::find(wgs.begin(), wgs.end(), w) == wgs.end()) wgs.push_back(w);
  // in-row weights matter only for the streaming kernels' work split
  std::vector<int> pcts = {100, 150, 200};
  struct Cand { int mm_min, tile; };
  std::vector<Cand> paths = {{1 << 30, 0}};  // streaming kernels
  if (nrhs >= 2) {
    paths.push_back({1, 16});
    if (nrhs > 16) paths.push_back({1, 32});
    if (nrhs > 32) paths.push_back({1, 64});
  }
  // one right-hand side of a symmetric problem: the half-storage product
  // too; with more right-hand sides the setting does not enter the timed
  // solves and keeps its value (it serves later one-RHS calls)
  std::vector<int> halves = {nrhs == 1 ? 2 : h->use_half};
  if (nrhs == 1 && h->half_ok) halves.push_back(1);
  // the matrix-core candidates with the K terms in one launch and per term
  const int multi0 = h->mm_multi_mode;
  hm_tuning bt{h->mm_min_rhs, h->term_wgs, h->rhs_tile, h->inrow_pct, halves[0], multi0};
  double bms = INFINITY;
  for (int w : wgs) {
    for (int pct : pcts) {
      if (w != h->term_wgs || pct != h->inrow_pct) {
        h->term_wgs = w;
        h->inrow_pct = pct;
        STCHK(build_lists(h, st));
      }
      for (int hs : halves) {
        h->use_half = hs;
        for (const Cand& c : paths) {
          if (pct != 100 && c.mm_min == 1) continue;  // MFMA lists have no in-row rows
          if (nrhs == 1 && hs == 1 && c.mm_min == 1) continue;  // the half product is one-RHS only
          h->mm_min_rhs = c.mm_min;
          h->rhs_tile = c.tile;
          const std::vector<int> multis = c.mm_min == 1 && h->mm_cnt ? std::vector<int>{1, 2}
                                                                      : std::vector<int>{multi0};
          for (int mu : multis) {
            h->mm_multi_mode = mu;
            double ms = 0;
            STCHK(time_one(&ms));
            if (ms < bms) {
              bms = ms;
              // the MFMA kernels were timed at nrhs only: they take over from
              // min(nrhs, the default threshold) on, so one right-hand side
              // (a GEMV, far below the MFMA ridge) keeps the streaming kernels
              bt = hm_tuning{c.mm_min == 1 ? std::min(nrhs, kMmMinRhsDefault) : nrhs + 1, w, c.tile,
                             pct, hs, mu};
            }
          }
        }
      }
    }
  }
  h->use_half = bt.half_storage;
  h->mm_min_rhs = bt.mm_min_rhs;
  h->rhs_tile = bt.rhs_tile;
  h->mm_multi_mode = bt.mm_multi;
  if (h->term_wgs != bt.term_wgs || h->inrow_pct != bt.inrow_pct) {
    h->term_wgs = bt.term_wgs;
    h->inrow_pct = bt.inrow_pct;
    STCHK(build_lists(h, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  if (best) *best = bt;
  if (best_ms) *best_ms = bms;
  return HM_OK;
}

int hm_profile_enable(hm_matrix_t h, int32_t enable) {
  if (!h) { set_error("null handle"); return HM_EINVAL; }
  if (h->host_only) { set_error("handle was built host-only"); return HM_ESTATE; }
  HIPCHK(hipSetDevice(h->device));
  HIPCHK(hipDeviceSynchronize());
  for (auto& r : h->prof_recs) { h->ev_pool.push_back(r.e0); h->ev_pool.push_back(r.e1); }
  h->prof_recs.clear();
  h->prof = enable != 0;
  return HM_OK;
}

int hm_profile_read(hm_matrix_t h, hm_kernel_time* out) {
  if (!h || !out) { set_error("null argument"); return HM_EINVAL; }
  for (int c = 0; c < HM_K_COUNT; ++c) out[c] = hm_kernel_time{0, 0.0};
  for (auto& r : h->prof_recs) {
    HIPCHK(hipEventSynchronize(r.e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, r.e0, r.e1));
    out[r.cls].launches += 1;
    out[r.cls].total_ms += ms;
  }
  return HM_OK;
}

int ps_solve_noalloc(hm_matrix_t h, const ps_opts* o, const void* b_dev, int64_t ldb,
                     void* x_dev, int64_t ldx, int32_t nrhs, void* hip_stream) {
  if (!h || !o) { set_error("null argument"); return HM_EINVAL; }
  if (h->host_only) { set_error("handle was built host-only"); return HM_ESTATE; }
  if (o->kind != PS_SERIES && o->kind != PS_REFINE_FIXED) {
    set_error("ps_solve_noalloc takes PS_SERIES and PS_REFINE_FIXED only");
    return HM_EINVAL;
  }
  if (nrhs <= 0) return nrhs == 0 ? HM_OK : (set_error("nrhs must be >= 0"), HM_EINVAL);
  const int64_t need = carve_workspace(h, nrhs, nullptr, nullptr);
  if (need > (int64_t)HM_NOALLOC_SCRATCH_BYTES) {
    set_error("ps_solve_noalloc: the workspace of " + std::to_string(nrhs) +
              " right-hand sides needs " + std::to_string(need) + " bytes, more than the " +
              std::to_string((int64_t)HM_NOALLOC_SCRATCH_BYTES) + "-byte static scratch");
    return HM_EINVAL;
  }
  HIPCHK(hipSetDevice(h->device));
  unsigned char* base = nullptr;
  STCHK(scratch_address(h->device, &base));
  WsView w{};
  carve_workspace(h, nrhs, base, &w);
  hipStream_t st = (hipStream_t)hip_stream;
  // the split-K counters must start at zero (the array keeps the last call's
  // contents); a fill kernel, not a memset node, so the call stays capturable
  HIPCHK(zero_words(w.counters, counter_count(h, nrhs), st));
  // the zero rows of the row-layout vectors (as 32-bit words)
  const int64_t ldin = h->N + h->T;
  for (void* zr : {(void*)(w.xr64_0 + ldin * w.ldr), (void*)(w.xr64_1 + ldin * w.ldr)})
    HIPCHK(zero_words(zr, 4 * w.ldr, st));
  for (void* zr : {(void*)(w.xr32_0 + ldin * w.ldr), (void*)(w.xr32_1 + ldin * w.ldr)})
    HIPCHK(zero_words(zr, 2 * w.ldr, st));
  WsSwap swap(h, w);
  return ps_solve_impl(h, o, b_dev, ldb, x_dev, ldx, nrhs, nullptr, hip_stream, false);
}

int hmat_free(hm_matrix_t h) {
  if (!h) return HM_OK;
  if (!h->host_only && h->device >= 0) {
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
  }
  delete h;
  return HM_OK;
}

}  // extern "C"

namespace hm {

int build_host_phase(const hm_problem* prob, const hm_build_opts* opts, hm_matrix_t* out) {
  return guarded([&]() -> int {
    if (!out) { set_error("null output handle"); return HM_EINVAL; }
    *out = nullptr;
    STCHK(validate_problem(prob, opts));
    std::unique_ptr<hm_matrix> h(new hm_matrix());
    const auto t0 = std::chrono::steady_clock::now();
    STCHK(build_host(copy_problem(prob), *opts, h->H));
    if (h->H.aca_pending) {
      // the far blocks are compressed here, so that the device bytes of the
      // handle are known before its device part is built
      std::string arch;
      if (!check_arch(&arch)) {
        set_error("no usable gfx950 device (found '" + arch + "')");
        return HM_EHIP;
      }
      hipStream_t st = nullptr;
      HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      const int s = device_aca(h->H, *opts, st);
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
      STCHK(s);
    }
    h->inst_off = {0, prob->n};
    hm_build_opts o = *opts;
    o.flags &= ~HM_BUILD_HOST_ONLY;
    prepare_fields(h.get(), &o);
    h->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h.release();
    return HM_OK;
  });
}

int build_device_phase(hm_matrix_t h, const hm_build_opts* opts, void* hip_stream) {
  return guarded([&]() -> int {
    const auto t0 = std::chrono::steady_clock::now();
    STCHK(device_part(h, opts, hip_stream));
    h->build_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return HM_OK;
  });
}

// Device bytes the device part of the build will allocate (panels FP64 and
// FP32, D^{-1}-premultiplied panels, LU and D^{-1}, stage-A W copies for both
// kernel families, in-row stacks), plus the workspace for nrhs right-hand
// sides; from block sizes only, to within a few percent.
int64_t device_bytes_estimate(hm_matrix_t h, int nrhs) {
  const HostH& H = h->H;
  int64_t P = 0, Dm = 0, Wn = 0, T = 0, Hn = 0, Hc = 0;
  const bool sym = h->want_half;  // half panels (surface, and volume on Z diag(1/chi))
  for (const NearBlock& nb : H.near) {
    const int64_t m = even_ld(H.leaf_size[nb.t_leaf]);
    P += m * H.leaf_size[nb.s_leaf];
    if (nb.t_leaf == nb.s_leaf) Dm += (int64_t)H.leaf_size[nb.t_leaf] * H.leaf_size[nb.t_leaf];
    if (sym && nb.t_leaf < nb.s_leaf) {
      Hn += m * H.leaf_size[nb.s_leaf];
      Hc += H.leaf_size[nb.s_leaf];
    }
  }
  int64_t Pf = 0;
  for (const FarBlock& fb : H.far) {
    const int64_t r = H.lowrank[fb.src].r;
    P += r * fb.m;
    Pf += r * fb.m;
    Wn += r * fb.n;
    T += r;
  }
  const int64_t f32 = h->has_f32 ? 1 : 0;
  const int64_t bytes =
      16 * (P + (P - Dm)) + 32 * Dm + 2 * 16 * Wn + f32 * (8 * (2 * P - Dm) + 2 * 8 * Wn);
  // half panels, their sources and v slots, the scaled far data, the
  // C^{-1}, C^{-T}, C and C^T panels and two N-vectors
  const int64_t half =
      Hn > 0 ? (16 + 8 * f32) * (Hn + Pf + Wn) + 20 * Hc + 32 * h->N + 64 * Dm : 0;
  return bytes + half + workspace_bytes(h, nrhs, T);
}

// Workspace of ensure_workspace for nrhs right-hand sides (t rows T when
// the device part is not built yet, else the handle's own).
int64_t workspace_bytes(hm_matrix_t h, int nrhs, int64_t T) {
  if (h->device >= 0) T = h->T;
  const int64_t partial = h->partial_rows > 0 ? h->partial_rows
                                              : 2 * h->N + (int64_t)h->term_wgs * h->max_m;
  const int64_t items = h->n_norm_items > 0 ? h->n_norm_items : h->N / kNormRows + 1;
  const int64_t ldr = row_ld(nrhs);
  return (int64_t)nrhs * (16 * 2 * (h->N + T) + 16 * 4 * h->N + 16 * (items + h->nseg)) +
         ldr * (24 * 2 * (h->N + T) + 16 * partial) + 4 * counter_count(h, nrhs);
}

int workspace_rhs(hm_matrix_t h) { return h->ws_nrhs; }

int gmres_restart(const ps_opts& o) {
  return o.restart > 0 ? o.restart : std::max(1, std::min(kDefaultRestart, o.max_passes));
}

int64_t gmres_growth_bytes(hm_matrix_t h, int m, int nrhs) {
  if (m <= h->gm_m && nrhs <= h->gm_nrhs) return 0;
  return gmres_bytes(h->N, std::max(m, h->gm_m), std::max(nrhs, h->gm_nrhs)) -
         gmres_bytes(h->N, h->gm_m, h->gm_nrhs);
}

int gmres_rhs(hm_matrix_t h, int m) { return m <= h->gm_m ? h->gm_nrhs : 0; }

int64_t resident_bytes(hm_matrix_t h) { return h->bytes + h->ws_bytes; }

int64_t matrix_n(hm_matrix_t h) { return h->N; }

}  // namespace hm
