// libhmps C-ABI: device packing of the H-matrix, batched leaf LU, the
// power-series solve and the H-matvec (Sec. III-IV).  The host only builds,
// packs and enqueues; every step of the solve runs in the kernels of
// device.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "dev.h"
#include "hm_internal.h"

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

struct WorkList {
  WorkItem* items = nullptr;   // device
  int32_t* ptr = nullptr;      // device, nleaves + 1
  int n = 0;
  int64_t rows = 0;            // partial rows
};

}  // namespace hm

struct hm_matrix {
  hm::HostH H;
  bool host_only = false;
  bool has_f32 = false;
  bool host_kept = true;
  int device = -1;
  int64_t N = 0, T = 0;
  int nl = 0, max_m = 0, L = 0, lmin = -1, nlev = 1;
  double build_ms = 0;
  int64_t bytes = 0;
  std::vector<void*> allocs;

  // per leaf
  int64_t* perm = nullptr;
  int32_t* leaf_off = nullptr;
  int32_t* leaf_m = nullptr;
  // apply panels [D | near | far], series panels D^{-1}[near | far]
  double2* R64 = nullptr;
  float2* R32 = nullptr;
  int64_t* R_off = nullptr;
  int32_t* src = nullptr;
  int64_t* R_col = nullptr;
  double2* M64 = nullptr;
  float2* M32 = nullptr;
  int64_t* M_off = nullptr;
  int64_t* M_col = nullptr;
  // D blocks, LU, inverse
  double2* LU = nullptr;
  double2* Dinv = nullptr;
  int64_t* D_off = nullptr;
  int32_t* piv = nullptr;
  int64_t* piv_off = nullptr;
  // stage A
  double2* W64 = nullptr;
  float2* W32 = nullptr;
  hm::StageABlock* blk = nullptr;
  std::vector<int> nA;          // per level index: active far blocks (prefix)
  std::vector<int64_t> bytes_R, bytes_M, bytes_W, ncoef;  // per level index, element counts
  // work lists
  std::vector<hm::WorkList> wl_apply, wl_series;
  hm::WorkList wl_dinv;
  int64_t partial_rows = 0;
  // workspace
  int ws_nrhs = 0;
  double2 *xin0 = nullptr, *xin1 = nullptr, *xt = nullptr, *bt = nullptr, *rt = nullptr,
          *dt = nullptr, *partial = nullptr;
  double *nscratch = nullptr, *norms = nullptr;
  double* norms_host = nullptr;  // pinned
  std::vector<void*> ws_allocs;
  // per-kernel timing
  bool prof = false;
  struct ProfRec { int cls; hipEvent_t e0, e1; };
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> ev_pool;

  ~hm_matrix() {
    for (auto& r : prof_recs) { (void)hipEventDestroy(r.e0); (void)hipEventDestroy(r.e1); }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (void* p : ws_allocs) (void)hipFree(p);
    for (void* p : allocs) (void)hipFree(p);
    if (norms_host) (void)hipHostFree(norms_host);
  }
};

namespace hm {

namespace {

int dalloc(hm_matrix* h, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    return HM_ENOMEM;
  }
  h->allocs.push_back(*p);
  h->bytes += (int64_t)bytes;
  return HM_OK;
}

template <typename T>
int upload(hm_matrix* h, T** dst, const std::vector<T>& v, hipStream_t st) {
  STCHK(dalloc(h, (void**)dst, v.size() * sizeof(T)));
  if (!v.empty()) HIPCHK(hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
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

// Split each leaf's active columns into work items.  `first` and `last`
// give the active column range of leaf a; target ~2048 items.
int make_worklist(hm_matrix* h, const std::vector<int64_t>& first, const std::vector<int64_t>& last,
                  WorkList& wl, hipStream_t st) {
  int64_t total = 0;
  for (int a = 0; a < h->nl; ++a) total += last[a] - first[a];
  const int64_t target = 2048;
  int64_t chunk = std::max<int64_t>(64, (total + target - 1) / target);
  chunk = (chunk + 31) / 32 * 32;
  std::vector<WorkItem> items;
  std::vector<int32_t> ptr(h->nl + 1, 0);
  int64_t rows = 0;
  for (int a = 0; a < h->nl; ++a) {
    ptr[a] = (int32_t)items.size();
    const int m = h->H.leaf_size[a];
    for (int64_t c = first[a]; c < last[a]; c += chunk) {
      items.push_back({a, (int32_t)c, (int32_t)std::min(last[a], c + chunk), (int32_t)rows});
      rows += m;
    }
  }
  ptr[h->nl] = (int32_t)items.size();
  wl.n = (int)items.size();
  wl.rows = rows;
  STCHK(upload(h, &wl.items, items, st));
  STCHK(upload(h, &wl.ptr, ptr, st));
  h->partial_rows = std::max(h->partial_rows, rows);
  return HM_OK;
}

int ensure_workspace(hm_matrix* h, int nrhs) {
  if (nrhs <= h->ws_nrhs) return HM_OK;
  for (void* p : h->ws_allocs) (void)hipFree(p);
  h->ws_allocs.clear();
  h->ws_nrhs = 0;
  const int64_t ldin = h->N + h->T;
  auto al = [&](void** p, size_t bytes) -> int {
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("workspace hipMalloc failed: " + std::string(hipGetErrorString(e)));
      return HM_ENOMEM;
    }
    h->ws_allocs.push_back(*p);
    return HM_OK;
  };
  STCHK(al((void**)&h->xin0, sizeof(double2) * ldin * nrhs));
  STCHK(al((void**)&h->xin1, sizeof(double2) * ldin * nrhs));
  STCHK(al((void**)&h->xt, sizeof(double2) * h->N * nrhs));
  STCHK(al((void**)&h->bt, sizeof(double2) * h->N * nrhs));
  STCHK(al((void**)&h->rt, sizeof(double2) * h->N * nrhs));
  STCHK(al((void**)&h->dt, sizeof(double2) * h->N * nrhs));
  STCHK(al((void**)&h->partial, sizeof(double2) * h->partial_rows * nrhs));
  STCHK(al((void**)&h->nscratch, sizeof(double) * kNormBlocks * nrhs * 2));
  STCHK(al((void**)&h->norms, sizeof(double) * nrhs * 2));
  if (h->norms_host) (void)hipHostFree(h->norms_host);
  h->norms_host = nullptr;
  HIPCHK(hipHostMalloc((void**)&h->norms_host, sizeof(double) * nrhs * 2, hipHostMallocDefault));
  h->ws_nrhs = nrhs;
  return HM_OK;
}

PanelSet apply_set(const hm_matrix* h, bool f32) {
  return PanelSet{f32 ? (const void*)h->R32 : (const void*)h->R64, h->R_off, h->src, h->R_col,
                  h->leaf_m};
}
PanelSet series_set(const hm_matrix* h, bool f32) {
  return PanelSet{f32 ? (const void*)h->M32 : (const void*)h->M64, h->M_off, h->src, h->M_col,
                  h->leaf_m};
}
PanelSet dinv_set(const hm_matrix* h) {
  return PanelSet{(const void*)h->Dinv, h->D_off, h->src, h->R_col, h->leaf_m};
}

EpilogueArgs epi(const hm_matrix* h, const WorkList& wl, int64_t ldp) {
  EpilogueArgs e{};
  e.leaf_off = h->leaf_off;
  e.leaf_m = h->leaf_m;
  e.item_ptr = wl.ptr;
  e.items = wl.items;
  e.partial = h->partial;
  e.ldp = ldp;
  e.alpha = 1.0;
  e.beta = 0.0;
  return e;
}

#define LCHK(x) HIPCHK(x)

hipEvent_t pool_event(hm_matrix* h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
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

// x_out = P_K rhs (tree order, ld N), as the power series of Sec. IV.
// y_0 = D^{-1} rhs; y_k = -(D^{-1} R_l) y_{k-1}; x = sum y_k.
int series_core(hm_matrix* h, int li, bool f32, int K, const double2* rhs, double2* x_out,
                int nrhs, bool want_norms, hipStream_t st) {
  const int64_t N = h->N, ldin = h->N + h->T, ldp = h->partial_rows;
  double2* y_cur = h->xin0;
  double2* y_nxt = h->xin1;
  {
    ProfScope ps(h, HM_K_PANEL_DINV, st);
    LCHK(launch_panel(false, h->max_m, dinv_set(h), h->wl_dinv.items, h->wl_dinv.n, rhs, N, nrhs,
                      h->partial, ldp, st));
    ps.done();
  }
  EpilogueArgs e = epi(h, h->wl_dinv, ldp);
  e.yout = y_cur;
  e.ldy = ldin;
  e.xacc = x_out;
  e.ldxa = N;
  e.accumulate = 0;
  {
    ProfScope ps(h, HM_K_EPILOGUE, st);
    LCHK(launch_epilogue(e, h->nl, h->max_m, nrhs, st));
    ps.done();
  }
  if (want_norms) LCHK(launch_norm2(y_cur, ldin, N, nrhs, h->nscratch, h->norms, st));
  const WorkList& wl = h->wl_series[li];
  const void* W = f32 ? (const void*)h->W32 : (const void*)h->W64;
  for (int k = 1; k <= K; ++k) {
    {
      ProfScope ps(h, HM_K_STAGEA, st);
      LCHK(launch_stageA(f32, W, h->blk, h->nA[li], y_cur, ldin, N, nrhs, st));
      ps.done();
    }
    {
      ProfScope ps(h, HM_K_PANEL_SERIES, st);
      LCHK(launch_panel(f32, h->max_m, series_set(h, f32), wl.items, wl.n, y_cur, ldin, nrhs,
                        h->partial, ldp, st));
      ps.done();
    }
    EpilogueArgs t = epi(h, wl, ldp);
    t.alpha = -1.0;
    t.yout = y_nxt;
    t.ldy = ldin;
    t.xacc = x_out;
    t.ldxa = N;
    t.accumulate = 1;
    {
      ProfScope ps(h, HM_K_EPILOGUE, st);
      LCHK(launch_epilogue(t, h->nl, h->max_m, nrhs, st));
      ps.done();
    }
    std::swap(y_cur, y_nxt);
  }
  if (want_norms)
    LCHK(launch_norm2(y_cur, ldin, N, nrhs, h->nscratch + kNormBlocks * nrhs, h->norms + nrhs, st));
  return HM_OK;
}

// out = alpha * Z_l x + beta * v (tree order, ld N); x_tree is read from
// xin0 (whose t part stage A fills).
int apply_core(hm_matrix* h, int li, bool f32, int nrhs, double alpha, double beta,
               const double2* v, double2* out, hipStream_t st) {
  const int64_t N = h->N, ldin = h->N + h->T, ldp = h->partial_rows;
  const void* W = f32 ? (const void*)h->W32 : (const void*)h->W64;
  {
    ProfScope ps(h, HM_K_STAGEA, st);
    LCHK(launch_stageA(f32, W, h->blk, h->nA[li], h->xin0, ldin, N, nrhs, st));
    ps.done();
  }
  const WorkList& wl = h->wl_apply[li];
  {
    ProfScope ps(h, HM_K_PANEL_APPLY, st);
    LCHK(launch_panel(f32, h->max_m, apply_set(h, f32), wl.items, wl.n, h->xin0, ldin, nrhs,
                      h->partial, ldp, st));
    ps.done();
  }
  EpilogueArgs e = epi(h, wl, ldp);
  e.alpha = alpha;
  e.beta = beta;
  e.v = v;
  e.ldv = N;
  e.yout = out;
  e.ldy = N;
  {
    ProfScope ps(h, HM_K_EPILOGUE, st);
    LCHK(launch_epilogue(e, h->nl, h->max_m, nrhs, st));
    ps.done();
  }
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

// ------------------------------------------------------------ device build
int build_device(hm_matrix* h, hipStream_t st) {
  const HostH& H = h->H;
  const int nl = h->nl;
  const int64_t N = h->N;
  // far blocks in device order (already finest first)
  const int nfar = (int)H.far.size();
  std::vector<int32_t> tb(nfar);
  int64_t T = 0;
  for (int b = 0; b < nfar; ++b) {
    tb[b] = (int32_t)T;
    T += H.lowrank[H.far[b].src].r;
  }
  h->T = T;
  // far slices per leaf, in device order
  std::vector<std::vector<std::pair<int, int>>> slices(nl);  // (block, row offset in block)
  {
    // leaf covering tree position: leaf_of
    for (int b = 0; b < nfar; ++b) {
      const FarBlock& fb = H.far[b];
      int a = H.tree.leaf_of[fb.t_off];
      while (a < nl && H.leaf_off[a] < fb.t_off + fb.m) {
        slices[a].push_back({b, H.leaf_off[a] - fb.t_off});
        ++a;
      }
    }
  }
  // levels
  h->nlev = (h->lmin < 0) ? 1 : (h->L - h->lmin + 1);
  std::vector<std::vector<int64_t>> far_end(h->nlev, std::vector<int64_t>(nl, 0));
  std::vector<int64_t> near_cols(nl, 0), ncols(nl, 0);
  std::vector<std::vector<int>> near_of(nl);
  for (int q = 0; q < (int)H.near.size(); ++q) {
    const NearBlock& nb = H.near[q];
    if (nb.t_leaf != nb.s_leaf) {
      near_of[nb.t_leaf].push_back(q);
      near_cols[nb.t_leaf] += H.leaf_size[nb.s_leaf];
    }
  }
  std::vector<int> diag_of(nl, -1);
  for (int q = 0; q < (int)H.near.size(); ++q)
    if (H.near[q].t_leaf == H.near[q].s_leaf) diag_of[H.near[q].t_leaf] = q;
  for (int a = 0; a < nl; ++a) {
    if (diag_of[a] < 0) { set_error("internal: missing diagonal block"); return HM_EINVAL; }
    int64_t fc = 0;
    for (auto& sl : slices[a]) fc += H.lowrank[H.far[sl.first].src].r;
    ncols[a] = H.leaf_size[a] + near_cols[a] + fc;
    for (int li = 0; li < h->nlev; ++li) {
      const int lev = (h->lmin < 0) ? h->L + 1 : h->lmin + li;
      int64_t e = 0;
      for (auto& sl : slices[a]) {
        const FarBlock& fb = H.far[sl.first];
        if (fb.level < lev) break;
        e += H.lowrank[fb.src].r;
      }
      far_end[li][a] = e;
    }
  }
  // stage-A prefix counts per level
  h->nA.assign(h->nlev, 0);
  for (int li = 0; li < h->nlev; ++li) {
    const int lev = (h->lmin < 0) ? h->L + 1 : h->lmin + li;
    int c = 0;
    while (c < nfar && H.far[c].level >= lev) ++c;
    h->nA[li] = c;
  }
  // ---- host panels, sources
  std::vector<int64_t> R_off(nl), R_col(nl), M_off(nl), M_col(nl), D_off(nl), piv_off(nl);
  int64_t rtot = 0, ctot = 0, mtot = 0, dtot = 0, ptot = 0;
  for (int a = 0; a < nl; ++a) {
    const int m = H.leaf_size[a];
    R_off[a] = rtot;
    rtot += (int64_t)m * ncols[a];
    R_col[a] = ctot;
    M_col[a] = ctot + m;
    ctot += ncols[a];
    M_off[a] = mtot;
    mtot += (int64_t)m * (ncols[a] - m);
    D_off[a] = dtot;
    dtot += (int64_t)m * m;
    piv_off[a] = ptot;
    ptot += m;
  }
  std::vector<double2> R((size_t)rtot);
  std::vector<int32_t> src((size_t)ctot);
  std::vector<double2> D((size_t)dtot);
  const double* chi = H.chi_tree.empty() ? nullptr : H.chi_tree.data();
#pragma omp parallel for schedule(dynamic, 1)
  for (int a = 0; a < nl; ++a) {
    const int m = H.leaf_size[a];
    double2* P = R.data() + R_off[a];
    int32_t* S = src.data() + R_col[a];
    int64_t c = 0;
    auto put_block = [&](const NearBlock& nb) {
      const int n = H.leaf_size[nb.s_leaf];
      const cplx* z = H.near_data.data() + nb.data;
      for (int j = 0; j < n; ++j, ++c) {
        S[c] = H.leaf_off[nb.s_leaf] + j;
        for (int i = 0; i < m; ++i) {
          const cplx v = z[i + (size_t)j * m];
          P[i + c * m] = make_double2(v.real(), v.imag());
        }
      }
    };
    put_block(H.near[diag_of[a]]);
    {
      const cplx* z = H.near_data.data() + H.near[diag_of[a]].data;
      for (int64_t e = 0; e < (int64_t)m * m; ++e) D[D_off[a] + e] = make_double2(z[e].real(), z[e].imag());
    }
    for (int q : near_of[a]) put_block(H.near[q]);
    for (auto& sl : slices[a]) {
      const FarBlock& fb = H.far[sl.first];
      const LowRank& lr = H.lowrank[fb.src];
      const std::vector<cplx>& U = fb.transposed ? lr.V : lr.U;  // m_b x r
      for (int q = 0; q < lr.r; ++q, ++c) {
        S[c] = (int32_t)(N + tb[sl.first] + q);
        for (int i = 0; i < m; ++i) {
          const cplx v = U[sl.second + i + (size_t)q * fb.m];
          P[i + c * m] = make_double2(v.real(), v.imag());
        }
      }
    }
  }
  // stage A: W_b = V^T diag(chi_s) row-major r x n
  std::vector<StageABlock> blk(nfar);
  int64_t wtot = 0;
  for (int b = 0; b < nfar; ++b) {
    const FarBlock& fb = H.far[b];
    const int r = H.lowrank[fb.src].r;
    blk[b] = StageABlock{fb.s_off, fb.n, r, tb[b], wtot};
    wtot += (int64_t)r * fb.n;
  }
  std::vector<double2> W((size_t)wtot);
#pragma omp parallel for schedule(dynamic, 16)
  for (int b = 0; b < nfar; ++b) {
    const FarBlock& fb = H.far[b];
    const LowRank& lr = H.lowrank[fb.src];
    const std::vector<cplx>& V = fb.transposed ? lr.U : lr.V;  // n_b x r
    double2* w = W.data() + blk[b].w_off;
    for (int q = 0; q < lr.r; ++q)
      for (int j = 0; j < fb.n; ++j) {
        cplx v = V[j + (size_t)q * fb.n];
        if (chi) v *= chi[fb.s_off + j];
        w[(int64_t)q * fb.n + j] = make_double2(v.real(), v.imag());
      }
  }
  // ---- upload
  std::vector<int32_t> loff(H.leaf_off), lm(H.leaf_size);
  STCHK(upload(h, &h->perm, H.tree.perm, st));
  STCHK(upload(h, &h->leaf_off, loff, st));
  STCHK(upload(h, &h->leaf_m, lm, st));
  STCHK(upload(h, &h->R64, R, st));
  std::vector<double2>().swap(R);
  STCHK(upload(h, &h->src, src, st));
  STCHK(upload(h, &h->R_off, R_off, st));
  STCHK(upload(h, &h->R_col, R_col, st));
  STCHK(upload(h, &h->M_off, M_off, st));
  STCHK(upload(h, &h->M_col, M_col, st));
  STCHK(upload(h, &h->D_off, D_off, st));
  STCHK(upload(h, &h->piv_off, piv_off, st));
  STCHK(upload(h, &h->LU, D, st));
  std::vector<double2>().swap(D);
  STCHK(upload(h, &h->W64, W, st));
  std::vector<double2>().swap(W);
  STCHK(upload(h, &h->blk, blk, st));
  STCHK(dalloc(h, (void**)&h->Dinv, sizeof(double2) * dtot));
  STCHK(dalloc(h, (void**)&h->piv, sizeof(int32_t) * ptot));
  STCHK(dalloc(h, (void**)&h->M64, sizeof(double2) * std::max<int64_t>(mtot, 1)));
  // ---- leaf LU with partial pivoting, then D^{-1} (eq. 12's near inverse)
  int* info = nullptr;
  STCHK(dalloc(h, (void**)&info, sizeof(int) * nl));
  HIPCHK(hipMemsetAsync(info, 0, sizeof(int) * nl, st));
  LCHK(launch_getrf(h->LU, h->D_off, h->leaf_m, h->piv, h->piv_off, nl, info, st));
  LCHK(launch_getri(h->LU, h->D_off, h->leaf_m, h->piv, h->piv_off, h->Dinv, nl, st));
  std::vector<int> info_h(nl);
  HIPCHK(hipMemcpyAsync(info_h.data(), info, sizeof(int) * nl, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int a = 0; a < nl; ++a)
    if (info_h[a] != 0) {
      set_error("leaf block " + std::to_string(a) + " is singular");
      return HM_EINVAL;
    }
  // ---- series panels M_a = D_a^{-1} [near | far] columns
  std::vector<int32_t> tiles, ncm(nl);
  for (int a = 0; a < nl; ++a) {
    ncm[a] = (int32_t)(ncols[a] - H.leaf_size[a]);
    for (int c = 0; c < ncm[a]; c += kPremulCols) { tiles.push_back(a); tiles.push_back(c); }
  }
  int32_t *d_tiles = nullptr, *d_ncm = nullptr;
  STCHK(upload(h, &d_tiles, tiles, st));
  STCHK(upload(h, &d_ncm, ncm, st));
  LCHK(launch_premul(h->Dinv, h->D_off, h->R64, h->R_off, h->leaf_m, d_ncm, h->M64, h->M_off,
                     d_tiles, (int)(tiles.size() / 2), h->max_m, st));
  // ---- FP32 copies
  if (h->has_f32) {
    STCHK(dalloc(h, (void**)&h->R32, sizeof(float2) * rtot));
    STCHK(dalloc(h, (void**)&h->M32, sizeof(float2) * std::max<int64_t>(mtot, 1)));
    STCHK(dalloc(h, (void**)&h->W32, sizeof(float2) * std::max<int64_t>(wtot, 1)));
    LCHK(launch_cast(h->R64, h->R32, rtot, st));
    LCHK(launch_cast(h->M64, h->M32, mtot, st));
    LCHK(launch_cast(h->W64, h->W32, wtot, st));
  }
  // ---- work lists
  std::vector<int64_t> zero(nl, 0), last(nl);
  h->wl_apply.assign(h->nlev, WorkList());
  h->wl_series.assign(h->nlev, WorkList());
  h->bytes_R.assign(h->nlev, 0);
  h->bytes_M.assign(h->nlev, 0);
  h->bytes_W.assign(h->nlev, 0);
  h->ncoef.assign(h->nlev, 0);
  for (int li = 0; li < h->nlev; ++li) {
    int64_t eR = 0, eM = 0, eW = 0, nc = 0;
    for (int a = 0; a < nl; ++a) {
      last[a] = H.leaf_size[a] + near_cols[a] + far_end[li][a];
      eR += (int64_t)H.leaf_size[a] * last[a];
    }
    STCHK(make_worklist(h, zero, last, h->wl_apply[li], st));
    for (int a = 0; a < nl; ++a) {
      last[a] = near_cols[a] + far_end[li][a];
      eM += (int64_t)H.leaf_size[a] * last[a];
    }
    STCHK(make_worklist(h, zero, last, h->wl_series[li], st));
    for (int b = 0; b < h->nA[li]; ++b) {
      eW += (int64_t)blk[b].r * blk[b].n;
      nc += blk[b].r;
    }
    h->ncoef[li] = nc;
    h->bytes_R[li] = eR;
    h->bytes_M[li] = eM;
    h->bytes_W[li] = eW;
  }
  for (int a = 0; a < nl; ++a) last[a] = H.leaf_size[a];
  STCHK(make_worklist(h, zero, last, h->wl_dinv, st));
  HIPCHK(hipStreamSynchronize(st));
  return HM_OK;
}

int validate_problem(const hm_problem* p, const hm_build_opts* o) {
  if (!p || !o) { set_error("null problem or options"); return HM_EINVAL; }
  if (p->n < 1 || !p->xyz) { set_error("n must be >= 1 and xyz non-null"); return HM_EINVAL; }
  if (p->n > (int64_t)1 << 30) { set_error("n too large"); return HM_EINVAL; }
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
    const int r = H.lowrank.empty() ? 0 : H.lowrank[fb.src].r;
    out->far_blocks[fb.level] += 1;
    out->far_rank_sum[fb.level] += r;
    out->far_entries[fb.level] += (int64_t)r * (fb.m + fb.n);
  }
  out->device_bytes = h->bytes;
  out->build_ms = h->build_ms;
  for (int li = 0; li < (int)h->bytes_M.size(); ++li) {
    const int lev = (h->lmin < 0) ? h->L : h->lmin + li;
    if (lev < 0 || lev >= HM_MAX_LEVELS) continue;
    out->series_entries[lev] = h->bytes_M[li];
    out->apply_entries[lev] = h->bytes_R[li];
    out->stageA_entries[lev] = h->bytes_W[li];
    out->coeffs[lev] = h->ncoef[li];
  }
}

}  // namespace
}  // namespace hm

using namespace hm;

// ====================================================================== C-ABI
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

int hmat_build(const hm_problem* prob, const hm_build_opts* opts, void* hip_stream,
               hm_matrix_t* out) {
  if (!out) { set_error("null output handle"); return HM_EINVAL; }
  *out = nullptr;
  STCHK(validate_problem(prob, opts));
  const auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<hm_matrix> h(new hm_matrix());
  Problem p;
  p.n = prob->n;
  p.kind = prob->kind;
  p.k = prob->k;
  p.h = prob->h;
  p.xyz.assign(prob->xyz, prob->xyz + 3 * prob->n);
  if (prob->kind == HM_VOLUME) p.chi.assign(prob->chi, prob->chi + prob->n);
  STCHK(build_host(p, *opts, h->H));
  h->N = p.n;
  h->nl = (int)h->H.leaf_size.size();
  h->max_m = h->H.max_leaf;
  h->L = h->H.tree.depth;
  h->lmin = h->H.min_far_level;
  h->host_only = (opts->flags & HM_BUILD_HOST_ONLY) != 0;
  h->has_f32 = (opts->flags & HM_BUILD_NO_F32) == 0;
  if (!h->host_only) {
    std::string arch;
    if (!check_arch(&arch)) {
      set_error("no usable gfx950 device (found '" + arch + "')");
      return HM_EHIP;
    }
    HIPCHK(hipGetDevice(&h->device));
    STCHK(build_device(h.get(), (hipStream_t)hip_stream));
    if (!(opts->flags & HM_BUILD_KEEP_HOST)) {
      std::vector<cplx>().swap(h->H.near_data);
      for (auto& lr : h->H.lowrank) {
        std::vector<cplx>().swap(lr.U);
        std::vector<cplx>().swap(lr.V);
      }
      h->host_kept = false;
    }
  }
  h->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h.release();
  return HM_OK;
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
  STCHK(ensure_workspace(h, nrhs));
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t ldin = h->N + h->T;
  LCHK(launch_permute_in((const double2*)x_dev, ldx, h->perm, h->xin0, ldin, h->N, nrhs, st));
  STCHK(apply_core(h, li, f32, nrhs, 1.0, 0.0, nullptr, h->bt, st));
  LCHK(launch_permute_out(h->bt, h->N, h->perm, (double2*)y_dev, ldy, h->N, nrhs, st));
  return HM_OK;
}

int ps_solve(hm_matrix_t h, const ps_opts* o, const void* b_dev, int64_t ldb, void* x_dev,
             int64_t ldx, int32_t nrhs, ps_stats* per_rhs, void* hip_stream) {
  if (!h || !o) { set_error("null argument"); return HM_EINVAL; }
  if (h->host_only) { set_error("handle was built host-only"); return HM_ESTATE; }
  if (nrhs < 0 || (nrhs > 0 && (!b_dev || !x_dev)) || ldb < h->N || ldx < h->N) {
    set_error("bad vector arguments");
    return HM_EINVAL;
  }
  if (o->K < 0 || o->K > 10000) { set_error("K must be in [0, 10000]"); return HM_EINVAL; }
  if (o->precision != HM_F64 && o->precision != HM_F32_APPLY) { set_error("bad precision"); return HM_EINVAL; }
  if (o->kind != PS_SERIES && o->kind != PS_REFINE) { set_error("bad kind"); return HM_EINVAL; }
  if (o->kind == PS_REFINE && (o->max_passes < 0 || !(o->refine_tol > 0))) {
    set_error("refinement needs max_passes >= 0 and refine_tol > 0");
    return HM_EINVAL;
  }
  const bool f32 = o->precision == HM_F32_APPLY;
  if (f32 && !h->has_f32) { set_error("FP32 copies were not kept"); return HM_ESTATE; }
  if (nrhs == 0) return HM_OK;
  int li = 0;
  STCHK(level_index(h, o->level, &li));
  HIPCHK(hipSetDevice(h->device));
  STCHK(ensure_workspace(h, nrhs));
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t N = h->N, ldin = h->N + h->T;
  const bool want = per_rhs != nullptr || o->kind == PS_REFINE;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (per_rhs) {
    HIPCHK(hipEventCreate(&ev0));
    HIPCHK(hipEventCreate(&ev1));
    HIPCHK(hipEventRecord(ev0, st));
  }
  LCHK(launch_permute_in((const double2*)b_dev, ldb, h->perm, h->bt, N, N, nrhs, st));
  STCHK(series_core(h, li, f32, o->K, h->bt, h->xt, nrhs, want, st));
  std::vector<double> growth(nrhs, 0.0), resid(nrhs, 0.0);
  std::vector<int> passes(nrhs, 0), done(nrhs, 0);
  auto read_norms = [&]() -> int {
    HIPCHK(hipMemcpyAsync(h->norms_host, h->norms, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return HM_OK;
  };
  if (want) {
    STCHK(read_norms());
    for (int c = 0; c < nrhs; ++c) {
      const double n0 = std::sqrt(h->norms_host[c]), nk = std::sqrt(h->norms_host[nrhs + c]);
      growth[c] = (n0 > 0) ? nk / n0 : (nk > 0 ? INFINITY : 0.0);
    }
  }
  if (o->kind == PS_REFINE) {
    for (int pass = 1; pass <= o->max_passes; ++pass) {
      // r = b - Z_l x in FP64 (all blocks including D)
      LCHK(launch_axpy(1.0, h->xt, N, h->xin0, ldin, N, nrhs, 0, st));
      STCHK(apply_core(h, li, false, nrhs, -1.0, 1.0, h->bt, h->rt, st));
      // d = P_K r, x += d
      STCHK(series_core(h, li, f32, o->K, h->rt, h->dt, nrhs, false, st));
      LCHK(launch_axpy(1.0, h->dt, N, h->xt, N, N, nrhs, 1, st));
      LCHK(launch_norm2(h->dt, N, N, nrhs, h->nscratch, h->norms, st));
      LCHK(launch_norm2(h->xt, N, N, nrhs, h->nscratch + kNormBlocks * nrhs, h->norms + nrhs, st));
      STCHK(read_norms());
      bool all = true;
      for (int c = 0; c < nrhs; ++c) {
        const double nd = std::sqrt(h->norms_host[c]), nx = std::sqrt(h->norms_host[nrhs + c]);
        const double rel = nx > 0 ? nd / nx : (nd > 0 ? INFINITY : 0.0);
        if (!done[c]) {
          resid[c] = rel;
          passes[c] = pass;
          if (rel <= o->refine_tol) done[c] = 1;
        }
        all = all && done[c];
      }
      if (all) break;
    }
  }
  LCHK(launch_permute_out(h->xt, N, h->perm, (double2*)x_dev, ldx, N, nrhs, st));
  int status = HM_OK;
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
      const bool bad = !(growth[c] <= 1.0) ||
                       (o->kind == PS_REFINE && !(resid[c] <= o->refine_tol));
      s.diverged = bad ? 1 : 0;
      if (bad) status = HM_EDIVERGED;
    }
  }
  return status;
}

int hmat_export(hm_matrix_t h, const char* path) {
  if (!h || !path) { set_error("null argument"); return HM_EINVAL; }
  if (!h->host_kept) { set_error("host blocks were released (build with HM_BUILD_KEEP_HOST)"); return HM_ESTATE; }
  if (h->host_only) return export_host(h->H, path, nullptr, nullptr);
  // add the device LU factors
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
