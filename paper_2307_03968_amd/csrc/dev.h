// Device-side data layout and kernel launchers of libhmps (internal).
//
// Layout in HBM (all tree order, complex elements, column-major):
//   * a "panel" per leaf row a with leading dimension ld_a = m_a rounded up
//     to even (zero pad row when m_a is odd, so FP32 panels can be read two
//     rows per 16-byte load).  The apply panel holds
//       [D_a | near blocks (a, s != a) | in-row far | global far]
//     and the series panel D_a^{-1} times the same columns without D_a; the
//     D^{-1} panel holds D_a^{-1}.
//   * a far block is "in-row" when its row cluster is a single leaf (every
//     leaf-level block is).  Its panel columns are U_b (m_a x r_b) and its W_b
//     (r_b x n_b) is a block of rows of the leaf's W stack, so one workgroup
//     forms t_b = W_b y_s and applies U_b t_b without a separate pass.
//     Other far blocks are "global": U_b is sliced into the panels of the
//     leaves of its row cluster and t_b comes from a separate stage-A pass
//     grouped by source cluster (W_g column-major, even leading dimension),
//     written into the t part of the combined input vector [y (N) | t (T)].
//   * far columns (and W stack rows) are ordered finest level first, so the
//     blocks of level >= l are a prefix of the in-row and of the global part.
//   * every dense panel column has a source index into [y | t].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

inline int even_ld(int m) { return m + (m & 1); }

struct PanelSet {
  const void* data;          // double2 (FP64) or float2 pairs (FP32) elements
  const int64_t* panel_off;  // per leaf: complex-element offset of the panel
  const int32_t* src;        // per panel column: row in the input vector
  const int64_t* col_off;    // per leaf: index of its first column in src
  const int32_t* leaf_m;     // per leaf: rows (ld = m rounded up to even)
};

// One piece of the work of a term kernel.  The pieces of all leaves are
// split evenly over a fixed number of persistent workgroups (one resident
// round), each workgroup taking a contiguous run of pieces.
//  kind 0: panel columns [c0, c1) against the input vector through src.
//  kind 1: in-row low-rank rows [r0, r1) of the leaf's W stack (at most
//          kInRowTile): first t = W_stack[r0:r1, :] y (each row has its own
//          source range), then the panel columns c0 .. c0 + (r1 - r0) against t.
struct TermItem {
  int32_t leaf, kind;
  int32_t c0, c1;
  int32_t r0, r1;
  int32_t prow;              // first row of its partial sums
  int32_t pad;
};

struct InRow {               // per-leaf W stacks of the in-row far blocks
  const void* W;             // double2 or float2 elements
  const int64_t* off;        // per leaf: complex-element offset of the stack
  const int32_t* ld;         // per leaf: leading dimension (even)
  const int32_t* ncol;       // per leaf: columns (largest source size)
  const int32_t* row0;       // per leaf: first row in soff / n
  const int32_t* soff;       // per stack row: source offset (tree order)
  const int32_t* n;          // per stack row: source size
};

struct Group {                // stage-A group (one source cluster)
  int32_t s_off, n;           // source points [s_off, s_off + n)
  int32_t t0, ld;             // first coefficient in t, leading dimension of W_g
  int64_t w_off;              // complex-element offset of W_g
};

struct GroupItem {            // one workgroup of a group product
  int32_t group;
  int32_t row0, rows;         // row tile start and active rows of the group
  int32_t pad;
};

struct TermArgs {
  PanelSet ps;
  InRow ir;
  const TermItem* items;     // pieces, grouped by workgroup
  const int32_t* wptr;       // per workgroup: first piece (count + 1 entries)
  const int32_t* lptr;       // per leaf: first entry in lprow (nleaves + 1)
  const int32_t* lprow;      // partial rows of each leaf's pieces, fixed order
  const int32_t* leaf_off;
  const double2* xin;        // [y | t] input, column stride ldx
  int64_t ldx;
  const int64_t* in_perm;    // non-null: kind-0 inputs read xin[in_perm[src]]
  double2* partial;
  int64_t ldp;
  int32_t* counters;         // per (leaf, rhs tile); zero between launches
  // epilogue of leaf a, run by its last workgroup: y = alpha z + beta v
  double alpha, beta;
  const double2* v;          // may be null (tree order, ld ldv)
  int64_t ldv;
  double2* yout;             // may be null (tree order, ld ldy)
  int64_t ldy;
  double2* xacc;             // may be null: x = y or x += y (tree order)
  int64_t ldxa;
  int accumulate;
  double2* out;              // may be null: out[out_perm[q]] = new x (or y)
  int64_t ldo;
  const int64_t* out_perm;
  // Matrix-core (many right-hand sides) kernels read [y | t] in ROW
  // layout: entry (p, c) at p * ldr + c, right-hand sides contiguous, ldr a
  // multiple of 16; FP64 (xr) or FP32 (xr32, the values the FP32 products
  // would round the FP64 ones to).  Their partial sums use the same layout
  // (partial[(prow + i) * ldr + c]).  The epilogue writes the new y in row
  // layout for the next term when yrow / yrow32 are set.
  const double2* xr;
  const float2* xr32;
  int64_t ldr;
  int32_t zrow;              // a row of xr / xr32 that holds zeros
  double2* yrow;
  float2* yrow32;
};

// Epilogue of one entry (row i of the leaf at tree offset off, right-hand
// side c) of a term: y = alpha z + beta v, then the y, x and output stores.
__device__ __forceinline__ void finish_entry(const TermArgs& A, int64_t off, int i, int c,
                                             double2 z) {
  double2 y = make_double2(A.alpha * z.x, A.alpha * z.y);
  if (A.v) {
    const double2 v = A.v[off + i + (int64_t)c * A.ldv];
    y.x = fma(A.beta, v.x, y.x);
    y.y = fma(A.beta, v.y, y.y);
  }
  if (A.yout) A.yout[off + i + (int64_t)c * A.ldy] = y;
  if (A.yrow) A.yrow[(off + i) * A.ldr + c] = y;
  if (A.yrow32) A.yrow32[(off + i) * A.ldr + c] = make_float2((float)y.x, (float)y.y);
  double2 res = y;
  if (A.xacc) {
    const int64_t q = off + i + (int64_t)c * A.ldxa;
    if (A.accumulate) {
      const double2 o = A.xacc[q];
      res.x += o.x;
      res.y += o.y;
    }
    A.xacc[q] = res;
  }
  if (A.out) A.out[A.out_perm[off + i] + (int64_t)c * A.ldo] = res;
}

struct NormItem {
  int64_t r0, r1;
};

// Half-storage product R y for symmetric (surface) problems, one
// right-hand side.  Z_st = Z_ts^T, so per row leaf t only the near blocks
// Z_ts with s > t are stored, side by side as the leaf's half panel (ld
// even(m_t), unpremultiplied).  Streaming a half-panel column j (row jj of
// source leaf s) gives both u_t += Z[:, j] y_s[jj] and v_j = Z[:, j]^T y_t,
// which is row jj of Z_st y_t: v_j goes to slot j of the vector vb and the
// epilogue of leaf s adds it in.  A far block between two leaves t < s is
// stored once too, as the pair of factors (U' of t's rows, W' of s's rows,
// S_ts = U' W'^T); one pass over the pair forms U'^T y_t and W'^T y_s and
// from them z_t += U' (W'^T y_s) and z_s += W' (U'^T y_t), the second into
// partial rows of its own that the epilogue of s adds.  Other far blocks
// (a row or column cluster above the leaves) keep their per-orientation
// form (in-row W stacks and the U columns of the far panels).  The
// workgroup that completes a leaf writes z = alpha R y + beta v through the
// TermArgs epilogue.
// Pieces are TermItems with the far panels as the panel set, taken by the
// persistent workgroups one at a time from a queue (a device counter):
//  kind 0: far-panel columns [c0, c1) through src (global far U slices)
//  kind 1: in-row far rows [r0, r1) of the W stack, far-panel columns c0..
//  kind 2: half-panel columns [c0, c1) of the leaf; its v values go to the
//          leaves vleaf[r0, r1) (the blocks the columns cover)
//  kind 3: far pairs [c0, c1) of the leaf (global pair indices); pair
//          c0 + k goes to leaf vleaf[r0 + k]
struct HalfArgs {
  TermArgs t;                // ps = scaled far panels; lptr/lprow: the leaf's
                             // u partial rows, then its v slots
  const void* hp;            // half panels: double2 (FP64) or float2 (FP32)
  const int64_t* hp_off;     // per leaf: element offset of its half panel
  const int32_t* hp_col;     // per leaf (+ end): first global half-panel column
  const int32_t* hsrc;       // per global half-panel column: row of y it reads
  int64_t vrow;              // v slot of global half-panel column j: partial row vrow + j
  const int32_t* lcnt;       // per leaf: counter increments before its epilogue
  const int32_t* vleaf;      // target leaves of the kind-2 pieces
  int npieces;               // pieces in t.items, taken in order from a queue
  int32_t* queue;            // [next piece, workgroups done]; zero between launches
  // far pairs: pair p is U' (even(m_t) x r) then W' (even(m_s) x r), both
  // column-major, at element offset fp_off[p]; its z_s rows are partial
  // rows frow + fp_slot[p] ..
  const void* fp;            // double2 (FP64) or float2 (FP32) elements
  const int64_t* fp_off;
  const int32_t* fp_rank;
  const int32_t* fp_slot;
  int64_t frow;
};
// All K terms of the scaled series in one launch of the half-storage kernel
// (lists whose far blocks are all pairs): term k reads y_{k-1} from
// y[(k - 1) & 1] (y_0 given) and writes y_k = alpha z to y[k & 1] and
// x += y_k, leaf by leaf; a piece of term k > 1 starts once the leaves it
// reads and writes are done with term k - 1.  done (nl entries) and the
// queue are zero between launches; err is set (and the launch still ends)
// if a wait gives up, which a consistent list never makes it do.
struct MultiArgs {
  int K;
  int nl;
  double2* y[2];
  double2* xacc;
  int32_t* done;
  int32_t* err;
};
hipError_t launch_half(bool f32, int max_m, const HalfArgs& a, int nwg, hipStream_t st);
hipError_t launch_half_multi(bool f32, int max_m, const HalfArgs& a, const MultiArgs& m, int nwg,
                             hipStream_t st);
int half_occupancy(bool f32, int max_m, bool multi = false);
constexpr int kMaxVLeaves = 8;  // target leaves (blocks) per kind-2 or kind-3 piece
constexpr int kHalfMaxLeaf = 128;  // largest leaf the half-storage product serves
constexpr int kHalfChunk = 1024;   // input columns of a kind-0 half-list piece (at most)
constexpr int kHalfPieceCols = 256;  // half-panel columns of a kind-2 piece (at most)
constexpr int kHalfInRowTile = 128;  // W-stack rows of a half-list in-row piece (at most)

constexpr int kInRowTile = 64;   // stack rows per kind-1 piece (one row per lane)
constexpr int kGroupTile = 128;  // rows per stage-A group item
// Many right-hand sides (MFMA path): stage A uses groups over all far blocks
// (in-row ones included) by source cluster, with their own W copies and t
// slots; items are 64-row tiles.
constexpr int kGroupTileMM = 64;


// ---- launchers (return hipError_t of the launch) ---------------------------
// one right-hand side, block-diagonal panels (D^{-1}, C^{-1}, C^{-T}): one
// workgroup per leaf, leaves of at most 128 points, epilogue as the term kernel
hipError_t launch_block_diag(const TermArgs& a, int nl, int max_m, hipStream_t st);
constexpr int kBlockDiagMaxLeaf = 128;
hipError_t launch_permute_in(const double2* b, int64_t ldb, const int64_t* perm, double2* out,
                             int64_t ldo, int64_t n, int nrhs, hipStream_t st);
hipError_t launch_permute_out(const double2* in, int64_t ldi, const int64_t* perm, double2* x,
                              int64_t ldx, int64_t n, int nrhs, hipStream_t st);
// many-RHS variants on MFMA (FP32 3M, FP64 4M), inputs and partial sums
// in row layout (TermArgs::xr / xr32, ldr), right-hand sides in tiles of
// `tile` = 16/32/64 (0: by nrhs).  Leaves of at most kMmWaveLeaf rows run
// one piece per wave (wave mode: nunits = waves, pieces grouped by wave);
// larger leaves (up to 256 rows) one piece per workgroup, wave w taking
// rows [w R, (w + 1) R) of the leaf, R = 32 or 64 (nunits = workgroups).
hipError_t launch_term_mm(bool f32, int max_m, const TermArgs& a, int nunits, int nrhs, int tile,
                          hipStream_t st);
constexpr int kMmWaveLeaf = 64;
// zeroed bytes after every panel set the matrix-core kernels read (their row
// tiles run up to 15 rows past a leaf's last column)
constexpr size_t kPanelPad = 4096;
inline bool mm_wave_mode(int max_m) { return max_m <= kMmWaveLeaf; }
// t rows of the listed group tiles (64 rows each) in row layout:
// x[(N + t0 + q) ldr + c] = sum_j W_g[q, j] x[(s_off + j) ldr + c]
hipError_t launch_stageA_mm(bool f32, const void* W, const Group* groups, const GroupItem* items,
                            int nitems, double2* xr, float2* xr32, int64_t ldr, int64_t N,
                            int zrow, int nrhs, int tile, hipStream_t st);
// The K terms of the series on the matrix cores in one persistent launch
// (wave mode: leaves of at most kMmWaveLeaf rows; one tile of at most 32
// right-hand sides).  Work comes from a queue of wave items, term by term:
// the stage-A tiles of every instance (64 rows of a group each), then the
// term pieces of every instance.  Term k reads [y_{k-1} | t_k] from
// rows r[(k - 1) & 1] and its leaf epilogues write y_k to rows r[k & 1] and
// x += y_k (TermArgs epilogue, alpha = -1).  Per (instance, term) two
// counters count the stage-A tiles done and the leaf epilogues done; a
// stage-A tile of term k starts once its instance's epilogues of term k - 1
// are all done, a term piece once its instance's stage-A tiles of term k are
// (and the epilogues of term k - 1).  Every wait is on items earlier in the
// queue, each taken by a running wave, so every wait ends; a wait that gives
// up sets *err.  Rows, x and the counters move through device-coherent
// loads and stores (the terms of one leaf run on any XCD).  The queue and
// the counters are zero between launches (the last wave out clears them).
struct MMItem {
  int32_t kind;              // 0: stage-A tile of group a; 1: term piece of leaf a
  int32_t inst;              // instance the item belongs to
  int32_t a;
  int32_t c0, c1;            // term piece: panel columns
  int32_t prow;              // term piece: first partial row
  int32_t row0, rows;        // stage-A tile: first row, active rows of the group
};
struct MMSeriesArgs {
  int K;
  int n_a, n_b;              // stage-A tiles and term pieces of one term
  const MMItem* items;       // n_a + n_b, the same for every term
  const Group* groups;       // stage-A groups and their W (FP64 or FP32)
  const void* W;
  double2* r64[2];
  float2* r32[2];
  int64_t N;                 // rows of y (t rows follow)
  int32_t* cnt;              // per (instance, term): [tiles done, epilogues done]
  int kmax;                  // terms the counters hold per instance
  const int32_t* need_a;     // per instance: stage-A tiles of one term
  const int32_t* need_b;     // per instance: leaf epilogues of one term
  int ninst;
  int32_t* queue;            // [next item, waves done]
  int32_t* err;
  // outputs of the last term only (the TermArgs yout / out are ignored)
  double2* yout;
  int64_t ldy;
  double2* out;
  int64_t ldo;
  const int64_t* out_perm;
};
constexpr int kMmSeriesMaxTerms = 16;
hipError_t launch_series_mm(bool f32, const TermArgs& a, const MMSeriesArgs& s, int nwg, int nrhs,
                            hipStream_t st);
// workgroups of the multi-term matrix-core kernel resident on one CU
int series_mm_occupancy(bool f32, int nrhs);
// column layout -> row layout: out[p ldr + c] = in[(perm ? perm[p] : p) + c ldi]
// for p < n, c < nrhs, zero for nrhs <= c < ldr; FP64 (out) and/or FP32 (out32)
hipError_t launch_rows(const double2* in, int64_t ldi, const int64_t* perm, int64_t n, int nrhs,
                       double2* out, float2* out32, int64_t ldr, hipStream_t st);
inline int64_t row_ld(int nrhs) { return ((int64_t)nrhs + 15) / 16 * 16; }
// nwg persistent workgroups; grid.y covers the right-hand sides
hipError_t launch_term(bool f32, int max_m, const TermArgs& a, int nwg, int nrhs,
                       hipStream_t st);
// workgroups of the 1-RHS term kernel that fit on one CU at once
int term_occupancy(bool f32, int max_m);
// number of right-hand sides one term workgroup handles for nrhs
int term_rhs_tile(int nrhs);
// t rows of the listed group tiles: xin[N + t0 + row] = W_g xin[s_off ...]
hipError_t launch_stageA(bool f32, const void* W, const Group* groups, const GroupItem* items,
                         int nitems, double2* xin, int64_t ldx, int64_t N, int nrhs,
                         hipStream_t st);
hipError_t launch_getrf(double2* A, const int64_t* off, const int32_t* m, int32_t* piv,
                        const int64_t* piv_off, int nblk, int* info, hipStream_t st);
// D^{-1} into panels of even leading dimension at dinv_off
hipError_t launch_getri(const double2* LU, const int64_t* off, const int32_t* m, const int32_t* piv,
                        const int64_t* piv_off, double2* Ainv, const int64_t* dinv_off, int nblk,
                        hipStream_t st);
// M panel columns c of leaf a = Dinv_a * (apply panel column m_a + c)
hipError_t launch_premul(const double2* Dinv, const int64_t* dinv_off, const double2* P,
                         const int64_t* p_off, const int32_t* leaf_m, const int32_t* ncols_m,
                         double2* M, const int64_t* m_off, const int32_t* tiles, int ntiles,
                         int max_m, hipStream_t st);
constexpr int kPremulCols = 32;  // columns per tile of launch_premul
hipError_t launch_cast(const double2* in, float2* out, int64_t n, hipStream_t st);
// per column c < nrhs: out[c] = sum_i |v[i + c*ld]|^2 in a fixed order
// squared norms per (segment, column) -> out[c * nseg + g]; scratch holds
// nitems * nrhs doubles
hipError_t launch_norm2(const double2* v, int64_t ld, const NormItem* items, int nitems,
                        const int32_t* seg_ptr, int nseg, int nrhs, double* scratch, double* out,
                        hipStream_t st);
// y[i + c*ldy] (+)= alpha x[i + c*ldx]
hipError_t launch_axpy(double alpha, const double2* x, int64_t ldx, double2* y, int64_t ldy,
                       int64_t n, int nrhs, int accumulate, hipStream_t st);

constexpr int64_t kNormRows = 8192;  // rows per norm item

}  // namespace hm
