// Device-side data layout and kernel launchers of libhmps (internal).
//
// Layout in HBM (all tree order):
//   * a "panel" per leaf row a: column-major m_a x C_a, complex, ld = m_a.
//     The apply panel holds [D_a | near blocks (a, s != a) | far slices]; the
//     series panel holds D_a^{-1} times the same columns without D_a.  Far
//     slices are the rows of the leaf inside U_b (m_b x r_b) of every far
//     block b whose row cluster contains the leaf, ordered finest level
//     first, so the blocks of level >= l are a prefix of the far columns.
//   * every panel column has a source index into the combined input vector
//     [y (N) | t (T)] of one right-hand side, where t holds the stage-A
//     coefficients t_b = W_b y_s of all far blocks (T = sum of ranks).
//   * W_b (r_b x n_b, row-major), finest level first, with the contrast of
//     the source points folded in for the volume case.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

struct WorkItem {      // one workgroup of the panel product
  int32_t leaf;
  int32_t c0, c1;      // panel column range [c0, c1)
  int32_t prow;        // first row of its partial sums in the partial buffer
};

struct PanelSet {
  const void* data;          // double2 or float2 elements
  const int64_t* panel_off;  // per leaf: element offset of the panel
  const int32_t* src;        // per panel column: row in the input vector
  const int64_t* col_off;    // per leaf: index of its first column in src
  const int32_t* leaf_m;     // per leaf: rows
};

struct StageABlock {
  int32_t s_off, n, r, tb_off;  // source range, rank, coefficient offset in t
  int64_t w_off;                // element offset of W_b
};

struct EpilogueArgs {
  const int32_t* leaf_off;
  const int32_t* leaf_m;
  const int32_t* item_ptr;   // per leaf: first work item (items sorted by leaf)
  const WorkItem* items;
  const double2* partial;
  int64_t ldp;
  double alpha;              // y = alpha * z + beta * v
  double beta;
  const double2* v;          // may be null
  int64_t ldv;
  double2* yout;             // may be null
  int64_t ldy;
  double2* xacc;             // may be null
  int64_t ldxa;
  int accumulate;            // xacc += y (1) or xacc = y (0)
};

// ---- launchers (return hipError_t of the launch) ---------------------------
hipError_t launch_permute_in(const double2* b, int64_t ldb, const int64_t* perm, double2* out,
                             int64_t ldo, int64_t n, int nrhs, hipStream_t st);
hipError_t launch_permute_out(const double2* in, int64_t ldi, const int64_t* perm, double2* x,
                              int64_t ldx, int64_t n, int nrhs, hipStream_t st);
hipError_t launch_panel(bool f32, int max_m, const PanelSet& ps, const WorkItem* items, int nitems,
                        const double2* xin, int64_t ldx, int nrhs, double2* partial, int64_t ldp,
                        hipStream_t st);
hipError_t launch_stageA(bool f32, const void* W, const StageABlock* blk, int nblk, double2* xin,
                         int64_t ldx, int64_t N, int nrhs, hipStream_t st);
hipError_t launch_epilogue(const EpilogueArgs& e, int nleaves, int max_m, int nrhs, hipStream_t st);
hipError_t launch_getrf(double2* A, const int64_t* off, const int32_t* m, int32_t* piv,
                        const int64_t* piv_off, int nblk, int* info, hipStream_t st);
hipError_t launch_getri(const double2* LU, const int64_t* off, const int32_t* m, const int32_t* piv,
                        const int64_t* piv_off, double2* Ainv, int nblk, hipStream_t st);
// M panel columns c of leaf a = Dinv_a * (apply panel column m_a + c)
hipError_t launch_premul(const double2* Dinv, const int64_t* dinv_off, const double2* P,
                         const int64_t* p_off, const int32_t* leaf_m, const int32_t* ncols_m,
                         double2* M, const int64_t* m_off, const int32_t* tiles, int ntiles,
                         int max_m, hipStream_t st);
constexpr int kPremulCols = 32;  // columns per tile of launch_premul
hipError_t launch_cast(const double2* in, float2* out, int64_t n, hipStream_t st);
// per column c < nrhs: out[c] = sum_i |v[i + c*ld]|^2 in a fixed order
hipError_t launch_norm2(const double2* v, int64_t ld, int64_t n, int nrhs, double* scratch,
                        double* out, hipStream_t st);
// y[i + c*ldy] (+)= alpha x[i + c*ldx]
hipError_t launch_axpy(double alpha, const double2* x, int64_t ldx, double2* y, int64_t ldy,
                       int64_t n, int nrhs, int accumulate, hipStream_t st);

constexpr int kNormBlocks = 128;  // partial sums per column in launch_norm2

}  // namespace hm
