// Device kernels of the half-storage build (internal): the symmetric leaf
// factors and the scaled operator S = C^{-1} R C^{-T} (the symmetric
// reading of the block-diagonal splitting of Sec. IV, on the symmetric
// operator of Sec. II).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

// Per leaf a (m_a <= kCsymMaxLeaf rows): the diagonal block D_a is the
// first m_a columns of the leaf's apply panel (column-major, leading
// dimension even(m_a), at element offset d_off[a] of d), with column k
// divided by chi[leaf_off[a] + k] when chi is not null (the volume
// operator's contrasts: D diag(1/chi) is symmetric).  The kernel
// factors D_a = C_a C_a^T without pivoting (C_a lower triangular, complex
// symmetric: no conjugation), forms C_a^{-1}, and writes C_a, C_a^T,
// C_a^{-1} and C_a^{-T} as m_a x m_a panels (leading dimension even(m_a),
// element offset c_off[a]) of cf, cft, ch, cht, whose other entries the
// caller has zeroed.  ok[a] = 1 when the factor is accepted: every pivot
// |d_jj - sum_k C_jk^2| above 1e-10 max_j |D_jj|, max |C_ij|^2 at most
// 1e2 max |D_ij| (element growth), ||C C^T - D||_F at most
// 1e-14 ||D||_F (backward error) and a finite inverse; else 0.
constexpr int kCsymMaxLeaf = 128;
hipError_t launch_csym(const double2* d, const int64_t* d_off, const int32_t* leaf_m,
                       const int32_t* leaf_off, const double* chi, int nl, int max_m, double2* cf,
                       double2* cft, double2* ch, double2* cht, const int64_t* c_off, int32_t* ok,
                       hipStream_t st);

// Block-diagonal m_a x m_a panels (leading dimension even(m_a), element
// offset c_off[a]) scaled by the contrasts of the leaf's points:
// out = diag(chi)^p in, p = -1 (mode 0), or out = in diag(chi)^p, p = -1
// (mode 1) or +1 (mode 2).  in and out may be the same panels.
hipError_t launch_panel_scale(const double2* in, double2* out, const int64_t* c_off,
                              const int32_t* leaf_m, const int32_t* leaf_off, const double* chi,
                              int nl, int mode, hipStream_t st);

// One product of a batch: C = op(A) op(B) with complex FP64 column-major
// operands (op(X) = X, or X^T when the flag is set; no conjugation); C is
// m x n, the inner dimension k; offsets are elements from the launch's
// base pointers.
struct GemmItem {
  int64_t a_off, b_off, c_off;
  int32_t lda, ldb, ldc;
  int32_t m, n, k;
  int32_t ta, tb;
};
// Runs every item of the batch (items on the device, count n_items; tiles:
// the items' 64 x 64 output tiles, (item, tile row, tile column), built by
// gemm_tiles).
struct GemmTile {
  int32_t item, i0, j0, pad;
};
hipError_t launch_cgemm(const double2* a, const double2* b, double2* c, const GemmItem* items,
                        const GemmTile* tiles, int n_tiles, hipStream_t st);
constexpr int kGemmTile = 64;

// Kernel parameters of one instance: kind 0 (surface) or 1 (volume), wave
// number k and spacing h.
struct EntryInst {
  int32_t kind, pad;
  double k, h;
};
// One near block of the entry fill: rows are the points of leaf t, columns
// the points of leaf s (both in tree order); entry (i, j) goes to
// out[dst + i + j ld], and rows m_t .. ld - 1 of each column are set to zero.
struct FillItem {
  int64_t dst;
  int32_t ld, t, s, pad;
};
// Computes every item's entries from the points (xyz: 3 doubles per point,
// tree order) with the formulas of the problem (Sec. II's integral
// equations on the synthetic point kernels): off the diagonal
// scale e^{-jkR} / (4 pi R), R the distance, scale h^2 (surface) or
// k^2 h^3 chi_j (volume, chi in tree order); on the diagonal 2h(1 + 0.1j)
// (surface) or 1/chi_i + 0.5 (volume).  Parameters per leaf through
// leaf_inst and inst.  *bad is set to 1 (never cleared here) when two
// distinct points of a block lie closer than 1e-12.
hipError_t launch_fill_near(const FillItem* items, int n_items, const double* xyz,
                            const double* chi, const int32_t* leaf_off, const int32_t* leaf_m,
                            const int32_t* leaf_inst, const EntryInst* inst, double2* out,
                            int32_t* bad, hipStream_t st);
// Segments (src_off, dst_off, len), three int64 each: len elements copied
// from src + src_off to dst + dst_off.
hipError_t launch_seg_copy(const double2* src, double2* dst, const int64_t* seg, int n_seg,
                           hipStream_t st);

}  // namespace hm
