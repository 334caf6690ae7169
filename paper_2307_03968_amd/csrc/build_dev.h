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
// One far block for the device compression (adaptive cross approximation
// with partial pivoting, then recompression; Sec. III): rows are the points
// t_off .. t_off + m - 1, columns s_off .. s_off + n - 1 (tree order), kernel
// part only (e^{-jkR} / (4 pi R) times h^2 or k^2 h^3; no contrast).
// Scratch (double2, offsets from the launch's base): U at u_off (m x rcap),
// V at v_off (n x rcap), four rcap x rcap matrices at w_off, and the output
// U' (m x rcap) then V' (n x rcap) at o_off.
struct AcaItem {
  int32_t t_off, m, s_off, n;
  int32_t inst, r_max, rcap, pad;
  int64_t u_off, v_off, w_off, o_off;
};
// k: rank of the cross approximation (0: no pivot above 1e-300 anywhere);
// rank: after recompression; status 1 when k reached rcap below r_max
// without meeting the stopping test (the block needs more columns).
struct AcaOut {
  int32_t k, rank, status, pad;
};
constexpr int kAcaMaxCols = 128;  // rcap limit of the device compression
// Cross approximation of every item (one workgroup each), rules:
//   start at row 0; residual row = A[i,:] - sum_l u_l[i] v_l;
//   if max|row| <= 1e-300 mark row i used and take the next unused row in
//   index order (stop when none is left);
//   pivot j = first index of max|row|; v = row / row[j];
//   u = A[:,j] - sum_l v_l[j] u_l;
//   ||S||_F^2 of S = sum_l u_l v_l^T updated with 2 Re(sum_l (u_l^H u)(v_l^H v))
//   + (||u|| ||v||)^2; stop after the step where ||u|| ||v|| <= eps ||S||_F
//   or the rank reaches r_max; next row = first index of max|u| over unused
//   rows.  max_m: largest m of the launch (its row marks live in LDS).
hipError_t launch_aca(const AcaItem* items, int n_items, int max_m, const double* xyz,
                      const EntryInst* inst, double eps, double2* ws, AcaOut* out,
                      hipStream_t st);
// Recompression of every item with status 0 and k >= 1: U = Qu Ru and
// V = Qv Rv (Gram-Schmidt with one reorthogonalisation), Ru Rv^T = Phi S Psi^H
// by one-sided Jacobi, and the smallest rank >= 1 whose discarded singular
// values have 2-norm <= eps times the 2-norm of all of them;
// U' = Qu Phi_r S_r and V' = Qv conj(Psi_r) written at o_off; rank set.
hipError_t launch_recompress(const AcaItem* items, int n_items, double eps, double2* ws,
                             AcaOut* out, hipStream_t st);

// Segments (src_off, dst_off, len), three int64 each: len elements copied
// from src + src_off to dst + dst_off.
hipError_t launch_seg_copy(const double2* src, double2* dst, const int64_t* seg, int n_seg,
                           hipStream_t st);

}  // namespace hm
