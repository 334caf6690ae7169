// Device kernels of the half-storage build: the symmetric factor of each
// leaf block (D = C C^T, C lower triangular, no pivoting) with its inverse,
// and a batched complex matrix product for the scaled blocks
// S_ts = C_t^{-1} Z_ts C_s^{-T} and the scaled far factors.
#include <hip/hip_runtime.h>

#include "build_dev.h"

namespace hm {

namespace {

constexpr int kT = 256;  // threads per workgroup

__device__ __forceinline__ double2 cz() { return make_double2(0.0, 0.0); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

// a / b = a conj(b) / |b|^2
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// principal square root (non-negative real part)
__device__ __forceinline__ double2 csqrt(double2 z) {
  const double r = hypot(z.x, z.y);
  if (r == 0.0) return cz();
  if (z.x >= 0.0) {
    const double t = sqrt(0.5 * (r + z.x));
    return make_double2(t, z.y / (2.0 * t));
  }
  const double t = sqrt(0.5 * (r - z.x));
  return make_double2(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}

__device__ __forceinline__ double cabs(double2 z) { return hypot(z.x, z.y); }

// Workgroup reductions (every thread receives the result).
__device__ double wg_max(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < kT / 64; ++w) r = fmax(r, red[w]);
  return r;
}

__device__ double wg_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < kT / 64; ++w) r += red[w];
  return r;
}

// One workgroup per leaf.  The lower triangle of D (then C, then C^{-1})
// lives in LDS, packed by columns: entry (i, k), i >= k, at k m - k (k - 1)
// / 2 + i - k.  Right-looking factorisation: for each column j the pivot
// C_jj = sqrt(updated D_jj), C_ij = updated D_ij / C_jj below it, and the
// trailing lower triangle is updated by C_ij C_kj.  The inverse is formed
// in place from the last column back: X_jj = 1 / C_jj and
// X[j+1:, j] = -X[j+1:, j+1:] C[j+1:, j] X_jj, where X[j+1:, j+1:] is the
// inverse of the trailing block already in place.
__global__ __launch_bounds__(kT) void k_csym(const double2* __restrict__ d,
                                             const int64_t* __restrict__ d_off,
                                             const int32_t* __restrict__ leaf_m,
                                             const int32_t* __restrict__ leaf_off,
                                             const double* __restrict__ chi, double2* cf,
                                             double2* cft, double2* ch, double2* cht,
                                             const int64_t* __restrict__ c_off, int32_t* ok) {
  extern __shared__ double2 P[];
  __shared__ double2 col[kCsymMaxLeaf];
  __shared__ double red[kT / 64];
  __shared__ double2 s_piv;
  __shared__ int s_fail;
  const int a = blockIdx.x;
  const int m = leaf_m[a];
  const int64_t ld = m + (m & 1);
  const int tid = threadIdx.x;
  const double2* D = d + d_off[a];
  const double* ch_a = chi ? chi + leaf_off[a] : nullptr;
  // entry (i, k) of the block to factor: D, or D diag(1/chi)
  auto dval = [&](int i, int k) {
    const double2 v = D[i + k * ld];
    if (!ch_a) return v;
    const double s = 1.0 / ch_a[k];
    return make_double2(v.x * s, v.y * s);
  };
  auto at = [m](int i, int k) { return k * m - (k * (k - 1)) / 2 + (i - k); };
  const int npk = m * (m + 1) / 2;
  // lower triangle of D into LDS; max |D_jj|, max |D_ij| and ||D||_F^2
  // (D symmetric: the upper triangle mirrors the lower one)
  double dmax = 0.0, amax = 0.0, dn2 = 0.0;
  for (int e = tid; e < m * m; e += kT) {
    const int i = e % m, k = e / m;
    if (i < k) continue;
    const double2 v = dval(i, k);
    P[at(i, k)] = v;
    const double av = cabs(v);
    amax = fmax(amax, av);
    dn2 += (i == k ? 1.0 : 2.0) * av * av;
    if (i == k) dmax = fmax(dmax, av);
  }
  dmax = wg_max(dmax, red);
  amax = wg_max(amax, red);
  dn2 = wg_sum(dn2, red);
  if (tid == 0) s_fail = !(dmax > 0.0);
  __syncthreads();
  // factor
  for (int j = 0; j < m; ++j) {
    if (tid == 0) {
      const double2 s = P[at(j, j)];
      const double mag = cabs(s);
      if (!(mag > 1e-10 * dmax)) s_fail = 1;
      const double2 r = csqrt(s);
      P[at(j, j)] = r;
      s_piv = mag > 0.0 ? r : make_double2(1.0, 0.0);
    }
    __syncthreads();
    const double2 piv = s_piv;
    for (int i = j + 1 + tid; i < m; i += kT) P[at(i, j)] = cdiv(P[at(i, j)], piv);
    __syncthreads();
    const int i = tid & (kCsymMaxLeaf - 1);
    for (int k = j + 1 + tid / kCsymMaxLeaf; k < m; k += kT / kCsymMaxLeaf)
      if (i >= k && i < m) {
        double2 v = P[at(i, k)];
        const double2 p = cmul(P[at(i, j)], P[at(k, j)]);
        v.x -= p.x;
        v.y -= p.y;
        P[at(i, k)] = v;
      }
    __syncthreads();
  }
  // element growth, C and C^T out
  double cmax = 0.0;
  const int64_t co = c_off[a];
  for (int e = tid; e < npk; e += kT) {
    int k = 0;
    while (at(m - 1, k) < e) ++k;  // column of packed entry e
    const int i = k + (e - at(k, k));
    const double2 v = P[e];
    cmax = fmax(cmax, cabs(v));
    cf[co + i + k * ld] = v;
    cft[co + k + i * ld] = v;
  }
  cmax = wg_max(cmax, red);
  // backward error ||C C^T - D||_F (lower triangle, off-diagonal twice)
  double rn2 = 0.0;
  for (int e = tid; e < npk; e += kT) {
    int k = 0;
    while (at(m - 1, k) < e) ++k;
    const int i = k + (e - at(k, k));  // entry (i, k) of C C^T, i >= k
    const double2 dv = dval(i, k);
    double2 acc = make_double2(-dv.x, -dv.y);
    for (int q = 0; q <= k; ++q) cfma(acc, P[at(i, q)], P[at(k, q)]);
    rn2 += (i == k ? 1.0 : 2.0) * (acc.x * acc.x + acc.y * acc.y);
  }
  rn2 = wg_sum(rn2, red);
  if (tid == 0 && !(cmax * cmax <= 1e2 * amax && rn2 <= 1e-28 * dn2)) s_fail = 1;
  __syncthreads();
  // inverse in place
  for (int j = m - 1; j >= 0; --j) {
    for (int i = j + 1 + tid; i < m; i += kT) col[i] = P[at(i, j)];
    __syncthreads();
    const double2 xjj = cdiv(make_double2(1.0, 0.0), P[at(j, j)]);
    for (int i = j + 1 + tid; i < m; i += kT) {
      double2 acc = cz();
      for (int k = j + 1; k <= i; ++k) cfma(acc, P[at(i, k)], col[k]);
      const double2 x = cmul(acc, xjj);
      P[at(i, j)] = make_double2(-x.x, -x.y);
    }
    __syncthreads();
    if (tid == 0) P[at(j, j)] = xjj;
    __syncthreads();
  }
  // C^{-1} and C^{-T} out; a non-finite entry rejects the factor
  int bad = 0;
  for (int e = tid; e < npk; e += kT) {
    int k = 0;
    while (at(m - 1, k) < e) ++k;
    const int i = k + (e - at(k, k));
    const double2 v = P[e];
    if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
    ch[co + i + k * ld] = v;
    cht[co + k + i * ld] = v;
  }
  const double anybad = wg_max((double)bad, red);
  if (tid == 0) ok[a] = (s_fail || anybad > 0.0) ? 0 : 1;
}

// C = op(A) op(B) per item, one 64 x 64 output tile per workgroup: thread
// (tx, ty) = (tid % 16, tid / 16) owns rows i0 + tx + 16 r and columns
// j0 + ty + 16 c (r, c < 4); k in steps of 16 through LDS, entries past the
// operands' edges read as zero.
__global__ __launch_bounds__(kT) void k_cgemm(const double2* __restrict__ A,
                                              const double2* __restrict__ B, double2* C,
                                              const GemmItem* __restrict__ items,
                                              const GemmTile* __restrict__ tiles) {
  constexpr int BK = 16;
  __shared__ double2 As[BK][kGemmTile + 1];
  __shared__ double2 Bs[BK][kGemmTile + 1];
  const GemmTile t = tiles[blockIdx.x];
  const GemmItem g = items[t.item];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  double2 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = cz();
  for (int k0 = 0; k0 < g.k; k0 += BK) {
    for (int e = tid; e < BK * kGemmTile; e += kT) {
      const int ii = e % kGemmTile, kk = e / kGemmTile;
      const int i = t.i0 + ii, k = k0 + kk;
      double2 v = cz();
      if (i < g.m && k < g.k)
        v = g.ta ? A[g.a_off + k + (int64_t)i * g.lda] : A[g.a_off + i + (int64_t)k * g.lda];
      As[kk][ii] = v;
    }
    for (int e = tid; e < BK * kGemmTile; e += kT) {
      const int kk = e % BK, jj = e / BK;
      const int k = k0 + kk, j = t.j0 + jj;
      double2 v = cz();
      if (k < g.k && j < g.n)
        v = g.tb ? B[g.b_off + j + (int64_t)k * g.ldb] : B[g.b_off + k + (int64_t)j * g.ldb];
      Bs[kk][jj] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < BK; ++kk) {
      double2 av[4], bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = As[kk][tx + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = Bs[kk][ty + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) cfma(acc[r][c], av[r], bv[c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = t.i0 + tx + 16 * r, j = t.j0 + ty + 16 * c;
      if (i < g.m && j < g.n) C[g.c_off + i + (int64_t)j * g.ldc] = acc[r][c];
    }
}

// Contrast scaling of block-diagonal panels (one workgroup per leaf).
__global__ __launch_bounds__(kT) void k_panel_scale(const double2* in, double2* out,
                                                    const int64_t* __restrict__ c_off,
                                                    const int32_t* __restrict__ leaf_m,
                                                    const int32_t* __restrict__ leaf_off,
                                                    const double* __restrict__ chi, int mode) {
  const int a = blockIdx.x;
  const int m = leaf_m[a];
  const int64_t ld = m + (m & 1), co = c_off[a];
  const double* c = chi + leaf_off[a];
  for (int e = threadIdx.x; e < m * m; e += kT) {
    const int i = e % m, k = e / m;
    const double s = mode == 0 ? 1.0 / c[i] : (mode == 1 ? 1.0 / c[k] : c[k]);
    const double2 v = in[co + i + k * ld];
    out[co + i + k * ld] = make_double2(v.x * s, v.y * s);
  }
}

// One workgroup per near block; consecutive threads take consecutive rows
// of a column, so the stores of a wave are contiguous.
__global__ __launch_bounds__(kT) void k_fill_near(const FillItem* __restrict__ items,
                                                  const double* __restrict__ xyz,
                                                  const double* __restrict__ chi,
                                                  const int32_t* __restrict__ leaf_off,
                                                  const int32_t* __restrict__ leaf_m,
                                                  const int32_t* __restrict__ leaf_inst,
                                                  const EntryInst* __restrict__ inst,
                                                  double2* __restrict__ out, int32_t* bad) {
  const FillItem it = items[blockIdx.x];
  const int m = leaf_m[it.t], n = leaf_m[it.s], ld = it.ld;
  const int t0 = leaf_off[it.t], s0 = leaf_off[it.s];
  const EntryInst P = inst[leaf_inst[it.t]];
  const bool surface = P.kind == 0;
  const double scale = surface ? P.h * P.h : P.k * P.k * P.h * P.h * P.h;
  double2* dst = out + it.dst;
  int close = 0;
  for (int e = threadIdx.x; e < ld * n; e += kT) {
    const int j = e / ld, i = e - j * ld;
    double2 v = cz();
    if (i < m) {
      const int gi = t0 + i, gj = s0 + j;
      if (gi == gj) {
        v = surface ? make_double2(2.0 * P.h, 0.2 * P.h) : make_double2(1.0 / chi[gi] + 0.5, 0.0);
      } else {
        const double dx = xyz[3 * gi] - xyz[3 * gj], dy = xyz[3 * gi + 1] - xyz[3 * gj + 1],
                     dz = xyz[3 * gi + 2] - xyz[3 * gj + 2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < 1e-24) close = 1;
        const double r = sqrt(r2);
        double sn, cs;
        sincos(P.k * r, &sn, &cs);
        double a = scale / (4.0 * M_PI * r);
        if (!surface) a *= chi[gj];
        v = make_double2(a * cs, -a * sn);
      }
    }
    dst[e] = v;
  }
  if (close) atomicOr(bad, 1);
}

__global__ __launch_bounds__(kT) void k_seg_copy(const double2* __restrict__ src,
                                                 double2* __restrict__ dst,
                                                 const int64_t* __restrict__ seg) {
  const int64_t so = seg[3 * blockIdx.x], d0 = seg[3 * blockIdx.x + 1], len = seg[3 * blockIdx.x + 2];
  for (int64_t e = threadIdx.x; e < len; e += kT) dst[d0 + e] = src[so + e];
}

}  // namespace

hipError_t launch_panel_scale(const double2* in, double2* out, const int64_t* c_off,
                              const int32_t* leaf_m, const int32_t* leaf_off, const double* chi,
                              int nl, int mode, hipStream_t st) {
  if (nl <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_panel_scale, dim3(nl), dim3(kT), 0, st, in, out, c_off, leaf_m, leaf_off,
                     chi, mode);
  return hipGetLastError();
}

hipError_t launch_csym(const double2* d, const int64_t* d_off, const int32_t* leaf_m,
                       const int32_t* leaf_off, const double* chi, int nl, int max_m, double2* cf,
                       double2* cft, double2* ch, double2* cht, const int64_t* c_off, int32_t* ok,
                       hipStream_t st) {
  if (nl <= 0) return hipSuccess;
  if (max_m > kCsymMaxLeaf) return hipErrorInvalidValue;
  const size_t lds = sizeof(double2) * (size_t)max_m * (max_m + 1) / 2;
  hipError_t e = hipFuncSetAttribute((const void*)k_csym,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_csym, dim3(nl), dim3(kT), lds, st, d, d_off, leaf_m, leaf_off, chi, cf, cft,
                     ch, cht, c_off, ok);
  return hipGetLastError();
}

hipError_t launch_fill_near(const FillItem* items, int n_items, const double* xyz,
                            const double* chi, const int32_t* leaf_off, const int32_t* leaf_m,
                            const int32_t* leaf_inst, const EntryInst* inst, double2* out,
                            int32_t* bad, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_near, dim3(n_items), dim3(kT), 0, st, items, xyz, chi, leaf_off, leaf_m,
                     leaf_inst, inst, out, bad);
  return hipGetLastError();
}

hipError_t launch_seg_copy(const double2* src, double2* dst, const int64_t* seg, int n_seg,
                           hipStream_t st) {
  if (n_seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seg_copy, dim3(n_seg), dim3(kT), 0, st, src, dst, seg);
  return hipGetLastError();
}

hipError_t launch_cgemm(const double2* a, const double2* b, double2* c, const GemmItem* items,
                        const GemmTile* tiles, int n_tiles, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cgemm, dim3(n_tiles), dim3(kT), 0, st, a, b, c, items, tiles);
  return hipGetLastError();
}

}  // namespace hm
