// Far-block compression on the device (Sec. III): adaptive cross
// approximation with partial pivoting, then recompression of the two
// factors by Gram-Schmidt QR and a one-sided Jacobi SVD of the small core.
// One workgroup per block; the factors live in a scratch buffer laid out by
// the host (AcaItem offsets).
#include <hip/hip_runtime.h>

#include <climits>

#include "build_dev.h"

namespace hm {

namespace {

constexpr int kT = 256;       // threads per workgroup
constexpr int kW = kT / 64;   // waves per workgroup

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double cnorm(double2 a) { return a.x * a.x + a.y * a.y; }

// a / b by Smith's method (scaled by the larger part of b)
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.x * r + b.y;
  return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}

// Kernel part of the entry between points i and j (tree order, i != j):
// scale e^{-jkR} / (4 pi R).
__device__ __forceinline__ double2 kern(const double* __restrict__ xyz, int i, int j, double k,
                                        double scale) {
  const double dx = xyz[3 * i] - xyz[3 * j], dy = xyz[3 * i + 1] - xyz[3 * j + 1],
               dz = xyz[3 * i + 2] - xyz[3 * j + 2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  double s, c;
  sincos(k * r, &s, &c);
  const double a = scale / (4.0 * M_PI * r);
  return make_double2(a * c, -a * s);
}

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Workgroup sum, every thread receives it (fixed summation order).
__device__ double gsum(double v, double* red) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < kW; ++w) r += red[w];
  return r;
}

// Largest v over the workgroup with the smallest index among equal values
// (values that are not numbers never win); every thread receives it.
__device__ void gargmax(double& v, int& idx, double* redv, int* redi) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o);
    const int oi = __shfl_xor(idx, o);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    redv[threadIdx.x >> 6] = v;
    redi[threadIdx.x >> 6] = idx;
  }
  __syncthreads();
  v = redv[0];
  idx = redi[0];
  for (int w = 1; w < kW; ++w)
    if (redv[w] > v || (redv[w] == v && redi[w] < idx)) {
      v = redv[w];
      idx = redi[w];
    }
}

__device__ int gmin(int v, int* red) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  int r = red[0];
  for (int w = 1; w < kW; ++w) r = min(r, red[w]);
  return r;
}

__device__ __forceinline__ bool is_used(const uint32_t* used, int q) {
  return (used[q >> 5] >> (q & 31)) & 1u;
}

__global__ __launch_bounds__(kT) void k_aca(const AcaItem* __restrict__ items,
                                            const double* __restrict__ xyz,
                                            const EntryInst* __restrict__ inst, double eps,
                                            double2* __restrict__ ws, AcaOut* __restrict__ out) {
  extern __shared__ uint32_t used[];  // row marks, (m + 31) / 32 words
  __shared__ double redv[kW];
  __shared__ int redi[kW];
  __shared__ double2 du[kAcaMaxCols], dv[kAcaMaxCols];
  const AcaItem it = items[blockIdx.x];
  const int m = it.m, n = it.n, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const EntryInst P = inst[it.inst];
  const double scale = P.kind == 0 ? P.h * P.h : P.k * P.k * P.h * P.h * P.h;
  double2* U = ws + it.u_off;
  double2* V = ws + it.v_off;
  for (int q = tid; q < ((m + 31) >> 5); q += kT) used[q] = 0u;
  __syncthreads();
  int i = 0, k = 0, status = 0;
  double s2 = 0.0;
  for (;;) {
    // residual row i into column k of V
    double best = -1.0;
    int jp = INT_MAX;
    for (int j = tid; j < n; j += kT) {
      double2 z = kern(xyz, it.t_off + i, it.s_off + j, P.k, scale);
      for (int l = 0; l < k; ++l) z = csub(z, cmul(U[i + (int64_t)l * m], V[j + (int64_t)l * n]));
      V[j + (int64_t)k * n] = z;
      const double a = hypot(z.x, z.y);
      if (a > best) {
        best = a;
        jp = j;
      }
    }
    if (tid == 0) used[i >> 5] |= 1u << (i & 31);
    gargmax(best, jp, redv, redi);
    if (best <= 1e-300) {
      // no pivot in this row: the next unused row in index order
      int nxt = INT_MAX;
      for (int q = tid; q < m; q += kT)
        if (!is_used(used, q)) {
          nxt = q;
          break;
        }
      nxt = gmin(nxt, redi);
      if (nxt == INT_MAX) break;
      i = nxt;
      continue;
    }
    const double2 piv = V[jp + (int64_t)k * n];
    __syncthreads();  // every thread holds the pivot before its entry is scaled
    for (int j = tid; j < n; j += kT) V[j + (int64_t)k * n] = cdiv(V[j + (int64_t)k * n], piv);
    // residual column jp into column k of U
    for (int q = tid; q < m; q += kT) {
      double2 z = kern(xyz, it.t_off + q, it.s_off + jp, P.k, scale);
      for (int l = 0; l < k; ++l) z = csub(z, cmul(V[jp + (int64_t)l * n], U[q + (int64_t)l * m]));
      U[q + (int64_t)k * m] = z;
    }
    __syncthreads();
    // u_l^H u and v_l^H v for the earlier columns (wave w takes l = w, w + 4, ...)
    for (int l = w; l < k; l += kW) {
      double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
      for (int q = lane; q < m; q += 64)
        a = cadd(a, cmulc(U[q + (int64_t)l * m], U[q + (int64_t)k * m]));
      for (int j = lane; j < n; j += 64)
        b = cadd(b, cmulc(V[j + (int64_t)l * n], V[j + (int64_t)k * n]));
      a.x = wsum(a.x);
      a.y = wsum(a.y);
      b.x = wsum(b.x);
      b.y = wsum(b.y);
      if (lane == 0) {
        du[l] = a;
        dv[l] = b;
      }
    }
    double nu2 = 0.0, nv2 = 0.0;
    for (int q = tid; q < m; q += kT) nu2 += cnorm(U[q + (int64_t)k * m]);
    for (int j = tid; j < n; j += kT) nv2 += cnorm(V[j + (int64_t)k * n]);
    nu2 = gsum(nu2, redv);
    nv2 = gsum(nv2, redv);  // its barriers also publish du and dv
    double2 cross = make_double2(0.0, 0.0);
    for (int l = 0; l < k; ++l) cross = cadd(cross, cmul(du[l], dv[l]));
    const double nuv = sqrt(nu2) * sqrt(nv2);
    s2 += 2.0 * cross.x + nuv * nuv;
    ++k;
    if (nuv <= eps * sqrt(s2) || k >= it.r_max) break;
    if (k >= it.rcap) {
      status = 1;
      break;
    }
    // next row: first index of max |u| over the unused rows
    double bu = -1.0;
    int nxt = INT_MAX;
    for (int q = tid; q < m; q += kT) {
      if (is_used(used, q)) continue;
      const double a = hypot(U[q + (int64_t)(k - 1) * m].x, U[q + (int64_t)(k - 1) * m].y);
      if (a > bu) {
        bu = a;
        nxt = q;
      }
    }
    gargmax(bu, nxt, redv, redi);
    if (nxt == INT_MAX) break;
    i = nxt;
  }
  if (tid == 0) out[blockIdx.x] = AcaOut{k, 0, status, 0};
}

// Orthonormal Q (in place of X, rows x k, leading dimension rows) and upper
// triangular R (leading dimension rc, zeroed by the caller) with X = Q R:
// classical Gram-Schmidt with one reorthogonalisation.  A column whose
// remainder falls to 1e-13 of its norm is dependent on the earlier ones: its
// Q column is set to zero with R_cc = 0 (X = Q R still holds to rounding).
__device__ void orthonormalize(double2* X, int rows, int k, double2* R, int rc, double2* dd,
                               double* red) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int c = 0; c < k; ++c) {
    double2* xc = X + (int64_t)c * rows;
    double n0 = 0.0;
    for (int q = tid; q < rows; q += kT) n0 += cnorm(xc[q]);
    n0 = gsum(n0, red);
    for (int pass = 0; pass < 2 && c > 0; ++pass) {
      for (int l = w; l < c; l += kW) {
        double2 a = make_double2(0.0, 0.0);
        for (int q = lane; q < rows; q += 64) a = cadd(a, cmulc(X[q + (int64_t)l * rows], xc[q]));
        a.x = wsum(a.x);
        a.y = wsum(a.y);
        if (lane == 0) dd[l] = a;
      }
      __syncthreads();
      for (int q = tid; q < rows; q += kT) {
        double2 z = xc[q];
        for (int l = 0; l < c; ++l) z = csub(z, cmul(dd[l], X[q + (int64_t)l * rows]));
        xc[q] = z;
      }
      for (int l = tid; l < c; l += kT) R[l + (int64_t)c * rc] = cadd(R[l + (int64_t)c * rc], dd[l]);
      __syncthreads();
    }
    double n2 = 0.0;
    for (int q = tid; q < rows; q += kT) n2 += cnorm(xc[q]);
    n2 = gsum(n2, red);
    const bool dep = !(n2 > 1e-26 * n0);
    const double inv = dep ? 0.0 : 1.0 / sqrt(n2);
    for (int q = tid; q < rows; q += kT) xc[q] = make_double2(xc[q].x * inv, xc[q].y * inv);
    if (tid == 0) R[c + (int64_t)c * rc] = make_double2(dep ? 0.0 : sqrt(n2), 0.0);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kT) void k_recompress(const AcaItem* __restrict__ items, double eps,
                                                   double2* __restrict__ ws,
                                                   AcaOut* __restrict__ out) {
  __shared__ double red[kW];
  __shared__ double2 dd[kAcaMaxCols];
  __shared__ double sig[kAcaMaxCols];
  __shared__ int ord[kAcaMaxCols];
  __shared__ int s_keep, s_rot;
  const AcaItem it = items[blockIdx.x];
  const AcaOut o = out[blockIdx.x];
  if (o.status != 0 || o.k < 1) return;
  const int k = o.k, m = it.m, n = it.n, rc = it.rcap, tid = threadIdx.x, lane = tid & 63,
            w = tid >> 6;
  double2* U = ws + it.u_off;
  double2* V = ws + it.v_off;
  double2* Ru = ws + it.w_off;
  double2* Rv = Ru + (int64_t)rc * rc;
  double2* C = Rv + (int64_t)rc * rc;
  double2* Psi = C + (int64_t)rc * rc;
  for (int e = tid; e < k * k; e += kT) {
    Ru[e % k + (int64_t)(e / k) * rc] = make_double2(0.0, 0.0);
    Rv[e % k + (int64_t)(e / k) * rc] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  orthonormalize(U, m, k, Ru, rc, dd, red);
  orthonormalize(V, n, k, Rv, rc, dd, red);
  // C = Ru Rv^T, Psi = I
  for (int e = tid; e < k * k; e += kT) {
    const int i = e % k, j = e / k;
    double2 acc = make_double2(0.0, 0.0);
    for (int l = 0; l < k; ++l)
      acc = cadd(acc, cmul(Ru[i + (int64_t)l * rc], Rv[j + (int64_t)l * rc]));
    C[i + (int64_t)j * rc] = acc;
    Psi[i + (int64_t)j * rc] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // one-sided Jacobi: C Psi -> Phi Sigma.  Each sweep takes every pair of
  // columns once, in rounds of disjoint pairs (circle method; index k is a
  // dummy when k is odd), one pair per wave at a time; a pair is rotated
  // while its columns' inner product exceeds 1e-15 of the product of their
  // norms (a tighter test sits at the rounding level of the inner product
  // and keeps rotating to the sweep limit).
  const int kk = k + (k & 1);
  for (int sweep = 0; sweep < 80; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int round = 0; round < kk - 1; ++round) {
      for (int pi = w; pi < kk / 2; pi += kW) {
        const int pa = pi == 0 ? 0 : (pi - 1 + round) % (kk - 1) + 1;
        const int qa = (kk - 1 - pi - 1 + round) % (kk - 1) + 1;
        if (pa >= k || qa >= k) continue;
        const int p = min(pa, qa), q = max(pa, qa);
        double a2 = 0.0, b2 = 0.0;
        double2 g = make_double2(0.0, 0.0);
        for (int i = lane; i < k; i += 64) {
          const double2 cp = C[i + (int64_t)p * rc], cq = C[i + (int64_t)q * rc];
          a2 += cnorm(cp);
          b2 += cnorm(cq);
          g = cadd(g, cmulc(cp, cq));
        }
        a2 = wsum(a2);
        b2 = wsum(b2);
        g.x = wsum(g.x);
        g.y = wsum(g.y);
        const double ag = hypot(g.x, g.y);
        if (ag == 0.0 || ag <= 1e-15 * sqrt(a2 * b2)) continue;
        if (lane == 0) s_rot = 1;
        const double2 eph = make_double2(g.x / ag, -g.y / ag);  // e^{-i phi}
        const double zeta = (b2 - a2) / (2.0 * ag);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
        for (int i = lane; i < k; i += 64) {
          const double2 cp = C[i + (int64_t)p * rc];
          const double2 cq = cmul(eph, C[i + (int64_t)q * rc]);
          C[i + (int64_t)p * rc] = make_double2(cs * cp.x - sn * cq.x, cs * cp.y - sn * cq.y);
          C[i + (int64_t)q * rc] = make_double2(sn * cp.x + cs * cq.x, sn * cp.y + cs * cq.y);
          const double2 vp = Psi[i + (int64_t)p * rc];
          const double2 vq = cmul(eph, Psi[i + (int64_t)q * rc]);
          Psi[i + (int64_t)p * rc] = make_double2(cs * vp.x - sn * vq.x, cs * vp.y - sn * vq.y);
          Psi[i + (int64_t)q * rc] = make_double2(sn * vp.x + cs * vq.x, sn * vp.y + cs * vq.y);
        }
      }
      __syncthreads();
    }
    const bool again = s_rot != 0;
    __syncthreads();  // s_rot read by all before the next sweep clears it
    if (!again) break;
  }
  // singular values (column norms), decreasing (stable), and the kept rank
  for (int j = tid; j < k; j += kT) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += cnorm(C[i + (int64_t)j * rc]);
    sig[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < k; j += kT) {
    int r = 0;
    for (int i = 0; i < k; ++i) r += (sig[i] > sig[j] || (sig[i] == sig[j] && i < j)) ? 1 : 0;
    ord[r] = j;
  }
  __syncthreads();
  if (tid == 0) {
    double total2 = 0.0;
    for (int r = 0; r < k; ++r) total2 += sig[ord[r]] * sig[ord[r]];
    const double total = sqrt(total2);
    int keep = k;
    for (int cand = 1; cand <= k; ++cand) {
      double tail2 = 0.0;
      for (int r = cand; r < k; ++r) tail2 += sig[ord[r]] * sig[ord[r]];
      if (sqrt(tail2) <= eps * total) {
        keep = cand;
        break;
      }
    }
    s_keep = keep;
  }
  __syncthreads();
  const int keep = s_keep;
  // U' = Qu (C Psi)[:, ord[:keep]], V' = Qv conj(Psi)[:, ord[:keep]]
  double2* Uo = ws + it.o_off;
  double2* Vo = Uo + (int64_t)m * rc;
  for (int q = tid; q < m; q += kT)
    for (int j = 0; j < keep; ++j) {
      const double2* cj = C + (int64_t)ord[j] * rc;
      double2 acc = make_double2(0.0, 0.0);
      for (int l = 0; l < k; ++l) acc = cadd(acc, cmul(U[q + (int64_t)l * m], cj[l]));
      Uo[q + (int64_t)j * m] = acc;
    }
  for (int q = tid; q < n; q += kT)
    for (int j = 0; j < keep; ++j) {
      const double2* pj = Psi + (int64_t)ord[j] * rc;
      double2 acc = make_double2(0.0, 0.0);
      for (int l = 0; l < k; ++l) acc = cadd(acc, cmulc(pj[l], V[q + (int64_t)l * n]));
      Vo[q + (int64_t)j * n] = acc;
    }
  if (tid == 0) out[blockIdx.x].rank = keep;
}

}  // namespace

hipError_t launch_aca(const AcaItem* items, int n_items, int max_m, const double* xyz,
                      const EntryInst* inst, double eps, double2* ws, AcaOut* out,
                      hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  const size_t lds = sizeof(uint32_t) * (size_t)((max_m + 31) / 32);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_aca,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_aca, dim3(n_items), dim3(kT), lds, st, items, xyz, inst, eps, ws, out);
  return hipGetLastError();
}

hipError_t launch_recompress(const AcaItem* items, int n_items, double eps, double2* ws,
                             AcaOut* out, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_recompress, dim3(n_items), dim3(kT), 0, st, items, eps, ws, out);
  return hipGetLastError();
}

}  // namespace hm
