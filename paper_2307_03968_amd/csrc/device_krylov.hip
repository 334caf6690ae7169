// Krylov kernels of libhmps: the vector work of restarted, right-
// preconditioned GMRES on Z_l (Saad and Schultz 1986; the flexible form of
// Saad 1993, which keeps the preconditioned vectors), one independent
// Krylov space per right-hand side.  The paper names GMRES as the iterative
// solver its power series is compared with; here the series P_K of Sec. IV
// serves as the preconditioner, which gives a converged solve also where
// rho(D^{-1} R_l) >= 1 and the series alone diverges.
//
// Vectors are N x nrhs column-major blocks (leading dimension ld); basis
// vector i of a block list starts at base + i * vs.  Per right-hand side c:
//   dots     h[i] = sum_r conj(V_i[r, c]) w[r, c], i < nvec, in two passes
//            (per-workgroup partial sums, then a fixed-order sum), so the
//            result does not depend on timing
//   update   y[r, c] += alpha sum_i V_i[r, c] coef[c, i]
//   step     the new Hessenberg column: previous Givens rotations, a new
//            rotation, the residual estimate |g_{j+1}| / ||b||
//   solve    the upper-triangular least-squares system R y = g
// The small per-column steps run one thread per right-hand side.
#include <hip/hip_runtime.h>

#include "dev.h"
#include "krylov.h"

namespace hm {

namespace {

constexpr int kKT = 256;  // threads per workgroup (one row each)

__device__ __forceinline__ double2 kzero() { return make_double2(0.0, 0.0); }

// conj(a) b
__device__ __forceinline__ double2 conj_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

unsigned blocks_of(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// partial[(c nvec + i) nblk + blk] = sum over the rows of workgroup blk of
// conj(V_i[r, c]) w[r, c]; grid (nblk, nrhs)
__global__ __launch_bounds__(kKT) void k_kdots(const double2* __restrict__ V, int64_t vs,
                                               int64_t ld, const double2* __restrict__ w,
                                               int64_t n, int nvec,
                                               double2* __restrict__ partial) {
  __shared__ double2 red[kKT / 64][kMaxKrylov + 1];
  const int blk = blockIdx.x, c = blockIdx.y, nblk = gridDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r = (int64_t)blk * kKT + threadIdx.x;
  const bool ok = r < n;
  const int64_t q = r + (int64_t)c * ld;
  const double2 wv = ok ? w[q] : kzero();
  for (int i = 0; i < nvec; ++i) {
    double2 p = conj_mul(ok ? V[(int64_t)i * vs + q] : kzero(), wv);
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) {
      p.x += __shfl_xor(p.x, sh);
      p.y += __shfl_xor(p.y, sh);
    }
    if (lane == 0) red[wave][i] = p;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nvec; i += kKT) {
    double2 s = red[0][i];
#pragma unroll
    for (int k = 1; k < kKT / 64; ++k) {
      s.x += red[k][i].x;
      s.y += red[k][i].y;
    }
    partial[((int64_t)c * nvec + i) * nblk + blk] = s;
  }
}

// out[c ldo + i] = sum_blk partial[(c nvec + i) nblk + blk], in order
__global__ void k_kreduce(const double2* __restrict__ partial, int nblk, int nvec, int nrhs,
                          double2* __restrict__ out, int ldo) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nvec * nrhs) return;
  const int c = t / nvec, i = t % nvec;
  const double2* p = partial + (int64_t)t * nblk;
  double2 s = kzero();
  for (int b = 0; b < nblk; ++b) {
    s.x += p[b].x;
    s.y += p[b].y;
  }
  out[(int64_t)c * ldo + i] = s;
}

// y[r, c] += alpha sum_{i < nvec} V_i[r, c] coef[c ldc + i]; grid (rows, nrhs)
__global__ __launch_bounds__(kKT) void k_kupdate(double alpha, const double2* __restrict__ V,
                                                 int64_t vs, int64_t ld,
                                                 const double2* __restrict__ coef, int ldc,
                                                 int nvec, double2* __restrict__ y, int64_t n) {
  const int c = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * kKT + threadIdx.x;
  if (r >= n) return;
  const int64_t q = r + (int64_t)c * ld;
  const double2* cf = coef + (int64_t)c * ldc;
  double2 s = kzero();
  for (int i = 0; i < nvec; ++i) {
    const double2 p = cmul(V[(int64_t)i * vs + q], cf[i]);
    s.x += p.x;
    s.y += p.y;
  }
  y[q].x += alpha * s.x;
  y[q].y += alpha * s.y;
}

// v[r, c] = s[c] v[r, c] (in place)
__global__ __launch_bounds__(kKT) void k_kscale(double2* v, int64_t ld, const double* __restrict__ s,
                                                int64_t n) {
  const int c = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * kKT + threadIdx.x;
  if (r >= n) return;
  const int64_t q = r + (int64_t)c * ld;
  const double f = s[c];
  v[q] = make_double2(f * v[q].x, f * v[q].y);
}

// Start of a cycle: r = b - Z x is in the first basis slot, rn2 = ||r||^2
// and bn2 = ||b||^2 per column (real parts of the dot results).
__global__ void k_kstart(KrylovState S, const double2* __restrict__ rn2,
                         const double2* __restrict__ bn2, double tol, int nrhs) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  // a NaN norm stays NaN (fmax would turn it into 0, i.e. b = 0)
  const double rq = rn2[c].x, bq = bn2[c].x;
  const double rn = rq > 0.0 ? sqrt(rq) : (rq <= 0.0 ? 0.0 : rq);
  const double bn = bq > 0.0 ? sqrt(bq) : (bq <= 0.0 ? 0.0 : bq);
  double2* g = S.g + (int64_t)c * (S.m + 1);
  g[0] = make_double2(rn, 0.0);
  for (int i = 1; i <= S.m; ++i) g[i] = kzero();
  // b = 0 has the solution x = 0: nothing to do; a non-finite b or r gives
  // a NaN or infinite estimate (inactive, reported as not converged)
  const double rel = bn > 0 ? rn / bn : (bn == 0.0 ? 0.0 : bn);
  const bool go = bn > 0 && rn > 0 && rel > tol && isfinite(rel);
  S.bnorm[c] = bn;
  S.resid[c] = rel;
  S.kc[c] = 0;
  S.act[c] = go ? 1 : 0;
  S.inv[c] = go ? 1.0 / rn : 0.0;
}

// Arnoldi step j of column c: h = h1 + h2 (the two Gram-Schmidt passes),
// h_{j+1,j} = ||w||; the column is rotated by the earlier rotations, the new
// rotation zeroes h_{j+1,j}, and g follows.  A column stays active while its
// residual estimate is above tol and the new basis vector is nonzero.
__global__ void k_kstep(KrylovState S, int j, const double2* __restrict__ h1,
                        const double2* __restrict__ h2, int ldh, const double2* __restrict__ hn2,
                        double tol, int nrhs) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  if (!S.act[c]) {
    S.inv[c] = 0.0;
    return;
  }
  const int m = S.m;
  double2* R = S.R + ((int64_t)c * m + j) * (m + 1);
  double* cs = S.cs + (int64_t)c * m;
  double2* sn = S.sn + (int64_t)c * m;
  double2* g = S.g + (int64_t)c * (m + 1);
  for (int i = 0; i <= j; ++i) {
    const double2 a = h1[(int64_t)c * ldh + i], b = h2[(int64_t)c * ldh + i];
    R[i] = make_double2(a.x + b.x, a.y + b.y);
  }
  const double hb = sqrt(fmax(hn2[c].x, 0.0));
  // earlier rotations: [a; b] <- [cs a + sn b; -conj(sn) a + cs b]
  for (int i = 0; i < j; ++i) {
    const double2 a = R[i], b = R[i + 1];
    const double2 sb = cmul(sn[i], b);
    const double2 sa = conj_mul(sn[i], a);
    R[i] = make_double2(cs[i] * a.x + sb.x, cs[i] * a.y + sb.y);
    R[i + 1] = make_double2(cs[i] * b.x - sa.x, cs[i] * b.y - sa.y);
  }
  // new rotation for (a, hb), hb real and >= 0: cs = |a| / t,
  // sn = (a / |a|) hb / t with t = sqrt(|a|^2 + hb^2); it maps (a, hb) to
  // ((a / |a|) t, 0).  For a = 0 it swaps the two rows (cs = 0, sn = 1),
  // which keeps |g| (no progress) when hb is zero too.
  const double2 a = R[j];
  const double aa = hypot(a.x, a.y), t = hypot(aa, hb);
  double cj;
  double2 sj;
  if (aa == 0.0) {
    cj = 0.0;
    sj = make_double2(1.0, 0.0);
    R[j] = make_double2(hb, 0.0);
  } else {
    cj = aa / t;
    sj = make_double2(a.x / aa * hb / t, a.y / aa * hb / t);
    R[j] = make_double2(a.x / aa * t, a.y / aa * t);
  }
  cs[j] = cj;
  sn[j] = sj;
  const double2 gj = g[j];
  const double2 sg = conj_mul(sj, gj);
  g[j] = make_double2(cj * gj.x, cj * gj.y);
  g[j + 1] = make_double2(-sg.x, -sg.y);
  const double rel = S.bnorm[c] > 0 ? hypot(sg.x, sg.y) / S.bnorm[c] : 0.0;
  const bool go = hb > 0.0 && rel > tol && isfinite(rel);
  S.kc[c] = j + 1;
  S.resid[c] = rel;
  S.act[c] = go ? 1 : 0;
  S.inv[c] = go ? 1.0 / hb : 0.0;
}

// y = R^{-1} g over the column's kc steps (zeros past kc, up to m)
__global__ void k_ksolve(KrylovState S, double2* __restrict__ y, int nrhs) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  const int m = S.m, k = S.kc[c];
  const double2* g = S.g + (int64_t)c * (m + 1);
  double2* yc = y + (int64_t)c * m;
  for (int i = k; i < m; ++i) yc[i] = kzero();
  for (int i = k - 1; i >= 0; --i) {
    double2 s = g[i];
    for (int l = i + 1; l < k; ++l) {
      const double2 p = cmul(S.R[((int64_t)c * m + l) * (m + 1) + i], yc[l]);
      s.x -= p.x;
      s.y -= p.y;
    }
    const double2 d = S.R[((int64_t)c * m + i) * (m + 1) + i];
    const double dd = d.x * d.x + d.y * d.y;
    // s / d = s conj(d) / |d|^2; a zero pivot (a zero column) gives 0
    yc[i] = dd > 0 ? make_double2((s.x * d.x + s.y * d.y) / dd, (s.y * d.x - s.x * d.y) / dd)
                   : kzero();
  }
}

}  // namespace

hipError_t launch_kdots(const double2* V, int64_t vs, int64_t ld, const double2* w, int64_t n,
                        int nvec, int nrhs, double2* partial, double2* out, int ldo,
                        hipStream_t st) {
  if (n <= 0 || nrhs <= 0 || nvec <= 0) return hipSuccess;
  if (nvec > kMaxKrylov + 1) return hipErrorInvalidValue;
  const unsigned nblk = blocks_of(n, kKT);
  hipLaunchKernelGGL(k_kdots, dim3(nblk, nrhs), dim3(kKT), 0, st, V, vs, ld, w, n, nvec, partial);
  hipLaunchKernelGGL(k_kreduce, dim3(blocks_of((int64_t)nvec * nrhs, 64)), dim3(64), 0, st,
                     partial, (int)nblk, nvec, nrhs, out, ldo);
  return hipGetLastError();
}

int64_t kdots_partials(int64_t n, int nvec, int nrhs) {
  return (int64_t)blocks_of(n, kKT) * nvec * nrhs;
}

hipError_t launch_kupdate(double alpha, const double2* V, int64_t vs, int64_t ld,
                          const double2* coef, int ldc, int nvec, double2* y, int64_t n, int nrhs,
                          hipStream_t st) {
  if (n <= 0 || nrhs <= 0 || nvec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kupdate, dim3(blocks_of(n, kKT), nrhs), dim3(kKT), 0, st, alpha, V, vs, ld,
                     coef, ldc, nvec, y, n);
  return hipGetLastError();
}

hipError_t launch_kscale(double2* v, int64_t ld, const double* s, int64_t n, int nrhs,
                         hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kscale, dim3(blocks_of(n, kKT), nrhs), dim3(kKT), 0, st, v, ld, s, n);
  return hipGetLastError();
}

hipError_t launch_kstart(const KrylovState& S, const double2* rn2, const double2* bn2, double tol,
                         int nrhs, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kstart, dim3(blocks_of(nrhs, 64)), dim3(64), 0, st, S, rn2, bn2, tol, nrhs);
  return hipGetLastError();
}

hipError_t launch_kstep(const KrylovState& S, int j, const double2* h1, const double2* h2, int ldh,
                        const double2* hn2, double tol, int nrhs, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  if (j < 0 || j >= S.m || j + 1 > ldh) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_kstep, dim3(blocks_of(nrhs, 64)), dim3(64), 0, st, S, j, h1, h2, ldh, hn2,
                     tol, nrhs);
  return hipGetLastError();
}

hipError_t launch_ksolve(const KrylovState& S, double2* y, int nrhs, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ksolve, dim3(blocks_of(nrhs, 64)), dim3(64), 0, st, S, y, nrhs);
  return hipGetLastError();
}

}  // namespace hm
