// HIP kernels of libhmps for gfx950 (CDNA4, wave64).
//
// Hot loop of the power series (Sec. IV, eq. 12-13 and 20-22), one term:
//   stage A   t_b = W_b y_s for every far block of level >= l   (k_stageA)
//   panel     z_a = sum over the leaf's series panel columns     (k_panel)
//             = D_a^{-1} (R_l y)_a, split over several workgroups per leaf
//   epilogue  y_a = -z_a, x_a += y_a                              (k_epilogue)
// The 1-RHS products are HBM-bound GEMVs (0.5 flop/B in FP64), so they stay
// on the vector ALUs with wide coalesced loads; no MFMA.
#include <hip/hip_runtime.h>

#include "dev.h"

namespace hm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ double2 zero2() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double2 widen(double2 a) { return a; }
__device__ __forceinline__ double2 widen(float2 a) { return make_double2((double)a.x, (double)a.y); }

// acc += a * x (complex)
__device__ __forceinline__ void cmac(double2& acc, double2 a, double2 x) {
  acc.x = fma(a.x, x.x, acc.x);
  acc.x = fma(-a.y, x.y, acc.x);
  acc.y = fma(a.x, x.y, acc.y);
  acc.y = fma(a.y, x.x, acc.y);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

template <typename TM>
__device__ __forceinline__ TM zero_elem();
template <>
__device__ __forceinline__ double2 zero_elem<double2>() { return make_double2(0.0, 0.0); }
template <>
__device__ __forceinline__ float2 zero_elem<float2>() { return make_float2(0.f, 0.f); }

// ---------------------------------------------------------------- permute
__global__ void k_permute_in(const double2* __restrict__ b, int64_t ldb,
                             const int64_t* __restrict__ perm, double2* __restrict__ out,
                             int64_t ldo, int64_t n) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (q < n) out[q + c * ldo] = b[perm[q] + c * ldb];
}

__global__ void k_permute_out(const double2* __restrict__ in, int64_t ldi,
                              const int64_t* __restrict__ perm, double2* __restrict__ x,
                              int64_t ldx, int64_t n) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (q < n) x[perm[q] + c * ldx] = in[q + c * ldi];
}

// ---------------------------------------------------------------- panel GEMV
// One workgroup = one work item (leaf row, column range).  Lane l of every
// wave owns rows l, l+64, ... of the leaf; the four waves take interleaved
// columns so that a workgroup streams consecutive panel columns; UNR columns
// per wave are loaded before they are used to keep enough bytes in flight.
template <typename TM, int RPL, int NR, int UNR>
__global__ __launch_bounds__(kThreads) void k_panel(PanelSet ps, const WorkItem* __restrict__ items,
                                                    const double2* __restrict__ xin, int64_t ldx,
                                                    int nrhs, double2* __restrict__ partial,
                                                    int64_t ldp) {
  const WorkItem it = items[blockIdx.x];
  const int m = ps.leaf_m[it.leaf];
  const TM* __restrict__ P = reinterpret_cast<const TM*>(ps.data) + ps.panel_off[it.leaf];
  const int32_t* __restrict__ src = ps.src + ps.col_off[it.leaf];
  const int rhs0 = blockIdx.y * NR;
  const int w = wave_id();
  const int lane = threadIdx.x & 63;

  double2 acc[RPL][NR];
#pragma unroll
  for (int q = 0; q < RPL; ++q)
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[q][r] = zero2();

  for (int c = it.c0 + w; c < it.c1; c += kWaves * UNR) {
    TM a[UNR][RPL];
    double2 xv[UNR][NR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int cc = c + kWaves * u;
      const bool ok = cc < it.c1;
      const int64_t s = ok ? (int64_t)src[cc] : 0;
#pragma unroll
      for (int r = 0; r < NR; ++r)
        xv[u][r] = (ok && rhs0 + r < nrhs) ? xin[s + (int64_t)(rhs0 + r) * ldx] : zero2();
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int i = lane + 64 * q;
        a[u][q] = (ok && i < m) ? P[i + (int64_t)cc * m] : zero_elem<TM>();
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int q = 0; q < RPL; ++q)
#pragma unroll
        for (int r = 0; r < NR; ++r) cmac(acc[q][r], widen(a[u][q]), xv[u][r]);
  }

  __shared__ double2 red[kWaves - 1][RPL][NR][64];
  if (w > 0) {
#pragma unroll
    for (int q = 0; q < RPL; ++q)
#pragma unroll
      for (int r = 0; r < NR; ++r) red[w - 1][q][r][lane] = acc[q][r];
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = lane + 64 * q;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        double2 s = acc[q][r];
#pragma unroll
        for (int v = 0; v < kWaves - 1; ++v) {
          s.x += red[v][q][r][lane].x;
          s.y += red[v][q][r][lane].y;
        }
        if (i < m && rhs0 + r < nrhs) partial[it.prow + i + (int64_t)(rhs0 + r) * ldp] = s;
      }
    }
  }
}

// ---------------------------------------------------------------- stage A
// One wave per far block: t_b = W_b y_s.  Lanes stride over the n source
// points (coalesced along the rows of W_b), QC coefficient rows at a time,
// then a butterfly reduction across the wave.
template <typename TM, int NR, int QC>
__global__ __launch_bounds__(kThreads) void k_stageA(const TM* __restrict__ W,
                                                     const StageABlock* __restrict__ blk, int nblk,
                                                     double2* __restrict__ xin, int64_t ldx,
                                                     int64_t N, int nrhs) {
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * kWaves + w;
  if (b >= nblk) return;  // whole wave leaves; no barrier in this kernel
  const StageABlock f = blk[b];
  const TM* __restrict__ Wb = W + f.w_off;
  const int rhs0 = blockIdx.y * NR;
  for (int q0 = 0; q0 < f.r; q0 += QC) {
    double2 acc[QC][NR];
#pragma unroll
    for (int qq = 0; qq < QC; ++qq)
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[qq][r] = zero2();
    for (int j = lane; j < f.n; j += 64) {
      double2 yv[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r)
        yv[r] = (rhs0 + r < nrhs) ? xin[f.s_off + j + (int64_t)(rhs0 + r) * ldx] : zero2();
#pragma unroll
      for (int qq = 0; qq < QC; ++qq) {
        if (q0 + qq < f.r) {
          const double2 wv = widen(Wb[(int64_t)(q0 + qq) * f.n + j]);
#pragma unroll
          for (int r = 0; r < NR; ++r) cmac(acc[qq][r], wv, yv[r]);
        }
      }
    }
#pragma unroll
    for (int qq = 0; qq < QC; ++qq)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        acc[qq][r].x = wave_sum(acc[qq][r].x);
        acc[qq][r].y = wave_sum(acc[qq][r].y);
      }
    if (lane == 0) {
#pragma unroll
      for (int qq = 0; qq < QC; ++qq)
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (q0 + qq < f.r && rhs0 + r < nrhs)
            xin[N + f.tb_off + q0 + qq + (int64_t)(rhs0 + r) * ldx] = acc[qq][r];
    }
  }
}

// ---------------------------------------------------------------- epilogue
// Per leaf: z = sum of the partial sums of its work items (fixed order),
// y = alpha z + beta v; optionally store y and add it to (or store it in) x.
__global__ __launch_bounds__(kThreads) void k_epilogue(EpilogueArgs e, int nrhs) {
  const int a = blockIdx.x;
  const int m = e.leaf_m[a];
  const int64_t off = e.leaf_off[a];
  const int p0 = e.item_ptr[a], p1 = e.item_ptr[a + 1];
  for (int c = blockIdx.y; c < nrhs; c += gridDim.y) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      double2 z = zero2();
      for (int p = p0; p < p1; ++p) {
        const double2 v = e.partial[e.items[p].prow + i + (int64_t)c * e.ldp];
        z.x += v.x;
        z.y += v.y;
      }
      double2 y = make_double2(e.alpha * z.x, e.alpha * z.y);
      if (e.v) {
        const double2 v = e.v[off + i + (int64_t)c * e.ldv];
        y.x = fma(e.beta, v.x, y.x);
        y.y = fma(e.beta, v.y, y.y);
      }
      if (e.yout) e.yout[off + i + (int64_t)c * e.ldy] = y;
      if (e.xacc) {
        const int64_t idx = off + i + (int64_t)c * e.ldxa;
        if (e.accumulate) {
          const double2 x = e.xacc[idx];
          y.x += x.x;
          y.y += x.y;
        }
        e.xacc[idx] = y;
      }
    }
  }
}

// ---------------------------------------------------------------- leaf LU
// Right-looking LU with partial pivoting of one leaf self-block per
// workgroup, in place (column-major).  Build-time only; works from L2.
__global__ __launch_bounds__(kThreads) void k_getrf(double2* __restrict__ A,
                                                    const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ mm,
                                                    int32_t* __restrict__ piv,
                                                    const int64_t* __restrict__ poff,
                                                    int* __restrict__ info) {
  const int b = blockIdx.x;
  const int m = mm[b];
  double2* a = A + off[b];
  int32_t* pv = piv + poff[b];
  const int tid = threadIdx.x;
  __shared__ double sval[kThreads];
  __shared__ int sidx[kThreads];
  for (int k = 0; k < m; ++k) {
    double best = -1.0;
    int bi = m;
    for (int i = k + tid; i < m; i += kThreads) {
      const double2 v = a[i + (int64_t)k * m];
      const double mag = hypot(v.x, v.y);
      if (mag > best) { best = mag; bi = i; }
    }
    sval[tid] = best;
    sidx[tid] = bi;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
      if (tid < s) {
        const double o = sval[tid + s];
        const int oi = sidx[tid + s];
        if (o > sval[tid] || (o == sval[tid] && oi < sidx[tid])) {
          sval[tid] = o;
          sidx[tid] = oi;
        }
      }
      __syncthreads();
    }
    const int p = sidx[0];
    const double pmag = sval[0];
    __syncthreads();
    if (tid == 0) {
      pv[k] = p;
      if (!(pmag > 0.0)) info[b] = k + 1;
    }
    if (p != k) {
      for (int j = tid; j < m; j += kThreads) {
        const double2 t = a[k + (int64_t)j * m];
        a[k + (int64_t)j * m] = a[p + (int64_t)j * m];
        a[p + (int64_t)j * m] = t;
      }
    }
    __syncthreads();
    if (pmag > 0.0) {
      const double2 d = a[k + (int64_t)k * m];
      const double dd = d.x * d.x + d.y * d.y;
      const double2 inv = make_double2(d.x / dd, -d.y / dd);
      for (int i = k + 1 + tid; i < m; i += kThreads) a[i + (int64_t)k * m] = cmul(a[i + (int64_t)k * m], inv);
    }
    __syncthreads();
    const int n2 = m - k - 1;
    for (int idx = tid; idx < n2 * n2; idx += kThreads) {
      const int i = k + 1 + idx % n2;
      const int j = k + 1 + idx / n2;
      const double2 l = a[i + (int64_t)k * m];
      const double2 u = a[k + (int64_t)j * m];
      double2 v = a[i + (int64_t)j * m];
      v.x -= l.x * u.x - l.y * u.y;
      v.y -= l.x * u.y + l.y * u.x;
      a[i + (int64_t)j * m] = v;
    }
    __syncthreads();
  }
}

// Inverse from the LU factors: column j of D^{-1} solves L U x = P e_j.
// One thread per column, working on its own column in the output.
__global__ __launch_bounds__(kThreads) void k_getri(const double2* __restrict__ LU,
                                                    const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ mm,
                                                    const int32_t* __restrict__ piv,
                                                    const int64_t* __restrict__ poff,
                                                    double2* __restrict__ Ainv) {
  const int b = blockIdx.x;
  const int m = mm[b];
  const double2* a = LU + off[b];
  const int32_t* pv = piv + poff[b];
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    double2* x = Ainv + off[b] + (int64_t)j * m;
    for (int i = 0; i < m; ++i) x[i] = zero2();
    x[j] = make_double2(1.0, 0.0);
    for (int k = 0; k < m; ++k) {
      const int p = pv[k];
      if (p != k) {
        const double2 t = x[k];
        x[k] = x[p];
        x[p] = t;
      }
    }
    for (int l = 0; l < m; ++l) {  // unit lower triangle
      const double2 xl = x[l];
      for (int i = l + 1; i < m; ++i) {
        const double2 L = a[i + (int64_t)l * m];
        double2 v = x[i];
        v.x -= L.x * xl.x - L.y * xl.y;
        v.y -= L.x * xl.y + L.y * xl.x;
        x[i] = v;
      }
    }
    for (int l = m - 1; l >= 0; --l) {  // upper triangle
      const double2 d = a[l + (int64_t)l * m];
      const double dd = d.x * d.x + d.y * d.y;
      const double2 inv = make_double2(d.x / dd, -d.y / dd);
      const double2 xl = cmul(x[l], inv);
      x[l] = xl;
      for (int i = 0; i < l; ++i) {
        const double2 U = a[i + (int64_t)l * m];
        double2 v = x[i];
        v.x -= U.x * xl.x - U.y * xl.y;
        v.y -= U.x * xl.y + U.y * xl.x;
        x[i] = v;
      }
    }
  }
}

// M panel tile: 32 columns c0.. of leaf a, M[:, c] = Dinv_a * P_a[:, m_a + c].
// Lane l owns rows l, l+64, ...; wave w owns columns w, w+4, ... of the tile.
template <int RPL>
__global__ __launch_bounds__(kThreads) void k_premul(const double2* __restrict__ Dinv,
                                                     const int64_t* __restrict__ dinv_off,
                                                     const double2* __restrict__ P,
                                                     const int64_t* __restrict__ p_off,
                                                     const int32_t* __restrict__ leaf_m,
                                                     const int32_t* __restrict__ ncols_m,
                                                     double2* __restrict__ M,
                                                     const int64_t* __restrict__ m_off,
                                                     const int32_t* __restrict__ tiles) {
  constexpr int TC = 8;  // columns per wave
  const int a = tiles[2 * blockIdx.x];
  const int c0 = tiles[2 * blockIdx.x + 1];
  const int m = leaf_m[a];
  const int nc = ncols_m[a];
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  const double2* Di = Dinv + dinv_off[a];
  const double2* Pa = P + p_off[a] + (int64_t)m * m;  // skip the D_a columns
  double2* Ma = M + m_off[a];
  double2 acc[RPL][TC];
#pragma unroll
  for (int q = 0; q < RPL; ++q)
#pragma unroll
    for (int u = 0; u < TC; ++u) acc[q][u] = zero2();
  for (int l = 0; l < m; ++l) {
    double2 d[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = lane + 64 * q;
      d[q] = (i < m) ? Di[i + (int64_t)l * m] : zero2();
    }
#pragma unroll
    for (int u = 0; u < TC; ++u) {
      const int c = c0 + w + kWaves * u;
      const double2 pv = (c < nc) ? Pa[l + (int64_t)c * m] : zero2();
#pragma unroll
      for (int q = 0; q < RPL; ++q) cmac(acc[q][u], d[q], pv);
    }
  }
#pragma unroll
  for (int u = 0; u < TC; ++u) {
    const int c = c0 + w + kWaves * u;
    if (c >= nc) continue;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = lane + 64 * q;
      if (i < m) Ma[i + (int64_t)c * m] = acc[q][u];
    }
  }
}

__global__ void k_cast(const double2* __restrict__ in, float2* __restrict__ out, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    out[q] = make_float2((float)in[q].x, (float)in[q].y);
}

// ---------------------------------------------------------------- norms
__global__ __launch_bounds__(kThreads) void k_norm2_partial(const double2* __restrict__ v,
                                                            int64_t ld, int64_t n,
                                                            double* __restrict__ scratch) {
  const int c = blockIdx.y;
  double s = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * kThreads) {
    const double2 z = v[q + c * ld];
    s = fma(z.x, z.x, s);
    s = fma(z.y, z.y, s);
  }
  __shared__ double sm[kThreads];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) scratch[(int64_t)c * gridDim.x + blockIdx.x] = sm[0];
}

__global__ void k_norm2_final(const double* __restrict__ scratch, int nb, int nrhs,
                              double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += scratch[(int64_t)c * nb + i];
  out[c] = s;
}

__global__ void k_axpy(double alpha, const double2* __restrict__ x, int64_t ldx,
                       double2* __restrict__ y, int64_t ldy, int64_t n, int accumulate) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (q >= n) return;
  const double2 a = x[q + c * ldx];
  double2 r = make_double2(alpha * a.x, alpha * a.y);
  if (accumulate) {
    const double2 b = y[q + c * ldy];
    r.x += b.x;
    r.y += b.y;
  }
  y[q + c * ldy] = r;
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ============================================================== launchers
hipError_t launch_permute_in(const double2* b, int64_t ldb, const int64_t* perm, double2* out,
                             int64_t ldo, int64_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_permute_in, dim3(blocks_for(n, 256), nrhs), dim3(256), 0, st, b, ldb, perm,
                     out, ldo, n);
  return hipGetLastError();
}

hipError_t launch_permute_out(const double2* in, int64_t ldi, const int64_t* perm, double2* x,
                              int64_t ldx, int64_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_permute_out, dim3(blocks_for(n, 256), nrhs), dim3(256), 0, st, in, ldi,
                     perm, x, ldx, n);
  return hipGetLastError();
}

template <typename TM, int RPL>
static hipError_t panel_rpl(const PanelSet& ps, const WorkItem* items, int nitems,
                            const double2* xin, int64_t ldx, int nrhs, double2* partial,
                            int64_t ldp, hipStream_t st) {
  constexpr int UNR = sizeof(TM) == 16 ? 8 : 16;
  if (nrhs == 1) {
    hipLaunchKernelGGL((k_panel<TM, RPL, 1, UNR>), dim3(nitems, 1), dim3(kThreads), 0, st, ps,
                       items, xin, ldx, nrhs, partial, ldp);
  } else if (nrhs == 2) {
    hipLaunchKernelGGL((k_panel<TM, RPL, 2, UNR / 2>), dim3(nitems, 1), dim3(kThreads), 0, st,
                       ps, items, xin, ldx, nrhs, partial, ldp);
  } else {
    hipLaunchKernelGGL((k_panel<TM, RPL, 4, UNR / 4>), dim3(nitems, (nrhs + 3) / 4),
                       dim3(kThreads), 0, st, ps, items, xin, ldx, nrhs, partial, ldp);
  }
  return hipGetLastError();
}

hipError_t launch_panel(bool f32, int max_m, const PanelSet& ps, const WorkItem* items, int nitems,
                        const double2* xin, int64_t ldx, int nrhs, double2* partial, int64_t ldp,
                        hipStream_t st) {
  if (nitems <= 0 || nrhs <= 0) return hipSuccess;
  if (max_m > 256) return hipErrorInvalidValue;
  const int rpl = (max_m + 63) / 64;
#define HM_PANEL_CASE(R)                                                                        \
  case R:                                                                                      \
    return f32 ? panel_rpl<float2, R>(ps, items, nitems, xin, ldx, nrhs, partial, ldp, st)     \
               : panel_rpl<double2, R>(ps, items, nitems, xin, ldx, nrhs, partial, ldp, st);
  switch (rpl) {
    HM_PANEL_CASE(1)
    HM_PANEL_CASE(2)
    HM_PANEL_CASE(3)
    HM_PANEL_CASE(4)
    default:
      return hipErrorInvalidValue;
  }
#undef HM_PANEL_CASE
}

hipError_t launch_stageA(bool f32, const void* W, const StageABlock* blk, int nblk, double2* xin,
                         int64_t ldx, int64_t N, int nrhs, hipStream_t st) {
  if (nblk <= 0 || nrhs <= 0) return hipSuccess;
  const unsigned gx = blocks_for(nblk, kWaves);
  if (nrhs == 1) {
    if (f32)
      hipLaunchKernelGGL((k_stageA<float2, 1, 8>), dim3(gx, 1), dim3(kThreads), 0, st,
                         (const float2*)W, blk, nblk, xin, ldx, N, nrhs);
    else
      hipLaunchKernelGGL((k_stageA<double2, 1, 8>), dim3(gx, 1), dim3(kThreads), 0, st,
                         (const double2*)W, blk, nblk, xin, ldx, N, nrhs);
  } else {
    const unsigned gy = (unsigned)((nrhs + 3) / 4);
    if (f32)
      hipLaunchKernelGGL((k_stageA<float2, 4, 4>), dim3(gx, gy), dim3(kThreads), 0, st,
                         (const float2*)W, blk, nblk, xin, ldx, N, nrhs);
    else
      hipLaunchKernelGGL((k_stageA<double2, 4, 4>), dim3(gx, gy), dim3(kThreads), 0, st,
                         (const double2*)W, blk, nblk, xin, ldx, N, nrhs);
  }
  return hipGetLastError();
}

hipError_t launch_epilogue(const EpilogueArgs& e, int nleaves, int max_m, int nrhs,
                           hipStream_t st) {
  if (nleaves <= 0 || nrhs <= 0) return hipSuccess;
  (void)max_m;
  const unsigned gy = (unsigned)(nrhs < 64 ? nrhs : 64);
  hipLaunchKernelGGL(k_epilogue, dim3(nleaves, gy), dim3(kThreads), 0, st, e, nrhs);
  return hipGetLastError();
}

hipError_t launch_getrf(double2* A, const int64_t* off, const int32_t* m, int32_t* piv,
                        const int64_t* piv_off, int nblk, int* info, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_getrf, dim3(nblk), dim3(kThreads), 0, st, A, off, m, piv, piv_off, info);
  return hipGetLastError();
}

hipError_t launch_getri(const double2* LU, const int64_t* off, const int32_t* m,
                        const int32_t* piv, const int64_t* piv_off, double2* Ainv, int nblk,
                        hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_getri, dim3(nblk), dim3(kThreads), 0, st, LU, off, m, piv, piv_off, Ainv);
  return hipGetLastError();
}

hipError_t launch_premul(const double2* Dinv, const int64_t* dinv_off, const double2* P,
                         const int64_t* p_off, const int32_t* leaf_m, const int32_t* ncols_m,
                         double2* M, const int64_t* m_off, const int32_t* tiles, int ntiles,
                         int max_m, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  const int rpl = (max_m + 63) / 64;
#define HM_PREMUL_CASE(R)                                                                      \
  case R:                                                                                     \
    hipLaunchKernelGGL(k_premul<R>, dim3(ntiles), dim3(kThreads), 0, st, Dinv, dinv_off, P,   \
                       p_off, leaf_m, ncols_m, M, m_off, tiles);                              \
    break;
  switch (rpl) {
    HM_PREMUL_CASE(1)
    HM_PREMUL_CASE(2)
    HM_PREMUL_CASE(3)
    HM_PREMUL_CASE(4)
    default:
      return hipErrorInvalidValue;
  }
#undef HM_PREMUL_CASE
  return hipGetLastError();
}

hipError_t launch_cast(const double2* in, float2* out, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t b = (n + 255) / 256;
  hipLaunchKernelGGL(k_cast, dim3((unsigned)(b < 65536 ? b : 65536)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

hipError_t launch_norm2(const double2* v, int64_t ld, int64_t n, int nrhs, double* scratch,
                        double* out, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_norm2_partial, dim3(kNormBlocks, nrhs), dim3(kThreads), 0, st, v, ld, n,
                     scratch);
  hipLaunchKernelGGL(k_norm2_final, dim3((nrhs + 63) / 64), dim3(64), 0, st, scratch,
                     kNormBlocks, nrhs, out);
  return hipGetLastError();
}

hipError_t launch_axpy(double alpha, const double2* x, int64_t ldx, double2* y, int64_t ldy,
                       int64_t n, int nrhs, int accumulate, hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n, 256), nrhs), dim3(256), 0, st, alpha, x, ldx, y,
                     ldy, n, accumulate);
  return hipGetLastError();
}

}  // namespace hm
