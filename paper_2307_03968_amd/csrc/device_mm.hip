// Many-right-hand-side kernels of libhmps for gfx950: the near/far panel
// products and the stage-A low-rank products become dense contractions
// (panel m x c times inputs c x nrhs), so they run on the matrix cores:
//   FP32 blocks: Gauss 3M complex product on v_mfma_f32_16x16x4f32,
//     T1 = Ar Xr, T2 = Ai Xi, T3 = (Ar + Ai)(Xr + Xi), Re = T1 - T2,
//     Im = T3 - T1 - T2 (three real products instead of four);
//   FP64 blocks: four real products on v_mfma_f64_16x16x4f64.
// MFMA 16x16x4 operand layout (lane l): A[i][k] with i = l % 16, k = l / 16;
// B[k][j] with k = l / 16, j = l % 16.  Result element v of lane l is
// D[4 (l / 16) + v][l % 16] for the FP32 instruction and D[l / 16 + 4 v][l % 16]
// for the FP64 one (both measured on gfx950).
// A workgroup of four waves covers up to 128 (or 256) panel rows: wave w owns
// the 16-row tiles w, w + 4, ...; the inputs of a column chunk are staged in
// LDS (converted to the compute precision) and shared by the waves.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dev.h"

namespace hm {

namespace {

constexpr int kThreads = 256;
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

template <bool F32>
struct Prec;

template <>
struct Prec<true> {                      // FP32 blocks, 3M
  using X = float2;                      // staged input element
  using Acc = f4v;
  static constexpr int NACC = 3;
  static constexpr int CH = 64;          // staged columns per chunk
  __device__ static __forceinline__ float2 load_a(const void* P, uint32_t idx) {
    const fvec2 v = __builtin_nontemporal_load(reinterpret_cast<const fvec2*>(P) + idx);
    return make_float2(v.x, v.y);
  }
  __device__ static __forceinline__ X cvt(double2 v) { return make_float2((float)v.x, (float)v.y); }
  __device__ static __forceinline__ void mac(Acc (&acc)[3], float2 a, X b) {
    acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc[1], 0, 0, 0);
    acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x + a.y, b.x + b.y, acc[2], 0, 0, 0);
  }
  __device__ static __forceinline__ double2 result(const Acc (&acc)[3], int v) {
    const double t1 = acc[0][v], t2 = acc[1][v], t3 = acc[2][v];
    return make_double2(t1 - t2, t3 - t1 - t2);
  }
  // row of result element v within the 16 x 16 tile (kq = lane / 16)
  __device__ static __forceinline__ int row(int kq, int v) { return 4 * kq + v; }
};

template <>
struct Prec<false> {                     // FP64 blocks, four real products
  using X = double2;
  using Acc = d4v;
  static constexpr int NACC = 2;
  static constexpr int CH = 32;
  __device__ static __forceinline__ double2 load_a(const void* P, uint32_t idx) {
    const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(P) + idx);
    return make_double2(v.x, v.y);
  }
  __device__ static __forceinline__ X cvt(double2 v) { return v; }
  __device__ static __forceinline__ void mac(Acc (&acc)[2], double2 a, X b) {
    acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, acc[0], 0, 0, 0);
    acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, acc[1], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, acc[1], 0, 0, 0);
  }
  __device__ static __forceinline__ double2 result(const Acc (&acc)[2], int v) {
    return make_double2(acc[0][v], acc[1][v]);
  }
  __device__ static __forceinline__ int row(int kq, int v) { return kq + 4 * v; }
};

template <bool F32, int RT, int NT>
struct MMAcc {
  typename Prec<F32>::Acc a[RT][NT][Prec<F32>::NACC];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q < Prec<F32>::NACC; ++q) a[r][t][q] = typename Prec<F32>::Acc{};
  }
};

// acc += P[rows of this wave's tiles, c0:c1) * Xs, the inputs of the chunk
// being fetched into LDS by fx(c, n) (c absolute column, n RHS within the
// tile; returns the FP64 value, zero outside the valid range).
template <bool F32, int RT, int NT, typename FX>
__device__ __forceinline__ void mm_core(const void* __restrict__ P, uint32_t ld, int row0,
                                        int c0, int c1, const FX& fx, MMAcc<F32, RT, NT>& acc,
                                        int w, int lane) {
  using PR = Prec<F32>;
  constexpr int NRT = 16 * NT;
  constexpr int CH = PR::CH;
  __shared__ typename PR::X xs[CH][NRT];  // the chunk's inputs, shared by the waves
  const int l16 = lane & 15, kq = lane >> 4;
  uint32_t ri[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) ri[r] = min<uint32_t>(row0 + (w + 4 * r) * 16 + l16, ld - 1);
  for (int cb = c0; cb < c1; cb += CH) {
    const int nc = min(CH, c1 - cb);
    __syncthreads();
    for (int t = threadIdx.x; t < CH * NRT; t += kThreads) {
      const int k = t % CH;
      const int n = t / CH;
      xs[k][n] = PR::cvt(k < nc ? fx(cb + k, n) : make_double2(0.0, 0.0));
    }
    __syncthreads();
    for (int kk = 0; kk < nc; kk += 16) {
      // four k-steps of four columns: A loads first, then the products
      float2 af[F32 ? 4 : 1][RT];
      double2 ad[F32 ? 1 : 4][RT];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int col = min(cb + kk + 4 * s + kq, c1 - 1);
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          if constexpr (F32)
            af[s][r] = PR::load_a(P, ri[r] + (uint32_t)col * ld);
          else
            ad[s][r] = PR::load_a(P, ri[r] + (uint32_t)col * ld);
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (kk + 4 * s >= nc) break;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const typename PR::X b = xs[kk + 4 * s + kq][t * 16 + l16];
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            if constexpr (F32)
              PR::mac(acc.a[r][t], af[s][r], b);
            else
              PR::mac(acc.a[r][t], ad[s][r], b);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- epilogue
// Partial-sum rows of the leaf's pieces come from LDS (STAGED, up to
// kThreads pieces) or straight from global memory.
template <int NRT, bool STAGED>
__device__ void epilogue_loop(const TermArgs& A, int a, int rhs0, int nrhs, const int* s_prow) {
  const int m = A.ps.leaf_m[a];
  const int64_t off = A.leaf_off[a];
  const int q0 = A.lptr[a], np = A.lptr[a + 1] - q0;
  for (int idx = threadIdx.x; idx < m * NRT; idx += kThreads) {
    const int i = idx % m;
    const int c = rhs0 + idx / m;
    if (c >= nrhs) continue;
    const double* pc = reinterpret_cast<const double*>(A.partial + i + (int64_t)c * A.ldp);
    double zr = 0.0, zi = 0.0;
    for (int p = 0; p < np; p += 8) {  // fixed order; loads in flight together
      double vr[8], vi[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (p + u < np) {
          int prow;
          if constexpr (STAGED)
            prow = s_prow[p + u];
          else
            prow = A.lprow[q0 + p + u];
          const double* q = pc + 2 * (int64_t)prow;
          vr[u] = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          vi[u] = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          vr[u] = 0.0;
          vi[u] = 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        zr += vr[u];
        zi += vi[u];
      }
    }
    double2 y = make_double2(A.alpha * zr, A.alpha * zi);
    if (A.v) {
      const double2 v = A.v[off + i + (int64_t)c * A.ldv];
      y.x = fma(A.beta, v.x, y.x);
      y.y = fma(A.beta, v.y, y.y);
    }
    if (A.yout) A.yout[off + i + (int64_t)c * A.ldy] = y;
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
}

template <int NRT>
__device__ void term_epilogue_mm(const TermArgs& A, int a, int rhs0, int nrhs) {
  __shared__ int s_prow[kThreads];
  const int q0 = A.lptr[a], np = A.lptr[a + 1] - q0;
  if (np <= kThreads) {
    __syncthreads();
    if ((int)threadIdx.x < np) s_prow[threadIdx.x] = A.lprow[q0 + threadIdx.x];
    __syncthreads();
    epilogue_loop<NRT, true>(A, a, rhs0, nrhs, s_prow);
  } else {
    epilogue_loop<NRT, false>(A, a, rhs0, nrhs, nullptr);
  }
}

// ---------------------------------------------------------------- term
// Persistent workgroup over its run of (dense) pieces; same publication and
// last-workgroup epilogue as the one-RHS term kernel.
template <bool F32, int RT, int NT>
__global__ __launch_bounds__(kThreads) void k_term_mm(TermArgs A, int nrhs) {
  using PR = Prec<F32>;
  constexpr int NRT = 16 * NT;
  __shared__ int s_last;
  const int rhs0 = blockIdx.y * NRT;
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  const int pe = A.wptr[blockIdx.x + 1];
  for (int p = A.wptr[blockIdx.x]; p < pe; ++p) {
    const TermItem it = A.items[p];
    const int a = it.leaf;
    const int m = A.ps.leaf_m[a];
    const uint32_t ld = (uint32_t)(m + (m & 1));
    const void* P = F32 ? (const void*)(reinterpret_cast<const float2*>(A.ps.data) + A.ps.panel_off[a])
                        : (const void*)(reinterpret_cast<const double2*>(A.ps.data) + A.ps.panel_off[a]);
    const int32_t* __restrict__ src = A.ps.src + A.ps.col_off[a];
    MMAcc<F32, RT, NT> acc;
    acc.zero();
    auto fx = [&](int c, int n) -> double2 {
      if (rhs0 + n >= nrhs) return make_double2(0.0, 0.0);
      int64_t s = src[c];
      if (A.in_perm) s = A.in_perm[s];
      return A.xin[s + (int64_t)(rhs0 + n) * A.ldx];
    };
    mm_core<F32, RT, NT>(P, ld, 0, it.c0, it.c1, fx, acc, w, lane);
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = (w + 4 * r) * 16 + PR::row(kq, v);
          const int c = rhs0 + t * 16 + l16;
          if (i < m && c < nrhs) {
            const double2 z = PR::result(acc.a[r][t], v);
            double* q = reinterpret_cast<double*>(A.partial + it.prow + i + (int64_t)c * A.ldp);
            __hip_atomic_store(q, z.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(q + 1, z.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
    __builtin_amdgcn_s_waitcnt(0);
    int32_t* cnt = A.counters + (int64_t)a * gridDim.y + blockIdx.y;
    __syncthreads();
    if (threadIdx.x == 0) {
      const int old = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_last = (old == A.lptr[a + 1] - A.lptr[a] - 1);
    }
    __syncthreads();
    if (s_last) {
      term_epilogue_mm<NRT>(A, a, rhs0, nrhs);
      if (threadIdx.x == 0) __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- stage A
// One workgroup = a 64-row tile of a source group (one 16-row tile per
// wave): t rows = W_g Y[s_off .. s_off + n), written to the t part of xin.
template <bool F32, int NT>
__global__ __launch_bounds__(kThreads) void k_stageA_mm(const void* __restrict__ W,
                                                        const Group* __restrict__ groups,
                                                        const GroupItem* __restrict__ items,
                                                        double2* __restrict__ xin, int64_t ldx,
                                                        int64_t N, int nrhs) {
  using PR = Prec<F32>;
  constexpr int NRT = 16 * NT;
  const GroupItem it = items[blockIdx.x];
  const Group g = groups[it.group];
  const void* Wg = F32 ? (const void*)(reinterpret_cast<const float2*>(W) + g.w_off)
                       : (const void*)(reinterpret_cast<const double2*>(W) + g.w_off);
  const int rhs0 = blockIdx.y * NRT;
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  MMAcc<F32, 1, NT> acc;
  acc.zero();
  auto fx = [&](int c, int n) -> double2 {
    return (rhs0 + n < nrhs) ? xin[g.s_off + c + (int64_t)(rhs0 + n) * ldx]
                             : make_double2(0.0, 0.0);
  };
  mm_core<F32, 1, NT>(Wg, (uint32_t)g.ld, it.row0, 0, g.n, fx, acc, w, lane);
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = it.row0 + w * 16 + PR::row(kq, v);
      const int c = rhs0 + t * 16 + l16;
      if (q < it.rows && c < nrhs)
        xin[N + g.t0 + q + (int64_t)c * ldx] = PR::result(acc.a[0][t], v);
    }
}

// 16-column RHS tiles per workgroup: the requested tile (16, 32 or 64), or
// by nrhs when 0
inline int pick_nt(int nrhs, int tile) {
  if (tile == 16 || tile == 32 || tile == 64) return tile / 16;
  return nrhs <= 16 ? 1 : (nrhs <= 32 ? 2 : 4);
}

template <bool F32, int RT>
hipError_t term_mm_rt(const TermArgs& a, int nwg, int nrhs, int tile, hipStream_t st) {
  const int nt = pick_nt(nrhs, tile);
  const dim3 grid(nwg, (nrhs + 16 * nt - 1) / (16 * nt));
  if (nt == 1)
    hipLaunchKernelGGL((k_term_mm<F32, RT, 1>), grid, dim3(kThreads), 0, st, a, nrhs);
  else if (nt == 2)
    hipLaunchKernelGGL((k_term_mm<F32, RT, 2>), grid, dim3(kThreads), 0, st, a, nrhs);
  else
    hipLaunchKernelGGL((k_term_mm<F32, RT, 4>), grid, dim3(kThreads), 0, st, a, nrhs);
  return hipGetLastError();
}

template <bool F32>
hipError_t stageA_mm_p(const void* W, const Group* groups, const GroupItem* items, int nitems,
                       double2* xin, int64_t ldx, int64_t N, int nrhs, int tile, hipStream_t st) {
  const int nt = pick_nt(nrhs, tile);
  const dim3 grid(nitems, (nrhs + 16 * nt - 1) / (16 * nt));
  if (nt == 1)
    hipLaunchKernelGGL((k_stageA_mm<F32, 1>), grid, dim3(kThreads), 0, st, W, groups, items, xin,
                       ldx, N, nrhs);
  else if (nt == 2)
    hipLaunchKernelGGL((k_stageA_mm<F32, 2>), grid, dim3(kThreads), 0, st, W, groups, items, xin,
                       ldx, N, nrhs);
  else
    hipLaunchKernelGGL((k_stageA_mm<F32, 4>), grid, dim3(kThreads), 0, st, W, groups, items, xin,
                       ldx, N, nrhs);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_term_mm(bool f32, int max_m, const TermArgs& a, int nwg, int nrhs, int tile,
                          hipStream_t st) {
  if (nwg <= 0 || nrhs <= 0) return hipSuccess;
  if (max_m > 256) return hipErrorInvalidValue;
  const int rt = (max_m + 63) / 64;  // 16-row tiles per wave
  if (f32) {
    if (rt <= 1) return term_mm_rt<true, 1>(a, nwg, nrhs, tile, st);
    if (rt <= 2) return term_mm_rt<true, 2>(a, nwg, nrhs, tile, st);
    return term_mm_rt<true, 4>(a, nwg, nrhs, tile, st);
  }
  if (rt <= 1) return term_mm_rt<false, 1>(a, nwg, nrhs, tile, st);
  if (rt <= 2) return term_mm_rt<false, 2>(a, nwg, nrhs, tile, st);
  return term_mm_rt<false, 4>(a, nwg, nrhs, tile, st);
}

hipError_t launch_stageA_mm(bool f32, const void* W, const Group* groups, const GroupItem* items,
                            int nitems, double2* xin, int64_t ldx, int64_t N, int nrhs, int tile,
                            hipStream_t st) {
  if (nitems <= 0 || nrhs <= 0) return hipSuccess;
  return f32 ? stageA_mm_p<true>(W, groups, items, nitems, xin, ldx, N, nrhs, tile, st)
             : stageA_mm_p<false>(W, groups, items, nitems, xin, ldx, N, nrhs, tile, st);
}

}  // namespace hm
