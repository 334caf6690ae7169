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
  __device__ static __forceinline__ float2 load_a(const void* P, uint32_t idx) {
    const fvec2 v = __builtin_nontemporal_load(reinterpret_cast<const fvec2*>(P) + idx);
    return make_float2(v.x, v.y);
  }
  __device__ static __forceinline__ X cvt(double2 v) { return make_float2((float)v.x, (float)v.y); }
  __device__ static __forceinline__ X cvt(float2 v) { return v; }
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

// acc += P[rows of this wave's tiles, c0:c1) * X[c0:c1, tile].  colp(c)
// points (XT: double2, or float2 for FP32 shadows of the inputs) at input
// column c's value for the tile's first right-hand side (right-hand side n
// at colp(c)[n * ldx]); nv right-hand sides of the tile are valid.
// Software pipelined one chunk of NG groups of 16 columns ahead: the inputs
// of chunk j + 1 are loaded into registers while chunk j is multiplied (two
// LDS buffers, one barrier per chunk), and each group's panel registers are
// refilled with the same group of the next chunk right after their
// products (NG register sets, no copies).  Every load is issued
// unconditionally at a clamped address (values past c1 or past the last
// right-hand side are replaced by zero), so the memory-counter waits before
// each group cover only the loads that group needs.
template <bool F32, int RT>
struct Groups {  // groups of 16 columns per staged chunk (4 measured no faster)
  static constexpr int NG = 2;
};

template <bool F32, int RT, int NT, typename XT, typename COLP>
__device__ __forceinline__ void mm_core(const void* __restrict__ P, uint32_t ld, int row0,
                                        int c0, int c1, const COLP& colp, int64_t ldx, int nv,
                                        MMAcc<F32, RT, NT>& acc, int w, int lane) {
  using PR = Prec<F32>;
  using AV = typename std::conditional<F32, float2, double2>::type;
  constexpr int NRT = 16 * NT;
  constexpr int NG = Groups<F32, RT>::NG;
  constexpr int CH = 16 * NG;                  // columns per staged chunk
  constexpr int NPT = kThreads / CH;           // right-hand sides apart per thread
  constexpr int XPT = CH * NRT / kThreads;     // staged inputs per thread
  __shared__ typename PR::X xs[2][CH][NRT + 1];  // +1: spreads the banks of column writes
  if (c1 <= c0) return;
  const int l16 = lane & 15, kq = lane >> 4;
  const int xk = threadIdx.x % CH, xn = threadIdx.x / CH;
  uint32_t ri[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) ri[r] = min<uint32_t>(row0 + (w + 4 * r) * 16 + l16, ld - 1);
  XT xr[XPT];
  bool xok[XPT];
  auto load_x = [&](int cb) {
    const bool col_ok = cb + xk < c1;
    const XT* base = colp(min(cb + xk, c1 - 1));
#pragma unroll
    for (int i = 0; i < XPT; ++i) {
      const int n = xn + i * NPT;
      xr[i] = base[(int64_t)min(n, nv - 1) * ldx];
      xok[i] = col_ok && n < nv;
    }
  };
  auto store_x = [&](int buf) {
#pragma unroll
    for (int i = 0; i < XPT; ++i) xs[buf][xk][xn + i * NPT] = PR::cvt(xok[i] ? xr[i] : XT{});
  };
  AV a[NG][4][RT];
  auto load_a = [&](int cg, AV (&dst)[4][RT]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int col = min(cg + 4 * s + kq, c1 - 1);
#pragma unroll
      for (int r = 0; r < RT; ++r) dst[s][r] = PR::load_a(P, ri[r] + (uint32_t)col * ld);
    }
  };
  // columns past c1 hold zero inputs (and clamped panel columns), so every
  // chunk runs all its groups of four k-steps without branches
  auto group = [&](const AV (&av)[4][RT], int buf, int kk) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const typename PR::X b = xs[buf][kk + 4 * s + kq][t * 16 + l16];
#pragma unroll
        for (int r = 0; r < RT; ++r) PR::mac(acc.a[r][t], av[s][r], b);
      }
    }
  };
  const int nchunks = (c1 - c0 + CH - 1) / CH;
  load_x(c0);
  store_x(0);
#pragma unroll
  for (int g = 0; g < NG; ++g) load_a(c0 + 16 * g, a[g]);
  __syncthreads();
  for (int j = 0; j < nchunks; ++j) {
    const int cb = c0 + j * CH;
    const int buf = j & 1;
    load_x(cb + CH);  // past the last chunk: zeros, never read
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      group(a[g], buf, 16 * g);
      load_a(cb + CH + 16 * g, a[g]);
    }
    store_x(buf ^ 1);
    __syncthreads();
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
    finish_entry(A, off, i, c, make_double2(zr, zi));
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
    const int64_t* inp = A.in_perm;
    if constexpr (F32) {
      // FP32 blocks take FP32 inputs: read the shadow copy (the values the
      // products would round the FP64 inputs to anyway)
      const float2* xbase = A.xin32 + (int64_t)rhs0 * A.ldx;
      auto colp = [&](int c) -> const float2* { return xbase + src[c]; };
      mm_core<F32, RT, NT, float2>(P, ld, 0, it.c0, it.c1, colp, A.ldx, nrhs - rhs0, acc, w, lane);
    } else {
      const double2* xbase = A.xin + (int64_t)rhs0 * A.ldx;
      auto colp = [&](int c) -> const double2* {
        int64_t s = src[c];
        if (inp) s = inp[s];
        return xbase + s;
      };
      mm_core<F32, RT, NT, double2>(P, ld, 0, it.c0, it.c1, colp, A.ldx, nrhs - rhs0, acc, w, lane);
    }
    if constexpr (RT == 1) {
      // small leaves: a leaf's only piece finishes its rows straight from the
      // registers (no partial sums, no counter); larger tiles keep the
      // register budget of the partial-sum path below
      if (A.lptr[a + 1] - A.lptr[a] == 1) {
        const int64_t off = A.leaf_off[a];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = w * 16 + PR::row(kq, v);
            const int c = rhs0 + t * 16 + l16;
            if (i < m && c < nrhs) finish_entry(A, off, i, c, PR::result(acc.a[0][t], v));
          }
        continue;
      }
    }
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
    if (A.lptr[a + 1] - A.lptr[a] == 1) {
      // the leaf's only piece: its epilogue needs no counter
      __syncthreads();
      term_epilogue_mm<NRT>(A, a, rhs0, nrhs);
      __syncthreads();
      continue;
    }
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
                                                        double2* __restrict__ xin,
                                                        float2* __restrict__ xin32, int64_t ldx,
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
  // FP32: inputs and the t coefficients live in the FP32 shadow [y | t]
  if constexpr (F32) {
    const float2* xbase = xin32 + g.s_off + (int64_t)rhs0 * ldx;
    auto colp = [&](int c) -> const float2* { return xbase + c; };
    mm_core<F32, 1, NT, float2>(Wg, (uint32_t)g.ld, it.row0, 0, g.n, colp, ldx, nrhs - rhs0, acc,
                                w, lane);
  } else {
    const double2* xbase = xin + g.s_off + (int64_t)rhs0 * ldx;
    auto colp = [&](int c) -> const double2* { return xbase + c; };
    mm_core<F32, 1, NT, double2>(Wg, (uint32_t)g.ld, it.row0, 0, g.n, colp, ldx, nrhs - rhs0, acc,
                                 w, lane);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = it.row0 + w * 16 + PR::row(kq, v);
      const int c = rhs0 + t * 16 + l16;
      if (q < it.rows && c < nrhs) {
        const double2 z = PR::result(acc.a[0][t], v);
        const int64_t o = N + g.t0 + q + (int64_t)c * ldx;
        if constexpr (F32)
          xin32[o] = make_float2((float)z.x, (float)z.y);
        else
          xin[o] = z;
      }
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
  // four row tiles per wave: at most 32 right-hand sides per workgroup (the
  // 64-wide tile does not fit the register file)
  const int nt = (RT == 4) ? min(2, pick_nt(nrhs, tile)) : pick_nt(nrhs, tile);
  const dim3 grid(nwg, (nrhs + 16 * nt - 1) / (16 * nt));
  if (nt == 1)
    hipLaunchKernelGGL((k_term_mm<F32, RT, 1>), grid, dim3(kThreads), 0, st, a, nrhs);
  else if (nt == 2 || RT == 4)
    hipLaunchKernelGGL((k_term_mm<F32, RT, 2>), grid, dim3(kThreads), 0, st, a, nrhs);
  else
    hipLaunchKernelGGL((k_term_mm<F32, RT, RT == 4 ? 2 : 4>), grid, dim3(kThreads), 0, st, a,
                       nrhs);
  return hipGetLastError();
}

template <bool F32>
hipError_t stageA_mm_p(const void* W, const Group* groups, const GroupItem* items, int nitems,
                       double2* xin, float2* xin32, int64_t ldx, int64_t N, int nrhs, int tile,
                       hipStream_t st) {
  const int nt = pick_nt(nrhs, tile);
  const dim3 grid(nitems, (nrhs + 16 * nt - 1) / (16 * nt));
  if (nt == 1)
    hipLaunchKernelGGL((k_stageA_mm<F32, 1>), grid, dim3(kThreads), 0, st, W, groups, items, xin,
                       xin32, ldx, N, nrhs);
  else if (nt == 2)
    hipLaunchKernelGGL((k_stageA_mm<F32, 2>), grid, dim3(kThreads), 0, st, W, groups, items, xin,
                       xin32, ldx, N, nrhs);
  else
    hipLaunchKernelGGL((k_stageA_mm<F32, 4>), grid, dim3(kThreads), 0, st, W, groups, items, xin,
                       xin32, ldx, N, nrhs);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_term_mm(bool f32, int max_m, const TermArgs& a, int nwg, int nrhs, int tile,
                          hipStream_t st) {
  if (nwg <= 0 || nrhs <= 0) return hipSuccess;
  if (f32 && (!a.xin32 || a.in_perm)) return hipErrorInvalidValue;  // FP32 reads the shadow
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
                            int nitems, double2* xin, float2* xin32, int64_t ldx, int64_t N,
                            int nrhs, int tile, hipStream_t st) {
  if (nitems <= 0 || nrhs <= 0) return hipSuccess;
  if (f32 && !xin32) return hipErrorInvalidValue;
  return f32 ? stageA_mm_p<true>(W, groups, items, nitems, xin, xin32, ldx, N, nrhs, tile, st)
             : stageA_mm_p<false>(W, groups, items, nitems, xin, xin32, ldx, N, nrhs, tile, st);
}

}  // namespace hm
