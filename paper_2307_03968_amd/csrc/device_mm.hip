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
//
// Every wave works on its own: the inputs are kept in row layout (the
// right-hand sides of one source point contiguous), so the B operand of a
// k-step (4 panel columns x 16 right-hand sides) is four 128- or 256-byte
// rows read straight from L2 with one load per lane, and no LDS staging or
// workgroup barrier is needed.  A piece (panel columns [c0, c1) of a leaf)
// streams D k-steps ahead of the products through a ring of registers (the
// source index of a column one more ring ahead, since the B address depends
// on it).  Leaves of at most 64 rows: one wave takes a whole leaf (up to
// four 16-row tiles, only the tiles the leaf has); larger leaves: the four
// waves of a workgroup take the same piece, each its own block of rows, so
// the B rows they share are read from L2 by one workgroup at a time.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dev.h"

namespace hm {

namespace {

#ifndef HM_MM_D32
#define HM_MM_D32 8  // k-steps of 4 columns in flight per wave, FP32 blocks
#endif
#ifndef HM_MM_D32_WIDE
#define HM_MM_D32_WIDE 12  // the same, FP32 blocks with 64-RHS tiles
#endif
#ifndef HM_MM_D64
#define HM_MM_D64 4  // the same, FP64 blocks
#endif

constexpr int kThreads = 256;
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Device-coherent (agent-scope) loads and stores of the row-layout vectors
// and x in the multi-term launch, where one term's values are read by
// waves of any XCD in the next term.
__device__ __forceinline__ float2 load_co(const float2* p) {
  const uint64_t v =
      __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  float2 r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}
__device__ __forceinline__ double2 load_co(const double2* p) {
  const double* d = reinterpret_cast<const double*>(p);
  return make_double2(__hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                      __hip_atomic_load(d + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void store_co(float2* p, float2 v) {
  uint64_t u;
  __builtin_memcpy(&u, &v, sizeof(u));
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_co(double2* p, double2 v) {
  double* d = reinterpret_cast<double*>(p);
  __hip_atomic_store(d, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(d + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-coherent load of a counter, the same value in every lane (a
// wave-uniform value: the control flow that depends on it stays uniform).
__device__ __forceinline__ int load_uniform(const int32_t* c) {
  return __builtin_amdgcn_readfirstlane(__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Wave-uniform fetch-and-add of one: every lane issues the atomic (lane 0
// adds one, the others zero), and every lane receives lane 0's result.
// No lane-0-only branch feeds the wave's control flow, so the compiler has
// no divergent region to split the wave's loop iterations over.
__device__ __forceinline__ int fetch_add_uniform(int32_t* c, int lane) {
  return __builtin_amdgcn_readfirstlane(
      __hip_atomic_fetch_add(c, lane == 0 ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Count of one finished item: a non-returning atomic from lane 0 (no value
// comes back into the wave's control flow, and the wave does not wait for
// it: increments of one shared counter queue at the device's coherence
// point instead of stalling every wave that makes them).
__device__ __forceinline__ void count_done(int32_t* c, int lane) {
  if (lane == 0) (void)__hip_atomic_fetch_add(c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool F32>
struct Prec;

template <>
struct Prec<true> {                      // FP32 blocks, 3M
  using A = float2;                      // panel element
  using X = float2;                      // input element (row layout)
  using Acc = f4v;
  static constexpr int NACC = 3;
  static constexpr int D = HM_MM_D32;    // k-steps in flight
  __device__ static __forceinline__ A load_a(const void* P, uint32_t byte_off) {
    const fvec2 v = __builtin_nontemporal_load(
        reinterpret_cast<const fvec2*>(reinterpret_cast<const char*>(P) + byte_off));
    return make_float2(v.x, v.y);
  }
  __device__ static __forceinline__ void mac(Acc (&acc)[3], float2 a, float as, X b, float bs) {
    acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc[1], 0, 0, 0);
    acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(as, bs, acc[2], 0, 0, 0);
  }
  __device__ static __forceinline__ float sum(float2 v) { return v.x + v.y; }
  __device__ static __forceinline__ double2 result(const Acc (&acc)[3], int v) {
    const double t1 = acc[0][v], t2 = acc[1][v], t3 = acc[2][v];
    return make_double2(t1 - t2, t3 - t1 - t2);
  }
  __device__ static __forceinline__ X from(double2 z) { return make_float2((float)z.x, (float)z.y); }
  // row of result element v within the 16 x 16 tile (kq = lane / 16)
  __device__ static __forceinline__ int row(int kq, int v) { return 4 * kq + v; }
};

template <>
struct Prec<false> {                     // FP64 blocks, four real products
  using A = double2;
  using X = double2;
  using Acc = d4v;
  static constexpr int NACC = 2;
  static constexpr int D = HM_MM_D64;
  __device__ static __forceinline__ A load_a(const void* P, uint32_t byte_off) {
    const dvec2 v = __builtin_nontemporal_load(
        reinterpret_cast<const dvec2*>(reinterpret_cast<const char*>(P) + byte_off));
    return make_double2(v.x, v.y);
  }
  __device__ static __forceinline__ void mac(Acc (&acc)[2], double2 a, double, X b, double) {
    acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, acc[0], 0, 0, 0);
    acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, acc[1], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, acc[1], 0, 0, 0);
  }
  __device__ static __forceinline__ double sum(double2) { return 0.0; }
  __device__ static __forceinline__ double2 result(const Acc (&acc)[2], int v) {
    return make_double2(acc[0][v], acc[1][v]);
  }
  __device__ static __forceinline__ X from(double2 z) { return z; }
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

// acc[r][t] += P[row0 + 16 r + (0..15), c0 : c1) X[src(c0 : c1), rhs0 + 16 t + (0..15)]
// for the RTL row tiles r < RTL of this wave.  P is column-major with
// leading dimension ld (its allocation extends at least 16 rows past the
// last column, so the row tiles need no clamp: rows past ld read the next
// column, and rows past m are never stored); srcf(c) is the X row holding
// column c's input, and X row zrow is all zero.
// The sources travel 64 columns (16 k-steps) at a time: lane l loads the
// source of column c0 + 64 j + l (zrow past c1) one block early and parks it
// in a per-wave ring of three blocks in LDS, from which a k-step reads its
// lane's value; so the loads of a k-step depend on no vector load issued
// after the ring slot was written.  Panel loads past c1 are issued at the
// clamped column c1 - 1 and read the zero row of X, so every k-step runs the same
// instructions; right-hand sides past the row length are read at the
// clamped column ldr - 1 (their products land in result columns that are
// never stored).  One loop iteration covers one block of 16 k-steps, so the
// code inside the loop is the same in every iteration.  CO: the inputs are
// read with device-coherent loads (the multi-term launch).
template <bool F32, int RT, int NT, int RTL, bool CO = false, typename SRCF>
__device__ __forceinline__ void mm_wave(const void* __restrict__ P, uint32_t ld, int row0, int c0,
                                        int c1, const SRCF& srcf,
                                        const typename Prec<F32>::X* __restrict__ xr, int64_t ldr,
                                        int zrow, int rhs0, MMAcc<F32, RT, NT>& acc, int lane,
                                        int* __restrict__ ring) {
  using PR = Prec<F32>;
  using AV = typename PR::A;
  using XV = typename PR::X;
  // a 64-RHS FP32 tile spends more matrix-core time per k-step, and a
  // deeper pipeline keeps its loads ahead (measured on the 32^3 cube)
  constexpr int D = (F32 && NT >= 4) ? HM_MM_D32_WIDE : PR::D;
  static_assert(D <= 16, "the loads of a k-step lie at most one block ahead");
  if (c1 <= c0) return;
  const int l16 = lane & 15, kq = lane >> 4;
  // byte offsets: panel entry (row0 + l16, column c) and the input rows stay
  // 32-bit (a panel set and a row-layout vector are below 2^32 bytes)
  constexpr uint32_t esz = sizeof(AV);
  const uint32_t a_first = (uint32_t)(row0 + l16 + (c0 + kq) * ld) * esz;
  const uint32_t a_last = (uint32_t)(row0 + l16 + (c1 - 1) * ld) * esz;
  const uint32_t a_step = 4u * ld * esz;
  uint32_t cx[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) cx[t] = (uint32_t)min<int64_t>(rhs0 + 16 * t + l16, ldr - 1);
  const uint32_t ldr32 = (uint32_t)ldr;
  const int nsteps = (c1 - c0 + 3) >> 2;
  auto block = [&](int j) -> int {
    const int c = c0 + 64 * j + lane;
    const int v = srcf(min(c, c1 - 1));
    return c < c1 ? v : zrow;
  };
  AV ab[D][RTL];
  XV bb[D][NT];
  auto load = [&](int s, AV (&a)[RTL], XV (&b)[NT]) {
    const uint32_t ao = min(a_first + (uint32_t)s * a_step, a_last);
#pragma unroll
    for (int r = 0; r < RTL; ++r) a[r] = PR::load_a(P, ao + r * 16 * esz);
    const int srow = ring[((s >> 4) % 3) * 64 + 4 * (s & 15) + kq];
    const uint32_t rb = (uint32_t)srow * ldr32;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if constexpr (CO) b[t] = load_co(xr + rb + cx[t]);
      else b[t] = xr[rb + cx[t]];
    }
  };
  ring[lane] = block(0);
  ring[64 + lane] = block(1);
#pragma unroll
  for (int d = 0; d < D; ++d) load(d, ab[d], bb[d]);
  for (int k = 0; k < nsteps; k += 16) {
    const int nxt = block((k >> 4) + 2);  // parked at the end of the block
#pragma unroll
    for (int d = 0; d < 16; ++d) {
      const int slot = d % D;
      decltype(PR::sum(XV{})) bs[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) bs[t] = PR::sum(bb[slot][t]);
#pragma unroll
      for (int r = 0; r < RTL; ++r) {
        const auto as = PR::sum(ab[slot][r]);
#pragma unroll
        for (int t = 0; t < NT; ++t) PR::mac(acc.a[r][t], ab[slot][r], as, bb[slot][t], bs[t]);
      }
      load(k + d + D, ab[slot], bb[slot]);
      // keep this k-step's products and the refill of its ring slot where
      // they are: otherwise the scheduler gathers the products of many
      // k-steps first and issues the loads after them, leaving no time
      // between a load and its use
      __builtin_amdgcn_sched_barrier(0);
    }
    ring[(((k >> 4) + 2) % 3) * 64 + lane] = nxt;
  }
}

// ---------------------------------------------------------------- term
// Sum of the partial rows of one leaf's pieces for rows [row0, row0 + nrow)
// and one tile of right-hand sides, then the term epilogue; one wave, the
// right-hand sides of a row on consecutive lanes.
// Epilogue of one entry in the multi-term launch: y = alpha z to the next
// term's rows and x += y, through device-coherent accesses (the leaf's
// earlier terms may have run on another XCD); the last term also writes
// the column-layout y and the output.
__device__ __forceinline__ void finish_entry_co(const TermArgs& A, const MMSeriesArgs& S,
                                                bool last, int64_t off, int i, int c, double2 z) {
  const double2 y = make_double2(A.alpha * z.x, A.alpha * z.y);
  if (A.yrow) store_co(A.yrow + (off + i) * A.ldr + c, y);
  if (A.yrow32) store_co(A.yrow32 + (off + i) * A.ldr + c, make_float2((float)y.x, (float)y.y));
  const int64_t q = off + i + (int64_t)c * A.ldxa;
  const double2 o = load_co(A.xacc + q);
  const double2 res = make_double2(y.x + o.x, y.y + o.y);
  store_co(A.xacc + q, res);
  if (last) {
    if (S.yout) S.yout[off + i + (int64_t)c * S.ldy] = y;
    if (S.out) S.out[S.out_perm[off + i] + (int64_t)c * S.ldo] = res;
  }
}

template <int NRT, bool MT = false>
__device__ void mm_epilogue(const TermArgs& A, int a, int row0, int nrow, int rhs0, int nrhs,
                            int lane, const MMSeriesArgs* S = nullptr, bool last = false) {
  const int64_t off = A.leaf_off[a];
  const int q0 = A.lptr[a], np = A.lptr[a + 1] - q0;
  for (int idx = lane; idx < nrow * NRT; idx += 64) {
    const int i = row0 + idx / NRT;
    const int c = rhs0 + idx % NRT;
    if (c >= nrhs) continue;
    double zr = 0.0, zi = 0.0;
    for (int p = 0; p < np; p += 8) {  // fixed order; loads in flight together
      double vr[8], vi[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (p + u < np) {
          const double* q =
              reinterpret_cast<const double*>(A.partial + ((int64_t)A.lprow[q0 + p + u] + i) * A.ldr + c);
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
    if constexpr (MT) finish_entry_co(A, *S, last, off, i, c, make_double2(zr, zi));
    else finish_entry(A, off, i, c, make_double2(zr, zi));
  }
}

// One piece on one wave: the products of its rows (RTL tiles), then either
// the epilogue straight from the registers (the leaf's only piece) or the
// partial sums published with agent-scope stores and the wave that brings
// the (leaf, row block) counter to the piece count sums them.  Returns
// whether this wave ran the epilogue.  MT: the multi-term launch (coherent
// inputs and epilogue, S and last as in finish_entry_co).
template <bool F32, int RT, int NT, int RTL, bool MT = false>
__device__ __forceinline__ bool term_piece(const TermArgs& A, const TermItem& it, int m, int rb,
                                           int row0, int rhs0, int nrhs, int lane, int* ring,
                                           const MMSeriesArgs* S = nullptr, bool last = false) {
  using PR = Prec<F32>;
  using XV = typename PR::X;
  constexpr int NRT = 16 * NT;
  const int a = it.leaf;
  const uint32_t ld = (uint32_t)(m + (m & 1));
  const int64_t poff = __builtin_amdgcn_readfirstlane((int)(A.ps.panel_off[a] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(A.ps.panel_off[a] >> 32)) << 32);
  const int64_t coff = __builtin_amdgcn_readfirstlane((int)(A.ps.col_off[a] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(A.ps.col_off[a] >> 32)) << 32);
  const void* P = F32 ? (const void*)(reinterpret_cast<const float2*>(A.ps.data) + poff)
                      : (const void*)(reinterpret_cast<const double2*>(A.ps.data) + poff);
  const int32_t* __restrict__ src = A.ps.src + coff;
  const XV* xr = F32 ? reinterpret_cast<const XV*>(A.xr32) : reinterpret_cast<const XV*>(A.xr);
  MMAcc<F32, RT, NT> acc;
  acc.zero();
  auto srcf = [&](int c) -> int { return src[c]; };
  mm_wave<F32, RT, NT, RTL, MT>(P, ld, row0, it.c0, it.c1, srcf, xr, A.ldr, A.zrow, rhs0, acc, lane,
                                ring);
  const int l16 = lane & 15, kq = lane >> 4;
  const int np = __builtin_amdgcn_readfirstlane(A.lptr[a + 1] - A.lptr[a]);
  if (np == 1) {
    const int64_t off = A.leaf_off[a];
#pragma unroll
    for (int r = 0; r < RTL; ++r)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = row0 + 16 * r + PR::row(kq, v);
          const int c = rhs0 + 16 * t + l16;
          if (i < m && c < nrhs) {
            if constexpr (MT) finish_entry_co(A, *S, last, off, i, c, PR::result(acc.a[r][t], v));
            else finish_entry(A, off, i, c, PR::result(acc.a[r][t], v));
          }
        }
    return true;
  }
#pragma unroll
  for (int r = 0; r < RTL; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0 + 16 * r + PR::row(kq, v);
        const int c = rhs0 + 16 * t + l16;
        if (i < m && c < nrhs) {
          const double2 z = PR::result(acc.a[r][t], v);
          double* q = reinterpret_cast<double*>(A.partial + ((int64_t)it.prow + i) * A.ldr + c);
          __hip_atomic_store(q, z.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(q + 1, z.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
  // the stores have completed at the device's coherence point before the
  // counter moves, so the wave that finishes the count reads them all
  __builtin_amdgcn_s_waitcnt(0);
  int32_t* cnt = A.counters + ((int64_t)a * 4 + rb) * gridDim.y + blockIdx.y;
  const int old = fetch_add_uniform(cnt, lane);
  if (old == np - 1) {
    mm_epilogue<NRT, MT>(A, a, row0, min(16 * RTL, m - row0), rhs0, nrhs, lane, S, last);
    if (lane == 0) __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
  }
  return false;
}

// Workgroups are dispatched to the eight XCDs in turn (workgroup b to XCD
// b mod 8), each XCD with its own L2.  Workgroup b runs list position
// (b mod 8) G/8 + b/8, so XCD x runs positions [x G/8, (x + 1) G/8): a
// contiguous range of the tree order, whose leaves read overlapping input
// rows from one L2.  The identity when G is not a multiple of 8.
__device__ __forceinline__ int xcd_order(int b, int G) {
  return (G & 7) ? b : (b & 7) * (G >> 3) + (b >> 3);
}

// Persistent term kernel.  WAVE: unit = wave (pieces grouped by wave), the
// wave takes all rows of its leaves (m <= 16 RT).  Otherwise unit =
// workgroup, wave w takes rows [16 RT w, 16 RT (w + 1)) of every piece of
// its workgroup.
template <bool F32, int RT, int NT, bool WAVE>
__global__ __launch_bounds__(kThreads) void k_term_mm(TermArgs A, int nrhs, int nunits) {
  const int lane = threadIdx.x & 63;
  const int w = wave_id();
  const int b = xcd_order((int)blockIdx.x, (int)gridDim.x);
  const int unit = WAVE ? b * 4 + w : b;
  if (unit >= nunits) return;
  const int rb = WAVE ? 0 : w;
  const int rhs0 = blockIdx.y * 16 * NT;
  __shared__ int rings[4][3 * 64];  // per wave: sources of three 64-column blocks
  int* ring = rings[w];
  const int pe = A.wptr[unit + 1];
  for (int p = A.wptr[unit]; p < pe; ++p) {
    // the piece is the same for the whole wave: keep it in scalar registers
    // (uniform branches, scalar base addresses)
    TermItem it = A.items[p];
    it.leaf = __builtin_amdgcn_readfirstlane(it.leaf);
    it.c0 = __builtin_amdgcn_readfirstlane(it.c0);
    it.c1 = __builtin_amdgcn_readfirstlane(it.c1);
    it.prow = __builtin_amdgcn_readfirstlane(it.prow);
    const int m = __builtin_amdgcn_readfirstlane(A.ps.leaf_m[it.leaf]);
    const int row0 = rb * 16 * RT;
    if (row0 >= m) continue;
    const int rtl = min(RT, (m - row0 + 15) >> 4);
    if constexpr (RT >= 4) {
      if (rtl == 4) { term_piece<F32, RT, NT, 4>(A, it, m, rb, row0, rhs0, nrhs, lane, ring); continue; }
      if (rtl == 3) { term_piece<F32, RT, NT, 3>(A, it, m, rb, row0, rhs0, nrhs, lane, ring); continue; }
    }
    if constexpr (RT >= 2) {
      if (rtl == 2) { term_piece<F32, RT, NT, 2>(A, it, m, rb, row0, rhs0, nrhs, lane, ring); continue; }
    }
    term_piece<F32, RT, NT, 1>(A, it, m, rb, row0, rhs0, nrhs, lane, ring);
  }
}

// ---------------------------------------------------------------- stage A
// One workgroup = a 64-row tile of a source group, wave w its rows
// [16 w, 16 w + 16): t rows = W_g X[s_off .. s_off + n), written to the t
// rows of the same row-layout vector.
template <bool F32, int NT>
__global__ __launch_bounds__(kThreads) void k_stageA_mm(const void* __restrict__ W,
                                                        const Group* __restrict__ groups,
                                                        const GroupItem* __restrict__ items,
                                                        typename Prec<F32>::X* __restrict__ xr,
                                                        int64_t ldr, int64_t N, int zrow, int nrhs) {
  using PR = Prec<F32>;
  const GroupItem it = items[blockIdx.x];
  const Group g = groups[it.group];
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  const int row0 = it.row0 + 16 * w;
  if (row0 >= it.rows) return;
  const void* Wg = F32 ? (const void*)(reinterpret_cast<const float2*>(W) + g.w_off)
                       : (const void*)(reinterpret_cast<const double2*>(W) + g.w_off);
  const int rhs0 = blockIdx.y * 16 * NT;
  MMAcc<F32, 1, NT> acc;
  acc.zero();
  const int s_off = g.s_off;
  auto srcf = [&](int c) -> int { return s_off + c; };
  __shared__ int rings[4][3 * 64];
  mm_wave<F32, 1, NT, 1>(Wg, (uint32_t)g.ld, row0, 0, g.n, srcf, xr, ldr, zrow, rhs0, acc, lane,
                         rings[w]);
  const int l16 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = row0 + PR::row(kq, v);
      const int c = rhs0 + 16 * t + l16;
      if (q < it.rows && c < nrhs) xr[(N + g.t0 + q) * ldr + c] = PR::from(PR::result(acc.a[0][t], v));
    }
}

// ---------------------------------------------------------------- multi-term
constexpr int kSeriesSpinLimit = 1 << 21;

// The wave waits (bounded) until *c reaches need; gives up setting *err.
__device__ __forceinline__ void wait_count(const int32_t* c, int need, int32_t* err) {
  if (need <= 0) return;
  for (int spins = 0; load_uniform(c) < need; ++spins) {
    if (spins >= kSeriesSpinLimit || load_uniform(err) != 0) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// The K series terms of MMSeriesArgs in one launch; every wave takes items
// from the queue on its own (no workgroup barrier anywhere).
template <bool F32, int NT>
__global__ __launch_bounds__(kThreads) void k_series_mm(TermArgs A, MMSeriesArgs S, int nrhs) {
  using PR = Prec<F32>;
  using XV = typename PR::X;
  const int lane = threadIdx.x & 63;
  const int w = wave_id();
  const int l16 = lane & 15, kq = lane >> 4;
  __shared__ int rings[4][3 * 64];
  int* ring = rings[w];
  const int per = S.n_a + S.n_b;
  const int total = S.K * per;
  for (;;) {
    // one ticket per fetch: items differ widely in size, and a wave holding
    // several consecutive tickets leaves a long tail (measured)
    const int tk = fetch_add_uniform(S.queue, lane);
    if (tk >= total) break;
    const int k = tk / per + 1, j = tk - (k - 1) * per;
    const int kind = __builtin_amdgcn_readfirstlane(S.items[j].kind);
    const int inst = __builtin_amdgcn_readfirstlane(S.items[j].inst);
    const int ia = __builtin_amdgcn_readfirstlane(S.items[j].a);
    const int cur = (k - 1) & 1;
    int32_t* cnt_k = S.cnt + ((int64_t)inst * S.kmax + (k - 1)) * 2;  // [tiles, epilogues] of term k
    const int need_b = S.need_b[inst];
    if (kind == 0) {
      // stage-A tile: t_k rows [row0, row0 + kGroupTileMM) of group ia from
      // y_{k-1}, 16 rows at a time
      if (k > 1) wait_count(cnt_k - 2 + 1, need_b, S.err);
      const int row0 = __builtin_amdgcn_readfirstlane(S.items[j].row0);
      const int rows = __builtin_amdgcn_readfirstlane(S.items[j].rows);
      const Group g = S.groups[ia];
      XV* xr = F32 ? reinterpret_cast<XV*>(S.r32[cur]) : reinterpret_cast<XV*>(S.r64[cur]);
      const void* Wg = F32 ? (const void*)(reinterpret_cast<const float2*>(S.W) + g.w_off)
                           : (const void*)(reinterpret_cast<const double2*>(S.W) + g.w_off);
      const int s_off = g.s_off;
      auto srcf = [&](int c) -> int { return s_off + c; };
      for (int r0 = row0; r0 < rows && r0 < row0 + kGroupTileMM; r0 += 16) {
        MMAcc<F32, 1, NT> acc;
        acc.zero();
        mm_wave<F32, 1, NT, 1, true>(Wg, (uint32_t)g.ld, r0, 0, g.n, srcf, xr, A.ldr, A.zrow, 0, acc,
                                     lane, ring);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int q = r0 + PR::row(kq, v);
            const int c = 16 * t + l16;
            if (q < rows && c < nrhs)
              store_co(xr + (S.N + g.t0 + q) * A.ldr + c, PR::from(PR::result(acc.a[0][t], v)));
          }
      }
      __builtin_amdgcn_s_waitcnt(0);  // the t rows are complete before the count moves
      count_done(cnt_k, lane);
    } else {
      // term piece of leaf ia: waits for its instance's t_k and y_{k-1}
      wait_count(cnt_k, S.need_a[inst], S.err);
      if (k > 1) wait_count(cnt_k - 2 + 1, need_b, S.err);
      TermArgs T = A;
      T.xr = S.r64[cur];
      T.xr32 = S.r32[cur];
      T.yrow = F32 ? nullptr : S.r64[cur ^ 1];
      T.yrow32 = F32 ? S.r32[cur ^ 1] : nullptr;
      TermItem it;
      it.leaf = ia;
      it.kind = 0;
      it.c0 = __builtin_amdgcn_readfirstlane(S.items[j].c0);
      it.c1 = __builtin_amdgcn_readfirstlane(S.items[j].c1);
      it.r0 = it.r1 = 0;
      it.prow = __builtin_amdgcn_readfirstlane(S.items[j].prow);
      it.pad = 0;
      const int m = __builtin_amdgcn_readfirstlane(A.ps.leaf_m[ia]);
      const int rtl = min(4, (m + 15) >> 4);
      const bool last = k == S.K;
      bool epi;
      if (rtl == 4) epi = term_piece<F32, 4, NT, 4, true>(T, it, m, 0, 0, 0, nrhs, lane, ring, &S, last);
      else if (rtl == 3) epi = term_piece<F32, 4, NT, 3, true>(T, it, m, 0, 0, 0, nrhs, lane, ring, &S, last);
      else if (rtl == 2) epi = term_piece<F32, 4, NT, 2, true>(T, it, m, 0, 0, 0, nrhs, lane, ring, &S, last);
      else epi = term_piece<F32, 4, NT, 1, true>(T, it, m, 0, 0, 0, nrhs, lane, ring, &S, last);
      if (epi) {
        __builtin_amdgcn_s_waitcnt(0);  // y_k and x of the leaf are complete before the count
        count_done(cnt_k + 1, lane);
      }
    }
  }
  // the last wave out clears the queue and the counters for the next launch.
  // Every count of a wave has landed before the wave counts itself out: its
  // later queue fetches return a value, and the wait for that value covers
  // all of the wave's earlier vector memory operations (gfx950 counts them
  // with one in-order counter), so no increment arrives after the clear.
  if (fetch_add_uniform(S.queue + 1, lane) == (int)gridDim.x * 4 - 1) {
    for (int i = lane; i < S.ninst * S.kmax * 2; i += 64)
      __hip_atomic_store(S.cnt + i, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (lane == 0) {
      __hip_atomic_store(S.queue, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(S.queue + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------- layout
// Column layout (n x nrhs, ld ldi, rows through perm when set) to row
// layout through a 64 x 16 LDS tile: reads coalesced along the rows, writes
// along the right-hand sides.
__global__ __launch_bounds__(kThreads) void k_rows(const double2* __restrict__ in, int64_t ldi,
                                                   const int64_t* __restrict__ perm, int64_t n,
                                                   int nrhs, double2* __restrict__ out,
                                                   float2* __restrict__ out32, int64_t ldr) {
  __shared__ double2 tile[16][65];
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 16;
  {
    const int pl = threadIdx.x & 63;
    const int64_t p = p0 + pl;
    const int64_t srow = (p < n) ? (perm ? perm[p] : p) : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cl = (threadIdx.x >> 6) + 4 * j;
      const int c = c0 + cl;
      tile[cl][pl] = (p < n && c < nrhs) ? in[srow + (int64_t)c * ldi] : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int cl = threadIdx.x & 15;
    const int pl = (threadIdx.x >> 4) + 16 * j;
    const int64_t p = p0 + pl;
    if (p >= n || c0 + cl >= ldr) continue;
    const double2 v = tile[cl][pl];
    if (out) out[p * ldr + c0 + cl] = v;
    if (out32) out32[p * ldr + c0 + cl] = make_float2((float)v.x, (float)v.y);
  }
}

// 16-column right-hand-side tiles per unit: the requested tile (16, 32 or
// 64), or by nrhs when 0; at most cap
inline int pick_nt(int nrhs, int tile, int cap) {
  int nt = (tile == 16 || tile == 32 || tile == 64) ? tile / 16 : (nrhs <= 16 ? 1 : (nrhs <= 32 ? 2 : 4));
  return nt < cap ? nt : cap;
}

template <bool F32, int RT, bool WAVE>
hipError_t term_mm_launch(const TermArgs& a, int nunits, int nrhs, int tile, hipStream_t st) {
  // accumulator registers: RT x NT tiles (at most 8 per wave)
  const int nt = pick_nt(nrhs, tile, RT >= 4 ? 2 : 4);
  const int nwg = WAVE ? (nunits + 3) / 4 : nunits;
  const dim3 grid(nwg, (nrhs + 16 * nt - 1) / (16 * nt));
  if (nt == 1)
    hipLaunchKernelGGL((k_term_mm<F32, RT, 1, WAVE>), grid, dim3(kThreads), 0, st, a, nrhs, nunits);
  else if (nt == 2)
    hipLaunchKernelGGL((k_term_mm<F32, RT, 2, WAVE>), grid, dim3(kThreads), 0, st, a, nrhs, nunits);
  else if constexpr (RT <= 2)
    hipLaunchKernelGGL((k_term_mm<F32, RT, 4, WAVE>), grid, dim3(kThreads), 0, st, a, nrhs, nunits);
  return hipGetLastError();
}

template <bool F32>
hipError_t stageA_mm_p(const void* W, const Group* groups, const GroupItem* items, int nitems,
                       typename Prec<F32>::X* xr, int64_t ldr, int64_t N, int zrow, int nrhs,
                       int tile, hipStream_t st) {
  const int nt = pick_nt(nrhs, tile, 4);
  const dim3 grid(nitems, (nrhs + 16 * nt - 1) / (16 * nt));
  if (nt == 1)
    hipLaunchKernelGGL((k_stageA_mm<F32, 1>), grid, dim3(kThreads), 0, st, W, groups, items, xr, ldr,
                       N, zrow, nrhs);
  else if (nt == 2)
    hipLaunchKernelGGL((k_stageA_mm<F32, 2>), grid, dim3(kThreads), 0, st, W, groups, items, xr, ldr,
                       N, zrow, nrhs);
  else
    hipLaunchKernelGGL((k_stageA_mm<F32, 4>), grid, dim3(kThreads), 0, st, W, groups, items, xr, ldr,
                       N, zrow, nrhs);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_term_mm(bool f32, int max_m, const TermArgs& a, int nunits, int nrhs, int tile,
                          hipStream_t st) {
  if (nunits <= 0 || nrhs <= 0) return hipSuccess;
  if (max_m > 256 || a.ldr < row_ld(nrhs) || (f32 ? !a.xr32 : !a.xr)) return hipErrorInvalidValue;
  if (mm_wave_mode(max_m))
    return f32 ? term_mm_launch<true, 4, true>(a, nunits, nrhs, tile, st)
               : term_mm_launch<false, 4, true>(a, nunits, nrhs, tile, st);
  if (max_m <= 128)
    return f32 ? term_mm_launch<true, 2, false>(a, nunits, nrhs, tile, st)
               : term_mm_launch<false, 2, false>(a, nunits, nrhs, tile, st);
  return f32 ? term_mm_launch<true, 4, false>(a, nunits, nrhs, tile, st)
             : term_mm_launch<false, 4, false>(a, nunits, nrhs, tile, st);
}

hipError_t launch_series_mm(bool f32, const TermArgs& a, const MMSeriesArgs& s, int nwg, int nrhs,
                            hipStream_t st) {
  if (nwg <= 0 || s.K <= 0) return hipSuccess;
  if (s.K > s.kmax || nrhs <= 0 || nrhs > 32 || a.ldr < row_ld(nrhs) || (f32 ? !a.xr32 : !a.xr) ||
      (int64_t)s.K * (s.n_a + s.n_b) >= ((int64_t)1 << 31))
    return hipErrorInvalidValue;
  if (nrhs <= 16) {
    if (f32) hipLaunchKernelGGL((k_series_mm<true, 1>), dim3(nwg), dim3(kThreads), 0, st, a, s, nrhs);
    else hipLaunchKernelGGL((k_series_mm<false, 1>), dim3(nwg), dim3(kThreads), 0, st, a, s, nrhs);
  } else {
    if (f32) hipLaunchKernelGGL((k_series_mm<true, 2>), dim3(nwg), dim3(kThreads), 0, st, a, s, nrhs);
    else hipLaunchKernelGGL((k_series_mm<false, 2>), dim3(nwg), dim3(kThreads), 0, st, a, s, nrhs);
  }
  return hipGetLastError();
}

int series_mm_occupancy(bool f32, int nrhs) {
  int n = 0;
  hipError_t e;
  if (nrhs <= 16)
    e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_series_mm<true, 1>, kThreads, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_series_mm<false, 1>, kThreads, 0);
  else
    e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_series_mm<true, 2>, kThreads, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_series_mm<false, 2>, kThreads, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_stageA_mm(bool f32, const void* W, const Group* groups, const GroupItem* items,
                            int nitems, double2* xr, float2* xr32, int64_t ldr, int64_t N,
                            int zrow, int nrhs, int tile, hipStream_t st) {
  if (nitems <= 0 || nrhs <= 0) return hipSuccess;
  if (ldr < row_ld(nrhs) || (f32 ? !xr32 : !xr)) return hipErrorInvalidValue;
  return f32 ? stageA_mm_p<true>(W, groups, items, nitems, xr32, ldr, N, zrow, nrhs, tile, st)
             : stageA_mm_p<false>(W, groups, items, nitems, xr, ldr, N, zrow, nrhs, tile, st);
}

hipError_t launch_rows(const double2* in, int64_t ldi, const int64_t* perm, int64_t n, int nrhs,
                       double2* out, float2* out32, int64_t ldr, hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (ldr < row_ld(nrhs)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)(ldr / 16));
  hipLaunchKernelGGL(k_rows, grid, dim3(kThreads), 0, st, in, ldi, perm, n, nrhs, out, out32, ldr);
  return hipGetLastError();
}

}  // namespace hm
