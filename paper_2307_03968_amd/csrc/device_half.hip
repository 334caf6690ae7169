// Half-storage product kernel of libhmps for symmetric (surface) problems,
// one right-hand side: z = alpha R y + beta v with every off-diagonal near
// block read once (the symmetric operator of Sec. II carried into the
// series of Sec. IV).
//
// The surface operator is symmetric, so the near block Z_st (s > t) is the
// transpose of Z_ts.  Each row leaf t keeps only its blocks Z_ts, s > t,
// side by side as one column-major half panel.  A workgroup streams a range
// of half-panel columns exactly as the ordinary term kernel streams panel
// columns (lane = row, 16-byte loads, eight columns in flight per wave) and
// forms two products from each loaded column j:
//   u_t += Z[:, j] y[src_j]                     (rows of t, like a panel)
//   v_j  = Z[:, j]^T y_t                        (one value per column)
// v_j is a sum over the rows, i.e. over the lanes of one wave: eight columns
// are reduced together with a butterfly whose first three exchanges halve
// the set of columns (ten exchanges for eight sums) and stored to slot j of
// vb.  v_j is row jj of Z_st y_t when column j is row jj of leaf s, so the
// epilogue of leaf s adds the vb slots of its blocks (t, s) to its partial
// sums.  A far block between two leaves t < s is stored once as its pair of
// factors and applied in both orientations from one read (far_pairs); the
// other far blocks keep one copy per orientation (in-row W stacks and the
// U columns of the far panels).
//
// Completion: each piece counts once for its own leaf and once for every
// leaf its v values or pair rows go to; the workgroup that brings a leaf's
// counter to its total sums the leaf's u partials, vb slots and pair rows
// in a fixed order and writes z.  The diagonal block is applied by a separate block-diagonal
// launch of the term kernel (D^{-1} z for a series term, D x + z for the
// H-matvec).  Relative to the D^{-1}-premultiplied panels this reads the
// off-diagonal near blocks once instead of twice.
#include <hip/hip_runtime.h>

#include "dev.h"

namespace hm {

namespace {

#include "gemv_inl.h"

// 32-bit lane moves within rows of the wave (DPP), applied to both halves
// of a double.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the sixteen lanes of each row of the wave (every lane of the
// row ends with the total): quad_perm [1,0,3,2], quad_perm [2,3,0,1], the
// mirror within each half row (lane i <-> 7 - i) pairs the quads, the
// mirror within the row (lane i <-> 15 - i) pairs the half rows.
__device__ __forceinline__ double sum16_lanes(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return v;
}

// Device-coherent (agent-scope) store of a value read by other workgroups
// of the same launch.
__device__ __forceinline__ void store_agent(double2* q, double2 z) {
  double* d = reinterpret_cast<double*>(q);
  __hip_atomic_store(d, z.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(d + 1, z.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double2 load_agent(const double2* q) {
  const double* d = reinterpret_cast<const double*>(q);
  return make_double2(__hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                      __hip_atomic_load(d + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// y entry of the term's input: a plain load within one term, a
// device-coherent load where an earlier term of the same launch wrote it.
template <bool MT>
__device__ __forceinline__ double2 ld_y(const double2* q) {
  if constexpr (MT) return load_agent(q);
  else return *q;
}

// acc += a * x (complex) with nxy = -x.y given: the negation sits on the
// operand shared by many products instead of on each loaded element.
__device__ __forceinline__ void cmac_n(double2& acc, double2 a, double2 x, double nxy) {
  acc.x = fma(a.x, x.x, acc.x);
  acc.x = fma(a.y, nxy, acc.x);
  acc.y = fma(a.x, x.y, acc.y);
  acc.y = fma(a.y, x.x, acc.y);
}

// 16-byte buffer load (non-temporal) of byte offset voff + IMM from the
// buffer rsrc: offsets past the buffer's size read zeros.
typedef int ivec4 __attribute__((ext_vector_type(4)));
template <int E>
__device__ __forceinline__ typename Elem<E>::T bload(__amdgpu_buffer_rsrc_t rs, uint32_t voff) {
  const ivec4 v = __builtin_bit_cast(ivec4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, 0, 2));
  if constexpr (E == 1) {
    const dvec2 d = __builtin_bit_cast(dvec2, v);
    return make_double2(d.x, d.y);
  } else {
    const fvec4 f = __builtin_bit_cast(fvec4, v);
    return make_float4(f.x, f.y, f.z, f.w);
  }
}

// Half-panel columns [cb, ce) of one leaf (column-major, leading dimension
// ld, nb bytes in all).  Lane (r, c) = (lane & 15, lane >> 4) reads rows
// 16E g + E r .. + E-1 (g < RG) of column c of a four-column step, so a load
// instruction reads 256 contiguous bytes of each of four columns and each
// tile is read once.  Loads go through a buffer descriptor of the panel:
// one offset register per step, the row groups as immediate offsets, and
// rows past the panel's end read zeros (rows past m of other columns are
// read but meet y_t = 0, and their u is never stored).  Wave w takes NC
// four-column steps at a time (columns j0 + 4 kWaves st + c) and issues
// all their loads before using them.  Per lane:
//   u[g] (the lane's rows, partial over its columns) += Z x_c
//   p    (column c, partial over the lane's rows)    += Z^T y_t
// p is summed over the sixteen row lanes of its column (DPP) and kept in
// LDS (vl[j - cb]); the caller writes the chunk's v values out in one
// coalesced pass, so the streaming loop issues no global stores.  Columns
// past ce re-read column ce - 1 with a zero input and keep no v.
template <int E, int RG, int NC>
__device__ __forceinline__ void half_tile(const void* __restrict__ P, uint32_t ld, uint32_t nb,
                                          int cb, int ce, int w, int lane, const double2* xs,
                                          const double2* ys, double2 (&u)[RG][E], double2* vl) {
  using T = typename Elem<E>::T;
  constexpr uint32_t kES = E == 1 ? 16 : 8;  // bytes per complex element
  const int r = lane & 15, c = lane >> 4;
  // the descriptor is wave-uniform (one leaf per piece); say so, so that it
  // lives in scalar registers
  const uint64_t pa = reinterpret_cast<uint64_t>(P);
  const uint32_t plo = __builtin_amdgcn_readfirstlane((uint32_t)pa);
  const uint32_t phi = __builtin_amdgcn_readfirstlane((uint32_t)(pa >> 32));
  void* pu = reinterpret_cast<void*>(((uint64_t)phi << 32) | plo);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      pu, 0, (int)__builtin_amdgcn_readfirstlane(nb), 0x00020000);
  const uint32_t lane_off = (uint32_t)(E * r) * kES;
  const uint32_t ldb = ld * kES;
  double2 yt[RG][E];
  double nyt[RG][E];
#pragma unroll
  for (int g = 0; g < RG; ++g)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      yt[g][e] = ys[16 * E * g + E * r + e];
      nyt[g][e] = -yt[g][e].y;
    }
  for (int j0 = cb + 4 * w; j0 < ce; j0 += 4 * kWaves * NC) {
    T a[NC][RG];
#pragma unroll
    for (int st = 0; st < NC; ++st) {
      const uint32_t vo = lane_off + (uint32_t)min(j0 + 4 * kWaves * st + c, ce - 1) * ldb;
#pragma unroll
      for (int g = 0; g < RG; ++g) a[st][g] = bload<E>(rs, vo + g * 16 * E * kES);
    }
#pragma unroll
    for (int st = 0; st < NC; ++st) {
      const int jj = j0 + 4 * kWaves * st + c;
      const bool ok = jj < ce;
      const double2 x = ok ? xs[jj - cb] : zero2();
      const double nx = -x.y;
      double2 pv = zero2();
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const double2 z = Elem<E>::get(a[st][g], e);
          cmac_n(u[g][e], z, x, nx);
          cmac_n(pv, z, yt[g][e], nyt[g][e]);
        }
      pv.x = sum16_lanes(pv.x);
      pv.y = sum16_lanes(pv.y);
      if (r == 0 && ok) vl[jj - cb] = pv;
    }
  }
}

// Far pairs [c0, c1) of leaf a (kind 3), pair c0 + k going to leaf
// vleaf[r0 + k]: wave w takes the pairs k = w, w + kWaves, ...  Pair p holds
// U' (rows of a, leading dimension lda) and W' (rows of its leaf s,
// leading dimension even(m_s)), r columns each, one after the other.  Each
// four-column step reads columns q of both factors with the half_tile lane
// layout and forms, per column,
//   sv = U'[:, q]^T y_a,  tv = W'[:, q]^T y_s   (sums over the 16 row lanes)
//   za += U'[:, q] tv,    zs += W'[:, q] sv,
// so za gathers S_as y_s = U' W'^T y_s and zs = W' U'^T y_a = S_sa y_a.
// Small tiles load two steps before using either.  zs is summed over the
// four column lanes and stored to the pair's partial rows when its pair is
// done; za stays in registers over the wave's pairs (summed by the caller).
// Columns past r re-read column r - 1 and are given sv = tv = 0; rows past
// a leaf meet y = 0 and their z is never stored.  y_a is read from LDS (ys)
// and y_s from the wave's own LDS rows yw (128 entries per pair, two pairs).
template <int E, int RG, bool MT>
__device__ __forceinline__ void far_pairs(const HalfArgs& A, const TermItem& it,
                                          const double2* xin, int lda, int w, int lane,
                                          const double2* ys, double2* yw, double2 (&za)[RG][E]) {
  using T = typename Elem<E>::T;
  constexpr uint32_t kES = E == 1 ? 16 : 8;  // bytes per complex element
  constexpr int NS = E * RG <= 4 ? 2 : 1;     // four-column steps in flight
  const TermArgs& Tm = A.t;
  const int r = lane & 15, c = lane >> 4;
  const uint32_t lane_off = (uint32_t)(E * r) * kES;
  const double2* ya = ys + E * r;  // y_a of the lane's rows (LDS): ya[16 E g + e]
  const int c0 = __builtin_amdgcn_readfirstlane(it.c0);
  const int np = __builtin_amdgcn_readfirstlane(it.c1) - c0;
  const int v0 = __builtin_amdgcn_readfirstlane(it.r0);
  static_assert(kMaxVLeaves <= 2 * kWaves, "a wave takes at most two pairs of a piece");
  static_assert(16 * E * RG <= 128, "the y_s rows of a wave's two pairs fit its 256 LDS entries");
  // the metadata of every pair of the piece at once (lane k: pair c0 + k),
  // then the y_s rows of the wave's (at most two) pairs, so that the
  // latencies of these loads overlap instead of adding up pair by pair
  int s_l = 0, rk_l = 0, slot_l = 0, ms_l = 0, off_l = 0;
  int64_t eoff_l = 0;
  if (lane < np) {
    s_l = A.vleaf[v0 + lane];
    rk_l = A.fp_rank[c0 + lane];
    slot_l = A.fp_slot[c0 + lane];
    eoff_l = A.fp_off[c0 + lane];
    ms_l = Tm.ps.leaf_m[s_l];
    off_l = Tm.leaf_off[s_l];
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int k = w + j * kWaves;
    if (k < np) {
      const int ms = __builtin_amdgcn_readlane(ms_l, k);
      const int offs = __builtin_amdgcn_readlane(off_l, k);
      for (int row = lane; row < 16 * E * RG; row += 64)
        yw[128 * j + row] = row < ms ? ld_y<MT>(xin + offs + row) : zero2();
    }
  }
  __builtin_amdgcn_wave_barrier();
  for (int k = w, j = 0; k < np; k += kWaves, ++j) {
    const int p = c0 + k;
    const int rk = __builtin_amdgcn_readlane(rk_l, k);
    const int ms = __builtin_amdgcn_readlane(ms_l, k);
    const int lds = ms + (ms & 1);
    const int slot = __builtin_amdgcn_readlane(slot_l, k);
    const uint32_t elo = __builtin_amdgcn_readlane((uint32_t)eoff_l, k);
    const uint32_t ehi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)eoff_l >> 32), k);
    const uint64_t eoff = ((uint64_t)ehi << 32) | elo;
    const uint64_t pa = reinterpret_cast<uint64_t>(A.fp) + eoff * kES;
    const uint32_t plo = __builtin_amdgcn_readfirstlane((uint32_t)pa);
    const uint32_t phi = __builtin_amdgcn_readfirstlane((uint32_t)(pa >> 32));
    void* pu = reinterpret_cast<void*>(((uint64_t)phi << 32) | plo);
    const uint32_t nbytes = (uint32_t)(lda + lds) * (uint32_t)rk * kES;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        pu, 0, (int)__builtin_amdgcn_readfirstlane(nbytes), 0x00020000);
    const uint32_t wb = (uint32_t)lda * (uint32_t)rk * kES;  // W' after U'
    double2 zs[RG][E];
#pragma unroll
    for (int g = 0; g < RG; ++g)
#pragma unroll
      for (int e = 0; e < E; ++e) zs[g][e] = zero2();
    const double2* yw_k = yw + 128 * j;
    const double2* yv = yw_k + E * r;  // y_s of the lane's rows: yv[16 E g + e]
    for (int q0 = 0; q0 < rk; q0 += 4 * NS) {
      T au[NS][RG], aw[NS][RG];
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        const uint32_t q = (uint32_t)min(q0 + 4 * st + c, rk - 1);
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          au[st][g] = bload<E>(rs, lane_off + q * (uint32_t)lda * kES + g * 16 * E * kES);
          aw[st][g] = bload<E>(rs, wb + lane_off + q * (uint32_t)lds * kES + g * 16 * E * kES);
        }
      }
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        double2 sv = zero2(), tv = zero2();
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
          for (int e = 0; e < E; ++e) {
            cmac(sv, Elem<E>::get(au[st][g], e), ya[16 * E * g + e]);
            cmac(tv, Elem<E>::get(aw[st][g], e), yv[16 * E * g + e]);
          }
        sv.x = sum16_lanes(sv.x);
        sv.y = sum16_lanes(sv.y);
        tv.x = sum16_lanes(tv.x);
        tv.y = sum16_lanes(tv.y);
        if (q0 + 4 * st + c >= rk) {
          sv = zero2();
          tv = zero2();
        }
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
          for (int e = 0; e < E; ++e) {
            cmac(za[g][e], Elem<E>::get(au[st][g], e), tv);
            cmac(zs[g][e], Elem<E>::get(aw[st][g], e), sv);
          }
      }
    }
#pragma unroll
    for (int g = 0; g < RG; ++g)
#pragma unroll
      for (int e = 0; e < E; ++e)
#pragma unroll
        for (int sh = 16; sh < 64; sh <<= 1) {
          zs[g][e].x += __shfl_xor(zs[g][e].x, sh);
          zs[g][e].y += __shfl_xor(zs[g][e].y, sh);
        }
    if (c == 0) {
      double2* zp = Tm.partial + A.frow + slot;
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int row = 16 * E * g + E * r + e;
          if (row < ms) store_agent(zp + row, zs[g][e]);
        }
    }
  }
}

// Epilogue of leaf a: z = the sum of its u partials and v slots (one list
// of partial rows), then y = alpha z + beta v and the stores of the TermArgs
// epilogue; the leaf's counter is cleared for the next launch.  P threads
// share a row (P = 256 / 128 or 256 / 64): thread (i, p) sums the list
// entries p, p + P, ... with all its loads in flight at once, and the P
// sums are added in a fixed order, so the result does not depend on timing.
template <bool MT>
__device__ void half_epilogue(const HalfArgs& A, const MultiArgs& M, int a, int term, int* s_off,
                              double2* s_z) {
  constexpr int kInFlight = 16;
  const int m = A.t.ps.leaf_m[a];
  const int P = m <= 64 ? 4 : 2;
  const int i = threadIdx.x % (kThreads / P), p = threadIdx.x / (kThreads / P);
  const int q0 = A.t.lptr[a], n = A.t.lptr[a + 1] - q0;
  double zr = 0.0, zi = 0.0;
  for (int c0 = 0; c0 < n; c0 += kThreads) {
    const int nc = min(kThreads, n - c0);
    __syncthreads();
    if ((int)threadIdx.x < nc) s_off[threadIdx.x] = A.t.lprow[q0 + c0 + threadIdx.x];
    __syncthreads();
    if (i < m) {
      const double* base = reinterpret_cast<const double*>(A.t.partial + i);
      for (int k0 = p; k0 < nc; k0 += P * kInFlight) {
        double vr[kInFlight], vi[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
          const int k = k0 + u * P;
          if (k < nc) {
            const double* q = base + 2 * (int64_t)s_off[k];
            vr[u] = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            vi[u] = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          } else {
            vr[u] = 0.0;
            vi[u] = 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
          zr += vr[u];
          zi += vi[u];
        }
      }
    }
  }
  if (i < m) s_z[p * 128 + i] = make_double2(zr, zi);
  __syncthreads();
  if ((int)threadIdx.x < m) {
    double2 z = s_z[threadIdx.x];
    for (int r = 1; r < P; ++r) {
      z.x += s_z[r * 128 + threadIdx.x].x;
      z.y += s_z[r * 128 + threadIdx.x].y;
    }
    if constexpr (MT) {
      // y_k = alpha z for the next term and x += y_k, read by other
      // workgroups of this launch: device-coherent stores and loads
      const int64_t q = A.t.leaf_off[a] + threadIdx.x;
      const double2 y = make_double2(A.t.alpha * z.x, A.t.alpha * z.y);
      store_agent(M.y[term & 1] + q, y);
      double2 x = load_agent(M.xacc + q);
      x.x += y.x;
      x.y += y.y;
      store_agent(M.xacc + q, x);
    } else {
      finish_entry(A.t, A.t.leaf_off[a], threadIdx.x, 0, z);
    }
  }
  if (threadIdx.x == 0)
    __hip_atomic_store(A.t.counters + a, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if constexpr (MT) {
    // every store of the epilogue (y, x, the counter) is complete before
    // the leaf is marked done with this term
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_store(M.done + a, term, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();  // s_z and s_off are free again
}

// Waits until leaf has finished term need (M.done[leaf] >= need).  The
// wait is bounded: past kSpinLimit polls, or once another wait has given
// up, it sets M.err and returns, so a launch always ends.
constexpr int kSpinLimit = 1 << 21;
__device__ void wait_done(const MultiArgs& M, int leaf, int need) {
  for (int spins = 0;
       __hip_atomic_load(M.done + leaf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need;
       ++spins) {
    if (spins >= kSpinLimit ||
        __hip_atomic_load(M.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
      __hip_atomic_store(M.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}


// Persistent workgroup over its run of pieces (see the file comment).
// Half-panel pieces use the row-group tiles of half_tile (RG groups of 16E
// rows); the far pieces use the lane-per-row GEMV of the term kernel (G
// groups of 64E rows).
//
// MT (multi-term): one launch runs the M.K terms of the scaled series.
// The queue holds the pieces of term 1, then those of term 2, ...; term k
// reads y_{k-1} from M.y[(k - 1) & 1] and the epilogue of each leaf writes
// y_k = alpha z to M.y[k & 1], adds it to M.xacc and then marks the leaf
// done with term k (M.done).  A piece of term k > 1 waits until its own
// leaf and the leaves of its columns or pairs are done with term k - 1.
// That orders every reuse of memory within the launch: (a) a piece writes
// partial rows only of those leaves, whose term k - 1 epilogues have read
// them; (b) every term k - 1 reader of y_{k-2} of a leaf L (the buffer L's
// term k epilogue overwrites) is L's own piece or writes v or pair rows of
// L, so it counts toward L's term k - 1 epilogue, which precedes L's term k
// pieces and so its term k epilogue; (c) L's epilogues, the only writers of
// its x rows, run in term order.  Data published by an epilogue (y, x, the
// leaf counter) is stored device-coherently and complete (s_waitcnt) before
// the mark, and the y of a later term is read device-coherently after the
// mark was seen.  Waits end: a piece waits only on pieces earlier in the
// queue, each taken by a running workgroup.  Only lists whose far blocks
// are all pairs (no kind 0 columns, no kind 1 rows) run this way.
template <int E, int G, int RG, int NC, bool MT>
__global__ __launch_bounds__(kThreads) void k_half(HalfArgs A, MultiArgs M) {
  constexpr int UNR = 8;
  constexpr int MR = 16 * E * RG;  // rows a half-panel piece covers
  static_assert(MR <= kHalfChunk / kWaves, "a wave's y_s rows of a far pair live in xs");
  const TermArgs& T = A.t;
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  // LDS of the wave reductions: the far GEMV (G x E rows per lane) and the
  // in-row stack product (kHalfInRowTile rows)
  __shared__ double2 red[(kWaves - 1) * (G * E > kHalfInRowTile / 64 ? G * E : kHalfInRowTile / 64) * 64];
  __shared__ double2 ured[kWaves][MR];
  __shared__ double2 ys[MR];
  __shared__ double2 tbuf[kHalfInRowTile];
  __shared__ double2 xs[kHalfChunk];
  __shared__ double2 vl[kHalfChunk];
  __shared__ int s_off[kThreads];
  __shared__ double2 s_z[4 * 128];
  __shared__ int s_last[kMaxVLeaves + 1];
  __shared__ int s_nlast, s_next, s_reset;
  __shared__ TermItem s_it;  // the piece about to start, and of its leaf:
  __shared__ int s_meta[4];  // rows, tree offset, first and end half-panel column
  __shared__ int64_t s_hpo;  // element offset of the half panel
  // Pieces come from a queue: a workgroup takes the next ticket once its
  // current piece's loads are done (the atomic completes with the piece's
  // stores), so faster workgroups take more pieces, no static split has to
  // predict how long each piece takes, and a workgroup holds one piece at
  // a time (no piece waits, unstarted, behind another).
  if (threadIdx.x == 0)
    s_next = __hip_atomic_fetch_add(A.queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int total = MT ? M.K * A.npieces : A.npieces;
  int p = s_next;
  // A piece's item and its leaf's metadata are loaded into LDS before the
  // piece starts: the next piece's item along with the current piece's
  // counter updates, the metadata along with its epilogues.
  auto item_word = [&](int q) -> int32_t {  // threads 0..7
    return reinterpret_cast<const int32_t*>(T.items + (MT ? q % A.npieces : q))[threadIdx.x];
  };
  auto meta_value = [&](int na) -> int64_t {  // threads 0..4
    switch (threadIdx.x) {
      case 0: return T.ps.leaf_m[na];
      case 1: return T.leaf_off[na];
      case 2: return A.hp_col[na];
      case 3: return A.hp_col[na + 1];
      default: return A.hp_off[na];
    }
  };
  auto put_meta = [&](int64_t v) {
    if (threadIdx.x < 4) s_meta[threadIdx.x] = (int)v;
    else s_hpo = v;
  };
  if (p < total && threadIdx.x < 8) reinterpret_cast<int32_t*>(&s_it)[threadIdx.x] = item_word(p);
  __syncthreads();
  if (p < total && threadIdx.x < 5) put_meta(meta_value(s_it.leaf));
  __syncthreads();
  while (p < total) {
    const int term = MT ? p / A.npieces + 1 : 1;
    const TermItem it = s_it;
    const double2* xin = MT ? M.y[(term - 1) & 1] : T.xin;
    const int a = it.leaf;
    const int m = s_meta[0];
    const int64_t ld = m + (m & 1);
    const int nc = it.c1 - it.c0;  // at most kHalfChunk for kinds 0 and 2
    if constexpr (MT) {
      if (term > 1) {
        const int nd = (it.kind >= 2 ? it.r1 - it.r0 : 0) + 1;
        if ((int)threadIdx.x < nd)
          wait_done(M, threadIdx.x == 0 ? a : A.vleaf[it.r0 + threadIdx.x - 1], term - 1);
        __syncthreads();
      }
    }
    if (it.kind == 2 || it.kind == 3) {
      const int64_t off = s_meta[1];
      for (int i = threadIdx.x; i < MR; i += kThreads) ys[i] = i < m ? ld_y<MT>(xin + off + i) : zero2();
      if (it.kind == 2) {
        const int32_t* __restrict__ hsrc = A.hsrc + s_meta[2];
        for (int k = threadIdx.x; k < nc; k += kThreads) xs[k] = ld_y<MT>(xin + hsrc[it.c0 + k]);
      }
      __syncthreads();
      double2 u[RG][E];
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e) u[g][e] = zero2();
      if (it.kind == 2) {
        const void* HP = Elem<E>::offset(A.hp, s_hpo);
        const uint32_t nbytes = (uint32_t)(ld * (s_meta[3] - s_meta[2]) * (E == 1 ? 16 : 8));
        half_tile<E, RG, NC>(HP, (uint32_t)ld, nbytes, it.c0, it.c1, w, lane, xs, ys, u, vl);
      } else {
        far_pairs<E, RG, MT>(A, it, xin, (int)ld, w, lane, ys, xs + w * (kHalfChunk / kWaves), u);
      }
      // u over the four column lanes of each row (lane bits 4, 5), then
      // over the waves in a fixed order
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
          for (int sh = 16; sh < 64; sh <<= 1) {
            u[g][e].x += __shfl_xor(u[g][e].x, sh);
            u[g][e].y += __shfl_xor(u[g][e].y, sh);
          }
      if ((lane >> 4) == 0) {
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
          for (int e = 0; e < E; ++e) ured[w][16 * E * g + E * lane + e] = u[g][e];
      }
      __syncthreads();
      for (int i = threadIdx.x; i < m; i += kThreads) {
        double2 z = ured[0][i];
#pragma unroll
        for (int v = 1; v < kWaves; ++v) {
          z.x += ured[v][i].x;
          z.y += ured[v][i].y;
        }
        store_agent(T.partial + it.prow + i, z);
      }
      if (it.kind == 2) {
        double2* vb = T.partial + A.vrow + A.hp_col[a] + it.c0;
        for (int k = threadIdx.x; k < nc; k += kThreads) store_agent(vb + k, vl[k]);
      }
    } else if constexpr (MT) {
      // a leaf with no work of its own publishes zeros
      for (int i = threadIdx.x; i < m; i += kThreads) store_agent(T.partial + it.prow + i, zero2());
    } else {
      // far pieces (kind 0, 1) and pieces of leaves with no work of their
      // own (which publish zeros): lane-per-row GEMV on the far panel
      double2 acc[G][E][1];
      zero_acc(acc);
      if (it.kind == 0) {
        const void* P = Elem<E>::offset(T.ps.data, T.ps.panel_off[a]);
        const int32_t* __restrict__ src = T.ps.src + T.ps.col_off[a];
        for (int k = threadIdx.x; k < nc; k += kThreads) xs[k] = T.xin[src[it.c0 + k]];
        __syncthreads();
        const double2* xq = xs - it.c0;
        auto X = [&](int c, int) -> double2 { return xq[c]; };
        tall_gemv<E, G, 1, UNR>(P, ld, m, 0, it.c0, it.c1, w, lane, X, acc);
      } else if (it.kind == 1) {
        constexpr int GW = kHalfInRowTile / (64 * E);  // stack rows per lane group
        const void* P = Elem<E>::offset(T.ps.data, T.ps.panel_off[a]);
        double2 tacc[GW][E][1];
        zero_acc(tacc);
        const int rb = T.ir.row0[a];
        inrow_t<E, GW, 1, 4>(Elem<E>::offset(T.ir.W, T.ir.off[a]), T.ir.ld[a], T.ir.ncol[a],
                             it.r0, it.r1, T.ir.soff + rb, T.ir.n + rb, T.xin, T.ldx, 0, 1, w,
                             lane, tacc);
        reduce_waves(tacc, w, lane, red);
        if (w == 0) {
#pragma unroll
          for (int g = 0; g < GW; ++g)
#pragma unroll
            for (int e = 0; e < E; ++e) tbuf[(g * 64 + lane) * E + e] = tacc[g][e][0];
        }
        __syncthreads();
        auto X = [&](int c, int) -> double2 { return tbuf[c - it.c0]; };
        tall_gemv<E, G, 1, UNR>(P, ld, m, 0, it.c0, it.c0 + (it.r1 - it.r0), w, lane, X, acc);
      }
      reduce_waves(acc, w, lane, red);
      if (w == 0) {
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const int i = (g * 64 + lane) * E + e;
            if (i < m) store_agent(T.partial + it.prow + i, acc[g][e][0]);
          }
      }
    }
    int ticket = 0;
    if (threadIdx.x == 0)
      ticket = __hip_atomic_fetch_add(A.queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // every store of the piece is complete before it is counted
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      s_nlast = 0;
      s_next = ticket;
    }
    __syncthreads();
    const int pn = s_next;
    const int32_t iw = pn < total && threadIdx.x < 8 ? item_word(pn) : 0;
    const int nv = it.kind >= 2 ? it.r1 - it.r0 : 0;
    if ((int)threadIdx.x <= nv) {
      const int leaf = threadIdx.x == 0 ? a : A.vleaf[it.r0 + threadIdx.x - 1];
      const int old = __hip_atomic_fetch_add(T.counters + leaf, 1, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
      if (old == A.lcnt[leaf] - 1) s_last[atomicAdd(&s_nlast, 1)] = leaf;
    }
    if (pn < total && threadIdx.x < 8) reinterpret_cast<int32_t*>(&s_it)[threadIdx.x] = iw;
    __syncthreads();
    const int64_t mv = pn < total && threadIdx.x < 5 ? meta_value(s_it.leaf) : 0;
    const int nlast = s_nlast;
    for (int k = 0; k < nlast; ++k) half_epilogue<MT>(A, M, s_last[k], term, s_off, s_z);
    if (pn < total && threadIdx.x < 5) put_meta(mv);
    __syncthreads();
    p = pn;
  }
  // the last workgroup out clears the queue (and the done marks) for the
  // next launch: every workgroup has taken its last ticket, and finished
  // its pieces and epilogues, before it counts itself out
  if (threadIdx.x == 0) {
    const int done = __hip_atomic_fetch_add(A.queue + 1, 1, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
    s_reset = done == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (s_reset) {
    if constexpr (MT)
      for (int i = threadIdx.x; i < M.nl; i += kThreads)
        __hip_atomic_store(M.done + i, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) {
      __hip_atomic_store(A.queue, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(A.queue + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <int E, int G, int RG, int NC, bool MT>
int occ_half() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_half<E, G, RG, NC, MT>, kThreads, 0) !=
      hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

// Variants by the largest leaf: G = row groups of 64E rows (far pieces),
// RG = row groups of 16E rows and NC = four-column steps in flight
// (half-panel tiles; RG * NC loads of 16 bytes per lane in flight).
#define HALF_VARIANTS(X)                                                       \
  X(true, 64, 2, 1, 2, 8) X(true, 96, 2, 1, 3, 5) X(true, 128, 2, 1, 4, 3)      \
  X(false, 64, 1, 1, 4, 6) X(false, 96, 1, 2, 6, 4) X(false, 128, 1, 2, 8, 2)

}  // namespace

hipError_t launch_half(bool f32, int max_m, const HalfArgs& a, int nwg, hipStream_t st) {
  if (nwg <= 0) return hipSuccess;
  if (max_m > kHalfMaxLeaf) return hipErrorInvalidValue;
  const MultiArgs none{};
#define X(F, MM, E, G, RG, NC)                                                                \
  if (f32 == F && max_m <= MM) {                                                             \
    hipLaunchKernelGGL((k_half<E, G, RG, NC, false>), dim3(nwg), dim3(kThreads), 0, st, a,   \
                       none);                                                                \
    return hipGetLastError();                                                                \
  }
  HALF_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_half_multi(bool f32, int max_m, const HalfArgs& a, const MultiArgs& m, int nwg,
                             hipStream_t st) {
  if (nwg <= 0 || m.K <= 0) return hipSuccess;
  if (max_m > kHalfMaxLeaf || (int64_t)m.K * a.npieces >= ((int64_t)1 << 31))
    return hipErrorInvalidValue;
#define X(F, MM, E, G, RG, NC)                                                                \
  if (f32 == F && max_m <= MM) {                                                             \
    hipLaunchKernelGGL((k_half<E, G, RG, NC, true>), dim3(nwg), dim3(kThreads), 0, st, a, m); \
    return hipGetLastError();                                                                \
  }
  HALF_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

int half_occupancy(bool f32, int max_m, bool multi) {
#define X(F, MM, E, G, RG, NC)                                                         \
  if (f32 == F && max_m <= MM)                                                        \
    return multi ? occ_half<E, G, RG, NC, true>() : occ_half<E, G, RG, NC, false>();
  HALF_VARIANTS(X)
#undef X
  return 1;
}

}  // namespace hm
