// HIP kernels of libhmps for gfx950 (CDNA4, wave64).
//
// Hot loop of the power series (Sec. IV, eq. 12-13 and 20-22): one launch
// of k_term per term.  Its workgroups cover a leaf's series panel
// D_a^{-1} [near | far] in column ranges, and the leaf's in-row low-rank
// blocks (t = W y in LDS, then D_a^{-1} U t); each writes partial sums, and
// the last workgroup of the leaf to finish (a device-scope counter) reduces
// them in a fixed order into y_a = -z_a and updates x_a.  Far blocks whose
// row cluster spans several leaves need t = W y first (k_stageA), one
// launch before k_term, only when levels above the leaf level are used.
// One-RHS products are HBM-bound GEMVs (0.5 flop/B in FP64, 1 in FP32), so
// they run on the vector ALUs: each lane owns one row (FP64) or two rows
// (FP32) of a column-major panel and every load is 16 bytes, so a wave
// reads 1 KiB of contiguous panel per instruction; UNR columns are loaded
// before they are used so that enough bytes are in flight per CU.
#include <hip/hip_runtime.h>

#include "dev.h"

namespace hm {

namespace {

#include "gemv_inl.h"

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

template <int E, int G, int NR>
constexpr int term_red_slots() {
  return G * E * NR;  // >= the in-row tile's 1 * E * NR
}

// Epilogue of leaf a for the RHS tile [rhs0, rhs0 + NR): z = sum of the
// leaf's partial sums in a fixed order, y = alpha z + beta v, y and x stores.
template <int NR>
__device__ void term_epilogue(const TermArgs& A, int a, int rhs0, int nrhs, int* s_prow) {
  constexpr int KE = (256 * NR + kThreads - 1) / kThreads;
  const int m = A.ps.leaf_m[a];
  const int64_t off = A.leaf_off[a];
  const int q0a = A.lptr[a], q1a = A.lptr[a + 1];
  double2 zacc[KE];
#pragma unroll
  for (int k = 0; k < KE; ++k) zacc[k] = zero2();
  for (int q0 = q0a; q0 < q1a; q0 += kThreads) {
    const int nq = min(kThreads, q1a - q0);
    __syncthreads();
    if ((int)threadIdx.x < nq) s_prow[threadIdx.x] = A.lprow[q0 + threadIdx.x];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KE; ++k) {
      const int idx = threadIdx.x + k * kThreads;
      if (idx >= m * NR) break;
      const int i = idx % m;
      const int c = rhs0 + idx / m;
      if (c >= nrhs) continue;
      const double* pc = reinterpret_cast<const double*>(A.partial + i + (int64_t)c * A.ldp);
      // fixed order, so results do not depend on timing; loads issued in
      // batches of 8 so that they are in flight together
      for (int p = 0; p < nq; p += 8) {
        double vr[8], vi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (p + u < nq) {
            const double* q = pc + 2 * (int64_t)s_prow[p + u];
            vr[u] = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            vi[u] = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          } else {
            vr[u] = 0.0;
            vi[u] = 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          zacc[k].x += vr[u];
          zacc[k].y += vi[u];
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int idx = threadIdx.x + k * kThreads;
    if (idx >= m * NR) break;
    const int i = idx % m;
    const int c = rhs0 + idx / m;
    if (c >= nrhs) continue;
    finish_entry(A, off, i, c, zacc[k]);
  }
}

// Persistent workgroup: processes its run of pieces; after each piece it
// publishes the partial sums and counts the piece for its leaf; the
// workgroup that completes a leaf runs the leaf's epilogue.
template <int E, int G, int NR, int UNR>
__global__ __launch_bounds__(kThreads) void k_term(TermArgs A, int nrhs) {
  constexpr int GW = 1;  // kInRowTile rows: one row per lane (E = 2: half the lanes)
  const int rhs0 = blockIdx.y * NR;
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  __shared__ double2 red[(kWaves - 1) * term_red_slots<E, G, NR>() * 64];
  constexpr int kXChunk = 1024 / NR;
  __shared__ double2 tbuf[NR][kInRowTile];
  __shared__ double2 xs[NR][kXChunk];
  __shared__ int s_prow[kThreads];
  __shared__ int s_last;
  const int pe = A.wptr[blockIdx.x + 1];
  for (int p = A.wptr[blockIdx.x]; p < pe; ++p) {
    const TermItem it = A.items[p];
    const int a = it.leaf;
    const int m = A.ps.leaf_m[a];
    const int64_t ld = m + (m & 1);
    const void* P = Elem<E>::offset(A.ps.data, A.ps.panel_off[a]);
    const int32_t* __restrict__ src = A.ps.src + A.ps.col_off[a];
    double2 acc[G][E][NR];
    zero_acc(acc);
    if (it.kind == 0) {
      // the piece's input values go to LDS first (chunks of kXChunk columns),
      // so the streaming loop reads them as LDS broadcasts
      for (int cb = it.c0; cb < it.c1; cb += kXChunk) {
        const int nc = min(kXChunk, it.c1 - cb);
        __syncthreads();
        for (int t = threadIdx.x; t < nc * NR; t += kThreads) {
          const int k = t % nc;
          const int r = t / nc;
          int64_t sidx = src[cb + k];
          if (A.in_perm) sidx = A.in_perm[sidx];
          xs[r][k] = (rhs0 + r < nrhs) ? A.xin[sidx + (int64_t)(rhs0 + r) * A.ldx] : zero2();
        }
        __syncthreads();
        auto X = [&](int c, int r) -> double2 { return xs[r][c - cb]; };
        tall_gemv<E, G, NR, UNR>(P, ld, m, 0, cb, cb + nc, w, lane, X, acc);
      }
    } else {
      double2 tacc[GW][E][NR];
      zero_acc(tacc);
      const int rb = A.ir.row0[a];
      inrow_t<E, GW, NR, (UNR > 4 ? 4 : UNR)>(Elem<E>::offset(A.ir.W, A.ir.off[a]), A.ir.ld[a], A.ir.ncol[a],
                            it.r0, it.r1, A.ir.soff + rb, A.ir.n + rb, A.xin, A.ldx, rhs0, nrhs,
                            w, lane, tacc);
      reduce_waves(tacc, w, lane, red);
      if (w == 0) {
#pragma unroll
        for (int g = 0; g < GW; ++g)
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const int k = (g * 64 + lane) * E + e;
#pragma unroll
            for (int r = 0; r < NR; ++r)
              if (k < kInRowTile) tbuf[r][k] = tacc[g][e][r];
          }
      }
      __syncthreads();
      auto X = [&](int c, int r) -> double2 { return tbuf[r][c - it.c0]; };
      tall_gemv<E, G, NR, UNR>(P, ld, m, 0, it.c0, it.c0 + (it.r1 - it.r0), w, lane, X, acc);
    }
    reduce_waves(acc, w, lane, red);
    // Partial sums are published with device-coherent (agent-scope) stores
    // and read back with device-coherent loads, so no writeback/invalidate
    // of the whole L2 is needed; the stores are complete (s_waitcnt) before
    // the workgroup's barrier and its counter increment.
    if (w == 0) {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int i = (g * 64 + lane) * E + e;
#pragma unroll
          for (int r = 0; r < NR; ++r)
            if (i < m && rhs0 + r < nrhs) {
              double* q = reinterpret_cast<double*>(A.partial + it.prow + i +
                                                    (int64_t)(rhs0 + r) * A.ldp);
              __hip_atomic_store(q, acc[g][e][r].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              __hip_atomic_store(q + 1, acc[g][e][r].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    if (A.lptr[a + 1] - A.lptr[a] == 1) {
      // the leaf's only piece: its epilogue needs no counter
      __syncthreads();
      term_epilogue<NR>(A, a, rhs0, nrhs, s_prow);
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
      term_epilogue<NR>(A, a, rhs0, nrhs, s_prow);
      if (threadIdx.x == 0) __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- stage A
// One workgroup = one row tile of a source group: t rows = W_g y_s.
template <int E, int G, int NR, int UNR>
__global__ __launch_bounds__(kThreads) void k_stageA(const void* __restrict__ W,
                                                     const Group* __restrict__ groups,
                                                     const GroupItem* __restrict__ items,
                                                     double2* __restrict__ xin, int64_t ldx,
                                                     int64_t N, int nrhs) {
  const GroupItem it = items[blockIdx.x];
  const Group g = groups[it.group];
  const void* Wg = Elem<E>::offset(W, g.w_off);
  const int rhs0 = blockIdx.y * NR;
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  auto X = [&](int c, int r) -> double2 {
    return (rhs0 + r < nrhs) ? xin[g.s_off + c + (int64_t)(rhs0 + r) * ldx] : zero2();
  };
  double2 acc[G][E][NR];
  zero_acc(acc);
  tall_gemv<E, G, NR, UNR>(Wg, g.ld, it.rows, it.row0, 0, g.n, w, lane, X, acc);
  __shared__ double2 red[(kWaves - 1) * G * E * NR * 64];
  reduce_waves(acc, w, lane, red);
  if (w == 0) {
#pragma unroll
    for (int gg = 0; gg < G; ++gg)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int row = it.row0 + (gg * 64 + lane) * E + e;
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (row < it.rows && rhs0 + r < nrhs)
            xin[N + g.t0 + row + (int64_t)(rhs0 + r) * ldx] = acc[gg][e][r];
      }
  }
}

// ---------------------------------------------------------------- leaf LU
// Right-looking LU with partial pivoting of one leaf self-block per
// workgroup, in place (column-major, ld = m).  Build-time only.
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

// D^{-1} from the LU factors: column j solves L U x = P e_j.  One thread
// per column works on its own column of the output (ld = m rounded up to
// even; the pad row is set to zero).
__global__ __launch_bounds__(kThreads) void k_getri(const double2* __restrict__ LU,
                                                    const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ mm,
                                                    const int32_t* __restrict__ piv,
                                                    const int64_t* __restrict__ poff,
                                                    double2* __restrict__ Ainv,
                                                    const int64_t* __restrict__ ioff) {
  const int b = blockIdx.x;
  const int m = mm[b];
  const int ld = m + (m & 1);
  const double2* a = LU + off[b];
  const int32_t* pv = piv + poff[b];
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    double2* x = Ainv + ioff[b] + (int64_t)j * ld;
    for (int i = 0; i < ld; ++i) x[i] = zero2();
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

// Series panel tile: 32 columns c0.. of leaf a, M[:, c] = Dinv_a P_a[:, m_a + c].
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
  constexpr int TC = kPremulCols / kWaves;  // columns per wave
  const int a = tiles[2 * blockIdx.x];
  const int c0 = tiles[2 * blockIdx.x + 1];
  const int m = leaf_m[a];
  const int64_t ld = m + (m & 1);
  const int nc = ncols_m[a];
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  const double2* Di = Dinv + dinv_off[a];
  const double2* Pa = P + p_off[a] + ld * m;  // skip the D_a columns
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
      d[q] = (i < m) ? Di[i + (int64_t)l * ld] : zero2();
    }
#pragma unroll
    for (int u = 0; u < TC; ++u) {
      const int c = c0 + w + kWaves * u;
      const double2 pv = (c < nc) ? Pa[l + (int64_t)c * ld] : zero2();
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
      if (i < m) Ma[i + (int64_t)c * ld] = acc[q][u];
    }
  }
}

__global__ void k_cast(const double2* __restrict__ in, float2* __restrict__ out, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    out[q] = make_float2((float)in[q].x, (float)in[q].y);
}

// ---------------------------------------------------------------- norms
// Squared 2-norms per (segment, right-hand side): a segment is one instance
// of a batched handle (the whole vector otherwise).  Item q covers rows
// [items[q].r0, items[q].r1) of segment items[q].seg; a workgroup reduces
// one item of one column, then the items of a segment are summed in order
// (the result does not depend on timing).
__global__ __launch_bounds__(kThreads) void k_norm2_items(const double2* __restrict__ v,
                                                          int64_t ld,
                                                          const NormItem* __restrict__ items,
                                                          double* __restrict__ scratch) {
  const int c = blockIdx.y;
  const NormItem it = items[blockIdx.x];
  double s = 0.0;
  for (int64_t q = it.r0 + threadIdx.x; q < it.r1; q += kThreads) {
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

__global__ void k_norm2_segments(const double* __restrict__ scratch, int nitems,
                                 const int32_t* __restrict__ seg_ptr, int nseg, int nrhs,
                                 double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nseg * nrhs) return;
  const int c = t / nseg, g = t % nseg;
  double s = 0.0;
  for (int i = seg_ptr[g]; i < seg_ptr[g + 1]; ++i) s += scratch[(int64_t)c * nitems + i];
  out[t] = s;
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

// NR (right-hand sides per workgroup) for nrhs; grid.y = ceil(nrhs / NR)
inline int pick_nr(int nrhs) { return nrhs == 1 ? 1 : (nrhs == 2 ? 2 : 4); }

// Block-diagonal product for one right-hand side (D^{-1}, C^{-1} or C^{-T}
// blocks): one workgroup per leaf a, z = P_a x_a with P_a the leaf's m x m
// block (column-major, leading dimension even m) and x_a gathered through
// the panel's column sources; the two halves of the workgroup take
// alternate columns (8 loads in flight per thread), their sums are added in
// a fixed order, and the epilogue stores of the term kernel follow.
__global__ __launch_bounds__(kThreads) void k_block_diag(TermArgs A) {
  constexpr int kRows = kBlockDiagMaxLeaf;  // rows per half: the largest leaf served
  static_assert(2 * kRows == kThreads, "two halves of one workgroup");
  constexpr int UNR = 8;
  __shared__ double2 xs[kRows];
  __shared__ double2 zs[2][kRows];
  const int a = blockIdx.x;
  const int m = A.ps.leaf_m[a];
  const int64_t ld = m + (m & 1);
  const double2* __restrict__ P = reinterpret_cast<const double2*>(A.ps.data) + A.ps.panel_off[a];
  const int32_t* __restrict__ src = A.ps.src + A.ps.col_off[a];
  for (int j = threadIdx.x; j < m; j += kThreads) {
    int64_t sidx = src[j];
    if (A.in_perm) sidx = A.in_perm[sidx];
    xs[j] = A.xin[sidx];
  }
  __syncthreads();
  const int i = threadIdx.x % kRows, h = threadIdx.x / kRows;
  double2 z = zero2();
  if (i < m) {
    int j = h;
    for (; j + 2 * (UNR - 1) < m; j += 2 * UNR) {
      double2 v[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const dvec2 q = __builtin_nontemporal_load(
            reinterpret_cast<const dvec2*>(P + i + (int64_t)(j + 2 * u) * ld));
        v[u] = make_double2(q.x, q.y);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) cmac(z, v[u], xs[j + 2 * u]);
    }
    for (; j < m; j += 2) {
      const dvec2 q = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(P + i + (int64_t)j * ld));
      cmac(z, make_double2(q.x, q.y), xs[j]);
    }
  }
  zs[h][i] = z;
  __syncthreads();
  if ((int)threadIdx.x < m) {
    const double2 z0 = zs[0][threadIdx.x], z1 = zs[1][threadIdx.x];
    finish_entry(A, A.leaf_off[a], threadIdx.x, 0, make_double2(z0.x + z1.x, z0.y + z1.y));
  }
}

}  // namespace

// ============================================================== launchers
hipError_t launch_block_diag(const TermArgs& a, int nl, int max_m, hipStream_t st) {
  if (nl <= 0) return hipSuccess;
  if (max_m > kBlockDiagMaxLeaf) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_block_diag, dim3(nl), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

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

int term_rhs_tile(int nrhs) { return pick_nr(nrhs); }

template <int E, int G>
static hipError_t term_eg(const TermArgs& a, int nwg, int nrhs, hipStream_t st) {
  const int nr = pick_nr(nrhs);
  const dim3 grid(nwg, (nrhs + nr - 1) / nr);
  if (nr == 1)
    hipLaunchKernelGGL((k_term<E, G, 1, 8>), grid, dim3(kThreads), 0, st, a, nrhs);
  else if (nr == 2)
    hipLaunchKernelGGL((k_term<E, G, 2, 4>), grid, dim3(kThreads), 0, st, a, nrhs);
  else
    hipLaunchKernelGGL((k_term<E, G, 4, 2>), grid, dim3(kThreads), 0, st, a, nrhs);
  return hipGetLastError();
}

hipError_t launch_term(bool f32, int max_m, const TermArgs& a, int nwg, int nrhs,
                       hipStream_t st) {
  if (nwg <= 0 || nrhs <= 0) return hipSuccess;
  if (max_m > 256) return hipErrorInvalidValue;
  if (f32) {
    if (max_m <= 128) return term_eg<2, 1>(a, nwg, nrhs, st);
    return term_eg<2, 2>(a, nwg, nrhs, st);
  }
  switch ((max_m + 63) / 64) {
    case 1: return term_eg<1, 1>(a, nwg, nrhs, st);
    case 2: return term_eg<1, 2>(a, nwg, nrhs, st);
    case 3: return term_eg<1, 3>(a, nwg, nrhs, st);
    default: return term_eg<1, 4>(a, nwg, nrhs, st);
  }
}

template <int E, int G>
static int occ_eg() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_term<E, G, 1, 8>, kThreads, 0) !=
      hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

int term_occupancy(bool f32, int max_m) {
  if (f32) return max_m <= 128 ? occ_eg<2, 1>() : occ_eg<2, 2>();
  switch ((max_m + 63) / 64) {
    case 1: return occ_eg<1, 1>();
    case 2: return occ_eg<1, 2>();
    case 3: return occ_eg<1, 3>();
    default: return occ_eg<1, 4>();
  }
}

// group tiles are kGroupTile = 128 rows: G = 2 for FP64, 1 for FP32
template <int E>
static hipError_t stageA_e(const void* W, const Group* groups, const GroupItem* items, int nitems,
                           double2* xin, int64_t ldx, int64_t N, int nrhs, hipStream_t st) {
  constexpr int G = kGroupTile / (64 * E);
  const int nr = pick_nr(nrhs);
  const dim3 grid(nitems, (nrhs + nr - 1) / nr);
  if (nr == 1)
    hipLaunchKernelGGL((k_stageA<E, G, 1, 4>), grid, dim3(kThreads), 0, st, W, groups, items,
                       xin, ldx, N, nrhs);
  else if (nr == 2)
    hipLaunchKernelGGL((k_stageA<E, G, 2, 2>), grid, dim3(kThreads), 0, st, W, groups, items,
                       xin, ldx, N, nrhs);
  else
    hipLaunchKernelGGL((k_stageA<E, G, 4, 1>), grid, dim3(kThreads), 0, st, W, groups, items,
                       xin, ldx, N, nrhs);
  return hipGetLastError();
}

hipError_t launch_stageA(bool f32, const void* W, const Group* groups, const GroupItem* items,
                         int nitems, double2* xin, int64_t ldx, int64_t N, int nrhs,
                         hipStream_t st) {
  if (nitems <= 0 || nrhs <= 0) return hipSuccess;
  return f32 ? stageA_e<2>(W, groups, items, nitems, xin, ldx, N, nrhs, st)
             : stageA_e<1>(W, groups, items, nitems, xin, ldx, N, nrhs, st);
}

hipError_t launch_getrf(double2* A, const int64_t* off, const int32_t* m, int32_t* piv,
                        const int64_t* piv_off, int nblk, int* info, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_getrf, dim3(nblk), dim3(kThreads), 0, st, A, off, m, piv, piv_off, info);
  return hipGetLastError();
}

hipError_t launch_getri(const double2* LU, const int64_t* off, const int32_t* m,
                        const int32_t* piv, const int64_t* piv_off, double2* Ainv,
                        const int64_t* dinv_off, int nblk, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_getri, dim3(nblk), dim3(kThreads), 0, st, LU, off, m, piv, piv_off, Ainv,
                     dinv_off);
  return hipGetLastError();
}

hipError_t launch_premul(const double2* Dinv, const int64_t* dinv_off, const double2* P,
                         const int64_t* p_off, const int32_t* leaf_m, const int32_t* ncols_m,
                         double2* M, const int64_t* m_off, const int32_t* tiles, int ntiles,
                         int max_m, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
#define HM_PREMUL_CASE(R)                                                                      \
  case R:                                                                                     \
    hipLaunchKernelGGL(k_premul<R>, dim3(ntiles), dim3(kThreads), 0, st, Dinv, dinv_off, P,   \
                       p_off, leaf_m, ncols_m, M, m_off, tiles);                              \
    break;
  switch ((max_m + 63) / 64) {
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

hipError_t launch_norm2(const double2* v, int64_t ld, const NormItem* items, int nitems,
                        const int32_t* seg_ptr, int nseg, int nrhs, double* scratch, double* out,
                        hipStream_t st) {
  if (nrhs <= 0 || nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_norm2_items, dim3(nitems, nrhs), dim3(kThreads), 0, st, v, ld, items,
                     scratch);
  hipLaunchKernelGGL(k_norm2_segments, dim3(blocks_for((int64_t)nseg * nrhs, 64)), dim3(64), 0, st,
                     scratch, nitems, seg_ptr, nseg, nrhs, out);
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
