// Streaming GEMV building blocks shared by the term kernels (included inside
// an anonymous namespace of each kernel source; needs hip_runtime.h and
// dev.h first).
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ double2 zero2() { return make_double2(0.0, 0.0); }

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

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

// E = complex rows per 16-byte lane load: 1 for FP64 (double2), 2 for FP32
// (float4 = two consecutive complex64 of one column).  Block data is read
// once per term and does not fit in the caches, so it is loaded with the
// non-temporal hint (streaming loads measured ~13% faster on gfx950).
template <int E>
struct Elem;
template <>
struct Elem<1> {
  using T = double2;
  __device__ static __forceinline__ T zero() { return make_double2(0.0, 0.0); }
  __device__ static __forceinline__ T load(const void* base, uint32_t idx) {
    const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(base) + idx);
    return make_double2(v.x, v.y);
  }
  __device__ static __forceinline__ double2 get(const T& a, int) { return a; }
  __device__ static __forceinline__ const void* offset(const void* base, int64_t n) {
    return reinterpret_cast<const double2*>(base) + n;
  }
};
template <>
struct Elem<2> {
  using T = float4;
  __device__ static __forceinline__ T zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  __device__ static __forceinline__ T load(const void* base, uint32_t idx) {  // idx even
    const fvec4 v = __builtin_nontemporal_load(reinterpret_cast<const fvec4*>(base) + (idx >> 1));
    return make_float4(v.x, v.y, v.z, v.w);
  }
  __device__ static __forceinline__ double2 get(const T& a, int e) {
    return e == 0 ? make_double2((double)a.x, (double)a.y) : make_double2((double)a.z, (double)a.w);
  }
  __device__ static __forceinline__ const void* offset(const void* base, int64_t n) {
    return reinterpret_cast<const float2*>(base) + n;
  }
};

// Lane l of wave w accumulates rows row0 + (g*64 + l)*E + e (g < G, e < E)
// of the column-major matrix P (leading dimension ld >= rows) against the
// input X(c, r), over columns c0 + w + kWaves*k < c1.  Loads are issued
// without branches: the row index is clamped into the column (lanes past
// `rows` re-read a valid element whose sum is never stored) and columns past
// c1 re-read column c1 - 1 with a zero input.
template <int E, int G, int NR, int UNR, typename XF>
__device__ __forceinline__ void tall_gemv(const void* __restrict__ P, int64_t ld, int rows,
                                          int row0, int c0, int c1, int w, int lane, const XF& X,
                                          double2 (&acc)[G][E][NR]) {
  using T = typename Elem<E>::T;
  (void)rows;
  // element offsets within one panel fit in 32 bits (checked at build time)
  uint32_t ri[G];
#pragma unroll
  for (int g = 0; g < G; ++g) ri[g] = (uint32_t)min<int64_t>(row0 + (g * 64 + lane) * E, ld - E);
  const uint32_t ld32 = (uint32_t)ld;
  for (int c = c0 + w; c < c1; c += kWaves * UNR) {
    T a[UNR][G];
    double2 xv[UNR][NR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int cc = c + kWaves * u;
      const bool ok = cc < c1;
      const uint32_t col = (uint32_t)(ok ? cc : c1 - 1) * ld32;
#pragma unroll
      for (int g = 0; g < G; ++g) a[u][g] = Elem<E>::load(P, ri[g] + col);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double2 v = X(ok ? cc : c1 - 1, r);
        xv[u][r] = ok ? v : zero2();
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
          for (int r = 0; r < NR; ++r) cmac(acc[g][e][r], Elem<E>::get(a[u][g], e), xv[u][r]);
  }
}

// Sum acc over the waves of the workgroup into wave 0 (through LDS).
template <int E, int G, int NR>
__device__ __forceinline__ void reduce_waves(double2 (&acc)[G][E][NR], int w, int lane,
                                             double2* red) {
  constexpr int S = G * E * NR;
  if (w > 0) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int e = 0; e < E; ++e)
#pragma unroll
        for (int r = 0; r < NR; ++r)
          red[((w - 1) * S + (g * E + e) * NR + r) * 64 + lane] = acc[g][e][r];
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int v = 0; v < kWaves - 1; ++v)
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const double2 o = red[(v * S + (g * E + e) * NR + r) * 64 + lane];
            acc[g][e][r].x += o.x;
            acc[g][e][r].y += o.y;
          }
  }
}

template <int E, int G, int NR>
__device__ __forceinline__ void zero_acc(double2 (&acc)[G][E][NR]) {
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int e = 0; e < E; ++e)
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[g][e][r] = zero2();
}

// ---------------------------------------------------------------- term
// In-row low-rank rows: lane l of wave w owns stack rows r0 + (g*64 + l)*E + e
// (each with its own source range) and accumulates W[row, j] y[soff + j] over
// the columns j = w + kWaves*k < ncol.
template <int E, int GW, int NR, int UNR>
__device__ __forceinline__ void inrow_t(const void* __restrict__ Wa, int64_t wld, int ncol,
                                        int r0, int r1, const int32_t* __restrict__ soff_a,
                                        const int32_t* __restrict__ n_a,
                                        const double2* __restrict__ xin, int64_t ldx, int rhs0,
                                        int nrhs, int w, int lane, double2 (&acc)[GW][E][NR]) {
  using T = typename Elem<E>::T;
  int so[GW][E], nn[GW][E];
  uint32_t ri[GW];
#pragma unroll
  for (int g = 0; g < GW; ++g) {
    ri[g] = (uint32_t)min<int64_t>(r0 + (g * 64 + lane) * E, wld - E);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int row = r0 + (g * 64 + lane) * E + e;
      so[g][e] = row < r1 ? soff_a[row] : 0;
      nn[g][e] = row < r1 ? n_a[row] : 0;
    }
  }
  for (int c = w; c < ncol; c += kWaves * UNR) {
    T wv[UNR][GW];
    double2 yv[UNR][GW][E][NR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int cc = c + kWaves * u;
      const uint32_t col = (uint32_t)(cc < ncol ? cc : ncol - 1) * (uint32_t)wld;
#pragma unroll
      for (int g = 0; g < GW; ++g) {
        wv[u][g] = Elem<E>::load(Wa, ri[g] + col);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const bool ok = cc < nn[g][e];
          const int64_t yi = so[g][e] + (ok ? cc : 0);
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const int rr = rhs0 + r < nrhs ? rhs0 + r : rhs0;
            const double2 v = xin[yi + (int64_t)rr * ldx];
            yv[u][g][e][r] = (ok && rhs0 + r < nrhs) ? v : zero2();
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int g = 0; g < GW; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
          for (int r = 0; r < NR; ++r) cmac(acc[g][e][r], Elem<E>::get(wv[u][g], e), yv[u][g][e][r]);
  }
}

