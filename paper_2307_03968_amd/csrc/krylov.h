// Declarations of the Krylov kernels of libhmps (device_krylov.hip): the
// vector work of restarted GMRES on the H-matrix, one Krylov space per
// right-hand side.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

constexpr int kMaxKrylov = 64;  // basis vectors per cycle (restart length), at most
// Per right-hand side c (arrays indexed by c first):
struct KrylovState {
  double2* R;      // m columns of m + 1 entries: the rotated Hessenberg matrix
  double* cs;      // m rotation cosines
  double2* sn;     // m rotation sines
  double2* g;      // m + 1: the rotated ||r|| e_1
  int32_t* act;    // 1 while the column iterates
  int32_t* kc;     // steps taken in this cycle
  double* resid;   // residual estimate |g_kc| / ||b||
  double* bnorm;   // ||b||
  double* inv;     // scale of the next basis vector (0 when inactive)
  int m;           // restart length
};
// h (ldo per column) = V_i^H w for i < nvec (conjugated dot products, fixed
// order); partial holds kdots_partials(n, nvec, nrhs) values
hipError_t launch_kdots(const double2* V, int64_t vs, int64_t ld, const double2* w, int64_t n,
                        int nvec, int nrhs, double2* partial, double2* out, int ldo,
                        hipStream_t st);
int64_t kdots_partials(int64_t n, int nvec, int nrhs);
// y[:, c] += alpha sum_{i < nvec} V_i[:, c] coef[c ldc + i]
hipError_t launch_kupdate(double alpha, const double2* V, int64_t vs, int64_t ld,
                          const double2* coef, int ldc, int nvec, double2* y, int64_t n, int nrhs,
                          hipStream_t st);
// v[:, c] *= s[c]
hipError_t launch_kscale(double2* v, int64_t ld, const double* s, int64_t n, int nrhs,
                         hipStream_t st);
hipError_t launch_kstart(const KrylovState& S, const double2* rn2, const double2* bn2, double tol,
                         int nrhs, hipStream_t st);
hipError_t launch_kstep(const KrylovState& S, int j, const double2* h1, const double2* h2, int ldh,
                        const double2* hn2, double tol, int nrhs, hipStream_t st);
hipError_t launch_ksolve(const KrylovState& S, double2* y, int nrhs, hipStream_t st);

}  // namespace hm
