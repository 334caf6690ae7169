// Far-block compression (Sec. III): adaptive cross approximation with
// partial pivoting, then recompression by QR of both factors and an SVD of
// the small core.  Host code.
//
// Rules (shared with the independent FP64 checker so both produce the same
// approximant up to rounding):
//   ACA on A (m x n), tolerance eps, rank cap r_max:
//     start at row 0; residual row = A[i,:] - sum_k u_k[i] v_k;
//     if max|row| <= 1e-300 mark it used, take the next unused row in index
//     order (stop when none is left);
//     pivot j = first index of max|row|; v = row / row[j];
//     u = A[:,j] - sum_k v_k[j] u_k;
//     ||S||_F^2 of S = sum_k u_k v_k^T updated incrementally;
//     stop after the step where ||u|| ||v|| <= eps ||S||_F or at r_max;
//     next row = first index of max|u| over unused rows.
//   Recompression: U = Qu Ru, V = Qv Rv (Householder), Ru Rv^T = Phi S Psi^H
//   (one-sided Jacobi), keep the smallest r >= 1 whose discarded singular
//   values have 2-norm <= eps times the 2-norm of all of them;
//   A ~ (Qu Phi_r S_r) (Qv conj(Psi_r))^T.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "hm_internal.h"

namespace hm {

namespace {

// Householder QR of A (m x r, column-major, m >= r).  On return Q (m x r)
// has orthonormal columns and R (r x r) is upper triangular, A = Q R.
void householder_qr(std::vector<cplx>& A, int m, int r, std::vector<cplx>& Q,
                    std::vector<cplx>& R) {
  std::vector<std::vector<cplx>> vs(r);
  for (int k = 0; k < r; ++k) {
    double nx2 = 0;
    for (int i = k; i < m; ++i) nx2 += std::norm(A[i + (size_t)k * m]);
    const double nx = std::sqrt(nx2);
    if (nx == 0.0) continue;
    const cplx x0 = A[k + (size_t)k * m];
    const cplx phase = (std::abs(x0) > 0) ? x0 / std::abs(x0) : cplx(1, 0);
    const cplx alpha = -phase * nx;
    std::vector<cplx> v(m - k);
    for (int i = k; i < m; ++i) v[i - k] = A[i + (size_t)k * m];
    v[0] -= alpha;
    double nv2 = 0;
    for (auto& z : v) nv2 += std::norm(z);
    const double nv = std::sqrt(nv2);
    if (nv == 0.0) continue;
    for (auto& z : v) z /= nv;
    for (int j = k; j < r; ++j) {
      cplx d = 0;
      for (int i = k; i < m; ++i) d += std::conj(v[i - k]) * A[i + (size_t)j * m];
      d *= 2.0;
      for (int i = k; i < m; ++i) A[i + (size_t)j * m] -= d * v[i - k];
    }
    vs[k] = std::move(v);
  }
  R.assign((size_t)r * r, cplx(0));
  for (int j = 0; j < r; ++j)
    for (int i = 0; i <= j; ++i) R[i + (size_t)j * r] = A[i + (size_t)j * m];
  Q.assign((size_t)m * r, cplx(0));
  for (int j = 0; j < r; ++j) Q[j + (size_t)j * m] = 1.0;
  for (int k = r - 1; k >= 0; --k) {
    const auto& v = vs[k];
    if (v.empty()) continue;
    for (int j = 0; j < r; ++j) {
      cplx d = 0;
      for (int i = k; i < m; ++i) d += std::conj(v[i - k]) * Q[i + (size_t)j * m];
      d *= 2.0;
      for (int i = k; i < m; ++i) Q[i + (size_t)j * m] -= d * v[i - k];
    }
  }
}

// One-sided Jacobi SVD of C (r x r, column-major).  On return C holds
// C Psi = Phi Sigma (columns sorted by decreasing norm), sig the singular
// values and Psi the right singular vectors.
void jacobi_svd(std::vector<cplx>& C, int r, std::vector<double>& sig,
                std::vector<cplx>& Psi) {
  Psi.assign((size_t)r * r, cplx(0));
  for (int j = 0; j < r; ++j) Psi[j + (size_t)j * r] = 1.0;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < r - 1; ++p) {
      for (int q = p + 1; q < r; ++q) {
        double a = 0, b = 0;
        cplx g = 0;
        for (int i = 0; i < r; ++i) {
          const cplx cp = C[i + (size_t)p * r], cq = C[i + (size_t)q * r];
          a += std::norm(cp);
          b += std::norm(cq);
          g += std::conj(cp) * cq;
        }
        const double ag = std::abs(g);
        if (ag == 0.0 || ag <= 1e-16 * std::sqrt(a * b)) continue;
        rotated = true;
        const cplx eph = std::conj(g) / ag;  // e^{-i phi}
        const double zeta = (b - a) / (2.0 * ag);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::abs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t);
        const double s = c * t;
        for (int i = 0; i < r; ++i) {
          const cplx cp = C[i + (size_t)p * r];
          const cplx cq = eph * C[i + (size_t)q * r];
          C[i + (size_t)p * r] = c * cp - s * cq;
          C[i + (size_t)q * r] = s * cp + c * cq;
          const cplx vp = Psi[i + (size_t)p * r];
          const cplx vq = eph * Psi[i + (size_t)q * r];
          Psi[i + (size_t)p * r] = c * vp - s * vq;
          Psi[i + (size_t)q * r] = s * vp + c * vq;
        }
      }
    }
    if (!rotated) break;
  }
  sig.assign(r, 0.0);
  for (int j = 0; j < r; ++j) {
    double s = 0;
    for (int i = 0; i < r; ++i) s += std::norm(C[i + (size_t)j * r]);
    sig[j] = std::sqrt(s);
  }
  std::vector<int> ord(r);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return sig[x] > sig[y]; });
  std::vector<cplx> C2(C.size()), P2(Psi.size());
  std::vector<double> s2(r);
  for (int j = 0; j < r; ++j) {
    s2[j] = sig[ord[j]];
    for (int i = 0; i < r; ++i) {
      C2[i + (size_t)j * r] = C[i + (size_t)ord[j] * r];
      P2[i + (size_t)j * r] = Psi[i + (size_t)ord[j] * r];
    }
  }
  C.swap(C2);
  Psi.swap(P2);
  sig.swap(s2);
}

void recompress(LowRank& lr, double eps) {
  const int m = lr.m, n = lr.n, r = lr.r;
  std::vector<cplx> Qu, Ru, Qv, Rv;
  householder_qr(lr.U, m, r, Qu, Ru);
  householder_qr(lr.V, n, r, Qv, Rv);
  std::vector<cplx> C((size_t)r * r, cplx(0));
  for (int j = 0; j < r; ++j)          // C = Ru Rv^T
    for (int l = 0; l < r; ++l) {
      const cplx rv = Rv[j + (size_t)l * r];
      if (rv == cplx(0)) continue;
      for (int i = 0; i < r; ++i) C[i + (size_t)j * r] += Ru[i + (size_t)l * r] * rv;
    }
  std::vector<double> sig;
  std::vector<cplx> Psi;
  jacobi_svd(C, r, sig, Psi);
  double total2 = 0;
  for (double s : sig) total2 += s * s;
  const double total = std::sqrt(total2);
  int keep = r;
  for (int cand = 1; cand <= r; ++cand) {
    double tail2 = 0;
    for (int i = cand; i < r; ++i) tail2 += sig[i] * sig[i];
    if (std::sqrt(tail2) <= eps * total) { keep = cand; break; }
  }
  LowRank out;
  out.m = m; out.n = n; out.r = keep;
  out.U.assign((size_t)m * keep, cplx(0));
  out.V.assign((size_t)n * keep, cplx(0));
  for (int j = 0; j < keep; ++j)
    for (int l = 0; l < r; ++l) {
      const cplx cu = C[l + (size_t)j * r];
      const cplx cv = std::conj(Psi[l + (size_t)j * r]);
      for (int i = 0; i < m; ++i) out.U[i + (size_t)j * m] += Qu[i + (size_t)l * m] * cu;
      for (int i = 0; i < n; ++i) out.V[i + (size_t)j * n] += Qv[i + (size_t)l * n] * cv;
    }
  lr = std::move(out);
}

}  // namespace

LowRank compress_block(const Problem& p, const int64_t* rows, int32_t m, const int64_t* cols,
                       int32_t n, double eps, int32_t max_rank) {
  const int r_max = (max_rank <= 0) ? std::min(m, n) : std::min({max_rank, m, n});
  std::vector<std::vector<cplx>> us, vs;
  std::vector<char> used(m, 0);
  std::vector<cplx> row(n), u(m);
  int i = 0;
  double s2 = 0;
  for (;;) {
    for (int j = 0; j < n; ++j) row[j] = kernel(p, rows[i], cols[j]);
    for (size_t k = 0; k < us.size(); ++k) {
      const cplx uk = us[k][i];
      const auto& vk = vs[k];
      for (int j = 0; j < n; ++j) row[j] -= uk * vk[j];
    }
    used[i] = 1;
    int jp = 0;
    double best = -1;
    for (int j = 0; j < n; ++j) {
      const double a = std::abs(row[j]);
      if (a > best) { best = a; jp = j; }
    }
    if (best <= 1e-300) {
      int nxt = -1;
      for (int q = 0; q < m; ++q)
        if (!used[q]) { nxt = q; break; }
      if (nxt < 0) break;
      i = nxt;
      continue;
    }
    const cplx piv = row[jp];
    std::vector<cplx> v(n);
    for (int j = 0; j < n; ++j) v[j] = row[j] / piv;
    for (int q = 0; q < m; ++q) u[q] = kernel(p, rows[q], cols[jp]);
    for (size_t k = 0; k < us.size(); ++k) {
      const cplx vk = vs[k][jp];
      const auto& uk = us[k];
      for (int q = 0; q < m; ++q) u[q] -= vk * uk[q];
    }
    cplx cross = 0;
    for (size_t k = 0; k < us.size(); ++k) {
      cplx du = 0, dv = 0;
      for (int q = 0; q < m; ++q) du += std::conj(us[k][q]) * u[q];
      for (int j = 0; j < n; ++j) dv += std::conj(vs[k][j]) * v[j];
      cross += du * dv;
    }
    double nu2 = 0, nv2 = 0;
    for (int q = 0; q < m; ++q) nu2 += std::norm(u[q]);
    for (int j = 0; j < n; ++j) nv2 += std::norm(v[j]);
    const double nuv = std::sqrt(nu2) * std::sqrt(nv2);
    s2 += 2.0 * cross.real() + nuv * nuv;
    us.push_back(u);
    vs.push_back(std::move(v));
    if (nuv <= eps * std::sqrt(s2) || (int)us.size() >= r_max) break;
    int nxt = -1;
    double bu = -1;
    for (int q = 0; q < m; ++q) {
      if (used[q]) continue;
      const double a = std::abs(u[q]);
      if (a > bu) { bu = a; nxt = q; }
    }
    if (nxt < 0) break;
    i = nxt;
  }
  LowRank lr;
  lr.m = m;
  lr.n = n;
  if (us.empty()) {
    lr.r = 1;
    lr.U.assign(m, cplx(0));
    lr.V.assign(n, cplx(0));
    return lr;
  }
  lr.r = (int)us.size();
  lr.U.resize((size_t)m * lr.r);
  lr.V.resize((size_t)n * lr.r);
  for (int k = 0; k < lr.r; ++k) {
    std::copy(us[k].begin(), us[k].end(), lr.U.begin() + (size_t)k * m);
    std::copy(vs[k].begin(), vs[k].end(), lr.V.begin() + (size_t)k * n);
  }
  recompress(lr, eps);
  return lr;
}

}  // namespace hm
