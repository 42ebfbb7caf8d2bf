// Small dense complex FP64 linear algebra for the host builder:
// Householder QR with column pivoting (rank-revealing, truncated by a
// relative tolerance), one-sided Jacobi SVD, pseudo-inverse and products.
// All matrices are column-major.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <numeric>
#include <vector>

namespace mbf {
namespace la {

using cd = std::complex<double>;

struct Mat {
  int64_t m = 0, n = 0;
  std::vector<cd> a;
  Mat() = default;
  Mat(int64_t m_, int64_t n_) : m(m_), n(n_), a((size_t)(m_ * n_), cd(0, 0)) {}
  cd& operator()(int64_t i, int64_t j) { return a[(size_t)(i + j * m)]; }
  const cd& operator()(int64_t i, int64_t j) const { return a[(size_t)(i + j * m)]; }
  cd* col(int64_t j) { return a.data() + j * m; }
  const cd* col(int64_t j) const { return a.data() + j * m; }
};

inline double norm2sq(const cd* x, int64_t n) {
  double s = 0;
  for (int64_t i = 0; i < n; ++i) s += x[i].real() * x[i].real() + x[i].imag() * x[i].imag();
  return s;
}

// <x, y> = sum conj(x_i) y_i
inline cd dotc(const cd* x, const cd* y, int64_t n) {
  double re = 0, im = 0;
  for (int64_t i = 0; i < n; ++i) {
    const double xr = x[i].real(), xi = x[i].imag(), yr = y[i].real(), yi = y[i].imag();
    re += xr * yr + xi * yi;
    im += xr * yi - xi * yr;
  }
  return cd(re, im);
}

// y += a x
inline void axpy(cd a, const cd* x, cd* y, int64_t n) {
  const double ar = a.real(), ai = a.imag();
  for (int64_t i = 0; i < n; ++i) {
    const double xr = x[i].real(), xi = x[i].imag();
    y[i] = cd(y[i].real() + ar * xr - ai * xi, y[i].imag() + ar * xi + ai * xr);
  }
}

inline Mat adjoint(const Mat& A) {
  Mat B(A.n, A.m);
  for (int64_t j = 0; j < A.n; ++j)
    for (int64_t i = 0; i < A.m; ++i) B(j, i) = std::conj(A(i, j));
  return B;
}

// C = A B
inline Mat matmul(const Mat& A, const Mat& B) {
  Mat C(A.m, B.n);
  for (int64_t j = 0; j < B.n; ++j)
    for (int64_t k = 0; k < A.n; ++k) {
      const cd b = B(k, j);
      if (b == cd(0, 0)) continue;
      axpy(b, A.col(k), C.col(j), A.m);
    }
  return C;
}

// C = A^* B
inline Mat matmul_ah(const Mat& A, const Mat& B) {
  Mat C(A.n, B.n);
  for (int64_t j = 0; j < B.n; ++j)
    for (int64_t i = 0; i < A.n; ++i) C(i, j) = dotc(A.col(i), B.col(j), A.m);
  return C;
}

// Householder QR with column pivoting: A P = Q R.  Stops after k steps when
// the largest remaining column norm is <= tol * (first pivot norm), or at
// kmax.  Returns Q (m x k), R (k x n, columns in pivoted order), piv (n).
struct QRP {
  Mat Q, R;
  std::vector<int64_t> piv;
  int64_t k = 0;
};
inline QRP pivoted_qr(Mat A, double tol, int64_t kmax, bool pivot = true);

inline QRP pivoted_qr(Mat A, double tol, int64_t kmax, bool pivot) {
  const int64_t m = A.m, n = A.n;
  QRP out;
  out.piv.resize(n);
  std::iota(out.piv.begin(), out.piv.end(), 0);
  kmax = std::min<int64_t>(kmax, std::min(m, n));
  // Partial column norms, downdated after every step and recomputed when
  // cancellation has eaten most of their digits.
  std::vector<double> cn(n), cn0(n);
  for (int64_t j = 0; j < n; ++j) cn0[j] = cn[j] = norm2sq(A.col(j), m);
  std::vector<cd> vs;
  std::vector<int64_t> voff;
  double first = -1;
  int64_t k = 0;
  for (; k < kmax; ++k) {
    int64_t p = k;
    if (pivot) {
      double best = -1;
      for (int64_t j = k; j < n; ++j)
        if (cn[j] > best) {
          best = cn[j];
          p = j;
        }
    }
    if (p != k) {
      std::swap_ranges(A.col(k), A.col(k) + m, A.col(p));
      std::swap(out.piv[k], out.piv[p]);
      std::swap(cn[k], cn[p]);
      std::swap(cn0[k], cn0[p]);
    }
    const double nrm = std::sqrt(norm2sq(A.col(k) + k, m - k));
    if (first < 0) first = nrm;
    if (nrm <= tol * first || nrm == 0.0) break;
    cd* x = A.col(k) + k;
    const int64_t len = m - k;
    const cd x0 = x[0];
    const double ax0 = std::abs(x0);
    const cd ph = ax0 > 0 ? x0 / ax0 : cd(1, 0);
    const cd alpha = -ph * nrm;
    // v = x - alpha e1, normalized
    voff.push_back((int64_t)vs.size());
    vs.insert(vs.end(), x, x + len);
    cd* v = vs.data() + voff.back();
    v[0] -= alpha;
    const double vn = std::sqrt(norm2sq(v, len));
    if (vn > 0)
      for (int64_t i = 0; i < len; ++i) v[i] /= vn;
    // apply H = I - 2 v v^* to columns k..n-1 and downdate the norms
    for (int64_t j = k; j < n; ++j) {
      cd* c = A.col(j) + k;
      const cd t = 2.0 * dotc(v, c, len);
      axpy(-t, v, c, len);
      if (pivot && j > k) {
        cn[j] -= std::norm(c[0]);
        if (cn[j] <= 1e-8 * cn0[j]) cn0[j] = cn[j] = norm2sq(c + 1, len - 1);
      }
    }
  }
  out.k = k;
  out.R = Mat(k, n);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < std::min<int64_t>(k, j + 1); ++i) out.R(i, j) = A(i, j);
  // Q = H_0 H_1 ... H_{k-1} [I_k; 0]
  out.Q = Mat(m, k);
  for (int64_t j = 0; j < k; ++j) out.Q(j, j) = cd(1, 0);
  for (int64_t r = k - 1; r >= 0; --r) {
    const cd* v = vs.data() + voff[r];
    const int64_t len = m - r;
    for (int64_t j = r; j < k; ++j) {
      cd* c = out.Q.col(j) + r;
      const cd t = 2.0 * dotc(v, c, len);
      axpy(-t, v, c, len);
    }
  }
  return out;
}

// One-sided Jacobi SVD of a tall matrix B (p x k, p >= k): B = U diag(s) V^*,
// U p x k with orthonormal columns (for s > 0), V k x k unitary, s sorted
// in decreasing order.
struct SVD {
  Mat U, V;
  std::vector<double> s;
};

inline SVD jacobi_svd_tall(Mat B) {
  const int64_t p = B.m, k = B.n;
  Mat V(k, k);
  for (int64_t i = 0; i < k; ++i) V(i, i) = cd(1, 0);
  std::vector<double> nr(k);
  for (int64_t j = 0; j < k; ++j) nr[j] = norm2sq(B.col(j), p);
  // Rotations stop at a relative off-diagonal level of 1e-12: the singular
  // values are then accurate far below any truncation tolerance used here,
  // and B V = U S holds to rounding whatever the level.
  const double eps = 1e-12;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0;
    for (int64_t i = 0; i < k - 1; ++i)
      for (int64_t j = i + 1; j < k; ++j) {
        const double a = nr[i], b = nr[j];
        if (a == 0.0 || b == 0.0) continue;
        const cd g = dotc(B.col(i), B.col(j), p);
        const double ag = std::abs(g);
        const double rel = ag / std::sqrt(a * b);
        off = std::max(off, rel);
        if (rel <= eps) continue;
        const double zeta = (b - a) / (2.0 * ag);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::abs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t);
        const double s = c * t;
        const cd e = std::conj(g) / ag;  // e^{-i phi}
        // [b_i, b_j] <- [b_i, e b_j] [[c, s], [-s, c]]
        cd* bi = B.col(i);
        cd* bj = B.col(j);
        for (int64_t r = 0; r < p; ++r) {
          const cd x = bi[r], y = e * bj[r];
          bi[r] = c * x - s * y;
          bj[r] = s * x + c * y;
        }
        cd* vi = V.col(i);
        cd* vj = V.col(j);
        for (int64_t r = 0; r < k; ++r) {
          const cd x = vi[r], y = e * vj[r];
          vi[r] = c * x - s * y;
          vj[r] = s * x + c * y;
        }
        nr[i] = norm2sq(bi, p);
        nr[j] = norm2sq(bj, p);
      }
    if (off <= eps) break;
  }
  std::vector<int64_t> ord(k);
  std::iota(ord.begin(), ord.end(), 0);
  std::vector<double> sv(k);
  for (int64_t j = 0; j < k; ++j) sv[j] = std::sqrt(norm2sq(B.col(j), p));
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return sv[x] > sv[y]; });
  SVD out;
  out.U = Mat(p, k);
  out.V = Mat(k, k);
  out.s.resize(k);
  for (int64_t jj = 0; jj < k; ++jj) {
    const int64_t j = ord[jj];
    out.s[jj] = sv[j];
    for (int64_t r = 0; r < p; ++r) out.U(r, jj) = sv[j] > 0 ? B(r, j) / sv[j] : cd(0, 0);
    for (int64_t r = 0; r < k; ++r) out.V(r, jj) = V(r, j);
  }
  return out;
}

// SVD of a tall matrix A (m >= n) preconditioned by a column-pivoted QR:
// A P = Q R, then one-sided Jacobi on R^* (n x k, few sweeps for such
// triangular factors): R^* = X S Y^*  =>  A = (Q Y) S (P X)^*.
inline SVD svd_tall_qr(const Mat& A) {
  QRP q = pivoted_qr(A, 0.0, A.n, true);
  const int64_t k = q.k, n = A.n;
  Mat RH(n, k);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < k; ++i) RH(j, i) = std::conj(q.R(i, j));
  SVD t = jacobi_svd_tall(RH);  // RH = X S Y^*  (X: n x k, Y: k x k)
  SVD out;
  out.s = t.s;
  out.U = Mat(A.m, k);
  // U = Q Y
  for (int64_t j = 0; j < k; ++j)
    for (int64_t l = 0; l < k; ++l) axpy(t.V(l, j), q.Q.col(l), out.U.col(j), A.m);
  out.V = Mat(n, k);
  for (int64_t j = 0; j < k; ++j)
    for (int64_t i = 0; i < n; ++i) out.V(q.piv[i], j) = t.U(i, j);
  return out;
}

// SVD of any matrix: A = U diag(s) V^*, economy size.
inline SVD svd(const Mat& A) {
  if (A.m >= A.n) return svd_tall_qr(A);
  SVD t = svd_tall_qr(adjoint(A));  // A^* = U' S V'^*  =>  A = V' S U'^*
  SVD out;
  out.U = t.V;
  out.V = t.U;
  out.s = t.s;
  return out;
}

inline int64_t trunc_rank(const std::vector<double>& s, double tol, int64_t rmax) {
  if (s.empty() || s[0] <= 0) return 0;
  int64_t r = 0;
  while (r < (int64_t)s.size() && s[r] > tol * s[0]) ++r;
  return std::min(r, rmax);
}

// Least-squares solution X = pinv(A) B for A (m x k) of full column rank,
// by Householder QR (A = Q R) and back substitution R X = Q^* B.
inline Mat lstsq(const Mat& A, const Mat& B) {
  QRP q = pivoted_qr(A, 0.0, A.n);
  const int64_t k = q.k;
  Mat QB = matmul_ah(q.Q, B);  // k x nb
  Mat X(A.n, B.n);
  for (int64_t j = 0; j < B.n; ++j) {
    std::vector<cd> y(k);
    for (int64_t i = k - 1; i >= 0; --i) {
      cd acc = QB(i, j);
      for (int64_t l = i + 1; l < k; ++l) acc -= q.R(i, l) * y[l];
      y[i] = acc / q.R(i, i);
    }
    for (int64_t i = 0; i < k; ++i) X(q.piv[i], j) = y[i];
  }
  return X;
}

// Moore-Penrose pseudo-inverse via SVD (singular values below 1e-13 s_1 dropped).
inline Mat pinv(const Mat& A) {
  SVD d = svd(A);
  const int64_t r = trunc_rank(d.s, 1e-13, (int64_t)d.s.size());
  Mat P(A.n, A.m);
  for (int64_t k = 0; k < r; ++k) {
    const double inv = 1.0 / d.s[k];
    for (int64_t j = 0; j < A.m; ++j) {
      const cd u = std::conj(d.U(j, k)) * inv;
      axpy(u, d.V.col(k), P.col(j), A.n);
    }
  }
  return P;
}

// Truncated SVD through a rank-revealing QR: W ~ Q R, R = U_R S V_R^*.
// Returns U0 (m x r), s (r), V0 (n x r) with W ~ U0 diag(s) V0^*.
struct Trunc {
  Mat U0, V0;
  std::vector<double> s;
};

inline Trunc truncated_svd(const Mat& W, double tol, int64_t rmax) {
  Trunc out;
  if (W.m == 0 || W.n == 0) {
    out.U0 = Mat(W.m, 0);
    out.V0 = Mat(W.n, 0);
    return out;
  }
  QRP q = pivoted_qr(W, tol * 1e-3, std::min(W.m, W.n));
  const int64_t k = q.k;
  if (k == 0) {
    out.U0 = Mat(W.m, 0);
    out.V0 = Mat(W.n, 0);
    return out;
  }
  // Rp = R P^T (k x n, columns back in the original order); Rp^* = Q2 R2
  // (n x k Householder QR), so Rp = R2^* Q2^* and the SVD needs only the
  // k x k matrix R2^* = U S V^*:  W ~ (Q U) S (Q2 V)^*.
  Mat RpH(W.n, k);
  for (int64_t j = 0; j < W.n; ++j)
    for (int64_t i = 0; i < k; ++i) RpH(q.piv[j], i) = std::conj(q.R(i, j));
  QRP q2 = pivoted_qr(RpH, 0.0, k);
  Mat Q2(W.n, k);  // undo the pivoting of q2: RpH P2 = Q2' R2'  =>  RpH = Q2' (R2' P2^T)
  Mat R2H(k, k);   // (R2' P2^T)^*  (k x k)
  for (int64_t j = 0; j < k; ++j)
    for (int64_t i = 0; i < q2.k; ++i) R2H(q2.piv[j], i) = std::conj(q2.R(i, j));
  Mat Q2p = q2.Q;  // n x q2.k
  // Rp = (RpH)^* = (R2' P2^T)^* Q2'^* = R2H Q2'^*   with R2H: k x q2.k
  Mat R2Hs(k, q2.k);
  for (int64_t j = 0; j < q2.k; ++j)
    for (int64_t i = 0; i < k; ++i) R2Hs(i, j) = R2H(i, j);
  SVD d = svd(R2Hs);  // R2Hs = U S V^*  (k x q2.k)
  const int64_t r = trunc_rank(d.s, tol, rmax);
  Mat UR(k, r), VR(q2.k, r);
  for (int64_t j = 0; j < r; ++j) {
    for (int64_t i = 0; i < k; ++i) UR(i, j) = d.U(i, j);
    for (int64_t i = 0; i < q2.k; ++i) VR(i, j) = d.V(i, j);
  }
  out.U0 = matmul(q.Q, UR);
  out.V0 = matmul(Q2p, VR);
  out.s.assign(d.s.begin(), d.s.begin() + r);
  (void)Q2;
  return out;
}

}  // namespace la
}  // namespace mbf
