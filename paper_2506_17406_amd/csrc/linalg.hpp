// Small dense FP64 linear algebra for the host-side reference-element build:
// row-major matrices, Householder QR with column pivoting (ranges and null
// spaces), the symmetric eigenproblem (Householder tridiagonalisation and
// implicit QL), and LU with partial pivoting.  Sizes are at most a few hundred, built once per
// (dimension, space, degree).
#pragma once
#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <vector>

namespace rz {

struct Dense {
  int r = 0, c = 0;
  std::vector<double> a;
  Dense() = default;
  Dense(int r_, int c_) : r(r_), c(c_), a(size_t(r_) * c_, 0.0) {}
  double &operator()(int i, int j) { return a[size_t(i) * c + j]; }
  double operator()(int i, int j) const { return a[size_t(i) * c + j]; }
  static Dense eye(int n) {
    Dense m(n, n);
    for (int i = 0; i < n; ++i) m(i, i) = 1.0;
    return m;
  }
};

inline Dense matmul(const Dense &A, const Dense &B) {
  if (A.c != B.r) throw std::runtime_error("matmul shape");
  Dense C(A.r, B.c);
  if (B.c == 0) return C;  // no columns: nothing to index
  for (int i = 0; i < A.r; ++i)
    for (int k = 0; k < A.c; ++k) {
      const double aik = A(i, k);
      if (aik == 0.0) continue;
      const double *b = B.a.data() + size_t(k) * B.c;
      double *cc = C.a.data() + size_t(i) * C.c;
      for (int j = 0; j < B.c; ++j) cc[j] += aik * b[j];
    }
  return C;
}

inline Dense transpose(const Dense &A) {
  Dense T(A.c, A.r);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) T(j, i) = A(i, j);
  return T;
}

inline Dense columns(const Dense &A, int j0, int j1) {
  Dense B(A.r, j1 - j0);
  for (int i = 0; i < A.r; ++i)
    for (int j = j0; j < j1; ++j) B(i, j - j0) = A(i, j);
  return B;
}

// Householder QR with column pivoting of A (m x n, m >= 1): returns the full
// orthogonal factor Q (m x m) and the numerical rank, judged by |R_kk| >
// rtol * |R_00| with a required gap below.
struct QRCP {
  Dense Q;
  int rank = 0;
  double gap_ratio = 0.0;  // |R_rank,rank| / |R_00|
};

inline QRCP qr_pivoted(Dense A, double rtol) {
  const int m = A.r, n = A.c;
  std::vector<double> colnorm(n);
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < m; ++i) s += A(i, j) * A(i, j);
    colnorm[j] = s;
  }
  std::vector<std::vector<double>> V;  // Householder vectors
  std::vector<double> beta;
  const int kmax = std::min(m, n);
  double r00 = 0.0;
  QRCP out;
  out.rank = kmax;
  for (int k = 0; k < kmax; ++k) {
    // pivot: column with the largest remaining norm (recomputed exactly)
    int piv = k;
    double best = -1;
    for (int j = k; j < n; ++j) {
      double s = 0;
      for (int i = k; i < m; ++i) s += A(i, j) * A(i, j);
      colnorm[j] = s;
      if (s > best) { best = s; piv = j; }
    }
    if (piv != k)
      for (int i = 0; i < m; ++i) std::swap(A(i, k), A(i, piv));
    double nrm = std::sqrt(best);
    if (k == 0) r00 = nrm;
    if (nrm <= rtol * r00 || nrm == 0.0) {
      out.rank = k;
      out.gap_ratio = r00 > 0 ? nrm / r00 : 0.0;
      break;
    }
    std::vector<double> v(m, 0.0);
    double alpha = A(k, k) >= 0 ? -nrm : nrm;
    for (int i = k; i < m; ++i) v[i] = A(i, k);
    v[k] -= alpha;
    double vv = 0;
    for (int i = k; i < m; ++i) vv += v[i] * v[i];
    double b = vv > 0 ? 2.0 / vv : 0.0;
    for (int j = k; j < n; ++j) {
      double s = 0;
      for (int i = k; i < m; ++i) s += v[i] * A(i, j);
      s *= b;
      for (int i = k; i < m; ++i) A(i, j) -= s * v[i];
    }
    V.push_back(std::move(v));
    beta.push_back(b);
  }
  // Q = H_0 H_1 ... H_{r-1} applied to the identity
  Dense Q = Dense::eye(m);
  for (int k = int(V.size()) - 1; k >= 0; --k) {
    const auto &v = V[k];
    for (int j = 0; j < m; ++j) {
      double s = 0;
      for (int i = k; i < m; ++i) s += v[i] * Q(i, j);
      s *= beta[k];
      for (int i = k; i < m; ++i) Q(i, j) -= s * v[i];
    }
  }
  out.Q = std::move(Q);
  return out;
}

// Orthonormal basis of range(S); throws unless the rank is `expected`.
inline Dense orth_range(const Dense &S, int expected) {
  QRCP f = qr_pivoted(S, 1e-10);
  if (f.rank != expected) throw std::runtime_error("space rank mismatch");
  return columns(f.Q, 0, f.rank);
}

// Orthonormal basis of the null space of C (rows are constraints).
inline Dense null_space(const Dense &C) {
  QRCP f = qr_pivoted(transpose(C), 1e-10);
  return columns(f.Q, f.rank, f.Q.r);
}

// Symmetric eigenproblem: eigenvalues ascending, and the corresponding
// orthonormal eigenvectors as columns of V.  Householder reduction to
// tridiagonal form (the reflections accumulated), then the implicit QL
// iteration with Wilkinson shifts on the tridiagonal matrix, the plane
// rotations applied to the accumulated basis: the published procedures tred2
// and tql2 of Wilkinson and Reinsch (Handbook for Automatic Computation,
// Vol. II, Linear Algebra, 1971; EISPACK), restated here in this file's
// dense-matrix type.
inline void sym_eig(Dense A, std::vector<double> &w, Dense &V) {
  const int n = A.r;
  w.assign(n, 0.0);
  if (n == 0) {
    V = Dense(0, 0);
    return;
  }
  std::vector<double> d(n), e(n, 0.0);
  // Householder: for i = n-1 .. 1 annihilate A(i, 0 .. i-2)
  std::vector<std::vector<double>> hv;  // reflection vectors u_i (length i), scaled
  std::vector<double> hh;               // their H = u^T u / 2
  for (int i = n - 1; i >= 1; --i) {
    const int l = i - 1;
    double scale = 0.0, h = 0.0;
    for (int k = 0; k <= l; ++k) scale += std::fabs(A(i, k));
    std::vector<double> u(i, 0.0);
    if (l == 0 || scale == 0.0) {
      e[i] = A(i, l);
      hv.push_back(u);
      hh.push_back(0.0);
      continue;
    }
    for (int k = 0; k <= l; ++k) {
      u[k] = A(i, k) / scale;
      h += u[k] * u[k];
    }
    const double f = u[l];
    const double g = f >= 0 ? -std::sqrt(h) : std::sqrt(h);
    e[i] = scale * g;
    h -= f * g;
    u[l] = f - g;
    // p = A u / h; K = u^T p / 2h; q = p - K u; A -= u q^T + q u^T (leading i x i block)
    std::vector<double> pvec(i, 0.0);
    for (int j = 0; j <= l; ++j) {
      double sacc = 0.0;
      const double *aj = A.a.data() + (size_t(j) * n);
      for (int k = 0; k <= l; ++k) sacc += aj[k] * u[k];
      pvec[j] = sacc / h;
    }
    double K = 0.0;
    for (int j = 0; j <= l; ++j) K += u[j] * pvec[j];
    K /= (h + h);
    for (int j = 0; j <= l; ++j) pvec[j] -= K * u[j];
    for (int j = 0; j <= l; ++j) {
      double *aj = A.a.data() + (size_t(j) * n);
      const double uj = u[j], qj = pvec[j];
      for (int k = 0; k <= l; ++k) aj[k] -= uj * pvec[k] + qj * u[k];
    }
    hv.push_back(u);
    hh.push_back(h);
  }
  for (int i = 0; i < n; ++i) d[i] = A(i, i);
  // accumulate Q = H_{n-1} ... H_1 applied to the identity (rows of Z)
  Dense Z = Dense::eye(n);
  for (int idx = int(hv.size()) - 1; idx >= 0; --idx) {
    const int i = n - 1 - idx;  // reflection acting on coordinates 0 .. i-1
    const double h = hh[idx];
    if (h == 0.0) continue;
    const std::vector<double> &u = hv[idx];
    // Z_rows: for every row r of Z (an eigenbasis vector), z[0..i-1] -= (u . z) u / h
    for (int r = 0; r < n; ++r) {
      double *zr = Z.a.data() + (size_t(r) * n);
      double sacc = 0.0;
      for (int k = 0; k < i; ++k) sacc += u[k] * zr[k];
      if (sacc == 0.0) continue;
      sacc /= h;
      for (int k = 0; k < i; ++k) zr[k] -= sacc * u[k];
    }
  }
  // row r of Z now holds column r of Q = H_{n-1} ... H_1: the basis in which
  // the matrix is tridiagonal, one vector per row
  Dense &Qt = Z;
  // implicit QL on (d, e): e[i] couples i-1 and i; shift to e[i-1] convention
  for (int i = 1; i < n; ++i) e[i - 1] = e[i];
  e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    for (;;) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-17 * dd) break;
      }
      if (m == l) break;
      if (++iter > 60) throw std::runtime_error("symmetric eigensolver did not converge");
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? std::fabs(r) : -std::fabs(r)));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      for (; i >= l; --i) {
        double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        // rotate basis vectors i and i+1 (rows of Qt)
        double *qa = Qt.a.data() + (size_t(i) * n), *qb = Qt.a.data() + (size_t(i + 1) * n);
        for (int k = 0; k < n; ++k) {
          f = qb[k];
          qb[k] = s * qa[k] + c * f;
          qa[k] = c * qa[k] - s * f;
        }
      }
      if (r == 0.0 && i >= l) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
  V = Dense(n, n);
  for (int j = 0; j < n; ++j) {
    w[j] = d[order[j]];
    const double *q = &Qt.a[size_t(order[j]) * n];
    for (int i = 0; i < n; ++i) V(i, j) = q[i];
  }
}

// Cyclic Jacobi method (the earlier solver, kept as a cross-check).
inline void sym_eig_jacobi(Dense A, std::vector<double> &w, Dense &V) {
  const int n = A.r;
  V = Dense::eye(n);
  double fro = 0;
  for (double x : A.a) fro += x * x;
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotations = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A(p, q);
        // rotate while the entry matters relative to its diagonal pair
        if (std::fabs(apq) <= 1e-17 * (std::fabs(A(p, p)) + std::fabs(A(q, q))) ||
            std::fabs(apq) <= 1e-19 * fro)
          continue;
        ++rotations;
        const double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A(k, p), akq = A(k, q);
          A(k, p) = cs * akp - sn * akq;
          A(k, q) = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A(p, k), aqk = A(q, k);
          A(p, k) = cs * apk - sn * aqk;
          A(q, k) = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V(k, p), vkq = V(k, q);
          V(k, p) = cs * vkp - sn * vkq;
          V(k, q) = sn * vkp + cs * vkq;
        }
      }
    if (rotations == 0) break;
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return A(a, a) < A(b, b); });
  w.resize(n);
  Dense Vs(n, n);
  for (int j = 0; j < n; ++j) {
    w[j] = A(order[j], order[j]);
    for (int i = 0; i < n; ++i) Vs(i, j) = V(i, order[j]);
  }
  V = std::move(Vs);
}

// Inverse by LU with partial pivoting; throws on a zero pivot.
inline Dense inverse(Dense A) {
  const int n = A.r;
  Dense Inv = Dense::eye(n);
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A(i, k)) > std::fabs(A(piv, k))) piv = i;
    if (A(piv, k) == 0.0) throw std::runtime_error("singular dof matrix");
    if (piv != k)
      for (int j = 0; j < n; ++j) {
        std::swap(A(k, j), A(piv, j));
        std::swap(Inv(k, j), Inv(piv, j));
      }
    const double d = 1.0 / A(k, k);
    for (int i = k + 1; i < n; ++i) {
      const double f = A(i, k) * d;
      if (f == 0.0) continue;
      for (int j = k; j < n; ++j) A(i, j) -= f * A(k, j);
      for (int j = 0; j < n; ++j) Inv(i, j) -= f * Inv(k, j);
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    const double d = 1.0 / A(k, k);
    for (int j = 0; j < n; ++j) {
      double s = Inv(k, j);
      for (int m = k + 1; m < n; ++m) s -= A(k, m) * Inv(m, j);
      Inv(k, j) = s * d;
    }
  }
  return Inv;
}

}  // namespace rz
