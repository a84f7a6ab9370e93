// Reference-element builder: the orthogonality-promoting dual bases of
// Brubeck, Farrell, Kirby & Parker (arXiv:2506.17406), Sec. 3-4.
//
// Steps (each on the equilateral reference simplex of edge length 2 with its
// centroid at the origin; the paper fixes only "equilateral", Sec. 3.3):
//  * polynomials: orthonormal Dubiner basis from its collapsed-coordinate
//    three-term recurrences, differentiated analytically through the
//    recurrences; Gauss-Legendre rules on the Duffy-collapsed cube;
//  * spaces X^k_p (eq:first-kind-def, eq:second-kind-def) as orthonormal
//    column spans inside P_p^c (Householder QR with column pivoting);
//  * bubble spaces (the definition opening Sec. 3.1) as null spaces of the
//    boundary trace moments;
//  * eigenbases of eq:ref-eval-problem-x through the augmented problem
//    eq:ref-eval-problem-x-aug: the stiffness form is diagonalised in an
//    L2-orthonormal bubble basis (cyclic Jacobi), the first N^{k-1}_S
//    eigenpairs (the kernel, eq:bubble-trace-dim-counts) are dropped, the
//    rest are scaled by mu^{-1/2};
//  * eigenspaces of (numerically) repeated mu are made unique by a rotation
//    that makes the matrix of probe values symmetric positive definite
//    (probes: point values along fixed directions at SplitMix64-drawn points;
//    the same convention is used everywhere these tables are compared);
//  * degrees of freedom eq:abstract-dofs in their concrete forms
//    (eq:hgrad-dofs, eq:hcurl-dofs, eq:hdiv-dofs; RT_p uses NedTwo_p
//    eigenfunctions for its type-II moments, Sec. 3.4.3) and the dual basis
//    C = D^{-1} (Sec. 4);
//  * the stacked reference matrices R_q: component products of the basis and
//    of its exterior derivative, whose geometric weighting gives every
//    affine cell's matrix (Sec. 2, eq:pullback-3d-def).
#include "refelem.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <thread>

namespace rz {

namespace {

// runs f(0 .. count-1) on up to 16 host threads (independent work items)
template <typename F>
void parallel_for(int count, F f) {
  const int nt = std::max(1, std::min({count, 16, int(std::thread::hardware_concurrency())}));
  if (nt <= 1) {
    for (int i = 0; i < count; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  for (int w = 0; w < nt; ++w)
    th.emplace_back([&, w]() {
      for (int i = w; i < count; i += nt) f(i);
    });
  for (auto &t : th) t.join();
}

constexpr double kClusterTol = 1e-7;

// ---------------------------------------------------------------- geometry
void eq_vertices_impl(int d, double *v) {
  const double s3 = std::sqrt(3.0), s6 = std::sqrt(6.0);
  if (d == 1) {
    v[0] = -1; v[1] = 1;
  } else if (d == 2) {
    const double t[6] = {-1, -1 / s3, 1, -1 / s3, 0, 2 / s3};
    for (int i = 0; i < 6; ++i) v[i] = t[i];
  } else if (d == 3) {
    const double t[12] = {-1, -1 / s3, -1 / s6, 1, -1 / s3, -1 / s6, 0, 2 / s3, -1 / s6, 0, 0, 3 / s6};
    for (int i = 0; i < 12; ++i) v[i] = t[i];
  }
}

struct Simplex {
  int d;
  std::vector<double> V;      // (d+1) x d vertices
  Dense E, Einv;              // columns v_m - v_0, and its inverse
  double absdetE = 1;
  explicit Simplex(int d_) : d(d_), V(size_t(d_ + 1) * d_), E(d_, d_) {
    eq_vertices_impl(d, V.data());
    for (int a = 0; a < d; ++a)
      for (int m = 0; m < d; ++m) E(a, m) = V[(m + 1) * d + a] - V[a];
    if (d > 0) {
      Einv = inverse(E);
      Dense Ecopy = E;
      // |det E| through the LU pivots of a copy
      double det = 1;
      for (int k = 0; k < d; ++k) {
        int piv = k;
        for (int i = k + 1; i < d; ++i)
          if (std::fabs(Ecopy(i, k)) > std::fabs(Ecopy(piv, k))) piv = i;
        if (piv != k) {
          for (int j = 0; j < d; ++j) std::swap(Ecopy(k, j), Ecopy(piv, j));
          det = -det;
        }
        det *= Ecopy(k, k);
        for (int i = k + 1; i < d; ++i) {
          double f = Ecopy(i, k) / Ecopy(k, k);
          for (int j = k; j < d; ++j) Ecopy(i, j) -= f * Ecopy(k, j);
        }
      }
      absdetE = std::fabs(det);
    }
  }
};

const Simplex &simplex(int d) {
  static std::once_flag once;
  static std::unique_ptr<Simplex> S[4];
  std::call_once(once, [] {
    for (int i = 0; i < 4; ++i) S[i] = std::make_unique<Simplex>(i);
  });
  return *S[d];
}

// -------------------------------------------------------------- quadrature
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.resize(n);
  w.resize(n);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = z;
      for (int k = 1; k < n; ++k) {
        double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1, p1 = z;
    for (int k = 1; k < n; ++k) {
      double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1);
    x[i] = z;
    w[i] = 2.0 / ((1 - z * z) * dp * dp);
  }
}

struct Quad {
  int d = 0;
  std::vector<double> x, w;  // points (npts x d) on the equilateral simplex
  int size() const { return int(w.size()); }
};

// Gauss-Legendre product rule on the Duffy-collapsed cube, mapped to the
// equilateral d-simplex; exact for degree 2n - d.
Quad simplex_quad(int d, int n) {
  Quad q;
  q.d = d;
  if (d == 0) {
    q.w = {1.0};
    return q;
  }
  std::vector<double> g, gw;
  gauss_legendre(n, g, gw);
  const Simplex &S = simplex(d);
  std::vector<double> r(d);
  auto push = [&](double weight) {
    for (int a = 0; a < d; ++a) {
      double xa = S.V[a];
      for (int m = 0; m < d; ++m) xa += S.E(a, m) * 0.5 * (r[m] + 1.0);
      q.x.push_back(xa);
    }
    q.w.push_back(weight * S.absdetE / std::pow(2.0, d));
  };
  if (d == 1) {
    for (int i = 0; i < n; ++i) { r[0] = g[i]; push(gw[i]); }
  } else if (d == 2) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double a = g[i], b = g[j];
        r[0] = 0.5 * (1 + a) * (1 - b) - 1;
        r[1] = b;
        push(gw[i] * gw[j] * 0.5 * (1 - b));
      }
  } else {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) {
          double a = g[i], b = g[j], c = g[k];
          r[0] = 0.25 * (1 + a) * (1 - b) * (1 - c) - 1;
          r[1] = 0.5 * (1 + b) * (1 - c) - 1;
          r[2] = c;
          push(gw[i] * gw[j] * gw[k] * 0.5 * (1 - b) * 0.25 * (1 - c) * (1 - c));
        }
  }
  return q;
}

// ------------------------------------------------------ Dubiner polynomials
// Scaled Jacobi recurrence: R_n = v^n P_n^{(alpha,0)}(xv / v) and gradients
// (D components), given xv, v, v^2 and their gradients.
void scaled_jacobi(int nmax, double alpha, double xv, const double *gxv, double v, const double *gv,
                   double v2, const double *gv2, int D, double *R, double *gR) {
  R[0] = 1;
  for (int a = 0; a < D; ++a) gR[a] = 0;
  if (nmax < 1) return;
  R[1] = 0.5 * ((alpha + 2) * xv + alpha * v);
  for (int a = 0; a < D; ++a) gR[D + a] = 0.5 * ((alpha + 2) * gxv[a] + alpha * gv[a]);
  for (int n = 1; n < nmax; ++n) {
    const double s = 2.0 * n + alpha;
    const double A0 = 2.0 * (n + 1) * (n + alpha + 1) * s;
    const double A1 = (s + 1) * (s + 2) * s;
    const double A2 = (s + 1) * alpha * alpha;
    const double A3 = 2.0 * (n + alpha) * n * (s + 2);
    R[n + 1] = (A1 * xv * R[n] + A2 * v * R[n] - A3 * v2 * R[n - 1]) / A0;
    for (int a = 0; a < D; ++a)
      gR[(n + 1) * D + a] = (A1 * (gxv[a] * R[n] + xv * gR[n * D + a]) + A2 * (gv[a] * R[n] + v * gR[n * D + a]) -
                             A3 * (gv2[a] * R[n - 1] + v2 * gR[(n - 1) * D + a])) / A0;
  }
}

struct PolyBasis {
  int d = 0, p = 0, n = 0;
  std::vector<std::array<int, 3>> idx;
  std::vector<int> degree;
  std::vector<double> scale;  // 1 / L2 norm

  PolyBasis() = default;
  PolyBasis(int d_, int p_) : d(d_), p(p_) {
    if (d == 0) {
      idx.push_back({0, 0, 0});
    } else if (d == 1) {
      for (int i = 0; i <= p; ++i) idx.push_back({i, 0, 0});
    } else if (d == 2) {
      for (int i = 0; i <= p; ++i)
        for (int j = 0; i + j <= p; ++j) idx.push_back({i, j, 0});
    } else {
      for (int i = 0; i <= p; ++i)
        for (int j = 0; i + j <= p; ++j)
          for (int k = 0; i + j + k <= p; ++k) idx.push_back({i, j, k});
    }
    n = int(idx.size());
    for (auto &m : idx) degree.push_back(m[0] + m[1] + m[2]);
    scale.assign(n, 1.0);
    if (d > 0) {
      Quad q = simplex_quad(d, p + 2);
      std::vector<double> val(size_t(q.size()) * n);
      eval(q.x.data(), q.size(), val.data(), nullptr);
      std::vector<double> nrm(n, 0.0);
      for (int t = 0; t < q.size(); ++t)
        for (int i = 0; i < n; ++i) nrm[i] += q.w[t] * val[size_t(t) * n + i] * val[size_t(t) * n + i];
      for (int i = 0; i < n; ++i) scale[i] = 1.0 / std::sqrt(nrm[i]);
    }
  }

  // values (npts x n) and gradients (npts x d x n) at equilateral points
  void eval(const double *x, int npts, double *val, double *grad) const {
    if (d == 0) {
      for (int t = 0; t < npts; ++t) val[t] = 1.0;
      return;
    }
    const Simplex &S = simplex(d);
    std::vector<double> R1(p + 1), gR1((p + 1) * 3), R2(p + 1), gR2((p + 1) * 3), R3(p + 1), gR3((p + 1) * 3);
    for (int t = 0; t < npts; ++t) {
      double r[3] = {0, 0, 0};
      for (int m = 0; m < d; ++m) {
        double s = 0;
        for (int a = 0; a < d; ++a) s += S.Einv(m, a) * (x[t * d + a] - S.V[a]);
        r[m] = 2 * s - 1;
      }
      const double zero[3] = {0, 0, 0};
      std::vector<double> gref(size_t(n) * d, 0.0);
      double *vout = val + size_t(t) * n;
      if (d == 1) {
        const double g1[1] = {1};
        scaled_jacobi(p, 0, r[0], g1, 1, zero, 1, zero, 1, R1.data(), gR1.data());
        for (int b = 0; b < n; ++b) {
          vout[b] = R1[idx[b][0]];
          gref[b] = gR1[idx[b][0]];
        }
      } else if (d == 2) {
        const double f1 = 0.5 * (1 + 2 * r[0] + r[1]), gf1[2] = {1, 0.5};
        const double u = 0.5 * (1 - r[1]), gu[2] = {0, -0.5};
        const double u2 = u * u, gu2[2] = {0, -u};
        scaled_jacobi(p, 0, f1, gf1, u, gu, u2, gu2, 2, R1.data(), gR1.data());
        const double gs[2] = {0, 1};
        int b = 0;
        for (int i = 0; i <= p; ++i) {
          scaled_jacobi(p - i, 2.0 * i + 1, r[1], gs, 1, zero, 1, zero, 2, R2.data(), gR2.data());
          for (int j = 0; i + j <= p; ++j, ++b) {
            vout[b] = R1[i] * R2[j];
            for (int a = 0; a < 2; ++a) gref[a * n + b] = gR1[i * 2 + a] * R2[j] + R1[i] * gR2[j * 2 + a];
          }
        }
      } else {
        const double f1 = 0.5 * (2 + 2 * r[0] + r[1] + r[2]), gf1[3] = {1, 0.5, 0.5};
        const double U = -0.5 * (r[1] + r[2]), gU[3] = {0, -0.5, -0.5};
        const double U2 = U * U, gU2[3] = {0, 0.5 * (r[1] + r[2]), 0.5 * (r[1] + r[2])};
        scaled_jacobi(p, 0, f1, gf1, U, gU, U2, gU2, 3, R1.data(), gR1.data());
        const double f3 = 0.5 * (1 + 2 * r[1] + r[2]), gf3[3] = {0, 1, 0.5};
        const double V = 0.5 * (1 - r[2]), gV[3] = {0, 0, -0.5};
        const double V2 = V * V, gV2[3] = {0, 0, -V};
        const double gt[3] = {0, 0, 1};
        int b = 0;
        for (int i = 0; i <= p; ++i) {
          scaled_jacobi(p - i, 2.0 * i + 1, f3, gf3, V, gV, V2, gV2, 3, R2.data(), gR2.data());
          for (int j = 0; i + j <= p; ++j) {
            scaled_jacobi(p - i - j, 2.0 * i + 2.0 * j + 2, r[2], gt, 1, zero, 1, zero, 3, R3.data(), gR3.data());
            for (int k = 0; i + j + k <= p; ++k, ++b) {
              vout[b] = R1[i] * R2[j] * R3[k];
              for (int a = 0; a < 3; ++a)
                gref[a * n + b] = gR1[i * 3 + a] * R2[j] * R3[k] + R1[i] * gR2[j * 3 + a] * R3[k] +
                                  R1[i] * R2[j] * gR3[k * 3 + a];
            }
          }
        }
      }
      for (int b = 0; b < n; ++b) vout[b] *= scale[b];
      if (grad) {
        // grad_x = 2 E^{-T} grad_r
        double *gout = grad + size_t(t) * d * n;
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < n; ++b) {
            double s = 0;
            for (int m = 0; m < d; ++m) s += S.Einv(m, a) * gref[m * n + b];
            gout[a * n + b] = 2.0 * s * scale[b];
          }
      }
    }
  }
};

// ------------------------------------------------------------------ spaces
int form_of(Family f) { return f == FAM_CG ? 0 : ((f == FAM_RT || f == FAM_BDM) ? 2 : 1); }

int binom(int n, int k) {
  if (k < 0 || n < k) return 0;
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return int(r);
}

int space_dim(int l, Family f, int p) {
  auto P = [&](int q) { return q < 0 ? 0 : binom(q + l, l); };
  switch (f) {
    case FAM_CG: return P(p);
    case FAM_NEDTWO:
    case FAM_BDM: return l * P(p);
    case FAM_NED: return l == 2 ? p * (p + 2) : p * (p + 2) * (p + 3) / 2;
    case FAM_RT: return p * (p + 1) * (p + 3) / 2;
  }
  return 0;
}

struct Space {
  int l = 0, c = 1, p = 0;
  Family fam = FAM_CG;
  PolyBasis poly;
  Dense B;  // (c * poly.n) x m, orthonormal columns

  // values (npts x c x c n) and jacobians of the primal basis e_comp (x) q_b
  // itself (the columns of the identity): the basis values put in place
  void field_primal(const double *x, int npts, std::vector<double> &vals, std::vector<double> &jac) const {
    const int n = poly.n, m = c * n;
    std::vector<double> V(size_t(npts) * n), G(size_t(npts) * std::max(l, 1) * n);
    poly.eval(x, npts, V.data(), l > 0 ? G.data() : nullptr);
    vals.assign(size_t(npts) * c * m, 0.0);
    jac.assign(size_t(npts) * c * std::max(l, 1) * m, 0.0);
    for (int t = 0; t < npts; ++t)
      for (int comp = 0; comp < c; ++comp)
        for (int b = 0; b < n; ++b) {
          const int j = comp * n + b;
          vals[(size_t(t) * c + comp) * m + j] = V[size_t(t) * n + b];
          for (int a = 0; a < l; ++a)
            jac[((size_t(t) * c + comp) * l + a) * m + j] = G[(size_t(t) * l + a) * n + b];
        }
  }

  // values (npts x c x m) and jacobians (npts x c x l x m) of columns of coef
  void field(const double *x, int npts, const Dense &coef, std::vector<double> &vals,
             std::vector<double> &jac) const {
    const int n = poly.n, m = coef.c;
    std::vector<double> V(size_t(npts) * n), G(size_t(npts) * std::max(l, 1) * n);
    poly.eval(x, npts, V.data(), l > 0 ? G.data() : nullptr);
    vals.assign(size_t(npts) * c * m, 0.0);
    jac.assign(size_t(npts) * c * std::max(l, 1) * m, 0.0);
    // points in chunks of 16 on host threads (each point's values are its own)
    const int nch = (npts + 15) / 16;
    parallel_for(nch, [&](int ch) {
      for (int t = ch * 16; t < std::min(npts, ch * 16 + 16); ++t)
        for (int comp = 0; comp < c; ++comp)
          for (int b = 0; b < n; ++b) {
            const double *crow = coef.a.data() + (size_t(comp * n + b) * m);
            const double vb = V[size_t(t) * n + b];
            double *vo = vals.data() + ((size_t(t) * c + comp) * m);
            for (int j = 0; j < m; ++j) vo[j] += vb * crow[j];
            for (int a = 0; a < l; ++a) {
              const double gb = G[(size_t(t) * l + a) * n + b];
              double *jo = jac.data() + (((size_t(t) * c + comp) * l + a) * m);
              for (int j = 0; j < m; ++j) jo[j] += gb * crow[j];
            }
          }
    });
  }
};

// exterior derivative on an l-simplex in its own coordinates: (npts x c' x m)
int dcomp(int k, int l) { return k == 0 ? l : (k == 1 && l == 3 ? 3 : 1); }

void d_op(int k, int l, int c, int npts, int m, const std::vector<double> &jac, std::vector<double> &out) {
  const int co = dcomp(k, l);
  out.assign(size_t(npts) * co * m, 0.0);
  auto J = [&](int t, int comp, int a, int j) { return jac[((size_t(t) * c + comp) * l + a) * m + j]; };
  for (int t = 0; t < npts; ++t)
    for (int j = 0; j < m; ++j) {
      double *o = out.data() + (size_t(t) * co * m + j);
      if (k == 0) {
        for (int a = 0; a < l; ++a) o[a * m] = J(t, 0, a, j);
      } else if (k == 1 && l == 2) {
        o[0] = J(t, 1, 0, j) - J(t, 0, 1, j);
      } else if (k == 1 && l == 3) {
        o[0] = J(t, 2, 1, j) - J(t, 1, 2, j);
        o[m] = J(t, 0, 2, j) - J(t, 2, 0, j);
        o[2 * m] = J(t, 1, 0, j) - J(t, 0, 1, j);
      } else if (k == 2 && l == 3) {
        o[0] = J(t, 0, 0, j) + J(t, 1, 1, j) + J(t, 2, 2, j);
      } else {
        throw std::runtime_error("d_op: unsupported (k, l)");
      }
    }
}

std::map<std::array<int, 3>, std::shared_ptr<Space>> &space_cache() {
  static std::map<std::array<int, 3>, std::shared_ptr<Space>> c;
  return c;
}

std::shared_ptr<Space> make_space(int l, Family fam, int p) {
  auto key = std::array<int, 3>{l, int(fam), p};
  auto &cache = space_cache();
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  auto sp = std::make_shared<Space>();
  sp->l = l;
  sp->p = p;
  sp->fam = fam;
  sp->poly = PolyBasis(l, p);
  const int n = sp->poly.n;
  if (fam == FAM_CG) {
    sp->c = 1;
    sp->B = Dense::eye(n);
  } else if (fam == FAM_NEDTWO || fam == FAM_BDM) {  // second kind: all of P_p^l
    sp->c = l;
    sp->B = Dense::eye(l * n);
  } else {
    const int c = l;
    sp->c = c;
    std::vector<int> low;
    for (int b = 0; b < n; ++b)
      if (sp->poly.degree[b] <= p - 1) low.push_back(b);
    Quad q = simplex_quad(l, p + 2);
    const int nq = q.size();
    std::vector<double> V(size_t(nq) * n);
    sp->poly.eval(q.x.data(), nq, V.data(), nullptr);
    std::vector<std::vector<double>> cols;
    for (int comp = 0; comp < c; ++comp)
      for (int b : low) {
        std::vector<double> e(c * n, 0.0);
        e[comp * n + b] = 1.0;
        cols.push_back(e);
      }
    // extra fields f (nq x c): the x-dependent generators, projected on P_p^c
    auto project = [&](const std::vector<double> &f) {
      std::vector<double> coef(c * n, 0.0);
      for (int t = 0; t < nq; ++t)
        for (int comp = 0; comp < c; ++comp) {
          const double fv = f[size_t(t) * c + comp] * q.w[t];
          for (int b = 0; b < n; ++b) coef[comp * n + b] += fv * V[size_t(t) * n + b];
        }
      cols.push_back(coef);
    };
    for (int b : low) {
      if (fam == FAM_NED && l == 3) {
        for (int comp = 0; comp < 3; ++comp) {
          std::vector<double> f(size_t(nq) * 3);
          for (int t = 0; t < nq; ++t) {
            double g[3] = {0, 0, 0};
            g[comp] = V[size_t(t) * n + b];
            const double *x = q.x.data() + (size_t(t) * 3);
            f[t * 3 + 0] = g[1] * x[2] - g[2] * x[1];
            f[t * 3 + 1] = g[2] * x[0] - g[0] * x[2];
            f[t * 3 + 2] = g[0] * x[1] - g[1] * x[0];
          }
          project(f);
        }
      } else if (fam == FAM_NED && l == 2) {
        std::vector<double> f(size_t(nq) * 2);
        for (int t = 0; t < nq; ++t) {
          const double vb = V[size_t(t) * n + b];
          f[t * 2 + 0] = -q.x[t * 2 + 1] * vb;
          f[t * 2 + 1] = q.x[t * 2 + 0] * vb;
        }
        project(f);
      } else if (fam == FAM_RT && l == 3) {
        std::vector<double> f(size_t(nq) * 3);
        for (int t = 0; t < nq; ++t)
          for (int a = 0; a < 3; ++a) f[t * 3 + a] = q.x[t * 3 + a] * V[size_t(t) * n + b];
        project(f);
      } else {
        throw std::runtime_error("unsupported space");
      }
    }
    Dense S(c * n, int(cols.size()));
    for (int j = 0; j < S.c; ++j)
      for (int i = 0; i < S.r; ++i) S(i, j) = cols[j][i];
    sp->B = orth_range(S, space_dim(l, fam, p));
  }
  cache[key] = sp;
  return sp;
}

// --------------------------------------------------------- subentity maps
struct EntityMap {
  std::vector<double> origin;  // d
  Dense A;                     // d x l
  std::vector<double> y0;      // l
};

EntityMap entity_map(int d, const std::vector<int> &verts) {
  const int l = int(verts.size()) - 1;
  const Simplex &T = simplex(d);
  EntityMap em;
  em.origin.assign(T.V.begin() + verts[0] * d, T.V.begin() + verts[0] * d + d);
  em.A = Dense(d, l);
  if (l == 0) return em;
  const Simplex &S = simplex(l);
  em.y0.assign(S.V.begin(), S.V.begin() + l);
  Dense Ed(d, l);
  for (int m = 0; m < l; ++m)
    for (int a = 0; a < d; ++a) Ed(a, m) = T.V[verts[m + 1] * d + a] - T.V[verts[0] * d + a];
  em.A = matmul(Ed, S.Einv);
  return em;
}

std::vector<double> map_points(const EntityMap &em, const Quad &q, int d) {
  const int l = em.A.c;
  std::vector<double> x(size_t(q.size()) * d);
  for (int t = 0; t < q.size(); ++t)
    for (int a = 0; a < d; ++a) {
      double s = em.origin[a];
      for (int m = 0; m < l; ++m) s += em.A(a, m) * (q.x[size_t(t) * l + m] - em.y0[m]);
      x[size_t(t) * d + a] = s;
    }
  return x;
}

std::vector<std::vector<std::vector<int>>> entities(int d) {
  std::vector<std::vector<std::vector<int>>> out(d + 1);
  for (int l = 0; l <= d; ++l) {
    std::vector<int> sel(l + 1);
    for (int i = 0; i <= l; ++i) sel[i] = i;
    while (true) {
      out[l].push_back(sel);
      int i = l;
      while (i >= 0 && sel[i] == d - l + i) --i;
      if (i < 0) break;
      ++sel[i];
      for (int j = i + 1; j <= l; ++j) sel[j] = sel[j - 1] + 1;
    }
  }
  return out;
}

// trace of a k-form field (npts x c x m) on a subsimplex with frame A (d x l):
// value (k=0), tangential components A^T v (k=1), normal n.v (k=2 on a face)
void trace(int k, const Dense &A, int npts, int c, int m, const std::vector<double> &vals,
           std::vector<double> &out, int &cout_) {
  const int d = A.r, l = A.c;
  if (k == 0 || l == d) {
    out = vals;
    cout_ = c;
    return;
  }
  if (k == 1) {
    cout_ = l;
    out.assign(size_t(npts) * l * m, 0.0);
    for (int t = 0; t < npts; ++t)
      for (int b = 0; b < l; ++b)
        for (int a = 0; a < d; ++a) {
          const double w = A(a, b);
          const double *vi = vals.data() + ((size_t(t) * c + a) * m);
          double *o = out.data() + ((size_t(t) * l + b) * m);
          for (int j = 0; j < m; ++j) o[j] += w * vi[j];
        }
    return;
  }
  if (k == 2 && l == 2 && d == 3) {
    const double nrm[3] = {A(1, 0) * A(2, 1) - A(2, 0) * A(1, 1), A(2, 0) * A(0, 1) - A(0, 0) * A(2, 1),
                           A(0, 0) * A(1, 1) - A(1, 0) * A(0, 1)};
    cout_ = 1;
    out.assign(size_t(npts) * m, 0.0);
    for (int t = 0; t < npts; ++t)
      for (int a = 0; a < 3; ++a) {
        const double *vi = vals.data() + ((size_t(t) * c + a) * m);
        double *o = out.data() + (size_t(t) * m);
        for (int j = 0; j < m; ++j) o[j] += nrm[a] * vi[j];
      }
    return;
  }
  throw std::runtime_error("trace: unsupported");
}

// --------------------------------------------------- bubbles and eigenbases
struct SplitMix64 {
  uint64_t s;
  double next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return double(z >> 11) * (1.0 / 9007199254740992.0);
  }
};

struct Eigen {
  int l = 0, k = 0, N = 0;
  std::shared_ptr<Space> sp;
  Dense Psi;  // primal coefficients (c * n) x N
  std::vector<double> mu;
  double cond_probe = 1.0, min_gap = 1e300;
};

Family kernel_family(Family f, int p, int &pk) {
  pk = p;
  if (f == FAM_NED) return FAM_CG;
  if (f == FAM_NEDTWO) { pk = p + 1; return FAM_CG; }
  if (f == FAM_RT) return FAM_NEDTWO;
  if (f == FAM_BDM) { pk = p + 1; return FAM_NEDTWO; }  // NedTwo_{p+1} for BDM_p
  return FAM_CG;
}

std::map<std::array<int, 3>, std::shared_ptr<Eigen>> &eigen_cache() {
  static std::map<std::array<int, 3>, std::shared_ptr<Eigen>> c;
  return c;
}

std::shared_ptr<Eigen> eigenbasis(int l, Family fam, int p) {
  auto key = std::array<int, 3>{l, int(fam), p};
  auto &cache = eigen_cache();
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  auto eb = std::make_shared<Eigen>();
  eb->l = l;
  eb->k = form_of(fam);
  auto sp = make_space(l, fam, p);
  eb->sp = sp;
  const int k = eb->k, c = sp->c, m = sp->B.c;
  // boundary trace moments against P_p on every facet
  std::vector<std::vector<double>> rows;
  auto facets = entities(l)[l - 1];
  for (auto &F : facets) {
    EntityMap em = entity_map(l, F);
    Quad fq = (l - 1 == 0) ? Quad{0, {}, {1.0}} : simplex_quad(l - 1, p + 2);
    std::vector<double> z = (l - 1 == 0) ? em.origin : map_points(em, fq, l);
    const int nq = fq.size();
    std::vector<double> vals, jac, tr;
    sp->field(z.data(), nq, sp->B, vals, jac);
    int ct = 1;
    trace(k, em.A, nq, c, m, vals, tr, ct);
    PolyBasis test(l - 1, p);
    std::vector<double> T(size_t(nq) * test.n);
    if (l - 1 == 0) T[0] = 1.0;
    else test.eval(fq.x.data(), nq, T.data(), nullptr);
    for (int comp = 0; comp < ct; ++comp)
      for (int b = 0; b < test.n; ++b) {
        std::vector<double> row(m, 0.0);
        for (int t = 0; t < nq; ++t) {
          const double wt = fq.w[t] * T[size_t(t) * test.n + b];
          const double *tv = tr.data() + ((size_t(t) * ct + comp) * m);
          for (int j = 0; j < m; ++j) row[j] += wt * tv[j];
        }
        rows.push_back(row);
      }
  }
  Dense C(int(rows.size()), m);
  for (int i = 0; i < C.r; ++i)
    for (int j = 0; j < m; ++j) C(i, j) = rows[i][j];
  Dense Bb = matmul(sp->B, null_space(C));  // L2-orthonormal bubble basis
  const int nb = Bb.c;
  if (nb == 0) {
    eb->Psi = Dense(sp->B.r, 0);
    cache[key] = eb;
    return eb;
  }
  // augmented eigenproblem: K = (d b_i, d b_j) in the orthonormal basis
  Quad q = simplex_quad(l, p + 2);
  const int nq = q.size();
  std::vector<double> vals, jac, dv;
  sp->field(q.x.data(), nq, Bb, vals, jac);
  d_op(k, l, c, nq, nb, jac, dv);
  const int cd = dcomp(k, l);
  Dense K(nb, nb);
  for (int t = 0; t < nq; ++t)
    for (int comp = 0; comp < cd; ++comp) {
      const double *v = dv.data() + ((size_t(t) * cd + comp) * nb);
      for (int i = 0; i < nb; ++i) {
        const double wi = q.w[t] * v[i];
        for (int j = 0; j < nb; ++j) K(i, j) += wi * v[j];
      }
    }
  std::vector<double> mu;
  Dense W;
  sym_eig(K, mu, W);
  int n_ker = 0;
  if (k > 0) {
    int pk;
    Family kf = kernel_family(fam, p, pk);
    n_ker = eigenbasis(l, kf, pk)->N;
  }
  const double mu_max = mu.back();
  for (int i = 0; i < n_ker; ++i)
    if (std::fabs(mu[i]) > 1e-10 * mu_max) throw std::runtime_error("bubble kernel is not null");
  if (n_ker < nb && mu[n_ker] < 1e-8 * mu_max) throw std::runtime_error("bubble kernel dimension mismatch");
  // clusters of equal mu and their canonical rotation
  std::vector<int> keep;
  for (int i = n_ker; i < nb; ++i) keep.push_back(i);
  Dense Wc(nb, int(keep.size()));
  std::vector<double> mu_out;
  int i0 = 0;
  const int nk = int(keep.size());
  while (i0 < nk) {
    int i1 = i0 + 1;
    while (i1 < nk && (mu[keep[i1]] - mu[keep[i1 - 1]]) < kClusterTol * mu[keep[i1]]) ++i1;
    if (i1 < nk) eb->min_gap = std::min(eb->min_gap, (mu[keep[i1]] - mu[keep[i1 - 1]]) / mu[keep[i1]]);
    const int mm = i1 - i0;
    Dense Wblk(nb, mm);
    for (int r = 0; r < nb; ++r)
      for (int j = 0; j < mm; ++j) Wblk(r, j) = W(r, keep[i0 + j]);
    // probe values Y_ij = e_i . w_j(z_i)
    SplitMix64 rng{uint64_t(0x5EED0000) + uint64_t(256 * l + c)};
    const Simplex &S = simplex(l);
    std::vector<double> pts(size_t(mm) * l), dirs(size_t(mm) * c, 1.0);
    for (int i = 0; i < mm; ++i) {
      std::vector<double> u(l + 1);
      double su = 0;
      for (int a = 0; a <= l; ++a) { u[a] = 0.25 + rng.next(); su += u[a]; }
      for (int a = 0; a < l; ++a) {
        double s = 0;
        for (int v = 0; v <= l; ++v) s += u[v] / su * S.V[v * l + a];
        pts[size_t(i) * l + a] = s;
      }
      if (c > 1)
        for (int a = 0; a < c; ++a) dirs[size_t(i) * c + a] = 2.0 * rng.next() - 1.0;
    }
    Dense coefb = matmul(Bb, Wblk);
    std::vector<double> pv, pj;
    sp->field(pts.data(), mm, coefb, pv, pj);
    Dense Y(mm, mm);
    for (int i = 0; i < mm; ++i)
      for (int j = 0; j < mm; ++j) {
        double s = 0;
        for (int a = 0; a < c; ++a) s += dirs[size_t(i) * c + a] * pv[(size_t(i) * c + a) * mm + j];
        Y(i, j) = s;
      }
    Dense YYt = matmul(Y, transpose(Y));
    std::vector<double> ev;
    Dense EV;
    sym_eig(YYt, ev, EV);
    if (ev[0] <= 0) throw std::runtime_error("degenerate canonicalisation probe");
    eb->cond_probe = std::max(eb->cond_probe, std::sqrt(ev.back() / ev[0]));
    Dense isq(mm, mm);
    for (int a = 0; a < mm; ++a)
      for (int b = 0; b < mm; ++b) {
        double s = 0;
        for (int e = 0; e < mm; ++e) s += EV(a, e) * EV(b, e) / std::sqrt(ev[e]);
        isq(a, b) = s;
      }
    Dense Rrot = matmul(transpose(Y), isq);
    Dense Wr = matmul(Wblk, Rrot);
    for (int j = 0; j < mm; ++j) {
      double rq = 0;
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) rq += Wr(a, j) * K(a, b) * Wr(b, j);
      const double s = 1.0 / std::sqrt(rq);
      for (int r = 0; r < nb; ++r) Wc(r, i0 + j) = Wr(r, j) * s;
      mu_out.push_back(rq);
    }
    i0 = i1;
  }
  eb->Psi = matmul(Bb, Wc);
  eb->mu = mu_out;
  eb->N = int(mu_out.size());
  cache[key] = eb;
  return eb;
}

// values of d_S psi (npts x c' x N) at points y of the l-simplex
void eigen_dvalues(const Eigen &eb, const std::vector<double> &y, int npts, std::vector<double> &dv) {
  std::vector<double> vals, jac;
  eb.sp->field(y.data(), npts, eb.Psi, vals, jac);
  d_op(eb.k, eb.l, eb.sp->c, npts, eb.N, jac, dv);
}

}  // namespace

void eq_vertices(int d, double *out) { eq_vertices_impl(d, out); }

namespace {
std::mutex &build_mutex() {
  static std::mutex mtx;
  return mtx;
}

// The element's dofs as functionals on the primal coefficients of its space
// (rows of L, in the element's dof order) and the dual basis in primal
// coefficients; `el` (if given) receives the dof list and the counts.
struct DualBasis {
  std::shared_ptr<Space> sp;
  Dense L, coef;
};

DualBasis dual_basis(int d, Family fam, int p, RefElement *el) {
  const int k = form_of(fam);
  auto sp = make_space(d, fam, p);
  const int c = sp->c, nfull = sp->B.r;
  std::vector<std::vector<double>> rows;
  RefElement scratch;
  RefElement &E = el ? *el : scratch;
  E.per_entity.assign(d + 1, 0);
  E.kind_start.assign(3 * (d + 1), -1);
  int p2 = p;  // the type-II family and degree: the next-lower space of the sequence
  const Family typeII = kernel_family(fam, p, p2);
  auto ents = entities(d);
  double cond = 1.0, gap = 1e300;
  for (int l = 0; l <= d; ++l) {
    for (int ei = 0; ei < int(ents[l].size()); ++ei) {
      EntityMap em = entity_map(d, ents[l][ei]);
      Quad q = (l == 0) ? Quad{0, {}, {1.0}} : simplex_quad(l, p + 2);
      std::vector<double> x = (l == 0) ? em.origin : map_points(em, q, d);
      const int nq = q.size();
      std::vector<double> vals, jac;
      sp->field_primal(x.data(), nq, vals, jac);  // the functionals act on the primal basis
      int count = 0;
      auto add_row = [&](const std::vector<double> &fn, const std::vector<double> &tr, int ct, int j) {
        // fn: (nq x ct) test values; tr: (nq x ct x nfull)
        std::vector<double> row(nfull, 0.0);
        for (int t = 0; t < nq; ++t)
          for (int a = 0; a < ct; ++a) {
            const double wv = q.w[t] * fn[size_t(t) * ct + a];
            const double *tv = tr.data() + ((size_t(t) * ct + a) * nfull);
            for (int b = 0; b < nfull; ++b) row[b] += wv * tv[b];
          }
        rows.push_back(row);
        (void)j;
      };
      // the rows of the N functionals (d_S psi_j, tr)_S of one eigenbasis, on
      // host threads (each row's sums run in the same order as add_row's)
      auto add_rows = [&](const std::vector<double> &dpsi, int N, const std::vector<double> &tr, int ct) {
        std::vector<std::vector<double>> blk(N);
        parallel_for(N, [&](int j) {
          std::vector<double> row(nfull, 0.0);
          for (int t = 0; t < nq; ++t)
            for (int a = 0; a < ct; ++a) {
              const double wv = q.w[t] * dpsi[(size_t(t) * ct + a) * N + j];
              const double *tv = tr.data() + ((size_t(t) * ct + a) * nfull);
              for (int b = 0; b < nfull; ++b) row[b] += wv * tv[b];
            }
          blk[j] = std::move(row);
        });
        for (auto &r : blk) rows.push_back(std::move(r));
      };
      if (l == k) {  // Whitney moment (1, tr v)_S (a point value when k = 0)
        std::vector<double> tr;
        int ct;
        trace(k, em.A, nq, c, nfull, vals, tr, ct);
        std::vector<double> one(nq, 1.0);
        add_row(one, tr, 1, 0);
        E.dofs.push_back({l, ei, KIND_W, 0});
        if (ei == 0) E.kind_start[3 * l + KIND_W] = count;
        ++count;
      }
      if (l > k) {  // type-I: (d_S psi_j, tr^{k+1} d v)_S
        auto eb = eigenbasis(l, fam, p);
        cond = std::max(cond, eb->cond_probe);
        gap = std::min(gap, eb->min_gap);
        std::vector<double> dpsi;
        eigen_dvalues(*eb, q.x, nq, dpsi);
        std::vector<double> dv, trdv;
        d_op(k, d, c, nq, nfull, jac, dv);
        int ct;
        trace(k + 1, em.A, nq, dcomp(k, d), nfull, dv, trdv, ct);
        if (ei == 0 && eb->N) E.kind_start[3 * l + KIND_I] = count;
        add_rows(dpsi, eb->N, trdv, ct);
        for (int j = 0; j < eb->N; ++j) {
          E.dofs.push_back({l, ei, KIND_I, j});
          ++count;
        }
      }
      if (k >= 1 && l >= k) {  // type-II: (d_S psi^{k-1}_j, tr v)_S
        auto eb = eigenbasis(l, typeII, p2);
        cond = std::max(cond, eb->cond_probe);
        gap = std::min(gap, eb->min_gap);
        std::vector<double> dpsi;
        eigen_dvalues(*eb, q.x, nq, dpsi);
        std::vector<double> tr;
        int ct;
        trace(k, em.A, nq, c, nfull, vals, tr, ct);
        if (ei == 0 && eb->N) E.kind_start[3 * l + KIND_II] = count;
        add_rows(dpsi, eb->N, tr, ct);
        for (int j = 0; j < eb->N; ++j) {
          E.dofs.push_back({l, ei, KIND_II, j});
          ++count;
        }
      }
      if (ei == 0) E.per_entity[l] = count;
    }
  }
  E.cond_probe = cond;
  E.min_cluster_gap = gap;
  const int n = int(rows.size());
  if (n != sp->B.c) throw std::runtime_error("dof count differs from the space dimension");
  E.n = n;
  DualBasis db;
  db.sp = sp;
  db.L = Dense(n, nfull);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < nfull; ++j) db.L(i, j) = rows[i][j];
  Dense D = matmul(db.L, sp->B);
  db.coef = matmul(sp->B, inverse(D));  // dual basis in primal coefficients
  return db;
}
}  // namespace

RefElement build_reference(int d, Family fam, int p) {
  if (d == 2 && fam == FAM_RT && p >= 1) {
    // 2D RT_p is the quarter turn R v = (v_1, -v_0) of 2D Ned_p (its dofs are
    // the H(curl) ones with n = R t, curl = R grad: the remark after
    // eq:hdiv-dofs): the same dofs and numbering, div R phi = rot phi, and
    // the component mass tables become R_00 <- R_11, R_11 <- R_00, R_01 <- -R_01
    RefElement el = build_reference(2, FAM_NED, p);
    el.fam = FAM_RT;
    const size_t nn = size_t(el.n) * el.n;
    std::vector<double> r00(el.R.begin(), el.R.begin() + nn);
    std::copy(el.R.begin() + nn, el.R.begin() + 2 * nn, el.R.begin());
    std::copy(r00.begin(), r00.end(), el.R.begin() + nn);
    for (size_t i = 2 * nn; i < 3 * nn; ++i) el.R[i] = -el.R[i];
    return el;
  }
  std::lock_guard<std::mutex> lock(build_mutex());
  if (d < 2 || d > 3 || p < 1 || (d == 2 && fam != FAM_CG && fam != FAM_NED))
    throw std::runtime_error("unsupported (dimension, space, degree)");
  RefElement el;
  el.d = d;
  el.fam = fam;
  el.p = p;
  el.k = form_of(fam);
  const int k = el.k;
  DualBasis db = dual_basis(d, fam, p, &el);
  auto sp = db.sp;
  const int c = sp->c;
  const int n = el.n;
  const Dense &coef = db.coef;
  // stacked reference matrices
  Quad q = simplex_quad(d, p + 2);
  const int nq = q.size();
  std::vector<double> vals, jac, dv;
  sp->field(q.x.data(), nq, coef, vals, jac);
  d_op(k, d, c, nq, n, jac, dv);
  const int cd = dcomp(k, d);
  std::vector<std::pair<int, int>> pairs;
  if (d == 3) pairs = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  else pairs = {{0, 0}, {1, 1}, {0, 1}};
  // R_ab = sum_t w_t F_a(t) F_b(t)^T, in 64 x 64 tiles of R (each entry
  // still sums over t in ascending order); the products run on threads
  auto prod = [&](const std::vector<double> &F, int cf, int a, int b) {
    Dense R(n, n);
    constexpr int TB = 64;
    for (int i0 = 0; i0 < n; i0 += TB)
      for (int j0 = 0; j0 < n; j0 += TB) {
        const int i1 = std::min(n, i0 + TB), j1 = std::min(n, j0 + TB);
        for (int t = 0; t < nq; ++t) {
          const double *fa = F.data() + ((size_t(t) * cf + a) * n);
          const double *fb = F.data() + ((size_t(t) * cf + b) * n);
          for (int i = i0; i < i1; ++i) {
            const double wi = q.w[t] * fa[i];
            double *rr = R.a.data() + (size_t(i) * n);
            for (int j = j0; j < j1; ++j) rr[j] += wi * fb[j];
          }
        }
      }
    if (a != b) {
      Dense Rt = transpose(R);
      for (size_t i = 0; i < R.a.size(); ++i) R.a[i] += Rt.a[i];
    }
    return R;
  };
  struct Job {
    const std::vector<double> *F;
    int cf, a, b;
  };
  std::vector<Job> jobs;
  for (const auto *F : {&vals, &dv}) {
    const int cf = F == &vals ? c : cd;
    if (cf == 1) jobs.push_back({F, cf, 0, 0});
    else
      for (auto &pr : pairs) jobs.push_back({F, cf, pr.first, pr.second});
  }
  std::vector<Dense> stack(jobs.size());
  parallel_for(int(jobs.size()), [&](int i) { stack[i] = prod(*jobs[i].F, jobs[i].cf, jobs[i].a, jobs[i].b); });
  el.Q = int(stack.size());
  el.R.resize(size_t(el.Q) * n * n);
  for (int qi = 0; qi < el.Q; ++qi)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)  // exact symmetry
        el.R[(size_t(qi) * n + i) * n + j] = 0.5 * (stack[qi](i, j) + stack[qi](j, i));
  return el;
}

// The exterior derivative X^{k-1}_p -> X^k_p on the reference cell in the two
// bases: D_hat (n_to x n_from), column j the coefficients of d phi_j in the
// X^k basis.  d phi_j lies in X^k_p (the discrete complex is exact), so its
// L2 projection onto the primal polynomial basis of X^k's space (Gram
// system by a rule exact to degree 2p + 3) is d phi_j itself; the X^k dofs
// applied to those coefficients give its expansion.
std::vector<double> derivative_reference(int d, Family from, Family to, int p) {
  std::lock_guard<std::mutex> lock(build_mutex());
  if (d != 3 || form_of(to) != form_of(from) + 1 || from == FAM_NEDTWO || to == FAM_NEDTWO)
    throw std::runtime_error("derivative_reference: needs consecutive first-kind 3D families");
  RefElement ea, eb;
  DualBasis da = dual_basis(d, from, p, &ea), dbb = dual_basis(d, to, p, &eb);
  Quad q = simplex_quad(d, p + 2);
  const int nq = q.size(), na = ea.n, nb = eb.n;
  std::vector<double> vals, jac, dv;
  da.sp->field(q.x.data(), nq, da.coef, vals, jac);
  d_op(form_of(from), d, da.sp->c, nq, na, jac, dv);  // (nq x c' x na)
  const int cd = dcomp(form_of(from), d);
  if (cd != dbb.sp->c) throw std::runtime_error("derivative_reference: component mismatch");
  const int nfull = dbb.sp->B.r;
  std::vector<double> pv, pj;
  dbb.sp->field_primal(q.x.data(), nq, pv, pj);  // primal basis values (nq x c x nfull)
  Dense proj(nfull, na);
  for (int t = 0; t < nq; ++t)
    for (int a = 0; a < cd; ++a) {
      const double *fb = pv.data() + ((size_t(t) * cd + a) * nfull);
      const double *fa = dv.data() + ((size_t(t) * cd + a) * na);
      for (int b = 0; b < nfull; ++b) {
        const double wb = q.w[t] * fb[b];
        if (wb == 0.0) continue;
        for (int j = 0; j < na; ++j) proj(b, j) += wb * fa[j];
      }
    }
  // Gram matrix of the primal basis under the same rule (the identity if
  // the polynomial basis is orthonormal on the reference cell)
  Dense G(nfull, nfull);
  for (int t = 0; t < nq; ++t)
    for (int a = 0; a < cd; ++a) {
      const double *fb = pv.data() + ((size_t(t) * cd + a) * nfull);
      for (int i = 0; i < nfull; ++i) {
        const double wi = q.w[t] * fb[i];
        if (wi == 0.0) continue;
        for (int j = 0; j < nfull; ++j) G(i, j) += wi * fb[j];
      }
    }
  Dense Dh = matmul(dbb.L, matmul(inverse(G), proj));
  std::vector<double> out(size_t(nb) * na);
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < na; ++j) out[size_t(i) * na + j] = Dh(i, j);
  return out;
}

// The divergence RT_p -> DG_{p-1} on the reference cell: n_dg x n_rt with
// entry (i, j) = (div phi_j, psi_i), psi the L2-orthonormal (Dubiner) basis
// of P_{p-1} on the reference cell (the DG_{p-1} basis: div phi_j lies in
// P_{p-1}, so these are its coefficients).
std::vector<double> divergence_reference_dg(int d, int p) {
  std::lock_guard<std::mutex> lock(build_mutex());
  if (d != 3 || p < 1) throw std::runtime_error("divergence_reference_dg: 3D, p >= 1");
  RefElement ea;
  DualBasis da = dual_basis(d, FAM_RT, p, &ea);
  Quad q = simplex_quad(d, p + 2);
  const int nq = q.size(), na = ea.n;
  std::vector<double> vals, jac, dv;
  da.sp->field(q.x.data(), nq, da.coef, vals, jac);
  d_op(2, d, da.sp->c, nq, na, jac, dv);  // (nq x 1 x na)
  PolyBasis pb(d, p - 1);
  std::vector<double> pv(size_t(nq) * pb.n);
  pb.eval(q.x.data(), nq, pv.data(), nullptr);
  std::vector<double> out(size_t(pb.n) * na, 0.0);
  for (int t = 0; t < nq; ++t)
    for (int i = 0; i < pb.n; ++i) {
      const double wi = q.w[t] * pv[size_t(t) * pb.n + i];  // eval applies the normalisation
      for (int j = 0; j < na; ++j) out[size_t(i) * na + j] += wi * dv[size_t(t) * na + j];
    }
  return out;
}

}  // namespace rz
