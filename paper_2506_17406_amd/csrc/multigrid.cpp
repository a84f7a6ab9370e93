// Geometric multigrid V-cycle on W^k: host set-up (prolongations, Galerkin
// operators, relaxation data, damping) and a host V-cycle.
//
// Relaxation (the solver diagrams of Sec. 7.1): k = 0 vertex patches of W^0,
// i.e. point-Jacobi; k = 1 Hiptmair-Jacobi, the additive Schwarz method of
// eq:hiptmair-smoothing at lowest order (vertex-hat gradients and Whitney
// edge functions, exact one-dimensional solves); k = 2 edge-star patches of
// W^2.  Each smoothing step is x += omega S (b - A x), omega = 1 / rho with
// rho = (lambda_min + 3 lambda_max) / 4 of S A (the paper's subspace-weight
// rule applied to the smoother), two steps before and after the coarse
// correction; Cholesky (here an explicit inverse) on the coarsest level.
#include "multigrid.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <stdexcept>
#include <string>

#include "linalg.hpp"

namespace rz {

Csr csr_from_triplets(int64_t n_rows, int64_t n_cols, const std::vector<int64_t> &r, const std::vector<int32_t> &c,
                      const std::vector<double> &v) {
  std::vector<int64_t> order(r.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = int64_t(i);
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return r[a] != r[b] ? r[a] < r[b] : c[a] < c[b]; });
  Csr A;
  A.n_rows = n_rows;
  A.n_cols = n_cols;
  A.ptr.assign(n_rows + 1, 0);
  for (size_t q = 0; q < order.size();) {
    const int64_t i = r[order[q]];
    const int32_t j = c[order[q]];
    double s = 0.0;
    while (q < order.size() && r[order[q]] == i && c[order[q]] == j) s += v[order[q++]];
    A.col.push_back(j);
    A.val.push_back(s);
    ++A.ptr[i + 1];
  }
  for (int64_t i = 0; i < n_rows; ++i) A.ptr[i + 1] += A.ptr[i];
  return A;
}

Csr csr_transpose(const Csr &A) {
  Csr T;
  T.n_rows = A.n_cols;
  T.n_cols = A.n_rows;
  T.ptr.assign(T.n_rows + 1, 0);
  for (int32_t j : A.col) ++T.ptr[j + 1];
  for (int64_t i = 0; i < T.n_rows; ++i) T.ptr[i + 1] += T.ptr[i];
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  std::vector<int64_t> fill(T.ptr.begin(), T.ptr.end() - 1);
  for (int64_t i = 0; i < A.n_rows; ++i)
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
      const int64_t q = fill[A.col[e]]++;
      T.col[q] = int32_t(i);
      T.val[q] = A.val[e];
    }
  return T;
}

Csr csr_multiply(const Csr &A, const Csr &B) {
  if (A.n_cols != B.n_rows) throw std::runtime_error("csr_multiply shape");
  Csr C;
  C.n_rows = A.n_rows;
  C.n_cols = B.n_cols;
  C.ptr.assign(C.n_rows + 1, 0);
  std::vector<double> acc(B.n_cols, 0.0);
  std::vector<int64_t> mark(B.n_cols, -1);
  std::vector<int32_t> cols;
  for (int64_t i = 0; i < A.n_rows; ++i) {
    cols.clear();
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
      for (int64_t f = B.ptr[A.col[e]]; f < B.ptr[A.col[e] + 1]; ++f) {
        const int32_t j = B.col[f];
        if (mark[j] != i) {
          mark[j] = i;
          acc[j] = 0.0;
          cols.push_back(j);
        }
        acc[j] += A.val[e] * B.val[f];
      }
    std::sort(cols.begin(), cols.end());
    for (int32_t j : cols) {
      C.col.push_back(j);
      C.val.push_back(acc[j]);
    }
    C.ptr[i + 1] = int64_t(C.col.size());
  }
  return C;
}

void csr_apply(const Csr &A, const double *x, double *y) {
  for (int64_t i = 0; i < A.n_rows; ++i) {
    double s = 0.0;
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) s += A.val[e] * x[A.col[e]];
    y[i] = s;
  }
}

namespace {

// barycentric coordinates lam(x) = L [x; 1] of a simplex (d + 1 vertices
// in d dimensions, coordinates with stride d)
Dense barycentric(int d, const double *X, const int64_t *v) {
  Dense M(d + 1, d + 1);
  for (int a = 0; a <= d; ++a) {
    for (int b = 0; b < d; ++b) M(b, a) = X[v[a] * d + b];
    M(d, a) = 1.0;
  }
  return inverse(M);
}

// the Whitney k-form of the local vertex tuple loc at x (d components for
// k = 1, 3 for k = 2)
void whitney_at(int d, int k, const Dense &L, const int *loc, const double *x, double *out) {
  double lam[4], g[4][3] = {};
  for (int a = 0; a <= d; ++a) {
    lam[a] = L(a, d);
    for (int b = 0; b < d; ++b) {
      lam[a] += L(a, b) * x[b];
      g[a][b] = L(a, b);
    }
  }
  auto cross = [](const double *u, const double *v, double *w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  if (k == 0) {
    out[0] = lam[loc[0]];
  } else if (k == 1) {
    const int a = loc[0], b = loc[1];
    for (int i = 0; i < d; ++i) out[i] = lam[a] * g[b][i] - lam[b] * g[a][i];
  } else {
    const int a = loc[0], b = loc[1], c = loc[2];
    double t1[3], t2[3], t3[3];
    cross(g[b], g[c], t1);
    cross(g[c], g[a], t2);
    cross(g[a], g[b], t3);
    for (int i = 0; i < 3; ++i) out[i] = 2.0 * (lam[a] * t1[i] + lam[b] * t2[i] + lam[c] * t3[i]);
  }
}

std::vector<std::vector<int>> subsets(int n, int m) {
  std::vector<std::vector<int>> out;
  std::vector<int> cur;
  std::function<void(int)> rec = [&](int s) {
    if (int(cur.size()) == m) {
      out.push_back(cur);
      return;
    }
    for (int i = s; i < n; ++i) {
      cur.push_back(i);
      rec(i + 1);
      cur.pop_back();
    }
  };
  rec(0);
  return out;
}

}  // namespace

Csr whitney_prolongation(int k, const Topology &tf, const double *Xf, const Topology &tc, const double *Xc) {
  const int d = tf.d, nv = tf.d + 1;
  if (tc.d != d || (d != 2 && d != 3) || k < 0 || k >= d)
    throw std::invalid_argument("the multigrid hierarchy is built for triangle and tetrahedral meshes");
  const int64_t nc = tc.n_cells;
  std::vector<Dense> L(nc);
  for (int64_t c = 0; c < nc; ++c) L[c] = barycentric(d, Xc, tc.cells.data() + (c * nv));
  // bucket grid over the coarse cells' bounding boxes
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < tc.n_vertices; ++v)
    for (int b = 0; b < d; ++b) lo[b] = std::min(lo[b], Xc[v * d + b]), hi[b] = std::max(hi[b], Xc[v * d + b]);
  const int G = std::max(1, d == 3 ? int(std::cbrt(double(nc) / 6.0) + 0.5) : int(std::sqrt(double(nc) / 2.0) + 0.5));
  auto bucket = [&](double x, int b) {
    const double t = (x - lo[b]) / std::max(1e-300, hi[b] - lo[b]) * G;
    return std::min(G - 1, std::max(0, int(std::floor(t))));
  };
  const size_t G2 = d == 3 ? size_t(G) : 1;  // extent of the third axis
  std::vector<std::vector<int64_t>> cells_in(size_t(G) * G * G2);
  for (int64_t c = 0; c < nc; ++c) {
    int b0[3] = {0, 0, 0}, b1[3] = {0, 0, 0};
    for (int b = 0; b < d; ++b) {
      double mn = 1e300, mx = -1e300;
      for (int a = 0; a < nv; ++a) mn = std::min(mn, Xc[tc.cells[c * nv + a] * d + b]), mx = std::max(mx, Xc[tc.cells[c * nv + a] * d + b]);
      b0[b] = bucket(mn - 1e-12, b);
      b1[b] = bucket(mx + 1e-12, b);
    }
    for (int i = b0[0]; i <= b1[0]; ++i)
      for (int j = b0[1]; j <= b1[1]; ++j)
        for (int l = b0[2]; l <= b1[2]; ++l) cells_in[(size_t(l) * G + j) * G + i].push_back(c);
  }
  const auto loc_sets = subsets(nv, k + 1);
  const int nsub = int(loc_sets.size());
  std::vector<int64_t> rows;
  std::vector<int32_t> cols;
  std::vector<double> vals;
  for (int64_t e = 0; e < tf.n_ent[k]; ++e) {
    const int64_t *tup = tf.ent[k].data() + (e * (k + 1));
    double xb[3] = {0, 0, 0};
    for (int a = 0; a <= k; ++a)
      for (int b = 0; b < d; ++b) xb[b] += Xf[tup[a] * d + b] / (k + 1);
    const int bz = d == 3 ? bucket(xb[2], 2) : 0;
    const auto &cand = cells_in[(size_t(bz) * G + bucket(xb[1], 1)) * G + bucket(xb[0], 0)];
    int64_t cell = -1;
    double best = -1e300;
    for (int64_t c : cand) {
      double mn = 1e300;
      for (int a = 0; a < nv; ++a) {
        double l = L[c](a, d);
        for (int b = 0; b < d; ++b) l += L[c](a, b) * xb[b];
        mn = std::min(mn, l);
      }
      if (mn > best) best = mn, cell = c;
    }
    if (cell < 0 || best < -1e-10)
      throw std::invalid_argument("multigrid: a fine entity lies in no cell of the next coarser mesh");
    for (int s = 0; s < nsub; ++s) {
      const int *loc = loc_sets[s].data();
      double w[3], v = 0.0;
      if (k == 0) {
        whitney_at(d, 0, L[cell], loc, &Xf[tup[0] * d], w);
        v = w[0];
      } else if (k == 1) {
        whitney_at(d, 1, L[cell], loc, xb, w);
        for (int b = 0; b < d; ++b) v += w[b] * (Xf[tup[1] * d + b] - Xf[tup[0] * d + b]);
      } else {
        whitney_at(3, 2, L[cell], loc, xb, w);
        double u[3], t[3], n[3];
        for (int b = 0; b < 3; ++b) u[b] = Xf[tup[1] * 3 + b] - Xf[tup[0] * 3 + b], t[b] = Xf[tup[2] * 3 + b] - Xf[tup[0] * 3 + b];
        n[0] = u[1] * t[2] - u[2] * t[1];
        n[1] = u[2] * t[0] - u[0] * t[2];
        n[2] = u[0] * t[1] - u[1] * t[0];
        for (int b = 0; b < 3; ++b) v += w[b] * n[b] / 2.0;
      }
      if (std::fabs(v) > 1e-14) {
        rows.push_back(e);
        cols.push_back(int32_t(tc.cell_ent[k][cell * nsub + s]));
        vals.push_back(v);
      }
    }
  }
  return csr_from_triplets(tf.n_ent[k], tc.n_ent[k], rows, cols, vals);
}

namespace {

void smooth_apply(const MgLevel &lv, int k, const double *r, double *z) {
  const int64_t n = lv.A.n_rows;
  for (int64_t i = 0; i < n; ++i) z[i] = lv.dinv.empty() ? 0.0 : lv.dinv[i] * r[i];
  if (k == 1) {
    std::vector<double> u(lv.Gt.n_rows);
    csr_apply(lv.Gt, r, u.data());
    for (size_t v = 0; v < u.size(); ++v) u[v] *= lv.gdiag[v];
    std::vector<double> t(n);
    csr_apply(lv.G, u.data(), t.data());
    for (int64_t i = 0; i < n; ++i) z[i] += t[i];
  } else if (k == 2) {
    for (int64_t i = 0; i < n; ++i) z[i] = 0.0;
    for (size_t s = 0; s + 1 < lv.star_ptr.size(); ++s) {
      const int64_t f0 = lv.star_ptr[s], m = lv.star_ptr[s + 1] - f0;
      const double *Ainv = &lv.inv[lv.inv_off[s]];
      for (int64_t a = 0; a < m; ++a) {
        double acc = 0.0;
        for (int64_t b = 0; b < m; ++b) acc += Ainv[a * m + b] * r[lv.star_face[f0 + b]];
        z[lv.star_face[f0 + a]] += acc;
      }
    }
  }
}

void cycle(const MgHierarchy &H, size_t l, const double *b, double *x) {
  const int64_t n = H.lev[l].A.n_rows;
  if (l + 1 == H.lev.size()) {
    for (int64_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int64_t j = 0; j < n; ++j) s += H.coarse_inv[i * n + j] * b[j];
      x[i] = s;
    }
    return;
  }
  const MgLevel &lv = H.lev[l];
  std::vector<double> t(n), z(n);
  std::fill(x, x + n, 0.0);
  auto smooth = [&]() {
    csr_apply(lv.A, x, t.data());
    for (int64_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
    smooth_apply(lv, H.k, t.data(), z.data());
    for (int64_t i = 0; i < n; ++i) x[i] += lv.omega * z[i];
  };
  for (int s = 0; s < H.nu; ++s) smooth();
  csr_apply(lv.A, x, t.data());
  for (int64_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
  const int64_t nc = lv.R.n_rows;
  std::vector<double> bc(nc), xc(nc);
  csr_apply(lv.R, t.data(), bc.data());
  cycle(H, l + 1, bc.data(), xc.data());
  csr_apply(lv.P, xc.data(), t.data());
  for (int64_t i = 0; i < n; ++i) x[i] += t[i];
  for (int s = 0; s < H.nu; ++s) smooth();
}

}  // namespace

double lanczos_weight(int64_t n, const std::function<void(const double *, double *)> &applyA,
                      const std::function<void(const double *, double *)> &applyB, uint64_t seed) {
  if (n == 0) return 1.0;
  std::vector<double> r(n), z(n), p(n), q(n);
  uint64_t state = seed;
  for (int64_t i = 0; i < n; ++i) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t zz = state;
    zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ull;
    zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBull;
    zz ^= zz >> 31;
    r[i] = 2.0 * (double(zz >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  }
  auto dot = [&](const std::vector<double> &a, const std::vector<double> &b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
  };
  const double bb = dot(r, r);
  applyB(r.data(), z.data());
  p = z;
  double rz = dot(r, z);
  std::vector<double> al, be;
  for (int it = 0; it < 10 && rz > 0.0; ++it) {
    applyA(p.data(), q.data());
    const double pq = dot(p, q);
    if (!(pq > 0.0)) throw std::runtime_error("weight estimate: p^T A p <= 0");
    const double a = rz / pq;
    al.push_back(a);
    for (int64_t i = 0; i < n; ++i) r[i] -= a * q[i];
    if (dot(r, r) <= 1e-24 * bb) break;
    applyB(r.data(), z.data());
    const double rz_new = dot(r, z);
    be.push_back(rz_new / rz);
    rz = rz_new;
    for (int64_t i = 0; i < n; ++i) p[i] = z[i] + be.back() * p[i];
  }
  const int kk = int(al.size());
  if (kk == 0) return 1.0;
  Dense T(kk, kk);
  for (int j = 0; j < kk; ++j) {
    T(j, j) = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j > 0) T(j, j - 1) = T(j - 1, j) = std::sqrt(be[j - 1]) / al[j - 1];
  }
  std::vector<double> ev;
  Dense V;
  sym_eig(T, ev, V);
  return (ev.front() + 3.0 * ev.back()) / 4.0;
}

MgHierarchy build_multigrid(int k, const Csr &AW, const std::vector<const Topology *> &tops,
                            const std::vector<const double *> &X, int nu) {
  const size_t L = tops.size();
  if (L < 2) throw std::invalid_argument("multigrid needs at least two meshes");
  MgHierarchy H;
  H.k = k;
  H.nu = nu;
  H.lev.resize(L);
  H.lev[0].A = AW;
  for (size_t l = 0; l + 1 < L; ++l) {
    MgLevel &lv = H.lev[l];
    lv.P = whitney_prolongation(k, *tops[l], X[l], *tops[l + 1], X[l + 1]);
    if (lv.P.n_rows != lv.A.n_rows) throw std::invalid_argument("multigrid: level sizes do not match");
    lv.R = csr_transpose(lv.P);
    H.lev[l + 1].A = csr_multiply(lv.R, csr_multiply(lv.A, lv.P));
  }
  for (size_t l = 0; l + 1 < L; ++l) {
    MgLevel &lv = H.lev[l];
    const Topology &t = *tops[l];
    const int64_t n = lv.A.n_rows;
    std::vector<double> diag(n, 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = lv.A.ptr[i]; e < lv.A.ptr[i + 1]; ++e)
        if (lv.A.col[e] == i) diag[i] = lv.A.val[e];
    if (k != 2) {
      lv.dinv.resize(n);
      for (int64_t i = 0; i < n; ++i) lv.dinv[i] = 1.0 / diag[i];
    }
    if (k == 1) {
      std::vector<int64_t> r;
      std::vector<int32_t> c;
      std::vector<double> v;
      for (int64_t e = 0; e < t.n_ent[1]; ++e) {
        r.push_back(e), c.push_back(int32_t(t.ent[1][e * 2])), v.push_back(-1.0);
        r.push_back(e), c.push_back(int32_t(t.ent[1][e * 2 + 1])), v.push_back(1.0);
      }
      lv.G = csr_from_triplets(t.n_ent[1], t.n_vertices, r, c, v);
      lv.Gt = csr_transpose(lv.G);
      // g_v^T A g_v, from the rows of A at the edges of v
      lv.gdiag.assign(t.n_vertices, 0.0);
      std::vector<double> gv(n, 0.0);
      for (int64_t vtx = 0; vtx < t.n_vertices; ++vtx) {
        for (int64_t e = lv.Gt.ptr[vtx]; e < lv.Gt.ptr[vtx + 1]; ++e) gv[lv.Gt.col[e]] = lv.Gt.val[e];
        double s = 0.0;
        for (int64_t e = lv.Gt.ptr[vtx]; e < lv.Gt.ptr[vtx + 1]; ++e) {
          const int32_t i = lv.Gt.col[e];
          for (int64_t f = lv.A.ptr[i]; f < lv.A.ptr[i + 1]; ++f) s += gv[i] * lv.A.val[f] * gv[lv.A.col[f]];
        }
        for (int64_t e = lv.Gt.ptr[vtx]; e < lv.Gt.ptr[vtx + 1]; ++e) gv[lv.Gt.col[e]] = 0.0;
        lv.gdiag[vtx] = 1.0 / s;
      }
    }
    if (k == 2) {
      // the faces of each edge, ascending
      std::map<std::pair<int64_t, int64_t>, int64_t> eid;
      for (int64_t e = 0; e < t.n_ent[1]; ++e) eid[{t.ent[1][e * 2], t.ent[1][e * 2 + 1]}] = e;
      std::vector<std::vector<int32_t>> faces(t.n_ent[1]);
      for (int64_t f = 0; f < t.n_ent[2]; ++f) {
        const int64_t *v = t.ent[2].data() + (f * 3);
        faces[eid.at({v[0], v[1]})].push_back(int32_t(f));
        faces[eid.at({v[0], v[2]})].push_back(int32_t(f));
        faces[eid.at({v[1], v[2]})].push_back(int32_t(f));
      }
      lv.star_ptr.push_back(0);
      for (auto &fl : faces) {
        std::sort(fl.begin(), fl.end());
        const int m = int(fl.size());
        Dense As(m, m);
        for (int a = 0; a < m; ++a)
          for (int64_t e = lv.A.ptr[fl[a]]; e < lv.A.ptr[fl[a] + 1]; ++e) {
            auto it = std::lower_bound(fl.begin(), fl.end(), lv.A.col[e]);
            if (it != fl.end() && *it == lv.A.col[e]) As(a, int(it - fl.begin())) = lv.A.val[e];
          }
        Dense Ai = inverse(As);
        lv.inv_off.push_back(int64_t(lv.inv.size()));
        lv.inv.insert(lv.inv.end(), Ai.a.begin(), Ai.a.end());
        lv.star_face.insert(lv.star_face.end(), fl.begin(), fl.end());
        lv.star_ptr.push_back(int64_t(lv.star_face.size()));
      }
    }
    const double rho = lanczos_weight(
        n, [&](const double *x, double *y) { csr_apply(lv.A, x, y); },
        [&](const double *r, double *z) { smooth_apply(lv, k, r, z); }, 0x5EED3000ull + l);
    lv.omega = 1.0 / rho;
  }
  // the coarsest level: an explicit inverse of the (small) operator
  const Csr &Ac = H.lev[L - 1].A;
  H.n_coarse = Ac.n_rows;
  Dense D(int(Ac.n_rows), int(Ac.n_rows));
  for (int64_t i = 0; i < Ac.n_rows; ++i)
    for (int64_t e = Ac.ptr[i]; e < Ac.ptr[i + 1]; ++e) D(int(i), Ac.col[e]) = Ac.val[e];
  H.coarse_inv = inverse(D).a;
  return H;
}

void mg_cycle_host(const MgHierarchy &H, const double *b, double *x) { cycle(H, 0, b, x); }

}  // namespace rz
