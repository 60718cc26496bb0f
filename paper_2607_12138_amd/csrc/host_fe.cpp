// Reference elements and reference mass tables (host side).
//
// Route: every integral is a collapsed-coordinate (Duffy) Gauss-Legendre
// quadrature in long double; the element space is spanned by an orthonormal
// basis obtained by Gram-Schmidt of a spanning set; the nodal basis solves
// the degree-of-freedom Vandermonde against that orthonormal basis (well
// conditioned) with pivoted LU; the mass tables are quadratures of nodal
// basis products (eq. piola_mass_pullbacks), rounded to double at the end.
//
// Element definitions (the paper names Firedrake's elements; readings):
//  H1 Lagrange P_p: point values at the recursive Gauss-Lobatto-Legendre
//    nodes (Isaac 2020): on an edge the p+1 GLL points; inside a k-simplex
//    the node of a barycentric multi-index alpha (entries >= 1, sum n) is the
//    average of its facet nodes (alpha without entry i, degree n - alpha_i)
//    weighted by n - alpha_i.
//  N1curl_k = [P_{k-1}]^d + {x x q} (3D) or (-y, x) P~_{k-1} (2D);
//  RT_k = [P_{k-1}]^d + x P~_{k-1}.  Integral moments on sorted-vertex
//    entities x(s) = v_a + s_1 (v_b - v_a) + s_2 (v_c - v_a): edge tangent
//    t = v_b - v_a (N1curl), 2D edge normal (t_y, -t_x) (RT), face normal
//    t_1 x t_2 (RT), face tangents t_1 then t_2 (N1curl), interior
//    components (component-major), each against the orthonormal polynomials
//    of the entity's parameter domain, Gram-Schmidt of monomials ordered by
//    total degree and then by descending exponent tuple.
//  N2curl_k = BDM_k = [P_k]^d with the classical second-kind moments: edge
//    tangents (N2curl) / facet normals (BDM) against P_k as above; N2curl
//    faces (u . t_1) q_1 + (u . t_2) q_2 for (q_1, q_2) in RT_{k-1} of the
//    face parameters; interiors u . q for q in RT_{k-1} (2D N2curl),
//    RT_{k-2} (3D N2curl) or N1curl_{k-1} (BDM).  Those RT / N1curl test
//    fields are monomial spanning fields in a fixed order (see test_fields),
//    orthonormalised in that order on the entity's parameter simplex.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <vector>

#include "internal.h"

namespace {

typedef long double ld;
using bras::fail;

struct Pt { ld x[3]; };

void gauss_legendre01(int n, std::vector<ld>& x, std::vector<ld>& w) {
  x.resize(n);
  w.resize(n);
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    ld t = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    ld dp = 0;
    for (int it = 0; it < 100; ++it) {
      ld p0 = 1, p1 = t;
      for (int k = 2; k <= n; ++k) {
        ld p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1);
      ld step = p1 / dp;
      t -= step;
      if (std::fabs(step) < 1e-21L) break;
    }
    {
      ld p0 = 1, p1 = t;
      for (int k = 2; k <= n; ++k) {
        ld p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1);
    }
    x[i] = (1 - t) / 2;
    w[i] = 1 / ((1 - t * t) * dp * dp);   // 2/((1-t^2)P'^2) on [-1,1], halved for [0,1]
  }
}

// Collapsed Gauss-Legendre rule on conv{0, e_1, .., e_d}, d in {1, 2, 3}.
void simplex_rule(int d, int n, std::vector<Pt>& pts, std::vector<ld>& wts) {
  std::vector<ld> g, w;
  gauss_legendre01(n, g, w);
  pts.clear();
  wts.clear();
  if (d == 1) {
    for (int i = 0; i < n; ++i) {
      Pt p{{g[i], 0, 0}};
      pts.push_back(p);
      wts.push_back(w[i]);
    }
  } else if (d == 2) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        Pt p{{g[i], (1 - g[i]) * g[j], 0}};
        pts.push_back(p);
        wts.push_back(w[i] * w[j] * (1 - g[i]));
      }
  } else {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) {
          Pt p{{g[i], (1 - g[i]) * g[j], (1 - g[i]) * (1 - g[j]) * g[k]}};
          pts.push_back(p);
          wts.push_back(w[i] * w[j] * w[k] * (1 - g[i]) * (1 - g[i]) * (1 - g[j]));
        }
  }
}

typedef std::array<int, 3> Exp;

// Exponents of total degree <= q in d variables: degree ascending, then
// exponent tuples in descending lexicographic order.
std::vector<Exp> monomials(int d, int q, bool homogeneous_only = false) {
  std::vector<Exp> out;
  for (int deg = homogeneous_only ? q : 0; deg <= q; ++deg) {
    std::vector<Exp> blk;
    for (int a = deg; a >= 0; --a) {
      if (d == 1) {
        if (a == deg) blk.push_back({a, 0, 0});
        continue;
      }
      for (int b = deg - a; b >= 0; --b) {
        if (d == 2) {
          if (a + b == deg) blk.push_back({a, b, 0});
          continue;
        }
        int c = deg - a - b;
        blk.push_back({a, b, c});
      }
    }
    out.insert(out.end(), blk.begin(), blk.end());
  }
  return out;
}

ld mono(const Exp& a, const ld* x, int d) {
  ld v = 1;
  for (int i = 0; i < d; ++i)
    for (int k = 0; k < a[i]; ++k) v *= x[i];
  return v;
}

// Values of the orthonormal polynomials of degree <= q on the reference
// k-simplex at the given points, by modified Gram-Schmidt (twice) of the
// ordered monomials under the exact rule `rule_pts`/`rule_w`.
// Returns coefficient matrix R with ON_m = sum_j R[m][j] mono_j.
std::vector<std::vector<ld>> orthonormal_coeffs(int k, int q) {
  std::vector<Exp> mons = monomials(k, q);
  std::vector<Pt> pts;
  std::vector<ld> wts;
  simplex_rule(k, q + 2, pts, wts);
  const int m = (int)mons.size(), np = (int)pts.size();
  std::vector<std::vector<ld>> val(m, std::vector<ld>(np)), R(m, std::vector<ld>(m, 0));
  for (int j = 0; j < m; ++j) {
    for (int p = 0; p < np; ++p) val[j][p] = mono(mons[j], pts[p].x, k);
    R[j][j] = 1;
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        ld c = 0;
        for (int p = 0; p < np; ++p) c += wts[p] * val[i][p] * val[j][p];
        for (int p = 0; p < np; ++p) val[j][p] -= c * val[i][p];
        for (int t = 0; t < m; ++t) R[j][t] -= c * R[i][t];
      }
    ld nrm = 0;
    for (int p = 0; p < np; ++p) nrm += wts[p] * val[j][p] * val[j][p];
    nrm = std::sqrt(nrm);
    for (int p = 0; p < np; ++p) val[j][p] /= nrm;
    for (int t = 0; t < m; ++t) R[j][t] /= nrm;
  }
  return R;
}

ld eval_poly(const std::vector<ld>& coef, const std::vector<Exp>& mons, const ld* x, int k) {
  ld s = 0;
  for (size_t j = 0; j < mons.size(); ++j) s += coef[j] * mono(mons[j], x, k);
  return s;
}

// ---- GLL points and recursive nodes -------------------------------------

std::vector<ld> gll01(int n) {
  std::vector<ld> out;
  out.push_back(0);
  if (n >= 2) {
    // interior points: roots of P_n' on [-1,1], Newton from Chebyshev-Gauss-Lobatto guesses
    const ld pi = 3.141592653589793238462643383279502884L;
    std::vector<ld> in;
    for (int i = 1; i < n; ++i) {
      ld t = -std::cos(pi * i / n);
      for (int it = 0; it < 200; ++it) {
        ld p0 = 1, p1 = t;
        for (int k = 2; k <= n; ++k) {
          ld p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        ld dp = n * (t * p1 - p0) / (t * t - 1);
        ld d2 = (2 * t * dp - n * (n + 1) * p1) / (1 - t * t);
        ld step = dp / d2;
        t -= step;
        if (std::fabs(step) < 1e-21L) break;
      }
      in.push_back((t + 1) / 2);
    }
    std::sort(in.begin(), in.end());
    out.insert(out.end(), in.begin(), in.end());
  }
  out.push_back(1);
  return out;
}

std::vector<ld> rec_full(const std::vector<int>& alpha) {
  int n = 0;
  for (int a : alpha) n += a;
  const int k = (int)alpha.size();
  if (k == 1) return {1};
  if (k == 2) {
    ld g = gll01(n)[alpha[1]];
    return {1 - g, g};
  }
  std::vector<ld> acc(k, 0);
  ld wsum = 0;
  for (int i = 0; i < k; ++i) {
    ld w = n - alpha[i];
    std::vector<int> facet;
    for (int j = 0; j < k; ++j)
      if (j != i) facet.push_back(alpha[j]);
    std::vector<ld> b = rec_full(facet);
    int q = 0;
    for (int j = 0; j < k; ++j)
      if (j != i) acc[j] += w * b[q++];
    wsum += w;
  }
  for (auto& a : acc) a /= wsum;
  return acc;
}

// multi-indices of length k, entries >= 1, sum n, descending lex order
void interior_multi(int k, int n, std::vector<std::vector<int>>& out) {
  out.clear();
  std::vector<int> cur(k, 1);
  std::function<void(int, int)> rec = [&](int pos, int rem) {
    if (pos == k - 1) {
      if (rem >= 1) {
        cur[pos] = rem;
        out.push_back(cur);
      }
      return;
    }
    for (int v = rem - (k - 1 - pos); v >= 1; --v) {
      cur[pos] = v;
      rec(pos + 1, rem - v);
    }
  };
  if (n >= k) rec(0, n);
}

std::vector<std::vector<int>> combos(int nv, int K) {
  std::vector<std::vector<int>> out;
  std::vector<int> cur(K);
  for (int i = 0; i < K; ++i) cur[i] = i;
  while (true) {
    out.push_back(cur);
    int pos = K - 1;
    while (pos >= 0 && cur[pos] == nv - K + pos) --pos;
    if (pos < 0) break;
    ++cur[pos];
    for (int q = pos + 1; q < K; ++q) cur[q] = cur[q - 1] + 1;
  }
  return out;
}

// ---- the element space ---------------------------------------------------

struct Field {           // spanning field: ncomp components, each a single monomial times a coefficient
  std::vector<std::pair<int, Exp>> terms;   // (component, exponent)
  std::vector<ld> coef;
  bool legendre = false;  // exponent a stands for prod_i P_{a_i}(2 x_i - 1) instead of x^a
};

// prod_i P_{a_i}(2 x_i - 1), Legendre polynomials by their three-term recurrence
ld legendre_product(const Exp& a, const ld* x, int d) {
  ld v = 1;
  for (int i = 0; i < d; ++i) {
    const ld t = 2 * x[i] - 1;
    ld p0 = 1, p1 = t;
    if (a[i] == 0) continue;
    for (int n = 2; n <= a[i]; ++n) {
      const ld p2 = ((2 * n - 1) * t * p1 - (n - 1) * p0) / n;
      p0 = p1;
      p1 = p2;
    }
    v *= p1;
  }
  return v;
}

void eval_field(const Field& f, const ld* x, int d, ld* out, int ncomp) {
  for (int c = 0; c < ncomp; ++c) out[c] = 0;
  for (size_t t = 0; t < f.terms.size(); ++t)
    out[f.terms[t].first] += f.coef[t] * (f.legendre ? legendre_product(f.terms[t].second, x, d)
                                                     : mono(f.terms[t].second, x, d));
}

std::vector<Field> spanning_set(int family, int d, int k) {
  std::vector<Field> S;
  // full P_k spaces: products of shifted Legendre polynomials span the same
  // space as the monomials and keep the Gram-Schmidt well conditioned
  if (family == BRAS_H1) {
    for (auto& a : monomials(d, k)) S.push_back(Field{{{0, a}}, {1}, true});
    return S;
  }
  if (family == BRAS_HCURL2 || family == BRAS_HDIV2) {
    for (int c = 0; c < d; ++c)
      for (auto& a : monomials(d, k)) S.push_back(Field{{{c, a}}, {1}, true});
    return S;
  }
  for (int c = 0; c < d; ++c)
    for (auto& a : monomials(d, k - 1)) S.push_back(Field{{{c, a}}, {1}});
  auto hom = monomials(d, k - 1, true);
  if (family == BRAS_HDIV) {
    for (auto& a : hom) {
      Field f;
      for (int c = 0; c < d; ++c) {
        Exp e = a;
        e[c] += 1;
        f.terms.push_back({c, e});
        f.coef.push_back(1);
      }
      S.push_back(f);
    }
  } else if (d == 2) {
    for (auto& a : hom) {
      Exp e0 = a, e1 = a;
      e0[1] += 1;
      e1[0] += 1;
      S.push_back(Field{{{0, e0}, {1, e1}}, {-1, 1}});
    }
  } else {
    // x cross (e_c x^a): (x cross e_c) x^a
    for (auto& a : hom)
      for (int c = 0; c < 3; ++c) {
        Field f;
        // x cross e_0 = (0, x2, -x1); x cross e_1 = (-x2, 0, x0); x cross e_2 = (x1, -x0, 0)
        int i1 = (c + 1) % 3, i2 = (c + 2) % 3;
        // component i1 gets +x_{i2}, component i2 gets -x_{i1}
        Exp ea = a, eb = a;
        ea[i2] += 1;
        eb[i1] += 1;
        f.terms.push_back({i1, ea});
        f.coef.push_back(1);
        f.terms.push_back({i2, eb});
        f.coef.push_back(-1);
        S.push_back(f);
      }
  }
  return S;
}

// Spanning fields of RT_j (rt) or N1curl_j on the m-simplex, the test fields
// of the second-kind moments: [P_{j-1}]^m component-major, then x q (RT),
// (-y q, x q) (2D N1curl) or x cross (e_c q) (3D N1curl: q outer, c inner;
// a field in the span of those kept before it is skipped), q over the
// homogeneous monomials of degree j - 1 in the order of monomials().
std::vector<Field> test_fields(bool rt, int m, int j) {
  std::vector<Field> S;
  if (j < 1) return S;
  // the [P_{j-1}]^m block as Legendre products: in degree order they span the
  // same nested spaces as the monomials (leading coefficients positive), so the
  // orthonormalised fields are the same, with a better conditioned Gram matrix
  for (int c = 0; c < m; ++c)
    for (auto& a : monomials(m, j - 1)) S.push_back(Field{{{c, a}}, {1}, true});
  auto hom = monomials(m, j - 1, true);
  if (rt) {
    for (auto& a : hom) {
      Field f;
      for (int c = 0; c < m; ++c) {
        Exp e = a;
        e[c] += 1;
        f.terms.push_back({c, e});
        f.coef.push_back(1);
      }
      S.push_back(f);
    }
  } else if (m == 2) {
    for (auto& a : hom) {
      Exp e0 = a, e1 = a;
      e0[1] += 1;
      e1[0] += 1;
      S.push_back(Field{{{0, e0}, {1, e1}}, {-1, 1}});
    }
  } else {
    // coefficient vectors over (component, degree-j homogeneous monomial);
    // independence by Gram-Schmidt against the kept ones (entries 0, +-1)
    auto homj = monomials(3, j, true);
    const int nh = (int)homj.size();
    auto col = [&](const Exp& e) {
      for (int i = 0; i < nh; ++i)
        if (homj[i] == e) return i;
      return -1;
    };
    std::vector<std::vector<ld>> basis;
    for (auto& a : hom)
      for (int c = 0; c < 3; ++c) {
        const int i1 = (c + 1) % 3, i2 = (c + 2) % 3;
        Exp ea = a, eb = a;
        ea[i2] += 1;
        eb[i1] += 1;
        std::vector<ld> v(3 * nh, 0);
        v[i1 * nh + col(ea)] = 1;
        v[i2 * nh + col(eb)] = -1;
        std::vector<ld> w = v;
        for (auto& b : basis) {
          ld dot = 0;
          for (int t = 0; t < 3 * nh; ++t) dot += b[t] * w[t];
          for (int t = 0; t < 3 * nh; ++t) w[t] -= dot * b[t];
        }
        ld nn = 0;
        for (ld x : w) nn += x * x;
        nn = std::sqrt(nn);
        if (nn < 1e-9L) continue;
        for (auto& x : w) x /= nn;
        basis.push_back(w);
        S.push_back(Field{{{i1, ea}, {i2, eb}}, {1, -1}});
      }
  }
  return S;
}

struct Functional {       // sum_q w_q (u(x_q) . dir_q) * weight_q  (weights include q_m and quadrature)
  std::vector<Pt> x;
  std::vector<std::array<ld, 3>> dir;   // direction per point (component selector for point values)
};

int build_functionals(int family, int d, int k, std::vector<Functional>& F) {
  F.clear();
  // reference vertices
  ld rv[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  if (family == BRAS_H1) {
    for (int edim = 0; edim <= d; ++edim) {
      for (auto& verts : combos(d + 1, edim + 1)) {
        std::vector<std::vector<int>> idxs;
        if (edim == 0)
          idxs = {{k}};
        else
          interior_multi(edim + 1, k, idxs);
        for (auto& beta : idxs) {
          std::vector<ld> b = rec_full(beta);
          Functional f;
          Pt p{{0, 0, 0}};
          for (size_t v = 0; v < verts.size(); ++v)
            for (int i = 0; i < d; ++i) p.x[i] += b[v] * rv[verts[v]][i];
          f.x.push_back(p);
          f.dir.push_back({1, 0, 0});
          F.push_back(f);
        }
      }
    }
    return BRAS_OK;
  }
  // moment functionals
  auto add_moments = [&](const std::vector<int>& verts, int qdeg, const std::vector<std::array<ld, 3>>& dirs) {
    const int ek = (int)verts.size() - 1;
    std::vector<Pt> pts;
    std::vector<ld> wts;
    simplex_rule(ek, k + 2, pts, wts);
    auto R = orthonormal_coeffs(ek, qdeg);
    auto mons = monomials(ek, qdeg);
    for (auto& dv : dirs)
      for (size_t m = 0; m < R.size(); ++m) {
        Functional f;
        for (size_t p = 0; p < pts.size(); ++p) {
          Pt x{{0, 0, 0}};
          for (int i = 0; i < d; ++i) {
            x.x[i] = rv[verts[0]][i];
            for (int j = 0; j < ek; ++j) x.x[i] += pts[p].x[j] * (rv[verts[j + 1]][i] - rv[verts[0]][i]);
          }
          ld q = eval_poly(R[m], mons, pts[p].x, ek) * wts[p];
          f.x.push_back(x);
          f.dir.push_back({dv[0] * q, dv[1] * q, dv[2] * q});
        }
        F.push_back(f);
      }
  };
  // moments int_entity sum_i (u . dirs_i) q_i of test fields given in the
  // entity's parameter coordinates, orthonormalised in their order on the
  // parameter simplex (modified Gram-Schmidt, twice, on their values at the
  // quadrature points: the moments need no other values)
  auto add_field_moments = [&](const std::vector<int>& verts, const std::vector<Field>& fields,
                               const std::vector<std::array<ld, 3>>& dirs) {
    const int ek = (int)verts.size() - 1;
    const int nf = (int)fields.size();
    if (nf == 0) return;
    std::vector<Pt> pts;
    std::vector<ld> wts;
    simplex_rule(ek, k + 2, pts, wts);
    const int np = (int)pts.size();
    const size_t len = (size_t)np * ek;
    std::vector<std::vector<ld>> q(nf, std::vector<ld>(len));
    auto ip = [&](const std::vector<ld>& a, const std::vector<ld>& b) {
      ld t = 0;
      for (int p = 0; p < np; ++p)
        for (int i = 0; i < ek; ++i) t += wts[p] * a[(size_t)p * ek + i] * b[(size_t)p * ek + i];
      return t;
    };
    for (int a = 0; a < nf; ++a) {
      for (int p = 0; p < np; ++p) eval_field(fields[a], pts[p].x, ek, &q[a][(size_t)p * ek], ek);
      for (int pass = 0; pass < 2; ++pass)
        for (int b = 0; b < a; ++b) {
          const ld c = ip(q[b], q[a]);
          for (size_t t = 0; t < len; ++t) q[a][t] -= c * q[b][t];
        }
      const ld nn = std::sqrt(ip(q[a], q[a]));
      for (auto& x : q[a]) x /= nn;
    }
    for (int a = 0; a < nf; ++a) {
      Functional f;
      for (int p = 0; p < np; ++p) {
        Pt x{{0, 0, 0}};
        for (int i = 0; i < d; ++i) {
          x.x[i] = rv[verts[0]][i];
          for (int j = 0; j < ek; ++j) x.x[i] += pts[p].x[j] * (rv[verts[j + 1]][i] - rv[verts[0]][i]);
        }
        std::array<ld, 3> dir = {0, 0, 0};
        for (int i = 0; i < ek; ++i) {
          const ld v = q[a][(size_t)p * ek + i] * wts[p];
          for (int c = 0; c < 3; ++c) dir[c] += v * dirs[i][c];
        }
        f.x.push_back(x);
        f.dir.push_back(dir);
      }
      F.push_back(f);
    }
  };
  auto sub = [&](int a, int b, int i) { return rv[b][i] - rv[a][i]; };
  if (family == BRAS_HCURL2 || family == BRAS_HDIV2) {
    const bool curl = family == BRAS_HCURL2;
    if (d == 2 || curl)
      for (auto& e : combos(d + 1, 2)) {
        std::array<ld, 3> t = {sub(e[0], e[1], 0), sub(e[0], e[1], 1), d == 3 ? sub(e[0], e[1], 2) : 0};
        add_moments(e, k, {curl ? t : std::array<ld, 3>{t[1], -t[0], 0}});
      }
    if (d == 3)
      for (auto& f : combos(4, 3)) {
        std::array<ld, 3> t1 = {sub(f[0], f[1], 0), sub(f[0], f[1], 1), sub(f[0], f[1], 2)};
        std::array<ld, 3> t2 = {sub(f[0], f[2], 0), sub(f[0], f[2], 1), sub(f[0], f[2], 2)};
        if (curl) {
          add_field_moments(f, test_fields(true, 2, k - 1), {t1, t2});
        } else {
          std::array<ld, 3> nrm = {t1[1] * t2[2] - t1[2] * t2[1], t1[2] * t2[0] - t1[0] * t2[2],
                                   t1[0] * t2[1] - t1[1] * t2[0]};
          add_moments(f, k, {nrm});
        }
      }
    std::vector<int> all;
    for (int i = 0; i <= d; ++i) all.push_back(i);
    std::vector<std::array<ld, 3>> unit = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    unit.resize(d);
    add_field_moments(all, curl ? test_fields(true, d, d == 2 ? k - 1 : k - 2) : test_fields(false, d, k - 1), unit);
    return BRAS_OK;
  }
  if (family == BRAS_HCURL || (family == BRAS_HDIV && d == 2)) {
    for (auto& e : combos(d + 1, 2)) {
      std::array<ld, 3> t = {sub(e[0], e[1], 0), sub(e[0], e[1], 1), d == 3 ? sub(e[0], e[1], 2) : 0};
      std::array<ld, 3> dir = family == BRAS_HCURL ? t : std::array<ld, 3>{t[1], -t[0], 0};
      add_moments(e, k - 1, {dir});
    }
  }
  if (d == 3) {
    for (auto& f : combos(4, 3)) {
      std::array<ld, 3> t1 = {sub(f[0], f[1], 0), sub(f[0], f[1], 1), sub(f[0], f[1], 2)};
      std::array<ld, 3> t2 = {sub(f[0], f[2], 0), sub(f[0], f[2], 1), sub(f[0], f[2], 2)};
      if (family == BRAS_HDIV) {
        std::array<ld, 3> nrm = {t1[1] * t2[2] - t1[2] * t2[1], t1[2] * t2[0] - t1[0] * t2[2],
                                 t1[0] * t2[1] - t1[1] * t2[0]};
        add_moments(f, k - 1, {nrm});
      } else if (k >= 2) {
        add_moments(f, k - 2, {t1, t2});
      }
    }
  }
  int qdeg = (family == BRAS_HDIV || d == 2) ? k - 2 : k - 3;
  if (qdeg >= 0) {
    std::vector<int> all;
    for (int i = 0; i <= d; ++i) all.push_back(i);
    for (int c = 0; c < d; ++c) {
      std::array<ld, 3> e = {0, 0, 0};
      e[c] = 1;
      add_moments(all, qdeg, {e});
    }
  }
  return BRAS_OK;
}

// Pivoted LU solve of A X = B (A n x n, B n x m), in place.
int lu_solve(int n, std::vector<ld>& A, int m, std::vector<ld>& B) {
  std::vector<int> piv(n);
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
    if (std::fabs(A[p * n + c]) < 1e-30L) return -1;
    if (p != c) {
      for (int j = 0; j < n; ++j) std::swap(A[p * n + j], A[c * n + j]);
      for (int j = 0; j < m; ++j) std::swap(B[p * m + j], B[c * m + j]);
    }
    for (int r = c + 1; r < n; ++r) {
      ld f = A[r * n + c] / A[c * n + c];
      if (f == 0) continue;
      for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
      for (int j = 0; j < m; ++j) B[r * m + j] -= f * B[c * m + j];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    for (int j = 0; j < m; ++j) {
      ld s = B[c * m + j];
      for (int t = c + 1; t < n; ++t) s -= A[c * n + t] * B[t * m + j];
      B[c * m + j] = s / A[c * n + c];
    }
  }
  return 0;
}

}  // namespace

// Bernstein reference mass in closed form: on the unit simplex
//   int B_a B_b = (k!)^2 (a+b)! / (a! b! (2k+d)!)
// (multi-index factorials are products over the d+1 barycentric entries),
// in the local order of the Lagrange nodes (vertices, edges, faces, interior;
// an entity's multi-indices in descending lexicographic order).
static void bernstein_mass(int d, int k, double* out) {
  std::vector<std::vector<int>> alphas;
  for (int edim = 0; edim <= d; ++edim)
    for (auto& verts : combos(d + 1, edim + 1)) {
      std::vector<std::vector<int>> idxs;
      if (edim == 0)
        idxs = {{k}};
      else
        interior_multi(edim + 1, k, idxs);
      for (auto& beta : idxs) {
        std::vector<int> a(d + 1, 0);
        for (size_t v = 0; v < verts.size(); ++v) a[verts[v]] = beta[v];
        alphas.push_back(a);
      }
    }
  auto fact = [](int m) {
    ld f = 1;
    for (int i = 2; i <= m; ++i) f *= i;
    return f;
  };
  const int nl = (int)alphas.size();
  for (int i = 0; i < nl; ++i)
    for (int j = 0; j < nl; ++j) {
      ld num = fact(k) * fact(k), den = fact(2 * k + d);
      for (int c = 0; c <= d; ++c) {
        num *= fact(alphas[i][c] + alphas[j][c]);
        den *= fact(alphas[i][c]) * fact(alphas[j][c]);
      }
      out[i * nl + j] = (double)(num / den);
    }
}

extern "C" int bras_reference_mass(int family, int dim, int degree, double* ref_h) {
  bras::clear_error();
  if (!ref_h) return fail(BRAS_EINVAL, "null output pointer");
  int nl, counts[4];
  int st = bras::element_counts(family, dim, degree, &nl, counts);
  if (st) return st;
  if (family == BRAS_H1_BERNSTEIN) {
    bernstein_mass(dim, degree, ref_h);
    return BRAS_OK;
  }
  const int d = dim, k = degree;
  const int ncomp = family == BRAS_H1 ? 1 : d;

  // cell quadrature, exact for degree 2k products
  std::vector<Pt> qp;
  std::vector<ld> qw;
  simplex_rule(d, k + 3, qp, qw);
  const int np = (int)qp.size();

  // orthonormal basis of the space by Gram-Schmidt of the spanning set
  std::vector<Field> S = spanning_set(family, d, k);
  const int ns = (int)S.size();
  std::vector<std::vector<ld>> val(ns, std::vector<ld>((size_t)np * ncomp));
  for (int s = 0; s < ns; ++s)
    for (int p = 0; p < np; ++p) eval_field(S[s], qp[p].x, d, &val[s][(size_t)p * ncomp], ncomp);
  auto ip = [&](const std::vector<ld>& a, const std::vector<ld>& b) {
    ld t = 0;
    for (int p = 0; p < np; ++p)
      for (int c = 0; c < ncomp; ++c) t += qw[p] * a[(size_t)p * ncomp + c] * b[(size_t)p * ncomp + c];
    return t;
  };
  std::vector<std::vector<ld>> onv, onc;   // values at quad points, coefficients over S
  for (int s = 0; s < ns; ++s) {
    std::vector<ld> v = val[s], coef(ns, 0);
    coef[s] = 1;
    ld n0 = std::sqrt(ip(v, v));
    for (int pass = 0; pass < 2; ++pass)
      for (size_t t = 0; t < onv.size(); ++t) {
        ld c = ip(onv[t], v);
        for (size_t q = 0; q < v.size(); ++q) v[q] -= c * onv[t][q];
        for (int q = 0; q < ns; ++q) coef[q] -= c * onc[t][q];
      }
    ld nn = std::sqrt(ip(v, v));
    if (nn < 1e-9L * n0) continue;   // dependent member of the spanning set
    for (auto& x : v) x /= nn;
    for (auto& x : coef) x /= nn;
    onv.push_back(v);
    onc.push_back(coef);
  }
  if ((int)onv.size() != nl) return fail(BRAS_EINVAL, "internal: space dimension %d != %d", (int)onv.size(), nl);

  // functionals applied to the orthonormal basis: V[i][t]
  std::vector<Functional> F;
  build_functionals(family, d, k, F);
  if ((int)F.size() != nl) return fail(BRAS_EINVAL, "internal: %d functionals for %d DOFs", (int)F.size(), nl);
  std::vector<ld> V((size_t)nl * nl, 0);
  std::vector<ld> fv(3);
  for (int i = 0; i < nl; ++i)
    for (size_t p = 0; p < F[i].x.size(); ++p) {
      // value of every spanning field at this point, then combine
      std::vector<ld> sv((size_t)ns * ncomp);
      for (int s = 0; s < ns; ++s) eval_field(S[s], F[i].x[p].x, d, &sv[(size_t)s * ncomp], ncomp);
      for (int t = 0; t < nl; ++t) {
        ld dot = 0;
        for (int c = 0; c < ncomp; ++c) {
          ld u = 0;
          for (int s = 0; s < ns; ++s) u += onc[t][s] * sv[(size_t)s * ncomp + c];
          dot += u * F[i].dir[p][c];
        }
        V[(size_t)i * nl + t] += dot;
      }
    }
  // nodal basis phi_j = sum_t C[t][j] ON_t with V C = I
  std::vector<ld> C((size_t)nl * nl, 0);
  for (int i = 0; i < nl; ++i) C[(size_t)i * nl + i] = 1;
  if (lu_solve(nl, V, nl, C)) return fail(BRAS_EINVAL, "internal: singular DOF Vandermonde");
  // nodal values at quadrature points: phi[j][p][c]
  std::vector<ld> phi((size_t)nl * np * ncomp, 0);
  for (int j = 0; j < nl; ++j)
    for (int t = 0; t < nl; ++t) {
      ld cj = C[(size_t)t * nl + j];
      if (cj == 0) continue;
      for (size_t q = 0; q < (size_t)np * ncomp; ++q) phi[(size_t)j * np * ncomp + q] += cj * onv[t][q];
    }
  if (family == BRAS_H1) {
    for (int i = 0; i < nl; ++i)
      for (int j = 0; j < nl; ++j) {
        ld s = 0;
        for (int p = 0; p < np; ++p) s += qw[p] * phi[(size_t)i * np + p] * phi[(size_t)j * np + p];
        ref_h[(size_t)i * nl + j] = (double)s;
      }
    for (int i = 0; i < nl; ++i)
      for (int j = 0; j < i; ++j) {
        double a = 0.5 * (ref_h[(size_t)i * nl + j] + ref_h[(size_t)j * nl + i]);
        ref_h[(size_t)i * nl + j] = ref_h[(size_t)j * nl + i] = a;
      }
    return BRAS_OK;
  }
  int pidx = 0;
  for (int a = 0; a < d; ++a)
    for (int b = a; b < d; ++b, ++pidx) {
      double* T = ref_h + (size_t)pidx * nl * nl;
      for (int i = 0; i < nl; ++i)
        for (int j = 0; j < nl; ++j) {
          ld s = 0;
          for (int p = 0; p < np; ++p) {
            const ld* fi = &phi[((size_t)i * np + p) * ncomp];
            const ld* fj = &phi[((size_t)j * np + p) * ncomp];
            s += qw[p] * (a == b ? fi[a] * fj[a] : fi[a] * fj[b] + fi[b] * fj[a]);
          }
          T[(size_t)i * nl + j] = (double)s;
        }
      for (int i = 0; i < nl; ++i)
        for (int j = 0; j < i; ++j) {
          double v = 0.5 * (T[(size_t)i * nl + j] + T[(size_t)j * nl + i]);
          T[(size_t)i * nl + j] = T[(size_t)j * nl + i] = v;
        }
    }
  return BRAS_OK;
}
