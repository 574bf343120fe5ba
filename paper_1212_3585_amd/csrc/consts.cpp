// Host-side generator of the reference-element constants (long double).
// Section 2.2: nodal basis at Gauss-Legendre nodes, stencil sets, per-stencil
// reconstruction matrices and the oscillation-indicator matrix Sigma.
// Section 2.3: the time factor of K^1 (time derivative integrated by parts)
// and the derivative matrix used by the dimension-by-dimension products.
#include "consts.hpp"

#include <cmath>

namespace ader {
namespace {

constexpr int kDeg = 2 * kMaxN;  // room for products of two basis polynomials

struct Poly {  // coefficients of t^k, t = xi - 1/2
  long double c[kDeg] = {};
};

Poly mul(const Poly& a, const Poly& b) {
  Poly r;
  for (int i = 0; i < kDeg; ++i)
    for (int j = 0; i + j < kDeg; ++j) r.c[i + j] += a.c[i] * b.c[j];
  return r;
}

Poly deriv(const Poly& a) {
  Poly r;
  for (int k = 1; k < kDeg; ++k) r.c[k - 1] = a.c[k] * k;
  return r;
}

long double eval(const Poly& a, long double xi) {
  long double t = xi - 0.5L, r = 0;
  for (int k = kDeg - 1; k >= 0; --k) r = r * t + a.c[k];
  return r;
}

// exact integral over [x0, x1] (in xi) from the antiderivative
long double integral(const Poly& a, long double x0, long double x1) {
  long double t0 = x0 - 0.5L, t1 = x1 - 0.5L, r = 0;
  for (int k = 0; k < kDeg; ++k) {
    r += a.c[k] * (std::pow(t1, (long double)(k + 1)) -
                   std::pow(t0, (long double)(k + 1))) / (k + 1);
  }
  return r;
}

// Gauss-Legendre nodes/weights on [0, 1] (ascending)
void gauss_legendre(int n, long double* x, long double* w) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double y = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    long double dp = 1;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = y;  // P_0, P_1
      if (n == 0) p1 = 1;
      for (int k = 2; k <= n; ++k) {
        long double p2 = ((2 * k - 1) * y * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // P_n(y) = p1, P_{n-1}(y) = p0
      dp = n * (y * p1 - p0) / (y * y - 1);
      long double dy = p1 / dp;
      y -= dy;
      if (std::fabs(dy) < 1e-30L) break;
    }
    // recompute the derivative at the converged root
    long double p0 = 1, p1 = y;
    for (int k = 2; k <= n; ++k) {
      long double p2 = ((2 * k - 1) * y * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (y * p1 - p0) / (y * y - 1);
    // y runs from near +1 downwards; map to ascending xi = (1 - y) / 2
    x[i] = 0.5L * (1 - y);
    w[i] = 1.0L / ((1 - y * y) * dp * dp);  // 2/((1-y^2)P'^2) scaled by 1/2
  }
}

bool invert(int n, const long double (*a)[kMaxN], long double (*inv)[kMaxN]) {
  long double m[kMaxN][2 * kMaxN];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j)
      m[i][j] = j < n ? a[i][j] : (j - n == i ? 1.0L : 0.0L);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(m[r][col]) > std::fabs(m[piv][col])) piv = r;
    if (std::fabs(m[piv][col]) < 1e-30L) return false;
    if (piv != col)
      for (int j = 0; j < 2 * n; ++j) {
        long double t = m[col][j];
        m[col][j] = m[piv][j];
        m[piv][j] = t;
      }
    long double d = m[col][col];
    for (int j = 0; j < 2 * n; ++j) m[col][j] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      long double f = m[r][col];
      for (int j = 0; j < 2 * n; ++j) m[r][j] -= f * m[col][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) inv[i][j] = m[i][n + j];
  return true;
}

// Lagrange basis psi_l(xi) = prod_{k != l} (xi - x_k) / (x_l - x_k)
void lagrange(int n, const long double* nodes, Poly* psi) {
  for (int l = 0; l < n; ++l) {
    Poly p;
    p.c[0] = 1;
    for (int k = 0; k < n; ++k) {
      if (k == l) continue;
      Poly f;  // (t - t_k) / (x_l - x_k) with t_k = x_k - 1/2
      long double den = nodes[l] - nodes[k];
      f.c[0] = -(nodes[k] - 0.5L) / den;
      f.c[1] = 1.0L / den;
      p = mul(p, f);
    }
    psi[l] = p;
  }
}

}  // namespace

bool build_amr_tables(int M, int r, AmrTables* out) {
  if (M < 0 || M + 1 > kMaxN || r < 2 || r > kMaxR) return false;
  AmrTables& t = *out;
  t = AmrTables();
  t.M = M;
  t.r = r;
  const int n = M + 1;
  long double x[kMaxN], w[kMaxN];
  gauss_legendre(n, x, w);
  if (n == 1) x[0] = 0.5L;
  Poly psi[kMaxN];
  lagrange(n, x, psi);
  for (int a = 0; a < r; ++a)
    for (int p = 0; p < n; ++p) {
      t.sub_avg[a][p] = r * integral(psi[p], (long double)a / r, (long double)(a + 1) / r);
      t.at_sub[a][p] = eval(psi[p], (long double)a / r);
      for (int side = 0; side < 2; ++side)
        t.at_face[a][side][p] = eval(psi[p], (long double)(a + side) / r);
      for (int b = 0; b < n; ++b) t.at_nodes[a][b][p] = eval(psi[p], (a + x[b]) / r);
    }
  return true;
}

bool build_ref_constants(int M, RefConstants* out) {
  if (M < 0 || M + 1 > kMaxN) return false;
  RefConstants& c = *out;
  c = RefConstants();
  const int n = M + 1;
  c.M = M;
  c.n = n;
  gauss_legendre(n, c.nodes, c.weights);
  gauss_legendre(kOsherNodes, c.path_s, c.path_w);
  if (n == 1) {
    c.nodes[0] = 0.5L;
    c.weights[0] = 1.0L;
  }

  Poly psi[kMaxN];
  lagrange(n, c.nodes, psi);
  Poly dpsi[kMaxN];
  for (int l = 0; l < n; ++l) dpsi[l] = deriv(psi[l]);

  for (int l = 0; l < n; ++l) {
    c.psi0[l] = eval(psi[l], 0.0L);
    c.psi1[l] = eval(psi[l], 1.0L);
  }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) c.dmat[a][b] = eval(dpsi[b], c.nodes[a]);

  // time factor of K^1: psi_s'(1) psi_s(1) - int_0^1 psi_s'' psi_s (test s')
  for (int sp = 0; sp < n; ++sp)
    for (int s = 0; s < n; ++s)
      c.time_mat[sp][s] = c.psi1[sp] * c.psi1[s] -
                          integral(mul(dpsi[sp], psi[s]), 0.0L, 1.0L);
  long double tinv[kMaxN][kMaxN];
  if (!invert(n, c.time_mat, tinv)) return false;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) c.time_inv_w[i][j] = tinv[i][j] * c.weights[j];

  // stencils (eq. stencildef): even M -> central, left, right;
  // odd M -> two central, left, right
  if (M % 2 == 0) {
    c.nstencils = 3;
    c.stencil_left[0] = M / 2;
    c.lambda[0] = kLambdaCentral;
    c.stencil_left[1] = M;
    c.lambda[1] = kLambdaOneSided;
    c.stencil_left[2] = 0;
    c.lambda[2] = kLambdaOneSided;
  } else {
    c.nstencils = 4;
    c.stencil_left[0] = M / 2 + 1;
    c.lambda[0] = kLambdaCentral;
    c.stencil_left[1] = M / 2;
    c.lambda[1] = kLambdaCentral;
    c.stencil_left[2] = M;
    c.lambda[2] = kLambdaOneSided;
    c.stencil_left[3] = 0;
    c.lambda[3] = kLambdaOneSided;
  }
  for (int s = 0; s < c.nstencils; ++s) {
    long double rec[kMaxN][kMaxN];
    const int L = c.stencil_left[s];
    for (int e = 0; e < n; ++e) {
      const long double o = e - L;  // stencil cell [o, o+1] in home coordinates
      for (int p = 0; p < n; ++p) rec[e][p] = integral(psi[p], o, o + 1);
    }
    if (!invert(n, rec, c.rec_inv[s])) return false;
  }

  // Legendre polynomials orthonormal on [0, 1] (Gram-Schmidt on powers of t)
  Poly leg[kMaxN];
  for (int i = 0; i < n; ++i) {
    Poly p;
    p.c[i] = 1;
    for (int j = 0; j < i; ++j) {
      const long double pr = integral(mul(p, leg[j]), 0.0L, 1.0L);
      for (int k = 0; k < kDeg; ++k) p.c[k] -= pr * leg[j].c[k];
    }
    const long double nrm = std::sqrt(integral(mul(p, p), 0.0L, 1.0L));
    for (int k = 0; k < kDeg; ++k) p.c[k] /= nrm;
    leg[i] = p;
  }
  // coefficient rows of the derivatives in that basis, then composed with
  // each stencil's inverse reconstruction matrix
  long double lrow[kMaxN * (kMaxN - 1) / 2][kMaxN];
  int nr = 0;
  Poly dp[kMaxN];
  for (int l = 0; l < n; ++l) dp[l] = psi[l];
  for (int alpha = 1; alpha <= M; ++alpha) {
    for (int l = 0; l < n; ++l) dp[l] = deriv(dp[l]);
    for (int i = 0; i <= M - alpha; ++i, ++nr)
      for (int p = 0; p < n; ++p) lrow[nr][p] = integral(mul(dp[p], leg[i]), 0.0L, 1.0L);
  }
  c.nsig_rows = nr;
  for (int s = 0; s < c.nstencils; ++s)
    for (int r = 0; r < nr; ++r)
      for (int e = 0; e < n; ++e) {
        long double acc = 0;
        for (int p = 0; p < n; ++p) acc += lrow[r][p] * c.rec_inv[s][p][e];
        c.sig_rows[s][r][e] = acc;
      }
  return true;
}

}  // namespace ader
