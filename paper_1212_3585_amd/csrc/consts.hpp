// Reference-element constants of the one-step ADER-WENO scheme, built on the
// host in long double at plan creation (Sections 2.2 and 2.3).
//
// Route: Gauss-Legendre nodes by Newton iteration on the three-term Legendre
// recurrence; Lagrange basis polynomials expanded as monomials in the
// centred variable t = xi - 1/2; every integral taken exactly from
// antiderivatives of those monomials; small inverses by Gauss-Jordan
// elimination with partial pivoting.
#pragma once

#include <cstdint>

namespace ader {

constexpr int kMaxN = 4;  // n = M + 1 <= 4  (M <= 3)

constexpr int kOsherNodes = 3;  // path-integral points (the paper asks for >= 2)

struct RefConstants {
  int M = 0;
  int n = 1;
  long double nodes[kMaxN];
  long double weights[kMaxN];
  long double psi0[kMaxN];         // psi_l(0)
  long double psi1[kMaxN];         // psi_l(1)
  long double dmat[kMaxN][kMaxN];  // dmat[a][b] = psi_b'(node_a)
  long double time_mat[kMaxN][kMaxN];  // K^1 time factor [test][trial]
  long double time_inv_w[kMaxN][kMaxN];  // time_mat^-1 diag(weights)
  int nstencils = 0;
  int stencil_left[kMaxN];  // L of each stencil (R = M - L)
  long double lambda[kMaxN];
  long double rec_inv[kMaxN][kMaxN][kMaxN];  // [stencil][p][e]
  // sig_rows[s][r][e]: stencil s's averages -> the coefficients, in Legendre
  // polynomials orthonormal on [0, 1], of the derivatives alpha = 1..M of its
  // reconstruction (r runs over alpha, then over the degrees 0..M-alpha).
  // By Parseval, the sum of their squares is the oscillation indicator of
  // eq. sigmas.
  int nsig_rows = 0;
  long double sig_rows[kMaxN][kMaxN * (kMaxN - 1) / 2][kMaxN];
  // Gauss-Legendre rule on [0, 1] of the Osher path integral (eq. osher)
  long double path_s[kOsherNodes], path_w[kOsherNodes];
};

// Fills 'out' for degree M (0..3). Returns false if a matrix is singular.
bool build_ref_constants(int M, RefConstants* out);

// Basis tables of the AMR operators for refinement factor r (2..kMaxR),
// psi_p the nodal basis of degree M on [0, 1], x_b its Gauss-Legendre nodes:
//   sub_avg[a][p]     = r * int_{a/r}^{(a+1)/r} psi_p   (projection, Sec. 3.1.3)
//   at_sub[j][p]      = psi_p(j / r)                      (mother-local time of substep j)
//   at_face[a][s][p]  = psi_p((a + s) / r)                (child face s = 0 / 1)
//   at_nodes[a][b][p] = psi_p((a + x_b) / r)              (child nodes, substep nodes)
constexpr int kMaxR = 4;
struct AmrTables {
  int M = 0, r = 2;
  long double sub_avg[kMaxR][kMaxN];
  long double at_sub[kMaxR][kMaxN];
  long double at_face[kMaxR][2][kMaxN];
  long double at_nodes[kMaxR][kMaxN][kMaxN];
};
bool build_amr_tables(int M, int r, AmrTables* out);

// WENO constants stated after eq. sigmas.
constexpr double kLambdaCentral = 1.0e5;
constexpr double kLambdaOneSided = 1.0;
constexpr double kWenoEpsilon = 1.0e-14;

}  // namespace ader
