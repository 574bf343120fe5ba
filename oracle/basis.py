"""Reference-element constants of the one-step ADER-WENO scheme, oracle side.

TEST INFRASTRUCTURE ONLY.  The oracle is the plain CPU definition that the HIP
path is checked against; nothing in the product path may import it.

Everything here is exact polynomial algebra (numpy's Polynomial class) on the
unit interval [0, 1] of the reference coordinates (Section 2.2, eq. xi):

* the M+1 Gauss-Legendre nodes lambda_k and weights on [0, 1];
* the nodal Lagrange basis psi_l with psi_l(lambda_k) = delta_lk (Section 2.2),
  used in space for the reconstruction and, by tensor products, in space-time
  for the predictor (Section 2.3);
* the one-dimensional integrals (mass, stiffness, end-point values) from which
  Section 2.3 assembles the space-time matrices K^1, K^xi and F^0.

Integrals are taken exactly from antiderivatives, not by quadrature, so that
the properties the scheme relies on (diagonal mass matrix, exactness of the
Gauss rule up to degree 2M+1) are results the tests can check, not inputs.

The tables are built in long double and rounded once to fp64: the stencil
integrals of Section 2.2 extrapolate the basis up to M cells away, where the
antiderivatives cancel badly, and the WENO weights raise the oscillation
indicators to the power r = 8, which turns table errors of a few hundred ulps
into visible changes of w_h.  Everything applied per cell stays fp64.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
from numpy.polynomial import Polynomial
from numpy.polynomial import legendre
from numpy.polynomial.legendre import leggauss


LD = np.longdouble


def gauss_legendre_ld(n: int) -> tuple[np.ndarray, np.ndarray]:
    """n Gauss-Legendre nodes and weights on [0, 1], in long double.

    numpy's fp64 rule, refined by Newton steps on the Legendre series P_n
    evaluated in long double; weights 2 / ((1 - x^2) P_n'(x)^2) on [-1, 1].
    """
    x, _ = leggauss(n)
    x = x.astype(LD)
    c = np.zeros(n + 1, dtype=LD)
    c[n] = 1
    dc = legendre.legder(c)
    for _ in range(3):
        x = x - legendre.legval(x, c) / legendre.legval(x, dc)
    dp = legendre.legval(x, dc)
    w = 2 / ((1 - x * x) * dp * dp)
    return (x + 1) / 2, w / 2


def gauss_legendre(n: int) -> tuple[np.ndarray, np.ndarray]:
    """n Gauss-Legendre nodes and weights mapped from [-1, 1] to [0, 1]."""
    x, w = gauss_legendre_ld(n)
    return x.astype(np.float64), w.astype(np.float64)


def inverse_ld(A: np.ndarray) -> np.ndarray:
    """Inverse of a small square matrix by Gauss-Jordan elimination with
    partial pivoting, in long double."""
    A = np.array(A, dtype=LD)
    n = A.shape[0]
    aug = np.concatenate([A, np.eye(n, dtype=LD)], axis=1)
    for c in range(n):
        piv = c + int(np.argmax(np.abs(aug[c:, c])))
        if aug[piv, c] == 0:
            raise np.linalg.LinAlgError("singular matrix")
        aug[[c, piv]] = aug[[piv, c]]
        aug[c] = aug[c] / aug[c, c]
        for r in range(n):
            if r != c:
                aug[r] = aug[r] - aug[r, c] * aug[c]
    return aug[:, n:]


def lagrange_basis(nodes: np.ndarray) -> list[Polynomial]:
    """Lagrange interpolation polynomials psi_l with psi_l(nodes[k]) = delta_lk."""
    n = len(nodes)
    basis = []
    for l in range(n):
        # product of (xi - lambda_k) over k != l, normalised to 1 at lambda_l;
        # stored in the variable 2 xi - 1 (domain [0,1] -> window [-1,1]),
        # which keeps the coefficients well conditioned
        roots = [nodes[k] for k in range(n) if k != l]
        p = (Polynomial.fromroots(roots, domain=[0.0, 1.0], window=[-1.0, 1.0])
             if roots else
             Polynomial([1.0], domain=[0.0, 1.0], window=[-1.0, 1.0]))
        basis.append(p / p(nodes[l]))
    return basis


def integral_ld(p: Polynomial, a, b):
    """Integral of a polynomial over [a, b] via its antiderivative, in the
    polynomial's own precision (long double for the tables' polynomials)."""
    P = p.integ()
    return P(LD(b)) - P(LD(a))


def integrate(p: Polynomial, a: float, b: float) -> float:
    """Exact integral of a polynomial over [a, b] via its antiderivative."""
    return float(integral_ld(p, a, b))


class Basis1D:
    """One-dimensional nodal basis of degree M on [0, 1] and its integrals.

    Attributes (n = M + 1):
      nodes, weights : Gauss-Legendre rule on [0, 1]
      psi            : list of n Lagrange polynomials
      dpsi           : their first derivatives
      psi0, psi1     : psi_l(0), psi_l(1)                      (n,)
      mass[i, j]     : int_0^1 psi_i psi_j                      (n, n)
      stiff[i, j]    : int_0^1 psi_i d(psi_j)/dxi  (test i, trial j)
      dmat[a, b]     : d(psi_b)/dxi evaluated at node a
    """

    def __init__(self, M: int):
        if M < 0:
            raise ValueError("degree M must be >= 0")
        self.M = M
        self.n = n = M + 1
        self.nodes_ld, self.weights_ld = gauss_legendre_ld(n)
        self.nodes = self.nodes_ld.astype(np.float64)
        self.weights = self.weights_ld.astype(np.float64)
        # long-double basis for the tables; fp64 copies for evaluations
        self.psi_ld = lagrange_basis(self.nodes_ld)
        self.psi = lagrange_basis(self.nodes)
        dpsi = [p.deriv() for p in self.psi_ld]
        self.dpsi = [p.deriv() for p in self.psi]
        f64 = lambda rows: np.array(rows, dtype=LD).astype(np.float64)
        self.psi0 = f64([p(LD(0)) for p in self.psi_ld])
        self.psi1 = f64([p(LD(1)) for p in self.psi_ld])
        self.mass = f64([[integral_ld(self.psi_ld[i] * self.psi_ld[j], 0, 1)
                          for j in range(n)] for i in range(n)])
        self.stiff = f64([[integral_ld(self.psi_ld[i] * dpsi[j], 0, 1)
                           for j in range(n)] for i in range(n)])
        self.dmat = f64([[dpsi[b](self.nodes_ld[a]) for b in range(n)]
                         for a in range(n)])

    def time_matrix(self) -> np.ndarray:
        """Time factor of K^1 (Section 2.3, definition of K^1).

        Integrating the time derivative by parts gives, for test function s'
        and trial function s, psi_s'(1) psi_s(1) - int_0^1 psi_s'' psi_s dtau.
        """
        n = self.n
        p1 = [p(LD(1)) for p in self.psi_ld]
        return np.array([[p1[sp] * p1[s]
                          - integral_ld(self.psi_ld[sp].deriv() * self.psi_ld[s], 0, 1)
                          for s in range(n)] for sp in range(n)], dtype=LD).astype(np.float64)


@lru_cache(maxsize=None)
def basis(M: int) -> Basis1D:
    return Basis1D(M)
