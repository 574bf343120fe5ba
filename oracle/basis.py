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
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
from numpy.polynomial import Polynomial
from numpy.polynomial.legendre import leggauss


def gauss_legendre(n: int) -> tuple[np.ndarray, np.ndarray]:
    """n Gauss-Legendre nodes and weights mapped from [-1, 1] to [0, 1]."""
    x, w = leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


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


def integrate(p: Polynomial, a: float, b: float) -> float:
    """Exact integral of a polynomial over [a, b] via its antiderivative."""
    P = p.integ()
    return float(P(b) - P(a))


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
        self.nodes, self.weights = gauss_legendre(n)
        self.psi = lagrange_basis(self.nodes)
        self.dpsi = [p.deriv() for p in self.psi]
        self.psi0 = np.array([p(0.0) for p in self.psi])
        self.psi1 = np.array([p(1.0) for p in self.psi])
        self.mass = np.array([[integrate(self.psi[i] * self.psi[j], 0.0, 1.0)
                               for j in range(n)] for i in range(n)])
        self.stiff = np.array([[integrate(self.psi[i] * self.dpsi[j], 0.0, 1.0)
                                for j in range(n)] for i in range(n)])
        self.dmat = np.array([[self.dpsi[b](self.nodes[a]) for b in range(n)]
                              for a in range(n)])

    def time_matrix(self) -> np.ndarray:
        """Time factor of K^1 (Section 2.3, definition of K^1).

        Integrating the time derivative by parts gives, for test function s'
        and trial function s, psi_s'(1) psi_s(1) - int_0^1 psi_s'' psi_s dtau.
        """
        n = self.n
        return np.array([[self.psi1[sp] * self.psi1[s]
                          - integrate(self.dpsi[sp] * self.psi[s], 0.0, 1.0)
                          for s in range(n)] for sp in range(n)])


@lru_cache(maxsize=None)
def basis(M: int) -> Basis1D:
    return Basis1D(M)
