"""Physical fluxes and wave speeds of the balance laws, oracle side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Euler equations of an ideal gas (Section 4.1, eq. Euler-system):
  u = (rho, rho v_x, rho v_y[, rho v_z], E), E = p/(gamma-1) + rho |v|^2 / 2.
  In two space dimensions v_z = 0 is exact for all time, so the 2D system keeps
  the four variables (rho, rho v_x, rho v_y, E).
* Scalar linear advection u_t + a . grad u = 0: the test system whose exact
  solution pins the predictor and the flux step.
* Ideal MHD with hyperbolic GLM divergence cleaning (Section 4.2): nine
  variables u = (rho, rho v (3), E, B (3), psi) in any space dimension, the
  magnetic terms in the paper's units (B^2 / 8 pi, B B / 4 pi).

The source term S of eq. governingPDE is zero for all systems.
"""
from __future__ import annotations

import numpy as np


class Euler:
    """Compressible Euler equations, ideal-gas closure (eq. Euler-system)."""

    def __init__(self, dim: int, gamma: float = 1.4):
        self.dim = dim
        self.gamma = gamma
        self.nv = dim + 2

    def primitive(self, q: np.ndarray):
        """(rho, velocity list, p) from conserved variables q[nv, ...]."""
        rho = q[0]
        vel = [q[1 + k] / rho for k in range(self.dim)]
        kinetic = 0.5 * sum(q[1 + k] * vel[k] for k in range(self.dim))
        p = (self.gamma - 1.0) * (q[self.dim + 1] - kinetic)
        return rho, vel, p

    def flux(self, q: np.ndarray, k: int) -> np.ndarray:
        """Physical flux along axis k (f, g, h of eq. Euler-system)."""
        rho, vel, p = self.primitive(q)
        vk = vel[k]
        out = np.empty_like(q)
        out[0] = q[1 + k]
        for m in range(self.dim):
            out[1 + m] = q[1 + m] * vk
        out[1 + k] = out[1 + k] + p
        out[self.dim + 1] = vk * (q[self.dim + 1] + p)
        return out

    def max_speed(self, q: np.ndarray, k: int) -> np.ndarray:
        """|v_k| + c: largest |eigenvalue| of the flux Jacobian along k."""
        rho, vel, p = self.primitive(q)
        c = np.sqrt(self.gamma * p / rho)
        return np.abs(vel[k]) + c


class LinearAdvection:
    """u_t + sum_k a_k u_{x_k} = 0 with constant velocity a."""

    def __init__(self, dim: int, velocity):
        self.dim = dim
        self.a = [float(v) for v in velocity][:dim]
        self.nv = 1

    def flux(self, q: np.ndarray, k: int) -> np.ndarray:
        return self.a[k] * q

    def max_speed(self, q: np.ndarray, k: int) -> np.ndarray:
        return np.full(q.shape[1:], abs(self.a[k]))


class GLMMHD:
    """Ideal MHD with hyperbolic GLM divergence cleaning (Section 4.2).

    State (rho, rho v_x, rho v_y, rho v_z, E, B_x, B_y, B_z, psi).  Flux along
    axis k (k < dim; the velocity and field always have three components):
      mass       rho v_k
      momentum   rho v_i v_k + (p + |B|^2 / 8 pi) delta_ik - B_i B_k / 4 pi
      energy     v_k (E + p + |B|^2 / 8 pi) - B_k (v . B) / 4 pi
      induction  v_k B_i - v_i B_k + psi delta_ik
      cleaning   c_h^2 B_k
    with p = (gamma - 1)(E - rho |v|^2 / 2 - |B|^2 / 8 pi).  The induction
    flux is the one of the ideal induction equation B_t = curl(v x B) plus the
    GLM term (the paper prints the dyads as v B - B v in its own ordering).
    The largest |eigenvalue| along k is max(|v_k| + c_f, c_h) with the fast
    magnetosonic speed c_f^2 = (a^2 + b^2 + sqrt((a^2 + b^2)^2 - 4 a^2 b_k^2)) / 2,
    a^2 = gamma p / rho, b^2 = |B|^2 / (4 pi rho), b_k^2 = B_k^2 / (4 pi rho)
    (the textbook fast speed; the paper does not print it).
    """

    def __init__(self, dim: int, gamma: float = 5.0 / 3.0, ch: float = 2.0):
        self.dim = dim
        self.gamma = gamma
        self.ch = ch
        self.nv = 9

    def primitive(self, q: np.ndarray):
        """(rho, [v_x, v_y, v_z], p, [B_x, B_y, B_z]) of q[9, ...]."""
        rho = q[0]
        vel = [q[1 + i] / rho for i in range(3)]
        B = [q[5 + i] for i in range(3)]
        kinetic = 0.5 * sum(q[1 + i] * vel[i] for i in range(3))
        magnetic = sum(b * b for b in B) / (8.0 * np.pi)
        p = (self.gamma - 1.0) * (q[4] - kinetic - magnetic)
        return rho, vel, p, B

    def flux(self, q: np.ndarray, k: int) -> np.ndarray:
        rho, vel, p, B = self.primitive(q)
        pm = sum(b * b for b in B) / (8.0 * np.pi)
        vB = sum(vel[i] * B[i] for i in range(3))
        out = np.empty_like(q)
        out[0] = q[1 + k]
        for i in range(3):
            out[1 + i] = q[1 + i] * vel[k] - B[i] * B[k] / (4.0 * np.pi)
        out[1 + k] = out[1 + k] + p + pm
        out[4] = vel[k] * (q[4] + p + pm) - B[k] * vB / (4.0 * np.pi)
        for i in range(3):
            out[5 + i] = vel[k] * B[i] - vel[i] * B[k]
        out[5 + k] = out[5 + k] + q[8]
        out[8] = self.ch * self.ch * B[k]
        return out

    def fast_speed(self, q: np.ndarray, k: int) -> np.ndarray:
        rho, vel, p, B = self.primitive(q)
        a2 = self.gamma * p / rho
        b2 = sum(b * b for b in B) / (4.0 * np.pi * rho)
        bk2 = B[k] * B[k] / (4.0 * np.pi * rho)
        s = a2 + b2
        return np.sqrt(0.5 * (s + np.sqrt(np.maximum(s * s - 4.0 * a2 * bk2, 0.0))))

    def max_speed(self, q: np.ndarray, k: int) -> np.ndarray:
        rho, vel, p, B = self.primitive(q)
        return np.maximum(np.abs(vel[k]) + self.fast_speed(q, k), self.ch)
