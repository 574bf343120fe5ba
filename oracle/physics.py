"""Physical fluxes and wave speeds of the balance laws, oracle side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Euler equations of an ideal gas (Section 4.1, eq. Euler-system):
  u = (rho, rho v_x, rho v_y[, rho v_z], E), E = p/(gamma-1) + rho |v|^2 / 2.
  In two space dimensions v_z = 0 is exact for all time, so the 2D system keeps
  the four variables (rho, rho v_x, rho v_y, E).
* Scalar linear advection u_t + a . grad u = 0: the test system whose exact
  solution pins the predictor and the flux step.

The source term S of eq. governingPDE is zero for both systems.
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
