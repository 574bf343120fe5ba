"""Seeded synthetic initial data shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the numerical method: it only builds
initial cell averages of analytic initial conditions (by a tensor
Gauss-Legendre rule with 8 points per axis and cell) and applies seeded
per-cell perturbations.  It imports nothing else from this package, so the
CPU tests can use it without the HIP library.

Arrays are returned as U[v, i, j(, k)] (x index first, conserved variables
first); ``to_soa`` converts to the library's layout u[v * ld + cell] with
cell = i + nx (j + ny k).

Workloads (conserved variables (rho, rho v, E), ideal gas):
  * isentropic vortex (Section 4.1, vortex test): strength 5, gamma 1.4, mean
    flow (1, 1) on the periodic square [0, 10]^2; the exact solution at time t
    is the initial condition translated by (t, t) modulo 10;
  * Kelvin-Helmholtz shear layer on the periodic unit square: rho = 2 and
    v_x = +0.5 for |y - 0.5| < 0.25, else rho = 1 and v_x = -0.5; p = 2.5;
    then v_x, v_y += 0.01 U(-1, 1) per cell (PCG64, seed 1);
  * circular explosion on [-1, 1]^2: (rho, p) = (1, 1) for r < 0.5 and
    (0.125, 0.1) outside, at rest; then rho *= 1 + 0.01 U(-1, 1) (seed 2);
  * spherical blast on [-1, 1]^3: rho = 1, p = 1 for r < 0.3 and 0.1 outside;
    then rho *= 1 + 0.01 U(-1, 1) (seed 3);
  * linear advection of a smooth sine wave, and a seeded random field;
  * a generic test state on the unit cube: smooth sinusoidal density,
    velocity and pressure with seeded phases, a discontinuity (density x1.5,
    pressure x1.8 for x < 0.4) and 1% seeded per-cell noise;
  * seeded tensor polynomials of degree <= M per axis (data every WENO
    stencil reproduces).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.legendre import leggauss

GAMMA = 1.4


def _cell_average(fn, n, lo, hi, nq=8):
    """Averages over each cell of fn(*coords) -> [nv, ...] by nq^d Gauss points."""
    d = len(n)
    x, w = leggauss(nq)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    h = [(hi[k] - lo[k]) / n[k] for k in range(d)]
    acc = None
    for idx in np.ndindex(*([nq] * d)):
        coords = np.meshgrid(*[lo[k] + (np.arange(n[k]) + x[idx[k]]) * h[k]
                               for k in range(d)], indexing="ij")
        wt = np.prod([w[i] for i in idx])
        val = np.asarray(fn(*coords)) * wt
        acc = val if acc is None else acc + val
    return acc


def conserved_from_primitive(rho, vel, p, gamma=GAMMA):
    kin = 0.5 * rho * sum(v * v for v in vel)
    return np.stack([rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + kin])


def vortex_state(x, y, t=0.0, eps=5.0, gamma=GAMMA, L=10.0):
    """Conserved variables of the isentropic vortex at time t (exact)."""
    xc = np.mod(x - t, L)
    yc = np.mod(y - t, L)
    dx = xc - 5.0
    dy = yc - 5.0
    r2 = dx * dx + dy * dy
    dT = -(eps * eps) * (gamma - 1.0) / (8.0 * gamma * np.pi ** 2) * np.exp(1.0 - r2)
    rho = (1.0 + dT) ** (1.0 / (gamma - 1.0))
    p = (1.0 + dT) ** (gamma / (gamma - 1.0))
    fac = eps / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2))
    vx = 1.0 - dy * fac
    vy = 1.0 + dx * fac
    return conserved_from_primitive(rho, [vx, vy], p, gamma)


def isentropic_vortex(n=20, t=0.0):
    return _cell_average(lambda x, y: vortex_state(x, y, t), (n, n),
                         (0.0, 0.0), (10.0, 10.0))


def kelvin_helmholtz(n=512, seed=1, amp=0.01, gamma=GAMMA):
    def prim(x, y):
        inner = np.abs(y - 0.5) < 0.25
        rho = np.where(inner, 2.0, 1.0)
        vx = np.where(inner, 0.5, -0.5)
        return np.stack([rho, vx, np.zeros_like(x), np.full_like(x, 2.5)])
    P = _cell_average(prim, (n, n), (0.0, 0.0), (1.0, 1.0))
    rng = np.random.Generator(np.random.PCG64(seed))
    vx = P[1] + amp * rng.uniform(-1.0, 1.0, size=P[1].shape)
    vy = P[2] + amp * rng.uniform(-1.0, 1.0, size=P[2].shape)
    return conserved_from_primitive(P[0], [vx, vy], P[3], gamma)


def explosion_2d(n=100, seed=2, amp=0.01, radius=0.5, gamma=GAMMA):
    def cons(x, y):
        inside = x * x + y * y < radius * radius
        rho = np.where(inside, 1.0, 0.125)
        p = np.where(inside, 1.0, 0.1)
        z = np.zeros_like(x)
        return conserved_from_primitive(rho, [z, z], p, gamma)
    U = _cell_average(cons, (n, n), (-1.0, -1.0), (1.0, 1.0))
    if seed is not None:
        rng = np.random.Generator(np.random.PCG64(seed))
        U[0] = U[0] * (1.0 + amp * rng.uniform(-1.0, 1.0, size=U[0].shape))
    return U


def blast_3d(n=64, seed=3, amp=0.01, radius=0.3, gamma=GAMMA, nq=4):
    def cons(x, y, z):
        inside = x * x + y * y + z * z < radius * radius
        rho = np.ones_like(x)
        p = np.where(inside, 1.0, 0.1)
        zero = np.zeros_like(x)
        return conserved_from_primitive(rho, [zero, zero, zero], p, gamma)
    U = _cell_average(cons, (n, n, n), (-1.0,) * 3, (1.0,) * 3, nq=nq)
    if seed is not None:
        rng = np.random.Generator(np.random.PCG64(seed))
        U[0] = U[0] * (1.0 + amp * rng.uniform(-1.0, 1.0, size=U[0].shape))
    return U


def mhd_conserved(rho, vel, p, B, psi=None, gamma=5.0 / 3.0):
    """GLM-MHD conserved variables (rho, rho v (3), E, B (3), psi) with
    E = p / (gamma - 1) + rho |v|^2 / 2 + |B|^2 / 8 pi."""
    z = np.zeros_like(rho)
    vel = [np.asarray(v) + z for v in vel]
    B = [np.asarray(b) + z for b in B]
    E = p / (gamma - 1.0) + 0.5 * rho * sum(v * v for v in vel) + \
        sum(b * b for b in B) / (8.0 * np.pi)
    psi = z if psi is None else psi + z
    return np.stack([rho] + [rho * v for v in vel] + [E] + B + [psi])


def orszag_tang(n, seed=None, amp=0.05, gamma=5.0 / 3.0):
    """Orszag-Tang vortex (Section 4.2) on the periodic square [0, 2 pi]^2:
    (rho, v_x, v_y, p, B_x, B_y) = (gamma^2, -sin y, sin x, gamma,
    -sqrt(4 pi) sin y, sqrt(4 pi) sin 2x), v_z = B_z = psi = 0.  With a seed,
    each sine gets a random phase and each amplitude a factor 1 + amp U(-1,1)
    (PCG64): a divergence-free family of the same shape."""
    ph = np.zeros(4)
    fac = np.ones(4)
    if seed is not None:
        r = np.random.Generator(np.random.PCG64(seed))
        ph = r.uniform(0.0, 2.0 * np.pi, 4)
        fac = 1.0 + amp * r.uniform(-1.0, 1.0, 4)
    s4 = np.sqrt(4.0 * np.pi)

    def fn(x, y):
        rho = gamma * gamma + 0 * x
        vel = [-fac[0] * np.sin(y + ph[0]), fac[1] * np.sin(x + ph[1]), 0 * x]
        B = [-s4 * fac[2] * np.sin(y + ph[2]), s4 * fac[3] * np.sin(2 * x + ph[3]), 0 * x]
        return mhd_conserved(rho, vel, gamma + 0 * x, B, gamma=gamma)
    L = 2.0 * np.pi
    return _cell_average(fn, (n, n), (0.0, 0.0), (L, L))


def sine_wave(n, dim=2, L=1.0):
    """Average of sin(2 pi (x + y [+ z]) / L) on the periodic cube [0, L]^d."""
    fn = lambda *c: np.sin(2.0 * np.pi * sum(c) / L)[None]
    return _cell_average(fn, (n,) * dim, (0.0,) * dim, (L,) * dim)


def perturbed_smooth_euler(n, seed, noise=0.01, gamma=GAMMA):
    """Smooth state + jump + per-cell noise on the unit cube, averages per cell.

    Cell-centre values (no sub-cell quadrature): a test input, not a solution.
    """
    dim = len(n)
    r = np.random.Generator(np.random.PCG64(seed))
    X = np.meshgrid(*[(np.arange(k) + 0.5) / k for k in n], indexing="ij")
    ph = r.uniform(0.0, 2.0 * np.pi, size=4)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * X[0] + ph[0]) * np.cos(2 * np.pi * X[-1] + ph[1])
    vel = [0.3 * np.sin(2 * np.pi * X[(k + 1) % dim] + ph[2 + k % 2]) for k in range(dim)]
    p = 1.0 + 0.2 * np.cos(2 * np.pi * X[0] + ph[3])
    jump = X[0] < 0.4
    rho = np.where(jump, 1.5 * rho, rho)
    p = np.where(jump, 1.8 * p, p)
    rho = rho * (1.0 + noise * r.uniform(-1.0, 1.0, size=rho.shape))
    vel = [v + noise * r.uniform(-1.0, 1.0, size=v.shape) for v in vel]
    return conserved_from_primitive(rho, vel, p, gamma)


def polynomial_state(n, M, nv, lo, hi, seed, amp=0.1):
    """Averages of seeded tensor polynomials of degree <= M per axis.

    Variable v is base[v] + amp * sum_e c_e prod_k ((x_k - lo_k)/(hi_k - lo_k))^e_k
    with c_e ~ U(-1, 1); the bases (1, 0, .., 0, 2.5) keep an Euler gas's
    density and pressure positive.  Every WENO stencil reproduces such data,
    so the reconstruction does not depend on the nonlinear weights.
    """
    d = len(n)
    r = np.random.Generator(np.random.PCG64(seed))
    base = np.zeros(nv)
    base[0] = 1.0
    if nv > 1:
        base[-1] = 2.5
    exps = list(np.ndindex(*([M + 1] * d)))
    coef = r.uniform(-1.0, 1.0, size=(nv, len(exps)))

    def fn(*c):
        s = [(c[k] - lo[k]) / (hi[k] - lo[k]) for k in range(d)]
        out = []
        for v in range(nv):
            acc = np.full(c[0].shape, base[v])
            for j, e in enumerate(exps):
                acc = acc + amp * coef[v, j] * np.prod([s[k] ** e[k] for k in range(d)], axis=0)
            out.append(acc)
        return np.stack(out)
    return _cell_average(fn, tuple(n), tuple(lo), tuple(hi))


def random_field(shape, seed, lo=-1.0, hi=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=shape)


def to_soa(U: np.ndarray, ld: int | None = None) -> np.ndarray:
    """U[v, i, j(, k)] -> u[v, ld] with cell = i + nx (j + ny k), zero padded."""
    nv = U.shape[0]
    # order="F" over the spatial axes puts the x index fastest
    flat = np.stack([U[v].reshape(-1, order="F") for v in range(nv)])
    C = flat.shape[1]
    ld = C if ld is None else ld
    out = np.zeros((nv, ld))
    out[:, :C] = flat
    return out


def from_soa(u: np.ndarray, shape) -> np.ndarray:
    """Inverse of to_soa: u[v, ld] -> U[v, i, j(, k)]."""
    C = int(np.prod(shape))
    return np.stack([u[v, :C].reshape(shape, order="F") for v in range(u.shape[0])])
