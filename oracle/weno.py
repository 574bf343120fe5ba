"""Dimension-by-dimension polynomial WENO reconstruction, oracle side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Section 2.2 step by step:

* stencil sets (eq. stencildef): for even M three stencils -- central with
  L = R = M/2, fully left (L = M, R = 0), fully right (L = 0, R = M); for odd
  M four stencils -- two central ones (L = floor(M/2)+1, R = floor(M/2)) and
  (L = floor(M/2), R = floor(M/2)+1), fully left and fully right;
* per-stencil reconstruction by integral conservation on every stencil cell
  (eqs. recpolydef.x, rec.x), solved with the inverse of the reference-element
  matrix, which depends only on the basis;
* oscillation indicator sigma_s = Sigma_pm w_p w_m with
  Sigma_pm = sum_{alpha=1..M} int_0^1 psi_p^(alpha) psi_m^(alpha) (eq. sigmas),
  i.e. sigma_s = sum_alpha int_0^1 (d^alpha w^s / dxi^alpha)^2; it is evaluated
  in that form, the squared derivative values at the Gauss nodes summed with
  the Gauss weights (exact: the integrand has degree 2(M - alpha) <= 2M + 1).
  The same number as the quadratic form with the assembled matrix, without
  its cancellation: Sigma has entries up to ~1e4 at M = 3 and annihilates
  constants, so w^T Sigma w loses digits that the weights' exponent r = 8
  then magnifies;
* nonlinear weights omega~_s = lambda_s / (sigma_s + eps)^r, normalised, with
  lambda = 1 for one-sided and 1e5 for central stencils, eps = 1e-14, r = 8
  (eq. omegas and the constants stated after it);
* the nonlinear combination (eq. weno), then the same procedure along y for
  every x degree of freedom (eqs. recpolydef.y .. weno.y) and along z for every
  (x, y) degree of freedom (eqs. recpolydef.z .. weno.z).

Readings where the text is silent: the y and z passes use one set of weights
per (variable, transverse degree of freedom) line; M = 1 keeps all four
stencils literally (the two "central" ones coincide with the one-sided ones);
both central stencils of odd M get lambda = 1e5; Sigma has no mesh-size
factors.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from .basis import LD, basis, integral_ld, inverse_ld

LAMBDA_CENTRAL = 1.0e5
LAMBDA_ONE_SIDED = 1.0
EPSILON = 1.0e-14
R_EXPONENT = 8


def stencils(M: int) -> list[tuple[int, int, float]]:
    """(L, R, lambda) of every stencil for degree M (eq. stencildef)."""
    if M % 2 == 0:
        h = M // 2
        return [(h, h, LAMBDA_CENTRAL),
                (M, 0, LAMBDA_ONE_SIDED),
                (0, M, LAMBDA_ONE_SIDED)]
    h = M // 2
    return [(h + 1, h, LAMBDA_CENTRAL),
            (h, h + 1, LAMBDA_CENTRAL),
            (M, 0, LAMBDA_ONE_SIDED),
            (0, M, LAMBDA_ONE_SIDED)]


def reconstruction_matrix(M: int, L: int, R: int) -> np.ndarray:
    """Matrix of the conservation system (eq. rec.x) on the reference element.

    Row e (stencil cell with offset o = e - L from the home cell, which is the
    interval [0, 1]) holds int_o^(o+1) psi_p(xi) dxi: the average over that
    cell of the p-th basis function, in the home cell's reference coordinate.
    """
    return reconstruction_matrix_ld(M, L, R).astype(np.float64)


def reconstruction_matrix_ld(M: int, L: int, R: int) -> np.ndarray:
    """reconstruction_matrix in long double (the inverse is taken from it)."""
    b = basis(M)
    offsets = range(-L, R + 1)
    return np.array([[integral_ld(b.psi_ld[p], o, o + 1) for p in range(b.n)]
                     for o in offsets], dtype=LD)


def oscillation_matrix(M: int) -> np.ndarray:
    """Sigma_pm of eq. sigmas (derivatives of order 1..M, no mesh scaling)."""
    b = basis(M)
    n = b.n
    S = np.zeros((n, n), dtype=LD)
    for alpha in range(1, M + 1):
        d = [p.deriv(alpha) for p in b.psi_ld]
        for p in range(n):
            for m in range(n):
                S[p, m] += integral_ld(d[p] * d[m], 0, 1)
    return S.astype(np.float64)


@lru_cache(maxsize=None)
def derivative_values(M: int) -> list:
    """[alpha-1][k, p] = d^alpha psi_p / dxi^alpha at Gauss node k, alpha = 1..M."""
    b = basis(M)
    return [np.array([[p.deriv(alpha)(x) for p in b.psi_ld] for x in b.nodes_ld],
                     dtype=LD).astype(np.float64)
            for alpha in range(1, M + 1)]


def oscillation_indicator(ws: np.ndarray, M: int) -> np.ndarray:
    """sigma = sum_alpha int_0^1 (d^alpha w / dxi^alpha)^2 for nodal w[..., n]."""
    b = basis(M)
    sigma = np.zeros(ws.shape[:-1])
    for D in derivative_values(M):
        sigma = sigma + ((ws @ D.T) ** 2) @ b.weights
    return sigma


@lru_cache(maxsize=None)
def weno_constants(M: int):
    """Per-stencil inverse matrices, stencil windows, lambdas and Sigma."""
    sts = stencils(M)
    inv = [inverse_ld(reconstruction_matrix_ld(M, L, R)).astype(np.float64)
           for (L, R, _) in sts]
    # window of stencil s inside the (2M+1)-cell line centred on the home cell
    windows = [(M - L, M + R + 1) for (L, R, _) in sts]
    lambdas = np.array([lam for (_, _, lam) in sts])
    return inv, windows, lambdas, oscillation_matrix(M)


def weno_1d(values: np.ndarray, M: int) -> np.ndarray:
    """One-dimensional WENO reconstruction along the last axis.

    values[..., 2M+1] are the averages of the cells i-M .. i+M (along the
    reconstruction direction) of the quantity being reconstructed; returns
    the n = M+1 nodal degrees of freedom w_p of the combined polynomial in the
    home cell i (eqs. rec.x, weno, omegas, sigmas).
    """
    inv, windows, lambdas, Sigma = weno_constants(M)
    polys = []
    omegas = []
    for s, (a, b) in enumerate(windows):
        ws = values[..., a:b] @ inv[s].T                  # w^s_p, eq. rec.x
        sigma = oscillation_indicator(ws, M)              # eq. sigmas
        omegas.append(lambdas[s] / (sigma + EPSILON) ** R_EXPONENT)
        polys.append(ws)
    total = sum(omegas)
    return sum((om / total)[..., None] * ws for om, ws in zip(omegas, polys))


def bc_index(i: np.ndarray, n: int, bc: str) -> np.ndarray:
    """Map (possibly ghost) cell indices to interior cells.

    periodic: wrap around; transmissive: zero-gradient ghost cells, i.e. a
    ghost takes the average of the nearest interior cell.
    """
    if bc == "periodic":
        return np.mod(i, n)
    if bc == "transmissive":
        return np.clip(i, 0, n - 1)
    raise ValueError(f"unknown boundary condition {bc!r}")


def gather_patches(U: np.ndarray, cells: np.ndarray, M: int,
                   bcs: list[str]) -> np.ndarray:
    """Averages on the (2M+1)^d patch around each requested cell.

    U[v, i, j(, k)] holds cell averages (x index first); cells[C, d] are the
    home cells.  Returns P[v, C, o_x, o_y(, o_z)] with o = offset + M.
    """
    d = cells.shape[1]
    off = np.arange(-M, M + 1)
    idx = []
    for k in range(d):
        shape = [1] * (d + 1)
        shape[1 + k] = 2 * M + 1
        ik = cells[:, k].reshape(-1, *([1] * d)) + off.reshape(shape)
        idx.append(bc_index(ik, U.shape[1 + k], bcs[k]))
    idx = np.broadcast_arrays(*idx)
    return U[(slice(None),) + tuple(idx)]


def reconstruct(U: np.ndarray, cells: np.ndarray, M: int,
                bcs: list[str]) -> np.ndarray:
    """Dimension-by-dimension WENO polynomial of each requested cell.

    Returns w[v, C, p_x, p_y(, p_z)]: the nodal degrees of freedom of w_h at
    the tensor Gauss-Legendre nodes (eq. weno.z).  The x pass is applied to
    every line of the patch that the later passes need, exactly as if it had
    been done once per cell of the mesh.
    """
    d = cells.shape[1]
    P = gather_patches(U, cells, M, bcs)          # [v, C, ox, oy(, oz)]
    # x pass: reconstruct along axis o_x -> nodal index p_x (appended last)
    Wx = weno_1d(np.moveaxis(P, 2, -1), M)         # [v, C, oy(, oz), px]
    if d == 2:
        # y pass for every x degree of freedom p_x: line along o_y
        Wxy = weno_1d(np.moveaxis(Wx, 2, -1), M)   # [v, C, px, py]
        return Wxy
    Wxy = weno_1d(np.moveaxis(Wx, 2, -1), M)       # [v, C, oz, px, py]
    Wxyz = weno_1d(np.moveaxis(Wxy, 2, -1), M)     # [v, C, px, py, pz]
    return Wxyz
