"""Element-local space-time DG predictor, oracle side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Section 2.3.  The PDE is written on the space-time reference element
[0,1]^(d+1) with f* = (dt/dx) f (eq. pde.ref).  The space-time basis is the
tensor product theta = psi_p(xi) psi_q(eta) [psi_r(zeta)] psi_s(tau) of the
one-dimensional nodal basis.  Fluxes are represented by their nodal values,
f*_hat = f*(q_hat) at every space-time node (eqs. st.fs, nodal.eval).  The
weak form with only the time derivative integrated by parts (eqs. pde.weak1
to pde.weak3) becomes the element-local system of eq. pde.weak4

    K^1 q_hat + sum_k K^(k) f*_k(q_hat) = F^0 w_hat        (S = 0),

whose matrices are tensor products of one-dimensional integrals; they are
assembled here as dense Kronecker products of exact 1D integrals, so every
entry is the integral the paper defines.  It is solved with the fixed-point
iteration of eq. stdg.final,

    K^1 q_hat^(k+1) = F^0 w_hat - sum_k K^(k) f*_k(q_hat^k),

from the initial guess q_hat^0 = w_hat at every time node (the paper cites a
MUSCL-type guess whose formula it does not give; the fixed point does not
depend on the guess).  The paper gives no stopping rule; a cell stops at
the first iteration with max |q^(k+1) - q^k| <= tol * max(1, max |w_hat|),
the maxima taken over the cell's variables and nodes, so the threshold is
fixed by the reconstructed data before the iteration starts.

Index conventions: spatial nodal index a = p_x + n p_y (+ n^2 p_z); the
space-time index is a + n^d s, time slowest.  F^0 is read with the spatial
multi-index of w_hat as its column index (the printed definition names it
with a different subscript than the system uses).
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from .basis import basis


def _kron_all(mats):
    out = np.array([[1.0]])
    for m in mats:
        out = np.kron(out, m)
    return out


@lru_cache(maxsize=None)
def spacetime_matrices(M: int, dim: int):
    """Dense K^1, [K^xi, K^eta(, K^zeta)] and F^0 (Section 2.3 definitions).

    The Kronecker factor order is (time, z, y, x) so that the flat index is
    a + n^d s with x fastest.
    """
    b = basis(M)
    Mt, Ms1, S1 = b.mass, b.mass, b.stiff
    # spatial factor lists, slowest (z) first, fastest (x) last
    space_mass = [Ms1] * dim
    K1 = _kron_all([b.time_matrix()] + space_mass)
    Kk = []
    for k in range(dim):                       # k = 0 -> x (fastest factor)
        facs = list(space_mass)
        facs[dim - 1 - k] = S1                 # derivative along axis k
        Kk.append(_kron_all([Mt] + facs))
    F0 = _kron_all([b.psi0[:, None]] + space_mass)
    return K1, Kk, F0


@lru_cache(maxsize=None)
def picard_operators(M: int, dim: int):
    """(K^1)^-1 F^0 and (K^1)^-1 K^(k): the two parts of eq. stdg.final."""
    K1, Kk, F0 = spacetime_matrices(M, dim)
    P0 = np.linalg.solve(K1, F0)
    Pk = [np.linalg.solve(K1, K) for K in Kk]
    return P0, Pk


def spatial_flat(w: np.ndarray, dim: int) -> np.ndarray:
    """w[v, C, p_x, p_y(, p_z)] -> w[v, C, a] with a = p_x + n p_y (+ n^2 p_z)."""
    axes = (0, 1) + tuple(range(2 + dim - 1, 1, -1))   # reverse nodal axes
    wt = np.transpose(w, axes)
    return wt.reshape(w.shape[0], w.shape[1], -1)


def predict(system, w: np.ndarray, courant: list, M: int, dim: int,
            tol: float = 1e-14, max_iter: int = 64):
    """Space-time predictor q_hat of every cell.

    w       : w_hat[v, C, p_x, p_y(, p_z)] from the reconstruction
    courant : per axis k, dt/dx_k (scalar or per-cell array of length C)
    Returns (q[v, C, n^(d+1)] with index a + n^d s, iterations[C], converged[C]).
    """
    n = M + 1
    P0, Pk = picard_operators(M, dim)
    wf = spatial_flat(w, dim)                              # [v, C, n^d]
    C = wf.shape[1]
    cour = [np.broadcast_to(np.asarray(c, dtype=float), (C,)) for c in courant]
    rhs0 = wf @ P0.T                                       # (K1^-1 F0) w_hat
    q = np.tile(wf, n)                                     # q^0 = w_hat
    iters = np.zeros(C, dtype=np.int64)
    done = np.zeros(C, dtype=bool)
    scale = np.maximum(1.0, np.max(np.abs(wf), axis=(0, 2)))   # per cell
    for it in range(1, max_iter + 1):
        act = ~done
        qa = q[:, act]
        qn = rhs0[:, act].copy()
        for k in range(dim):
            fk = system.flux(qa, k) * cour[k][act][None, :, None]
            qn -= fk @ Pk[k].T
        delta = np.max(np.abs(qn - qa), axis=(0, 2))
        q[:, act] = qn
        iters[act] = it
        newly = delta <= tol * scale[act]
        idx = np.flatnonzero(act)
        done[idx[newly]] = True
        if done.all():
            break
    return q, iters, done
