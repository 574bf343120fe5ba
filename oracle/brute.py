"""Brute-force routes that pin the oracle, written independently of it.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Nothing here reuses the oracle's basis, matrices or contractions:

* ``weno_1d_monomial`` rebuilds every stencil polynomial in the monomial basis
  by solving the conservation conditions of eq. rec.x with exact monomial
  moments, evaluates the oscillation indicator of eq. sigmas from monomial
  derivatives, and samples the combined polynomial at the Gauss nodes;
* ``predictor_newton`` assembles the element-local system of eq. pde.weak3 by
  direct (d+1)-dimensional tensor quadrature of the space-time test and trial
  functions (no Kronecker structure), and solves it with Newton's method and a
  finite-difference Jacobian instead of the Picard iteration.
"""
from __future__ import annotations

import itertools

import numpy as np
from numpy.polynomial.legendre import leggauss


def _gl01(n):
    x, w = leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _stencil_list(M, lam_central, lam_side):
    """Stencil extents (L, R) and linear weights, from Section 2.2's rules."""
    if M % 2 == 0:
        return [(M // 2, M // 2, lam_central), (M, 0, lam_side), (0, M, lam_side)]
    h = M // 2
    return [(h + 1, h, lam_central), (h, h + 1, lam_central),
            (M, 0, lam_side), (0, M, lam_side)]


def weno_1d_monomial(values: np.ndarray, M: int, lam_central: float,
                     lam_side: float, eps: float, r: int) -> np.ndarray:
    """WENO along the last axis (2M+1 averages) via monomial polynomials.

    The constants are passed in (the tests take them from the values the
    paper states) so that this route shares nothing with the oracle.
    """
    n = M + 1
    nodes, _ = _gl01(n)
    out_polys, om = [], []
    for (L, R, lam) in _stencil_list(M, lam_central, lam_side):
        offs = np.arange(-L, R + 1)
        # exact averages of xi^m over [o, o+1]
        A = np.array([[((o + 1.0) ** (m + 1) - float(o) ** (m + 1)) / (m + 1)
                       for m in range(n)] for o in offs])
        win = values[..., M - L:M + R + 1]
        coef = np.linalg.solve(A, win.reshape(-1, n).T).T.reshape(win.shape)
        # sigma = sum_{alpha=1..M} int_0^1 (d^alpha P)^2
        sigma = np.zeros(values.shape[:-1])
        for alpha in range(1, M + 1):
            # derivative coefficients c'_j for monomial j >= alpha
            dco = np.zeros(coef.shape[:-1] + (n,))
            for j in range(alpha, n):
                fac = np.prod(np.arange(j - alpha + 1, j + 1, dtype=float))
                dco[..., j - alpha] = coef[..., j] * fac
            # int_0^1 (sum_i d_i xi^i)^2 = sum_ij d_i d_j / (i + j + 1)
            H = np.array([[1.0 / (i + j + 1) for j in range(n)] for i in range(n)])
            sigma = sigma + np.einsum('...i,ij,...j->...', dco, H, dco)
        om.append(lam / (sigma + eps) ** r)
        V = np.vander(nodes, n, increasing=True)          # [node, m]
        out_polys.append(coef @ V.T)                       # values at nodes
    tot = sum(om)
    return sum((o / tot)[..., None] * p for o, p in zip(om, out_polys))


def _lagrange_values(nodes, pts):
    """psi_l(pts) and d psi_l / dx (pts) for the Lagrange basis on nodes."""
    n = len(nodes)
    V = np.ones((len(pts), n))
    dV = np.zeros((len(pts), n))
    for l in range(n):
        for i, x in enumerate(pts):
            prod = 1.0
            for k in range(n):
                if k != l:
                    prod *= (x - nodes[k]) / (nodes[l] - nodes[k])
            V[i, l] = prod
            s = 0.0
            for j in range(n):
                if j == l:
                    continue
                term = 1.0 / (nodes[l] - nodes[j])
                for k in range(n):
                    if k != l and k != j:
                        term *= (x - nodes[k]) / (nodes[l] - nodes[k])
                s += term
            dV[i, l] = s
    return V, dV


def predictor_newton(system, w: np.ndarray, courant, M: int, dim: int,
                     newton_tol=1e-14, max_newton=50):
    """Solve eq. pde.weak3 for one cell by quadrature assembly + Newton.

    w[v, p_x, p_y(, p_z)] nodal reconstruction of ONE cell.  Returns
    q[v, a + n^d s] (same ordering as the oracle predictor).
    """
    n = M + 1
    nodes, _ = _gl01(n)
    nq = n + 2                                   # over-integrating rule
    qx, qw = _gl01(nq)
    V, dV = _lagrange_values(nodes, qx)          # [quad pt, basis]
    V1, _ = _lagrange_values(nodes, [1.0])
    V0, _ = _lagrange_values(nodes, [0.0])
    nst = n ** (dim + 1)
    nsp = n ** dim
    # multi-index lists: flat = a + n^d s with a = px + n py (+ n^2 pz)
    idx = [tuple(np.unravel_index(f, (n,) * (dim + 1), order="F"))
           for f in range(nst)]                  # (px, py, [pz,] s)
    sp_idx = [tuple(np.unravel_index(a, (n,) * dim, order="F"))
              for a in range(nsp)]
    qpts = list(itertools.product(range(nq), repeat=dim + 1))   # (x, y, [z,] t)

    def theta(f, qp, dk=None):
        val = 1.0
        for ax in range(dim + 1):
            b = idx[f][ax]
            if dk == ax:
                val *= dV[qp[ax], b]
            else:
                val *= V[qp[ax], b]
        return val

    # dense matrices by quadrature
    Th = np.array([[theta(f, qp) for f in range(nst)] for qp in qpts])
    Wq = np.array([np.prod([qw[i] for i in qp]) for qp in qpts])
    dTh_t = np.array([[theta(f, qp, dk=dim) for f in range(nst)] for qp in qpts])
    dTh = [np.array([[theta(f, qp, dk=k) for f in range(nst)] for qp in qpts])
           for k in range(dim)]
    # spatial quadrature on the time slices tau = 1 and tau = 0
    spts = list(itertools.product(range(nq), repeat=dim))
    Ws = np.array([np.prod([qw[i] for i in sp]) for sp in spts])
    def space_val(f, sp):
        val = 1.0
        for ax in range(dim):
            val *= V[sp[ax], idx[f][ax]]
        return val
    S = np.array([[space_val(f, sp) for f in range(nst)] for sp in spts])
    T1 = np.array([V1[0, idx[f][dim]] for f in range(nst)])
    T0 = np.array([V0[0, idx[f][dim]] for f in range(nst)])
    Psp = np.array([[np.prod([V[sp[ax], sp_idx[m][ax]] for ax in range(dim)])
                     for m in range(nsp)] for sp in spts])
    # K1 = int theta_q(x,1) theta_p(x,1) - int d_tau theta_q theta_p
    K1 = (S * T1).T @ (Ws[:, None] * (S * T1)) - dTh_t.T @ (Wq[:, None] * Th)
    Kk = [Th.T @ (Wq[:, None] * dTh[k]) for k in range(dim)]
    F0 = (S * T0).T @ (Ws[:, None] * Psp)

    wf = np.stack([np.transpose(w[v], tuple(range(dim - 1, -1, -1))).ravel()
                   for v in range(w.shape[0])])        # [v, a]
    rhs = (F0 @ wf.T).T                                 # [v, nst]
    nv = w.shape[0]

    def residual(x):
        q = x.reshape(nv, nst)
        r = (K1 @ q.T).T - rhs
        for k in range(dim):
            r = r + courant[k] * (Kk[k] @ system.flux(q, k).T).T
        return r.ravel()

    x = np.tile(wf, n).ravel()
    for _ in range(max_newton):
        r = residual(x)
        J = np.empty((x.size, x.size))
        h = 1e-7
        for i in range(x.size):
            xp = x.copy()
            xp[i] += h
            xm = x.copy()
            xm[i] -= h
            J[:, i] = (residual(xp) - residual(xm)) / (2 * h)
        dx = np.linalg.solve(J, -r)
        x = x + dx
        if np.max(np.abs(dx)) <= newton_tol * max(1.0, np.max(np.abs(x))):
            break
    return x.reshape(nv, nst)
