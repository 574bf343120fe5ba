"""One-step ADER-WENO finite-volume scheme on a uniform Cartesian mesh, oracle side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

One step (Section 2):
  1. time step from the CFL condition on the current averages;
  2. WENO reconstruction w_h of every cell (Section 2.2, oracle/weno.py);
  3. space-time predictor q_h of every cell (Section 2.3, oracle/predictor.py);
  4. numerical fluxes: Rusanov flux (eq. rusanov), or the Osher-type flux
     (eq. osher) with a 3-point Gauss-Legendre path integral of |A| taken
     from the eigendecomposition of the flux Jacobian, between the two predictor
     traces at the tensor Gauss-Legendre points of each face in the transverse
     directions and in time, summed with the Gauss weights, which is the
     space-time average of eqs. flux:F, flux:G, flux:H on the unit reference
     face (the same nodes as the predictor);
  5. conservative update of the cell averages (eq. finite_vol, S = 0).

Readings where the text is silent:
  * CFL: dt = CFL / max_cells sum_k (|v_k| + c) / dx_k on the averages at t^n,
    clipped to the end time;
  * |s_max| of the Rusanov flux is taken per space-time point as the larger of
    |v_n| + c over the two traces (|a_n| for advection);
  * transmissive boundaries: zero-gradient ghost averages for the stencils, and
    at a boundary face the outer trace equals the inner trace (outflow).

State arrays are U[v, i, j(, k)] with the x index first.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .basis import basis
from .predictor import predict
from .weno import bc_index, reconstruct


@dataclass
class Problem:
    dim: int
    M: int
    system: object                    # physics.Euler or physics.LinearAdvection
    n: tuple                          # cells per axis
    lo: tuple
    hi: tuple
    bc: list = field(default_factory=lambda: ["periodic"] * 3)
    cfl: float = 0.9
    tol: float = 1e-14
    max_iter: int = 64
    flux: str = "rusanov"             # "rusanov" (eq. rusanov) or "osher" (eq. osher)

    @property
    def dx(self):
        return [(self.hi[k] - self.lo[k]) / self.n[k] for k in range(self.dim)]

    @property
    def ncells(self):
        return int(np.prod(self.n[:self.dim]))


def all_cells(prob: Problem) -> np.ndarray:
    """[C, d] index array of every cell, x fastest (cell = i + nx j + ...)."""
    grids = np.meshgrid(*[np.arange(prob.n[k]) for k in range(prob.dim)],
                        indexing="ij")
    cells = np.stack([g.ravel(order="F") for g in grids], axis=1)
    return cells


def cfl_dt(prob: Problem, U: np.ndarray, t: float = 0.0,
           t_end: float = np.inf) -> float:
    """dt = CFL / max over cells of sum_k (largest |eigenvalue|_k) / dx_k."""
    s = sum(prob.system.max_speed(U, k) / prob.dx[k] for k in range(prob.dim))
    dt = prob.cfl / float(np.max(s))
    return min(dt, t_end - t)


def traces(q: np.ndarray, prob: Problem, k: int, side: int) -> np.ndarray:
    """Predictor values on the face xi_k = side (0 or 1) of each cell.

    q[v, C, a + n^d s] -> T[v, C, s, remaining transverse nodal axes]; the
    trace is sum_a psi_a(side) q_(..a..) along axis k.
    """
    b = basis(prob.M)
    n, d = b.n, prob.dim
    Q = q.reshape(q.shape[0], q.shape[1], *([n] * (d + 1)))  # [v,C,s,(pz),py,px]
    psi = b.psi1 if side == 1 else b.psi0
    return np.moveaxis(Q, 2 + d - k, -1) @ psi


def rusanov(system, qL: np.ndarray, qR: np.ndarray, k: int) -> np.ndarray:
    """Rusanov / local Lax-Friedrichs flux of eq. rusanov along axis k."""
    smax = np.maximum(system.max_speed(qL, k), system.max_speed(qR, k))
    return 0.5 * (system.flux(qL, k) + system.flux(qR, k)) - 0.5 * smax * (qR - qL)


def flux_jacobian(system, Q: np.ndarray, k: int) -> np.ndarray:
    """A = d f_k / d u at the states Q[nv, N] -> [N, nv, nv], by complex-step
    differentiation (exact to rounding for the rational fluxes used here)."""
    nv, npts = Q.shape
    J = np.empty((npts, nv, nv))
    h = 1e-30
    for j in range(nv):
        dq = Q.astype(complex)
        dq[j] += 1j * h
        J[:, :, j] = (system.flux(dq, k).imag / h).T
    return J


def abs_matrix(A: np.ndarray) -> np.ndarray:
    """|A| = R |Lambda| R^-1 from the eigendecomposition of A[..., nv, nv]
    (hyperbolic: real eigenvalues, a complete set of eigenvectors)."""
    lam, R = np.linalg.eig(A)
    return np.real(R @ (np.abs(lam)[..., :, None] * np.linalg.inv(R)))


OSHER_NODES = 3  # Gauss-Legendre points of the path integral (the paper asks for >= 2)


def osher(system, qL: np.ndarray, qR: np.ndarray, k: int) -> np.ndarray:
    """Osher-type flux of eq. osher along axis k: the path integral of |A|
    along psi(s) = qL + s (qR - qL) by Gauss-Legendre quadrature in s."""
    from .basis import gauss_legendre
    s, w = gauss_legendre(OSHER_NODES)
    shape = qL.shape
    a = qL.reshape(shape[0], -1)
    dq = qR.reshape(shape[0], -1) - a
    Aint = sum(w[j] * abs_matrix(flux_jacobian(system, a + s[j] * dq, k))
               for j in range(OSHER_NODES))                      # [N, nv, nv]
    diss = np.einsum("pij,jp->ip", Aint, dq)
    central = 0.5 * (system.flux(qL, k) + system.flux(qR, k))
    return central - 0.5 * diss.reshape(shape)


def numerical_flux(prob, qL: np.ndarray, qR: np.ndarray, k: int) -> np.ndarray:
    if prob.flux == "osher":
        return osher(prob.system, qL, qR, k)
    return rusanov(prob.system, qL, qR, k)


def face_average(Ft: np.ndarray, prob: Problem) -> np.ndarray:
    """Gauss-Legendre tensor sum over (time, transverse) points: Ft[v, F, ...]."""
    w = basis(prob.M).weights
    out = Ft
    for _ in range(prob.dim):            # time + (d-1) transverse axes
        out = out @ w
    return out


def _predict_cells(prob, U, cells, dt, chunk=16384):
    """Reconstruction + predictor of the given cells, processed in chunks."""
    cour = [dt / h for h in prob.dx]
    qs, its = [], []
    for start in range(0, len(cells), chunk):
        cc = cells[start:start + chunk]
        w = reconstruct(U, cc, prob.M, prob.bc[:prob.dim])
        q, it, ok = predict(prob.system, w, cour, prob.M, prob.dim,
                            prob.tol, prob.max_iter)
        if not ok.all():
            raise RuntimeError("predictor fixed-point iteration did not converge"
                               f" within {prob.max_iter} iterations")
        qs.append(q)
        its.append(it)
    return np.concatenate(qs, axis=1), np.concatenate(its)


def step(prob: Problem, U: np.ndarray, dt: float):
    """One full-mesh step; every face flux is computed exactly once.

    Returns (U_new, info) with info['picard_iters'] per cell.
    """
    d = prob.dim
    cells = all_cells(prob)
    C = len(cells)
    shape = tuple(prob.n[:d])
    q, iters = _predict_cells(prob, U, cells, dt)
    lin = np.arange(C).reshape(shape, order="F")        # lin[i, j(, k)] -> cell
    Unew = U.copy()
    for k in range(d):
        nk = shape[k]
        periodic = prob.bc[k] == "periodic"
        # faces along k indexed by the cell on their right, 0..nk (nk+1 faces)
        nf = nk if periodic else nk + 1
        right_idx = np.arange(nf)
        left_idx = right_idx - 1
        # lin arranged with axis k first: [nk, rest]
        link = np.moveaxis(lin, k, 0).reshape(nk, -1)
        rest = link.shape[1]
        tr1 = traces(q, prob, k, 1)          # [v, C, ...] at xi_k = 1
        tr0 = traces(q, prob, k, 0)          # at xi_k = 0
        li = bc_index(left_idx, nk, prob.bc[k])
        ri = bc_index(right_idx, nk, prob.bc[k])
        Lc = link[li].ravel()
        Rc = link[ri].ravel()
        qL = tr1[:, Lc]
        qR = tr0[:, Rc]
        if not periodic:
            # outflow at the two boundary faces: outer trace = inner trace
            qL = qL.reshape(qL.shape[0], nf, rest, *qL.shape[2:])
            qR = qR.reshape(qR.shape[0], nf, rest, *qR.shape[2:])
            qL[:, 0] = qR[:, 0]
            qR[:, nf - 1] = qL[:, nf - 1]
            qL = qL.reshape(qL.shape[0], nf * rest, *qL.shape[3:])
            qR = qR.reshape(qR.shape[0], nf * rest, *qR.shape[3:])
        F = face_average(numerical_flux(prob, qL, qR, k), prob)  # [v, nf*rest]
        F = F.reshape(F.shape[0], nf, rest)
        lo_face = np.arange(nk)
        hi_face = np.arange(1, nk + 1) % nf if periodic else np.arange(1, nk + 1)
        dU = (F[:, hi_face] - F[:, lo_face]).reshape(F.shape[0], nk, rest)
        # back to the mesh layout
        dU_full = np.empty((U.shape[0], C))
        dU_full[:, link.ravel()] = dU.reshape(U.shape[0], -1)
        Unew -= (dt / prob.dx[k]) * dU_full.reshape(
            (U.shape[0],) + shape, order="F")
    return Unew, {"picard_iters": iters}


def step_cells(prob: Problem, U: np.ndarray, dt: float, cells: np.ndarray):
    """Updated averages of selected cells only (sampled checks at large sizes).

    Computes, for each requested cell, its own predictor and those of its 2d
    face neighbours, the fluxes through its 2d faces, and the update.
    Returns (values[v, len(cells)], picard iterations of the requested cells).
    """
    d = prob.dim
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, d)
    shape = np.array(prob.n[:d])
    nb = [cells]
    for k in range(d):
        for sgn in (-1, 1):
            c = cells.copy()
            c[:, k] = bc_index(c[:, k] + sgn, shape[k], prob.bc[k])
            nb.append(c)
    allc = np.unique(np.concatenate(nb), axis=0)
    q, iters = _predict_cells(prob, U, allc, dt)
    key = {tuple(c): i for i, c in enumerate(allc)}
    pos = lambda cc: np.array([key[tuple(c)] for c in cc])
    me = pos(cells)
    out = U[(slice(None),) + tuple(cells.T)].copy()
    for k in range(d):
        tr1 = traces(q, prob, k, 1)
        tr0 = traces(q, prob, k, 0)
        fluxes = []
        for sgn in (-1, 1):
            raw = cells[:, k] + sgn
            c = cells.copy()
            c[:, k] = bc_index(raw, shape[k], prob.bc[k])
            other = pos(c)
            outside = (raw < 0) | (raw >= shape[k])
            if sgn < 0:           # low face: left = neighbour, right = me
                qL, qR = tr1[:, other].copy(), tr0[:, me].copy()
                if prob.bc[k] != "periodic":
                    qL[:, outside] = qR[:, outside]
            else:                 # high face: left = me, right = neighbour
                qL, qR = tr1[:, me].copy(), tr0[:, other].copy()
                if prob.bc[k] != "periodic":
                    qR[:, outside] = qL[:, outside]
            fluxes.append(face_average(numerical_flux(prob, qL, qR, k), prob))
        out -= (dt / prob.dx[k]) * (fluxes[1] - fluxes[0])
    return out, iters[me]


def run(prob: Problem, U: np.ndarray, t_end: float, max_steps: int = 10**9):
    """Advance to t_end (or max_steps); returns (U, t, steps, dts)."""
    t = 0.0
    dts = []
    while t < t_end and len(dts) < max_steps:
        dt = cfl_dt(prob, U, t, t_end)
        U, _ = step(prob, U, dt)
        t += dt
        dts.append(dt)
    return U, t, len(dts), dts
