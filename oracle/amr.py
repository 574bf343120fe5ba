"""Cell-by-cell AMR with time-accurate local time stepping (Section 3), oracle side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Mesh.  Level 0 is the uniform mesh of the Problem; level l refines it by
r^l along every axis (eq. refine-factor, r >= M).  Every level is held as a
dense array over its whole index space, with a status per cell:
    ACTIVE  (sigma = 0)   updated by the finite volume scheme on its level;
    VCHILD  (sigma = 1)   virtual child of an active mother: its average is
                          the projection of the mother's space-time predictor
                          (Section 3.1.3);
    VMOTHER (sigma = -1)  virtual mother: the average of its r^d children
                          (eq. average);
    ABSENT                not part of the mesh.
The mother of level-l cell i is i // r on level l-1; the children of a cell
are the r^d cells i*r + a, 0 <= a < r (consecutive blocks).

Refinement (built from the initial data, then changed by regrid()).  A cell of level l < L is
flagged when the Loehner indicator (eq. indicator) of its level's initial
averages exceeds chi_ref, and so are its Voronoi neighbours up to 'buffer'
layers (the paper names no buffer; without one, a single unflagged cell on a
front leaves a hole of virtual cells in the refined region, whose projected
averages spoil the fine stencils next to the front).  Flags are closed so that the rules of Section 3.1
hold: the mother of any cell within the Voronoi neighbourhood of a flagged
cell is flagged (levels of Voronoi neighbours differ by at most one, and a
refined cell's Voronoi neighbours exist on the finer level), and flags nest.
Children of flagged cells are ACTIVE (VMOTHER if flagged themselves); the
children of the active Voronoi neighbours of flagged cells are VCHILD.  With
r >= M the (2M+1)^d reconstruction patch of every active cell lies in cells
that are not ABSENT (checked).

Local time stepping (Section 3.1.2).  Delta t_l = r Delta t_(l+1); one
level-0 step advances level l by r^l substeps, finest first.  advance(l, t)
(all levels >= l are at time t):
  1. VMOTHER averages of levels >= l from their children, finest first;
  2. VCHILD averages of level l: projection of the mother's predictor at the
     mother-local time of t;
  3. reconstruction (Section 2.2) and predictor (Section 2.3) of the active
     cells of level l over [t, t + Delta t_l];
  4. r substeps of level l+1 (its memory variables cleared first);
  5. update of the active cells of level l (eq. finite_vol):
       - face to an active cell of the same level: the usual flux;
       - face to a VCHILD (the neighbour is coarser): the flux between this
         cell's predictor and the coarse mother's predictor evaluated at this
         face's Gauss points and this substep's time nodes; it updates this
         cell and is added to the VCHILD's memory variable for that face;
       - face to a VMOTHER (the neighbour is finer): the average of the
         memory variables of this cell's virtual children on that face, which
         hold the fine fluxes of all r substeps (eq. memory.sum);
       - face through a transmissive boundary: outflow.
Delta t_0 = min over levels of r^l * CFL / max_active sum_k speed_k / dx_(l,k),
clipped to the end time.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from .basis import basis
from .predictor import predict
from .scheme import Problem, face_average, numerical_flux, traces
from .weno import bc_index, reconstruct

ABSENT, VMOTHER, ACTIVE, VCHILD = -2, -1, 0, 1


# ------------------------------------------------------------ indicator
def _shift(Phi, offs, bcs):
    """Phi at index + offs on a dense level grid (periodic wrap or
    transmissive clamp)."""
    idx = np.ix_(*[bc_index(np.arange(n) + o, n, bc) for n, o, bc in zip(Phi.shape, offs, bcs)])
    return Phi[idx]


def lohner(Phi: np.ndarray, bcs, eps: float = 0.01) -> np.ndarray:
    """Loehner indicator chi (eq. indicator) on a dense level grid, in index
    units (the mesh widths cancel).  Per axis pair (k, l):
      k == l: D = P+ - 2 P + P-, den = |P+ - P| + |P - P-| + eps (|P+| + 2|P| + |P-|);
      k != l: with A = P(+k+l) - P(-k+l), B = P(+k-l) - P(-k-l):
              D = (A - B) / 4, den = (|A| + |B|) / 4 + eps (sum of |P| at the
              four diagonal points) / 4;
    chi = sqrt(sum D^2 / sum den^2), 0 where the denominator vanishes."""
    d = Phi.ndim
    num = np.zeros_like(Phi)
    den = np.zeros_like(Phi)
    for k in range(d):
        for m in range(d):
            if k == m:
                e = [0] * d
                e[k] = 1
                p, q = _shift(Phi, e, bcs), _shift(Phi, [-x for x in e], bcs)
                D = p - 2.0 * Phi + q
                De = np.abs(p - Phi) + np.abs(Phi - q) + eps * (np.abs(p) + 2.0 * np.abs(Phi) + np.abs(q))
            else:
                def s(a, b):
                    o = [0] * d
                    o[k], o[m] = a, b
                    return _shift(Phi, o, bcs)
                pp, pm, mp, mm = s(1, 1), s(1, -1), s(-1, 1), s(-1, -1)
                A, B = pp - mp, pm - mm
                D = 0.25 * (A - B)
                De = 0.25 * (np.abs(A) + np.abs(B)) + 0.25 * eps * (
                    np.abs(pp) + np.abs(pm) + np.abs(mp) + np.abs(mm))
            num += D * D
            den += De * De
    out = np.zeros_like(Phi)
    ok = den > 0
    out[ok] = np.sqrt(num[ok] / den[ok])
    return out


# ------------------------------------------------------------ hierarchy
def _dilate(F: np.ndarray, bcs) -> np.ndarray:
    """Voronoi (3^d) neighbourhood of the True cells; no wrap through a
    transmissive boundary."""
    out = F.copy()
    d = F.ndim
    for offs in np.ndindex(*([3] * d)):
        o = [x - 1 for x in offs]
        if not any(o):
            continue
        idx = []
        valid = np.ones(F.shape, dtype=bool)
        for ax, (n, oo, bc) in enumerate(zip(F.shape, o, bcs)):
            raw = np.arange(n) + oo
            if bc == "periodic":
                idx.append(np.mod(raw, n))
            else:
                inside = (raw >= 0) & (raw < n)
                idx.append(np.clip(raw, 0, n - 1))
                sh = [1] * d
                sh[ax] = n
                valid &= inside.reshape(sh)
        out |= F[np.ix_(*idx)] & valid
    return out


def _mothers(F: np.ndarray, r: int) -> np.ndarray:
    """Cells of the coarser level with at least one True child."""
    d = F.ndim
    sh = []
    for n in F.shape:
        sh += [n // r, r]
    G = F.reshape(sh)
    return G.any(axis=tuple(range(1, 2 * d, 2)))


def _children(F: np.ndarray, r: int) -> np.ndarray:
    out = F
    for ax in range(F.ndim):
        out = np.repeat(out, r, axis=ax)
    return out


def _close_flags(F, bcs, r: int, L: int):
    """Rules 4 and 5 of Section 3.1 on refinement flags F[0..L-1]: the mother
    of every cell in the Voronoi neighbourhood of a flagged level-l cell is
    flagged on level l-1 (so Voronoi neighbours differ by at most one level
    and a refined cell's Voronoi neighbours exist on the finer level), and
    flags nest (a flagged cell has a flagged mother)."""
    F = [np.asarray(f, dtype=bool).copy() for f in F]
    for l in range(L - 1, 0, -1):
        F[l - 1] |= _mothers(_dilate(F[l], bcs), r)
    for l in range(1, L):
        F[l] &= _children(F[l - 1], r)
    return F


def _status_from_flags(F, shape, bcs, r: int, L: int):
    """Status arrays of all levels from closed flags: children of flagged
    cells are active (virtual mothers if flagged themselves); children of the
    unflagged Voronoi neighbours of flagged cells are virtual children;
    every other cell of levels >= 1 is absent."""
    st = [np.full(shape[0], ACTIVE, dtype=np.int8)]
    if L > 0:
        st[0][F[0]] = VMOTHER
    for l in range(1, L + 1):
        s = np.full(shape[l], ABSENT, dtype=np.int8)
        near = _dilate(F[l - 1], bcs) & ~F[l - 1]
        assert np.all(st[l - 1][near] == ACTIVE)
        s[_children(near, r)] = VCHILD
        kids = _children(F[l - 1], r)
        s[kids] = ACTIVE
        if l < L:
            s[kids & F[l]] = VMOTHER
        st.append(s)
    return st


class Hierarchy:
    """Dense per-level state and status arrays of an AMR mesh."""

    def __init__(self, prob: Problem, r: int, L: int, U_levels, chi_ref: float = 0.2,
                 eps: float = 0.01, indicator_var: int = 0, flags=None, buffer: int = 1,
                 chi_rec: float | None = None):
        if r < max(prob.M, 2):
            raise ValueError("the refinement factor must satisfy r >= M (and r >= 2)")
        self.prob, self.r, self.L, self.d = prob, r, L, prob.dim
        self.chi_ref, self.eps, self.indicator_var, self.buffer = chi_ref, eps, indicator_var, buffer
        self.chi_rec = chi_ref if chi_rec is None else chi_rec
        d = self.d
        self.bcs = list(prob.bc[:d])
        self.shape = [tuple(prob.n[k] * r ** l for k in range(d)) for l in range(L + 1)]
        if flags is None:
            flags = [lohner(U_levels[l][indicator_var], self.bcs, eps) > chi_ref
                     for l in range(L)]
            for _ in range(buffer):          # buffer layers around indicator flags
                flags = [_dilate(f, self.bcs) for f in flags]
        F = _close_flags(flags, self.bcs, r, L)
        self.flags = F
        st = _status_from_flags(F, self.shape, self.bcs, r, L)
        self.status = st
        self.U = []
        for l in range(L + 1):
            U = np.array(U_levels[l], dtype=float, copy=True)
            U[:, st[l] == ABSENT] = np.nan
            self.U.append(U)
        self.mem = [None] + [np.zeros((d, 2, prob.system.nv) + self.shape[l])
                             for l in range(1, L + 1)]
        self.q = [None] * (L + 1)
        self.pos = [None] * (L + 1)
        self.sub = [0] * (L + 1)
        self.picard_iters = 0
        self.cell_updates = 0
        self._check_patches()

    # ------------------------------------------------------------ helpers
    def level_problem(self, l: int) -> Problem:
        return replace(self.prob, n=self.shape[l])

    def dx(self, l: int):
        return [h / self.r ** l for h in self.prob.dx]

    def active(self, l: int) -> np.ndarray:
        """[C, d] active cells of level l, x fastest."""
        A = self.status[l] == ACTIVE
        idx = np.argwhere(A)                      # C-order: last axis fastest
        order = np.lexsort(tuple(idx[:, k] for k in range(self.d)))
        return idx[order]

    def counts(self):
        return [{name: int((s == val).sum()) for name, val in
                 (("active", ACTIVE), ("vchild", VCHILD), ("vmother", VMOTHER))}
                for s in self.status]

    def _check_patches(self):
        M = self.prob.M
        for l in range(self.L + 1):
            cells = self.active(l)
            for offs in np.ndindex(*([2 * M + 1] * self.d)):
                idx = tuple(bc_index(cells[:, k] + offs[k] - M, self.shape[l][k], self.bcs[k])
                            for k in range(self.d))
                if np.any(self.status[l][idx] == ABSENT):
                    raise AssertionError(f"level {l}: an active cell's stencil leaves the mesh")

    def total(self) -> np.ndarray:
        """Integral of the conserved variables over the domain (active cells)."""
        tot = 0.0
        for l in range(self.L + 1):
            vol = np.prod(self.dx(l))
            tot = tot + vol * self.U[l][:, self.status[l] == ACTIVE].sum(axis=1)
        return tot


# ------------------------------------------------------------ operators
def subcell_average_matrix(M: int, r: int) -> np.ndarray:
    """P[a, p] = r * int_{a/r}^{(a+1)/r} psi_p(xi) dxi: the average of basis
    function p over child interval a (projection, Section 3.1.3)."""
    b = basis(M)
    P = np.empty((r, b.n))
    for p in range(b.n):
        ant = b.psi[p].integ()
        for a in range(r):
            P[a, p] = r * (ant((a + 1) / r) - ant(a / r))
    return P


def _eval_1d(M: int, x: np.ndarray) -> np.ndarray:
    """E[p, i] = psi_p(x_i)."""
    b = basis(M)
    return np.array([b.psi[p](x) for p in range(b.n)])


def average_down(H: Hierarchy, l: int):
    """VMOTHER averages of levels L-1 .. l from their children (eq. average)."""
    r, d = H.r, H.d
    for lev in range(H.L - 1, l - 1, -1):
        st = H.status[lev]
        vm = st == VMOTHER
        if not vm.any():
            continue
        sh = [H.U[lev + 1].shape[0]]
        for n in H.shape[lev]:
            sh += [n, r]
        Uc = H.U[lev + 1].reshape(sh)
        mean = Uc.mean(axis=tuple(range(2, 2 + 2 * d, 2)))
        H.U[lev][:, vm] = mean[:, vm]


def project(H: Hierarchy, l: int):
    """VCHILD averages of level l: the mother's predictor at the mother-local
    time sub / r, averaged over the child's sub-cell."""
    r, d, M = H.r, H.d, H.prob.M
    n = M + 1
    vc = np.argwhere(H.status[l] == VCHILD)
    if len(vc) == 0:
        return
    P = subcell_average_matrix(M, r)
    tau = H.sub[l] / r
    ptime = np.array([basis(M).psi[s](tau) for s in range(n)])
    mothers = vc // r
    offs = vc % r
    pos = H.pos[l - 1][tuple(mothers.T)]
    assert np.all(pos >= 0), "a virtual child's mother is not active"
    q = H.q[l - 1][:, pos]                                # [v, C, n^(d+1)]
    Q = q.reshape(q.shape[0], q.shape[1], *([n] * (d + 1)))  # [v, C, s, (pz), py, px]
    val = np.einsum("vcs...,s->vc...", Q, ptime)          # [v, C, (pz), py, px]
    for k in range(d):                                    # contract px, then py, ...
        Pk = P[offs[:, k]]                                # [C, n]
        val = np.einsum("vc...p,cp->vc...", val, Pk)
    H.U[l][(slice(None),) + tuple(vc.T)] = val


def coarse_trace(H: Hierarchy, l: int, vchild: np.ndarray, k: int, side: int) -> np.ndarray:
    """Traces of VCHILD cells of level l on their face (axis k, side) at the
    face's Gauss points and at the time nodes of substep H.sub[l]: the
    mother's (level l-1) predictor evaluated at the mapped points.
    Returns T[v, C, s, transverse axes (z, y, x order without k)]."""
    r, d, M = H.r, H.d, H.prob.M
    b = basis(M)
    n = b.n
    mothers, offs = vchild // r, vchild % r
    pos = H.pos[l - 1][tuple(mothers.T)]
    q = H.q[l - 1][:, pos]
    Q = q.reshape(q.shape[0], q.shape[1], *([n] * (d + 1)))   # [v, C, s, (pz), py, px]
    Et = _eval_1d(M, (H.sub[l] + b.nodes) / r)                  # [s', s]
    Q = np.einsum("vcs...,sj->vcj...", Q, Et)                   # time nodes of the substep
    for ax in range(d):                                         # spatial axes x, y, z
        dim_axis = 2 + d - ax                                   # position of p_ax in Q
        if ax == k:
            x = (offs[:, ax] + side) / r                        # [C]
            E = np.stack([_eval_1d(M, x[c:c + 1])[:, 0] for c in range(len(x))])  # [C, p]
            Q = np.moveaxis(Q, dim_axis, -1)
            Q = np.einsum("vc...p,cp->vc...", Q, E)
            Q = np.expand_dims(Q, dim_axis)                     # keep axis positions
        else:
            x = (offs[:, ax][:, None] + b.nodes[None, :]) / r   # [C, nodes]
            E = np.stack([_eval_1d(M, x[c]) for c in range(len(x))])   # [C, p, i]
            Q = np.moveaxis(Q, dim_axis, -1)
            Q = np.einsum("vc...p,cpi->vc...i", Q, E)
            Q = np.moveaxis(Q, -1, dim_axis)
    return np.squeeze(Q, axis=2 + d - k)


def _cell_traces(H: Hierarchy, l: int, pos: np.ndarray, k: int, side: int) -> np.ndarray:
    return traces(H.q[l][:, pos], H.level_problem(l), k, side)


def predict_level(H: Hierarchy, l: int, dt: float):
    prob = H.level_problem(l)
    cells = H.active(l)
    pos = np.full(H.shape[l], -1, dtype=np.int64)
    pos[tuple(cells.T)] = np.arange(len(cells))
    H.pos[l] = pos
    if len(cells) == 0:
        H.q[l] = np.zeros((prob.system.nv, 0, (prob.M + 1) ** (H.d + 1)))
        return
    w = reconstruct(H.U[l], cells, prob.M, H.bcs)
    cour = [dt / h for h in H.dx(l)]
    q, it, ok = predict(prob.system, w, cour, prob.M, H.d, prob.tol, prob.max_iter)
    if not ok.all():
        raise RuntimeError("predictor fixed-point iteration did not converge")
    H.q[l] = q
    H.picard_iters += int(it.sum())


def update_level(H: Hierarchy, l: int, dt: float):
    prob = H.level_problem(l)
    cells = H.active(l)
    if len(cells) == 0:
        return
    r, d = H.r, H.d
    pos = H.pos[l]
    me = pos[tuple(cells.T)]
    st = H.status[l]
    nv = prob.system.nv
    out = H.U[l][(slice(None),) + tuple(cells.T)].copy()
    for k in range(d):
        nk = H.shape[l][k]
        Fs = []
        for side in (0, 1):
            raw = cells[:, k] + (1 if side else -1)
            nb = cells.copy()
            nb[:, k] = bc_index(raw, nk, H.bcs[k])
            outside = (raw < 0) | (raw >= nk)
            nst = st[tuple(nb.T)]
            F = np.full((nv, len(cells)), np.nan)
            mine = _cell_traces(H, l, me, k, side)            # [v, C, s, t...]
            # same-level active neighbour, or a transmissive boundary
            sel = (nst == ACTIVE) | ((H.bcs[k] != "periodic") & outside)
            if sel.any():
                qa = mine[:, sel]
                npos = pos[tuple(nb[sel].T)]
                qb = _cell_traces(H, l, np.maximum(npos, 0), k, 1 - side)
                out_b = outside[sel]
                if H.bcs[k] != "periodic":
                    qb[:, out_b] = qa[:, out_b]
                qL, qR = (qa, qb) if side else (qb, qa)
                F[:, sel] = face_average(numerical_flux(prob, qL, qR, k), prob)
            # coarser neighbour (virtual child of an active mother)
            sel = (nst == VCHILD) & ~((H.bcs[k] != "periodic") & outside)
            if sel.any():
                qa = mine[:, sel]
                qb = coarse_trace(H, l, nb[sel], k, 1 - side)
                qL, qR = (qa, qb) if side else (qb, qa)
                Ff = face_average(numerical_flux(prob, qL, qR, k), prob)
                F[:, sel] = Ff
                slot = H.mem[l][k, 1 - side]                   # view [v, *shape]
                slot[(slice(None),) + tuple(nb[sel].T)] += Ff
            # finer neighbour (virtual mother): sum of the memory variables
            sel = (nst == VMOTHER) & ~((H.bcs[k] != "periodic") & outside)
            if sel.any():
                c = cells[sel]
                acc = np.zeros((nv, len(c)))
                for a in np.ndindex(*([r] * (d - 1))):
                    child = np.empty_like(c)
                    t = 0
                    for ax in range(d):
                        if ax == k:
                            child[:, ax] = c[:, ax] * r + (r - 1 if side else 0)
                        else:
                            child[:, ax] = c[:, ax] * r + a[t]
                            t += 1
                    assert np.all(H.status[l + 1][tuple(child.T)] == VCHILD)
                    acc += H.mem[l + 1][k, side][(slice(None),) + tuple(child.T)]
                F[:, sel] = acc / r ** d
            assert not np.isnan(F).any(), "a face of an active cell has no flux"
            Fs.append(F)
        out -= (dt / H.dx(l)[k]) * (Fs[1] - Fs[0])
    H.U[l][(slice(None),) + tuple(cells.T)] = out
    H.cell_updates += len(cells)


def children_from_mothers(H: Hierarchy, l: int, target: np.ndarray):
    """Averages of the level-l cells in the mask 'target' from their mothers'
    reconstruction (Section 2.2 on level l-1, at the current averages): the
    average of w_h over the child's sub-cell (the projection of Section 3.1.3
    applied to w_h).  The mean of the r^d sub-cell averages is the mother's
    average, so refinement is conservative."""
    r, d, M = H.r, H.d, H.prob.M
    cells = np.argwhere(target)
    if len(cells) == 0:
        return
    moth, inv = np.unique(cells // r, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    idx = tuple(bc_index(moth[:, k][:, None] + np.arange(-M, M + 1)[None, :],
                         H.shape[l - 1][k], H.bcs[k]) for k in range(d))
    for offs in np.ndindex(*([2 * M + 1] * d)):        # every mother's stencil lies in the mesh
        pidx = tuple(idx[k][:, offs[k]] for k in range(d))
        assert np.all(H.status[l - 1][pidx] != ABSENT), "a mother's stencil leaves the mesh"
    w = reconstruct(H.U[l - 1], moth, M, H.bcs)          # [v, Cm, px, py(, pz)]
    P = subcell_average_matrix(M, r)
    val = w[:, inv]                                       # [v, C, px, py(, pz)]
    offs = cells % r
    for k in range(d - 1, -1, -1):                        # contract pz, then py, then px
        val = np.einsum("vc...p,cp->vc...", val, P[offs[:, k]])
    H.U[l][(slice(None),) + tuple(cells.T)] = val


def refinement_flags(H: Hierarchy):
    """Raw flags of levels 0..L-1 at a regrid (Section 3.1.1): an active cell
    is refined when chi > chi_ref; a refined cell (virtual mother) stays
    refined unless chi < chi_rec.  Virtual children are never flagged by the
    indicator (rule 2: a virtual child is activated first)."""
    out = []
    for l in range(H.L):
        with np.errstate(invalid="ignore"):
            chi = lohner(H.U[l][H.indicator_var], H.bcs, H.eps)
        st = H.status[l]
        out.append(((st == ACTIVE) & (chi > H.chi_ref)) | ((st == VMOTHER) & (chi >= H.chi_rec)))
    return out


def regrid(H: Hierarchy, flags=None):
    """Refinement and recoarsening at a common time of all levels (after a
    level-0 step, virtual mothers averaged):
      1. virtual children take the sub-cell averages of their mothers'
         reconstruction, coarse to fine, so every cell holds a value at this
         time;
      2. raw flags (refinement_flags, or the caller's), widened by 'buffer'
         Voronoi layers when they come from the indicator, closed by rules 4
         and 5 (flags nest, which keeps a cell with grandchildren refined:
         rule 7);
      3. the new status of every cell (recoarsened cells are active again with
         the average of their children, eq. average; their children become
         virtual or are removed);
      4. cells that did not exist take the sub-cell averages of their
         mothers' reconstruction, coarse to fine (a new cell's mother may be
         new itself).
    Returns True when the mesh changed."""
    L, r = H.L, H.r
    if L == 0:
        return False
    average_down(H, 0)
    for l in range(1, L + 1):
        children_from_mothers(H, l, H.status[l] == VCHILD)
    if flags is None:
        F = refinement_flags(H)
        for _ in range(H.buffer):
            F = [_dilate(f, H.bcs) for f in F]
    else:
        F = [np.asarray(f, dtype=bool) for f in flags]
    F = _close_flags(F, H.bcs, r, L)
    old = H.status
    new = _status_from_flags(F, H.shape, H.bcs, r, L)
    changed = any(not np.array_equal(a, b) for a, b in zip(old, new))
    H.status, H.flags = new, F
    H._check_patches()
    for l in range(1, L + 1):
        children_from_mothers(H, l, (new[l] != ABSENT) & (old[l] == ABSENT))
    for l in range(L + 1):
        H.U[l][:, new[l] == ABSENT] = np.nan
    H.q = [None] * (L + 1)
    H.pos = [None] * (L + 1)
    return changed


def cfl_dt0(H: Hierarchy, t: float, t_end: float) -> float:
    prob = H.prob
    best = np.inf
    for l in range(H.L + 1):
        A = H.status[l] == ACTIVE
        if not A.any():
            continue
        q = H.U[l][:, A]
        s = sum(prob.system.max_speed(q, k) / H.dx(l)[k] for k in range(H.d))
        best = min(best, H.r ** l * prob.cfl / np.max(s))
    return min(best, t_end - t)


def advance(H: Hierarchy, l: int, t: float, dt: float):
    average_down(H, l)
    if l > 0:
        project(H, l)
    predict_level(H, l, dt)
    if l < H.L:
        H.mem[l + 1][:] = 0.0
        for sub in range(H.r):
            H.sub[l + 1] = sub
            advance(H, l + 1, t + sub * (dt / H.r), dt / H.r)
    update_level(H, l, dt)


def amr_step(H: Hierarchy, t: float, t_end: float) -> float:
    """One level-0 step with local time stepping; returns Delta t_0."""
    dt0 = cfl_dt0(H, t, t_end)
    advance(H, 0, t, dt0)
    average_down(H, 0)
    return dt0


def amr_run(H: Hierarchy, t_end: float, max_steps: int = 10 ** 9):
    t, steps = 0.0, 0
    while t < t_end and steps < max_steps:
        t += amr_step(H, t, t_end)
        steps += 1
    return t, steps
