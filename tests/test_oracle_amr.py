"""Pins of the oracle's AMR with local time stepping (Section 3).

Independent facts: a mesh refined everywhere is the uniform fine mesh (one
level-0 step = r^L fine steps, bitwise); no refinement is the uniform scheme;
the scheme is conservative and keeps a free stream with refined patches;
linear advection over a refined patch converges at the design order; the
projection operator gives exact sub-cell averages of polynomials; the mesh
obeys the rules of Section 3.1; the Loehner indicator's closed forms."""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from oracle import Euler, LinearAdvection, Problem
from oracle.amr import (ABSENT, ACTIVE, VCHILD, VMOTHER, Hierarchy, amr_run, amr_step,
                        lohner, subcell_average_matrix)
from oracle.basis import basis
from paper_1212_3585_amd import workloads as wl


def _coarsen(U, r):
    nv, *n = U.shape
    sh = [nv]
    for k in n:
        sh += [k // r, r]
    return U.reshape(sh).mean(axis=tuple(range(2, 2 + 2 * len(n), 2)))


def _levels(Ufine, r, L):
    Us = [Ufine]
    for _ in range(L):
        Us.insert(0, _coarsen(Us[0], r))
    return Us


@pytest.mark.parametrize("L", [1, 2])
def test_refined_everywhere_is_the_fine_uniform_mesh(L):
    n0, r, M = 4, 3, 2
    prob = Problem(2, M, Euler(2), (n0, n0), (0.0, 0.0), (1.0, 1.0), ["periodic"] * 2)
    nf = n0 * r ** L
    Us = _levels(wl.perturbed_smooth_euler((nf, nf), 5), r, L)
    flags = [np.ones((n0 * r ** l,) * 2, bool) for l in range(L)]
    H = Hierarchy(prob, r, L, Us, flags=flags)
    assert H.counts()[L]["active"] == nf * nf
    dt0 = amr_step(H, 0.0, 1.0)
    fine = Problem(2, M, Euler(2), (nf, nf), (0.0, 0.0), (1.0, 1.0), ["periodic"] * 2)
    np.testing.assert_allclose(dt0, r ** L * oracle.cfl_dt(fine, Us[L]), rtol=1e-15)
    dtf = dt0
    for _ in range(L):
        dtf = dtf / r                     # the substep of each level, as LTS forms it
    U = Us[L]
    for _ in range(r ** L):
        U, _ = oracle.step(fine, U, dtf)
    np.testing.assert_array_equal(H.U[L], U)


def test_unrefined_is_the_uniform_scheme():
    prob = Problem(2, 3, Euler(2), (10, 8), (0.0, 0.0), (1.0, 0.8), ["periodic", "transmissive"])
    U = wl.perturbed_smooth_euler((10, 8), 6)
    H = Hierarchy(prob, 3, 0, [U], flags=[])
    dt = amr_step(H, 0.0, 1.0)
    ref, _ = oracle.step(prob, U, oracle.cfl_dt(prob, U))
    assert dt == oracle.cfl_dt(prob, U)
    np.testing.assert_array_equal(H.U[0], ref)


def _patch_flags(n0, r):
    F0 = np.zeros((n0, n0), bool)
    F0[2:4, 2:4] = True
    F1 = np.zeros((n0 * r, n0 * r), bool)
    F1[7:9, 7:9] = True
    return [F0, F1]


def test_conservation_with_refined_patches():
    n0, r = 6, 3
    prob = Problem(2, 2, Euler(2), (n0, n0), (0.0, 0.0), (1.0, 1.0), ["periodic"] * 2)
    Us = _levels(wl.perturbed_smooth_euler((n0 * 9, n0 * 9), 5), r, 2)
    H = Hierarchy(prob, r, 2, Us, flags=_patch_flags(n0, r))
    c = H.counts()
    assert c[1]["vchild"] > 0 and c[2]["vchild"] > 0 and c[1]["vmother"] > 0
    tot0 = H.total()
    for _ in range(2):
        amr_step(H, 0.0, 1.0)
    assert np.all(np.abs(H.total() - tot0) <= 1e-13 * np.abs(tot0).max())


def test_free_stream_with_refined_patches():
    n0, r = 6, 3
    prob = Problem(2, 2, Euler(2), (n0, n0), (0.0, 0.0), (1.0, 1.0), ["periodic"] * 2)
    state = np.array([1.0, 0.3, -0.2, 2.5 + 0.5 * 0.13])
    Us = [np.broadcast_to(state[:, None, None], (4, n0 * r ** l, n0 * r ** l)).copy()
          for l in range(3)]
    H = Hierarchy(prob, r, 2, Us, flags=_patch_flags(n0, r))
    amr_step(H, 0.0, 1.0)
    for l in range(3):
        A = H.status[l] == ACTIVE
        np.testing.assert_allclose(H.U[l][:, A], Us[l][:, A], rtol=1e-13, atol=1e-13)


def test_3d_conservation():
    n0, r = 4, 2
    prob = Problem(3, 2, Euler(3), (n0,) * 3, (0.0,) * 3, (1.0,) * 3, ["periodic"] * 3)
    Us = _levels(wl.perturbed_smooth_euler((n0 * r,) * 3, 8), r, 1)
    F0 = np.zeros((n0,) * 3, bool)
    F0[1, 1, 1] = True
    H = Hierarchy(prob, r, 1, Us, flags=[F0])
    tot0 = H.total()
    amr_step(H, 0.0, 1.0)
    assert np.all(np.abs(H.total() - tot0) <= 1e-13 * np.abs(tot0).max())


def test_design_order_through_a_refined_patch():
    from paper_1212_3585_amd.workloads import _cell_average
    M, r, errs = 2, 3, []
    for n0 in (12, 24):
        prob = Problem(2, M, LinearAdvection(2, [1.0, 0.5]), (n0, n0), (0.0, 0.0), (1.0, 1.0),
                       ["periodic"] * 2)
        Us = [wl.sine_wave(n0 * r ** l) for l in range(2)]
        F0 = np.zeros((n0, n0), bool)
        F0[n0 // 3:2 * n0 // 3, n0 // 3:2 * n0 // 3] = True
        H = Hierarchy(prob, r, 1, Us, flags=[F0])
        t, _ = amr_run(H, 0.1)
        err = 0.0
        for l in range(2):
            ex = _cell_average(lambda x, y: np.sin(2 * np.pi * (x + y - 1.5 * t))[None],
                               (n0 * r ** l,) * 2, (0.0, 0.0), (1.0, 1.0))
            A = H.status[l] == ACTIVE
            err += np.abs(H.U[l] - ex)[:, A].sum() * np.prod(H.dx(l))
        errs.append(err)
    order = np.log2(errs[0] / errs[1])
    assert abs(order - (M + 1)) <= 0.2, (errs, order)


@pytest.mark.parametrize("M,r", [(1, 2), (2, 3), (3, 3), (3, 4)])
def test_projection_gives_exact_subcell_averages(M, r):
    b = basis(M)
    rng = np.random.Generator(np.random.PCG64(M + 10 * r))
    coef = rng.normal(size=M + 1)
    poly = np.polynomial.Polynomial(coef)
    P = subcell_average_matrix(M, r)
    got = P @ poly(b.nodes)                        # nodal values -> child averages
    want = [r * quad(poly, a / r, (a + 1) / r)[0] for a in range(r)]
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(P.sum(axis=1), 1.0, rtol=1e-14)   # constants kept


def test_mesh_rules_on_random_flags():
    rng = np.random.Generator(np.random.PCG64(3))
    n0, r = 8, 3
    for bc in ("periodic", "transmissive"):
        prob = Problem(2, 2, Euler(2), (n0, n0), (0.0, 0.0), (1.0, 1.0), [bc] * 2)
        flags = [rng.uniform(size=(n0, n0)) < 0.08, rng.uniform(size=(n0 * r,) * 2) < 0.01]
        Us = [np.ones((4, n0 * r ** l, n0 * r ** l)) for l in range(3)]
        H = Hierarchy(prob, r, 2, Us, flags=flags)     # checks every active stencil
        for l in range(1, 3):
            st, up = H.status[l], H.status[l - 1]
            mom = np.repeat(np.repeat(up, r, 0), r, 1)
            assert np.all(mom[st == VCHILD] == ACTIVE)          # virtual child: active mother
            assert np.all(mom[st == ACTIVE] == VMOTHER)         # active child: refined mother
            assert np.all(st[mom == VMOTHER] >= VMOTHER)        # children of refined cells exist
            assert np.all(st[mom == VMOTHER] != VCHILD)
            # Voronoi neighbours of an active cell differ by at most one level:
            # no active cell of level l touches an ABSENT cell of level l whose
            # mother is not active (that would be a jump of two levels)
            A = np.argwhere(st == ACTIVE)
            for o in np.ndindex(3, 3):
                nb = A + np.array(o) - 1
                ok = np.all((nb >= 0) & (nb < st.shape[0]), axis=1) if bc != "periodic" else \
                    np.ones(len(nb), bool)
                nb = np.mod(nb, st.shape[0])[ok]
                assert np.all(st[tuple(nb.T)] != ABSENT)


def test_lohner_closed_forms():
    x = np.arange(12.0)
    X, Y = np.meshgrid(x, x, indexing="ij")
    lin = 3.0 + 0.5 * X - 0.25 * Y
    chi = lohner(lin, ["transmissive"] * 2, eps=0.0)
    assert np.all(chi[1:-1, 1:-1] < 1e-12)            # no second derivative
    step = np.where(X < 6, 1.0, 2.0)
    chi = lohner(step, ["transmissive"] * 2, eps=0.0)
    # at the step: D_xx = +-1 over |jump| = 1; the cross terms have D = 0; the
    # pair (x, y) differentiates along x at the y-neighbours (den = 1/2), the
    # pair (y, x) along y at the x-neighbours (den = 0): chi = sqrt(1 / (1 + 1/4))
    np.testing.assert_allclose(chi[5, 3:9], np.sqrt(1 / 1.25), rtol=1e-14)
    np.testing.assert_allclose(chi[6, 3:9], np.sqrt(1 / 1.25), rtol=1e-14)
    assert np.all(chi[:4] == 0) and np.all(chi[8:] == 0)
    ripple = 100.0 + 0.01 * (-1.0) ** X
    assert lohner(ripple, ["periodic"] * 2, eps=0.01).max() < 0.01   # filtered
