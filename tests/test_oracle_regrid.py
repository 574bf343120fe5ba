"""Pins of the oracle's dynamic refinement and recoarsening (Section 3.1,
rules 1-7, and the thresholds of Section 3.1.1).

Independent facts: a regrid conserves the integral of the conserved
variables (eq. average and sub-cell averages of a conservative
reconstruction); new children of polynomial data are the exact sub-cell
averages of that polynomial (closed-form integrals); recoarsened cells hold
the exact average of their children; the refine/keep decisions follow the
two thresholds as stated; the refined region follows an advected front; a
regrid that keeps the flags keeps every active average."""
import numpy as np
import pytest

from oracle import Euler, LinearAdvection, Problem
from oracle.amr import (ABSENT, ACTIVE, VCHILD, VMOTHER, Hierarchy, amr_step, refinement_flags,
                        regrid)
from paper_1212_3585_amd import workloads as wl


def _poly_averages(n, lo, hi):
    """Exact cell averages of P(x, y) = 1 + 0.3x - 0.2y + 0.5x^2 + 0.1xy - 0.4y^2
    + 0.2x^2 y on an n x n mesh (antiderivatives, no quadrature)."""
    e = [np.linspace(lo, hi, n + 1)] * 2
    def m(k, a, b):                       # average of t^k over [a, b]
        return (b ** (k + 1) - a ** (k + 1)) / ((k + 1) * (b - a))
    xa, xb = e[0][:-1, None], e[0][1:, None]
    ya, yb = e[1][None, :-1], e[1][None, 1:]
    X = lambda k: m(k, xa, xb)
    Y = lambda k: m(k, ya, yb)
    return (1 + 0.3 * X(1) - 0.2 * Y(1) + 0.5 * X(2) + 0.1 * X(1) * Y(1) - 0.4 * Y(2)
            + 0.2 * X(2) * Y(1))[None]


def _poly_hierarchy(n0, r, F0):
    prob = Problem(2, 2, LinearAdvection(2, [1.0, 0.5]), (n0, n0), (0.0, 0.0), (1.0, 1.0),
                   ["transmissive"] * 2)
    Us = [_poly_averages(n0 * r ** l, 0.0, 1.0) for l in range(2)]
    return prob, Hierarchy(prob, r, 1, Us, flags=[F0])


def test_new_children_of_polynomial_data_are_exact():
    n0, r = 10, 3
    F0 = np.zeros((n0, n0), bool)
    F0[4:6, 4:6] = True
    prob, H = _poly_hierarchy(n0, r, F0)
    G0 = np.zeros_like(F0)
    G0[3:7, 3:6] = True                    # grows the refined region; no mother's
    assert regrid(H, flags=[G0])           # stencil reaches the boundary
    exact = _poly_averages(n0 * r, 0.0, 1.0)
    A = H.status[1] == ACTIVE
    assert A.sum() == 12 * 9
    np.testing.assert_allclose(H.U[1][:, A], exact[:, A], rtol=1e-12, atol=1e-12)
    V = H.status[1] == VCHILD
    np.testing.assert_allclose(H.U[1][:, V], exact[:, V], rtol=1e-12, atol=1e-12)
    assert np.isnan(H.U[1][:, H.status[1] == ABSENT]).all()


def test_recoarsened_cells_hold_the_average_of_their_children():
    n0, r = 10, 3
    F0 = np.zeros((n0, n0), bool)
    F0[2:8, 3:6] = True
    prob, H = _poly_hierarchy(n0, r, F0)
    rng = np.random.Generator(np.random.PCG64(5))
    A = H.status[1] == ACTIVE
    H.U[1][:, A] += 0.01 * rng.normal(size=(1, A.sum()))   # children differ from the mother
    fine = H.U[1].copy()
    G0 = np.zeros_like(F0)
    G0[4:6, 4:6] = True                    # shrinks it
    assert regrid(H, flags=[G0])
    for i, j in [(2, 3), (7, 5), (3, 4)]:
        assert H.status[0][i, j] == ACTIVE
        kids = fine[0, 3 * i:3 * i + 3, 3 * j:3 * j + 3]
        np.testing.assert_allclose(H.U[0][0, i, j], kids.mean(), rtol=1e-14)
    # cells that stay refined keep their children's averages bitwise
    keep = (H.status[1] == ACTIVE)
    np.testing.assert_array_equal(H.U[1][:, keep], fine[:, keep])


def test_regrid_conserves_and_keeps_the_mesh_rules():
    n0, r, L = 8, 3, 2
    # periodic: on a mesh this coarse the numerical domain of dependence reaches a
    # transmissive boundary within three steps, and real boundary fluxes appear
    prob = Problem(2, 2, Euler(2), (n0, n0), (-1.0, -1.0), (1.0, 1.0), ["periodic"] * 2,
                   cfl=0.5)
    Us = [wl.explosion_2d(n0 * r ** l, seed=2) for l in range(L + 1)]
    H = Hierarchy(prob, r, L, Us, chi_ref=0.2, eps=0.01, indicator_var=3, buffer=1,
                  chi_rec=0.1)
    tot0 = H.total()
    t = 0.0
    changed = 0
    for _ in range(3):
        t += amr_step(H, t, 1.0)
        before = H.total()
        changed += regrid(H)
        np.testing.assert_allclose(H.total(), before, rtol=1e-13, atol=1e-13)
        for l in range(1, L + 1):
            st, up = H.status[l], H.status[l - 1]
            mom = np.repeat(np.repeat(up, r, 0), r, 1)
            assert np.all(mom[st == VCHILD] == ACTIVE)
            assert np.all(mom[st == ACTIVE] == VMOTHER)
            assert np.all(st[mom == VMOTHER] != ABSENT)
    assert changed >= 1
    np.testing.assert_allclose(H.total(), tot0, rtol=1e-12, atol=1e-13)


def test_refine_and_keep_thresholds():
    n0, r = 12, 3
    prob = Problem(2, 2, LinearAdvection(2, [1.0, 0.0]), (n0, n0), (0.0, 0.0), (1.0, 1.0),
                   ["transmissive"] * 2)
    x = np.arange(n0)
    X, _ = np.meshgrid(x, x, indexing="ij")
    step = np.where(X < 6, 1.0, 2.0)[None]          # chi = sqrt(1 / 1.25) on rows 5, 6 (eps = 0)
    Us = [step, np.repeat(np.repeat(step, r, 1), r, 2)]
    F0 = np.zeros((n0, n0), bool)
    F0[5:7, 0:6] = True                               # half the step cells are refined
    H = Hierarchy(prob, r, 1, Us, flags=[F0], chi_ref=0.95, eps=0.0, chi_rec=0.5)
    F = refinement_flags(H)[0]
    chi = np.sqrt(1 / 1.25)
    assert chi < 0.95 and chi >= 0.5
    assert np.array_equal(F, F0)                       # refined cells kept, none new
    H.chi_ref, H.chi_rec = 0.5, 0.5
    F = refinement_flags(H)[0]
    assert np.array_equal(F[5:7], np.ones((2, n0), bool)) and not F[:5].any() and not F[7:].any()
    H.chi_ref, H.chi_rec = 0.95, 0.9
    assert not refinement_flags(H)[0].any()            # everything recoarsened


def test_refined_region_follows_an_advected_front():
    n0, r, M = 24, 3, 2
    prob = Problem(2, M, LinearAdvection(2, [1.0, 0.0]), (n0, 4), (0.0, 0.0), (1.0, 1.0 / 6),
                   ["periodic"] * 2, cfl=0.5)
    def front(n, shift=0.0):
        xc = (np.arange(n[0]) + 0.5) / n[0]
        v = 1.0 + np.tanh((0.25 - np.abs(((xc - 0.35 - shift) % 1.0) - 0.5)) * 60.0)
        return np.broadcast_to(v[:, None], n)[None].copy()
    Us = [front((n0 * r ** l, 4 * r ** l)) for l in range(2)]
    H = Hierarchy(prob, r, 1, Us, chi_ref=0.2, eps=0.01, buffer=1, chi_rec=0.1)
    def centre():
        cols = np.where((H.status[0] == VMOTHER).any(axis=1))[0]
        return cols.mean()
    c0, t = centre(), 0.0
    while t < 0.25 - 1e-12:
        t += amr_step(H, t, 0.25)
        regrid(H)
    moved = centre() - c0
    assert abs(moved - 0.25 * n0) <= 1.0, moved      # 6 cells in 0.25 time units


def test_regrid_with_unchanged_flags_keeps_active_averages():
    n0, r = 6, 3
    prob = Problem(2, 2, Euler(2), (n0, n0), (0.0, 0.0), (1.0, 1.0), ["periodic"] * 2)
    Us = [wl.perturbed_smooth_euler((n0 * r ** l,) * 2, 5) for l in range(2)]
    F0 = np.zeros((n0, n0), bool)
    F0[2:4, 1:4] = True
    H = Hierarchy(prob, r, 1, Us, flags=[F0])
    amr_step(H, 0.0, 1.0)
    keep = [u.copy() for u in H.U]
    assert not regrid(H, flags=[F0])
    for l in range(2):
        A = H.status[l] != VCHILD
        np.testing.assert_array_equal(H.U[l][:, A], keep[l][:, A])
