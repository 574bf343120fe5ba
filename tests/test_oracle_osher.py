"""Pins of the oracle's Osher-type flux (eq. osher) and of the scheme with it.

The oracle takes |A| from numpy's eigendecomposition of a complex-step
Jacobian; the checks below use other facts: |A|^2 = A^2 with the spectrum
|lambda|, the consistency F(q, q) = f(q), upwinding of a flow whose
characteristic speeds all have one sign (the path integral of A along the
segment is f(qR) - f(qL)), the analytic Euler eigenvectors, and exact upwind
fluxes for linear advection."""
import numpy as np

import oracle
from oracle import Euler, LinearAdvection, Problem
from oracle.scheme import abs_matrix, flux_jacobian, osher, rusanov


def _euler_states(n, seed, mach=0.5, dim=2):
    r = np.random.Generator(np.random.PCG64(seed))
    rho = r.uniform(0.5, 2.0, n)
    p = r.uniform(0.5, 2.0, n)
    c = np.sqrt(1.4 * p / rho)
    v = [mach * c * r.uniform(-1, 1, n) for _ in range(dim)]
    E = p / 0.4 + 0.5 * rho * sum(x * x for x in v)
    return np.stack([rho] + [rho * x for x in v] + [E])


def test_abs_matrix_squares_to_A_squared():
    q = _euler_states(20, 1)
    for k in range(2):
        A = flux_jacobian(Euler(2), q, k)
        absA = abs_matrix(A)
        np.testing.assert_allclose(absA @ absA, A @ A, rtol=1e-10, atol=1e-10)
        lam = np.sort(np.abs(np.linalg.eigvals(A)), axis=-1)
        mu = np.sort(np.linalg.eigvals(absA).real, axis=-1)
        np.testing.assert_allclose(mu, lam, rtol=1e-10, atol=1e-12)


def test_abs_matrix_against_analytic_euler_eigenvectors():
    """|A| = sum |lambda_i| r_i l_i with the textbook eigenvectors of the 2D
    Euler flux along x (left eigenvectors with b1 = (gamma-1)/c^2)."""
    g = 1.4
    q = _euler_states(8, 2)
    A = flux_jacobian(Euler(2, g), q, 0)
    for p in range(q.shape[1]):
        rho, mx, my, E = q[:, p]
        u, v = mx / rho, my / rho
        pr = (g - 1) * (E - 0.5 * rho * (u * u + v * v))
        c = np.sqrt(g * pr / rho)
        H = (E + pr) / rho
        q2 = u * u + v * v
        b1 = (g - 1) / c ** 2
        b2 = 0.5 * b1 * q2
        R = np.array([[1, 1, 0, 1], [u - c, u, 0, u + c], [v, v, 1, v],
                      [H - u * c, 0.5 * q2, v, H + u * c]])
        L = np.array([[0.5 * (b2 + u / c), -0.5 * (b1 * u + 1 / c), -0.5 * b1 * v, 0.5 * b1],
                      [1 - b2, b1 * u, b1 * v, -b1],
                      [-v, 0, 1, 0],
                      [0.5 * (b2 - u / c), -0.5 * (b1 * u - 1 / c), -0.5 * b1 * v, 0.5 * b1]])
        np.testing.assert_allclose(L @ R, np.eye(4), atol=1e-12)
        lam = np.array([u - c, u, u, u + c])
        np.testing.assert_allclose(abs_matrix(A[p]), R @ np.diag(np.abs(lam)) @ L,
                                   rtol=1e-10, atol=1e-10)


def test_consistency():
    q = _euler_states(12, 3)
    for k in range(2):
        np.testing.assert_allclose(osher(Euler(2), q, q, k), Euler(2).flux(q, k), rtol=1e-14)


def test_supersonic_flow_is_upwinded():
    """All speeds positive along the path (Mach > 1 along +x): the path
    integral of A is f(qR) - f(qL) up to the 3-point rule's error, so the
    flux is f(qL); mirrored, it is f(qR)."""
    qL = _euler_states(10, 4, mach=0.0)
    rho, p = qL[0], 0.4 * (qL[3] - 0.5 * (qL[1] ** 2 + qL[2] ** 2) / qL[0])
    c = np.sqrt(1.4 * p / rho)
    for sgn in (1.0, -1.0):
        qa = qL.copy()
        qa[1] = sgn * 2.5 * c * rho
        qa[3] = p / 0.4 + 0.5 * (qa[1] ** 2 + qa[2] ** 2) / rho
        qb = qa * (1 + 0.01 * np.sin(np.arange(10)))[None]
        F = osher(Euler(2), qa, qb, 0)
        up = Euler(2).flux(qa if sgn > 0 else qb, 0)
        np.testing.assert_allclose(F, up, rtol=1e-9, atol=1e-9)


def test_linear_advection_is_exact_upwind():
    r = np.random.Generator(np.random.PCG64(5))
    qL, qR = r.uniform(-1, 1, (1, 7)), r.uniform(-1, 1, (1, 7))
    for a in (0.7, -1.3):
        sysa = LinearAdvection(2, [a, 0.4])
        np.testing.assert_allclose(osher(sysa, qL, qR, 0), a * (qL if a > 0 else qR), rtol=1e-14)
        np.testing.assert_allclose(osher(sysa, qL, qR, 0), rusanov(sysa, qL, qR, 0), rtol=1e-14)


def test_scheme_with_osher_conserves_and_keeps_free_stream():
    from paper_1212_3585_amd import workloads as wl
    prob = Problem(2, 2, Euler(2), (10, 10), (-1.0, -1.0), (1.0, 1.0), ["periodic"] * 2,
                   flux="osher")
    U = wl.explosion_2d(10, seed=2)
    U1, _ = oracle.step(prob, U, oracle.cfl_dt(prob, U))
    scale = np.maximum(np.abs(U).sum(axis=(1, 2)), np.abs(U[0]).sum())
    assert np.all(np.abs(U1.sum(axis=(1, 2)) - U.sum(axis=(1, 2))) <= 1e-12 * scale)
    # a uniform moving state (rho 1, v (0.3, -0.2), p 1) is kept
    Uc = np.empty_like(U)
    Uc[0], Uc[1], Uc[2] = 1.0, 0.3, -0.2
    Uc[3] = 1.0 / 0.4 + 0.5 * (0.09 + 0.04)
    Uc1, _ = oracle.step(prob, Uc, oracle.cfl_dt(prob, Uc))
    np.testing.assert_allclose(Uc1, Uc, rtol=1e-13, atol=1e-13)
