"""Osher-type flux (eq. osher) on the GPU against the oracle, whose |A| comes
from numpy's eigendecomposition of the complex-step Jacobian (the kernels use
the analytic Euler eigenvectors): fused 2D path, generic 3D path, level
path; for linear advection the flux equals Rusanov bitwise."""
import numpy as np
import pytest

import oracle
from paper_1212_3585_amd import workloads as wl

from gpu_helpers import check_parity, from_device, make_pair, rel_l1, say, to_device
from level_views import mesh_level_view

pytestmark = pytest.mark.gpu


def _run(ader, op, gp, U, nsteps):
    s = ader.Solver(gp)
    u = to_device(U)
    out = s.empty_state()
    Uo = U.copy()
    for _ in range(nsteps):
        dt = oracle.cfl_dt(op, Uo)
        s.compute_dt(u)
        assert abs(float(s.dt.item()) - dt) <= 1e-13 * dt
        s.step(u, out)
        u, out = out, u
        Uo, _ = oracle.step(op, Uo, dt)
    return from_device(u, U.shape[1:]), Uo, s


@pytest.mark.parametrize("M,n", [(1, 24), (2, 20), (3, 16)])
def test_osher_2d_parity(ader, M, n):
    say(f"Osher 2D explosion {n}^2 M={M}, transmissive: 3 steps vs oracle")
    op, gp = make_pair(ader, 2, M, (n, n), (-1, -1), (1, 1), "transmissive", flux="osher")
    U = wl.explosion_2d(n, seed=2)
    got, ref, s = _run(ader, op, gp, U, 3)
    check_parity(got, ref)
    assert s.read_status()[0] == 0


def test_osher_differs_from_rusanov(ader):
    """The selector reaches the kernels: on a discontinuity the two fluxes
    give different results (and each matches its oracle, above)."""
    say("Osher vs Rusanov on the explosion 20^2 M=2")
    U = wl.explosion_2d(20, seed=2)
    outs = []
    for flux in ("rusanov", "osher"):
        op, gp = make_pair(ader, 2, 2, (20, 20), (-1, -1), (1, 1), "transmissive", flux=flux)
        got, _, _ = _run(ader, op, gp, U, 1)
        outs.append(got)
    assert rel_l1(outs[0], outs[1]) > 1e-6


def test_osher_3d_parity(ader):
    say("Osher 3D 7x6x5 M=2 periodic: 2 steps vs oracle")
    n = (7, 6, 5)
    op, gp = make_pair(ader, 3, 2, n, (0,) * 3, (1,) * 3, flux="osher")
    U = wl.perturbed_smooth_euler(n, 41)
    got, ref, _ = _run(ader, op, gp, U, 2)
    check_parity(got, ref)


def test_osher_level_path(ader):
    say("Osher on the level path: whole 2D mesh 16x12 M=2 vs oracle")
    import torch
    shape = (16, 12)
    op, gp = make_pair(ader, 2, 2, shape, (0, 0), (1, 1), flux="osher")
    U = wl.perturbed_smooth_euler(shape, 42)
    s = ader.Solver(gp)
    pc, pp, up, nb = mesh_level_view(shape, 2, ["periodic"] * 2)
    dev = lambda a: torch.tensor(a, dtype=torch.int32, device="cuda")
    u = to_device(U)
    out = u.clone()
    s.compute_dt(u)
    s.step_level(dev(pc), dev(pp), dev(up), dev(nb), op.dx, u, out)
    ref, _ = oracle.step(op, U, oracle.cfl_dt(op, U))
    check_parity(from_device(out, shape), ref)


def test_osher_is_rusanov_for_advection(ader):
    say("linear advection: Osher selector gives the Rusanov result bitwise")
    res = []
    for flux in ("rusanov", "osher"):
        op, gp = make_pair(ader, 2, 3, (24, 24), (0, 0), (1, 1), system="linadv", flux=flux)
        s = ader.Solver(gp)
        u, _, _ = s.run(to_device(wl.sine_wave(24)), 0.05)
        res.append(from_device(u, (24, 24)))
    assert np.array_equal(res[0], res[1])
