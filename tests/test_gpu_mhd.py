"""GLM-MHD (Section 4.2) on the GPU against the oracle: step parity for
M = 1..3 on seeded Orszag-Tang data, the unperturbed vortex to t = 0.1,
a 3D transmissive step (generic kernels), the fp32-predictor form's error,
and MHD solves in the solve server."""
import numpy as np
import pytest

import oracle
from paper_1212_3585_amd import workloads as wl

from gpu_helpers import check_parity, from_device, make_pair, max_rel, rel_l1, say, to_device

pytestmark = pytest.mark.gpu
L = 2.0 * np.pi


def _steps(ader, op, gp, U, nsteps, same_dt=True):
    """nsteps steps on both sides, each with its own CFL step; same_dt
    asserts the two time steps agree (fp64 form)."""
    s = ader.Solver(gp)
    u = to_device(U)
    out = s.empty_state()
    Uo = U.copy()
    for _ in range(nsteps):
        dt = oracle.cfl_dt(op, Uo)
        s.compute_dt(u)
        if same_dt:
            assert abs(float(s.dt.item()) - dt) <= 1e-13 * dt
        s.step(u, out)
        u, out = out, u
        Uo, _ = oracle.step(op, Uo, dt)
    return from_device(u, U.shape[1:]), Uo, s


@pytest.mark.parametrize("M,n", [(1, 20), (2, 16), (3, 12)])
def test_mhd_step_parity(ader, M, n):
    say(f"MHD Orszag-Tang {n}^2 M={M}: 3 steps vs oracle")
    op, gp = make_pair(ader, 2, M, (n, n), (0, 0), (L, L), system="mhd")
    U = wl.orszag_tang(n, seed=10 + M)
    got, ref, s = _steps(ader, op, gp, U, 3)
    check_parity(got, ref)
    assert s.read_status()[0] == 0


def test_mhd_orszag_tang_to_t(ader):
    say("MHD Orszag-Tang 32^2 M=2 to t = 0.1 vs oracle.run")
    op, gp = make_pair(ader, 2, 2, (32, 32), (0, 0), (L, L), system="mhd")
    U0 = wl.orszag_tang(32)
    s = ader.Solver(gp)
    u, t, steps = s.run(to_device(U0), 0.1)
    Uo, to, so, _ = oracle.run(op, U0, 0.1)
    assert steps == so and abs(t - to) <= 1e-14
    check_parity(from_device(u, (32, 32)), Uo)


def test_mhd_3d_transmissive(ader):
    say("MHD 3D 7x6x5 M=2 transmissive: 2 steps vs oracle")
    n = (7, 6, 5)
    op, gp = make_pair(ader, 3, 2, n, (0,) * 3, (1,) * 3, "transmissive", system="mhd")
    r = np.random.Generator(np.random.PCG64(31))
    X = np.meshgrid(*[(np.arange(k) + 0.5) / k for k in n], indexing="ij")
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * X[0]) * (1 + 0.01 * r.uniform(-1, 1, n))
    vel = [0.3 * np.sin(2 * np.pi * X[1]), 0.2 * np.cos(2 * np.pi * X[2]), 0.1 + 0 * rho]
    B = [1.5 + 0 * rho, 0.8 * np.sin(2 * np.pi * X[0]), 0.5 * np.cos(2 * np.pi * X[1])]
    U = wl.mhd_conserved(rho, vel, 1.0 + 0 * rho, B)
    got, ref, _ = _steps(ader, op, gp, U, 2)
    check_parity(got, ref)


def test_mhd_mixed_precision_error_is_stated(ader):
    say("MHD fp32 predictor, Orszag-Tang 24^2 M=2: 3 steps vs fp64 oracle")
    op, gp = make_pair(ader, 2, 2, (24, 24), (0, 0), (L, L), system="mhd", precision=1,
                       tol=1e-6)
    op.tol = 1e-14
    U = wl.orszag_tang(24, seed=3)
    got, ref, s = _steps(ader, op, gp, U, 3, same_dt=False)
    err = rel_l1(got, ref)
    print(f"fp32-predictor MHD relative L1 vs fp64 oracle: {err:.3e}, "
          f"element-wise {max_rel(got, ref):.3e}")
    # about ten times the measured 5.1e-8
    assert err <= 5e-7
    assert s.read_status()[0] == 0


def test_mhd_in_the_server(ader):
    say("server: MHD and Euler solves mixed vs alone")
    cases = []
    for M, n, seed in [(1, 32, 1), (2, 24, 2), (3, 16, 3)]:
        p = ader.Problem(dim=2, M=M, system=ader.SYS_MHD_GLM, gamma=5.0 / 3.0, ch=2.0,
                         n=(n, n, 1), lo=(0, 0, 0), hi=(L, L, 1))
        cases.append((p, wl.orszag_tang(n, seed=seed), 0.05))
    p = ader.Problem(dim=2, M=2, n=(32, 32, 1))
    cases.append((p, wl.kelvin_helmholtz(32, seed=4), 0.02))
    alone = []
    for c in cases:
        srv = ader.Server(hbm_bytes=1 << 30, max_slots=2)
        rid = srv.submit(*c)
        srv.drain([rid])
        alone.append((srv.result(rid).copy(), srv.info(rid)))
        srv.close()
    srv = ader.Server(hbm_bytes=1 << 30, max_slots=8)
    ids = [srv.submit(*c) for c in cases]
    srv.drain(ids)
    for rid, (ref, info) in zip(ids, alone):
        assert srv.info(rid)["state"] == ader.REQ_DONE
        assert srv.info(rid)["steps"] == info["steps"]
        assert np.array_equal(srv.result(rid), ref)
    # the first MHD solve equals the single-solve step loop
    p, U0, te = cases[0]
    s = ader.Solver(p)
    u, t, steps = s.run(to_device(U0), te)
    assert np.array_equal(from_device(u, U0.shape[1:]), alone[0][0])
    srv.close()
