"""Autotuning of the fused 2D cell kernel's tile height (ader_tune,
ader_set_tile_rows): every height gives the same bits (a wavefront is one
tile row whatever the height), the tuner returns a candidate and its timings,
and GLM-MHD never gets the 16-row block."""
import numpy as np
import pytest

from paper_1212_3585_amd import workloads as wl

from gpu_helpers import say

pytestmark = pytest.mark.gpu


def _steps(ader, torch, prob, U, rows, nsteps=2, tune=False):
    s = ader.Solver(prob)
    u = torch.tensor(wl.to_soa(U), dtype=torch.float64, device="cuda")
    if tune:
        s.compute_dt(u)
        chosen, ms = s.tune(u, reps=2)
    else:
        s.set_tile_rows(rows)
        chosen, ms = rows, {}
    s.clear_status()
    b = torch.empty_like(u)
    for _ in range(nsteps):
        s.compute_dt(u)
        s.step(u, b)
        u, b = b, u
    flags, iters = s.read_status()
    return u.cpu().numpy(), flags, iters, chosen, ms


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("M,n,bc", [(3, (40, 37), 0), (2, (23, 50), 1)])
def test_tile_heights_give_the_same_bits(ader, precision, M, n, bc):
    import torch
    say(f"tile heights 2/4/8/16: KH-like {n} M={M} bc={bc} precision={precision}")
    U = wl.kelvin_helmholtz(n[0]) if n[0] == n[1] else wl.perturbed_smooth_euler(n, 3)
    prob = ader.Problem(dim=2, M=M, n=(n[0], n[1], 1), bc=(bc, bc, bc), precision=precision,
                        picard_tol=1e-14 if precision == 0 else 1e-6)
    ref = _steps(ader, torch, prob, U, 8)
    assert ref[1] == 0
    for rows in (2, 4, 16):
        got = _steps(ader, torch, prob, U, rows)
        assert np.array_equal(got[0], ref[0]), rows
        assert got[1:3] == ref[1:3], rows
    tuned = _steps(ader, torch, prob, U, None, tune=True)
    assert tuned[3] in (2, 4, 8, 16) and set(tuned[4]) == {2, 4, 8, 16}
    assert all(v > 0 for v in tuned[4].values())
    assert np.array_equal(tuned[0], ref[0])


def test_mhd_tile_heights(ader):
    import torch
    say("tile heights for GLM-MHD: 2/4/8 equal, 16 refused, tuner skips it")
    n = 24
    U = wl.orszag_tang(n, seed=3)
    prob = ader.Problem(dim=2, M=2, n=(n, n, 1), system=ader.SYS_MHD_GLM)
    ref = _steps(ader, torch, prob, U, 8)
    for rows in (2, 4):
        assert np.array_equal(_steps(ader, torch, prob, U, rows)[0], ref[0])
    with pytest.raises(RuntimeError):
        _steps(ader, torch, prob, U, 16)
    tuned = _steps(ader, torch, prob, U, None, tune=True)
    assert set(tuned[4]) == {2, 4, 8} and tuned[3] in (2, 4, 8)
    assert np.array_equal(tuned[0], ref[0])
