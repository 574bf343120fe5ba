"""AMR with local time stepping (ader_amr_*) against the oracle's AMR
(oracle/amr.py): the same mesh from the same initial data (bit-exact status
arrays), level averages of the active cells within 1e-11 pooled relative L1
and element by element after level-0 steps, conservation, graph replay equal to direct launches,
and the fp32-predictor form's stated error."""
import numpy as np
import pytest

from oracle import Euler, Problem as OProblem
from oracle.amr import Hierarchy, amr_step
from paper_1212_3585_amd import workloads as wl

from gpu_helpers import max_rel, say

pytestmark = pytest.mark.gpu


def _coarsen(U, r):
    nv, *n = U.shape
    sh = [nv]
    for k in n:
        sh += [k // r, r]
    return U.reshape(sh).mean(axis=tuple(range(2, 2 + 2 * len(n), 2)))


def _levels_from_fine(Uf, r, L):
    Us = [Uf]
    for _ in range(L):
        Us.insert(0, _coarsen(Us[0], r))
    return Us


def _make(ader, dim, M, n0, r, L, Us, bc="periodic", flags=None, lo=0.0, hi=1.0,
          precision=0, use_graph=True, indicator_var=0, chi_ref=0.2, cfl=0.9, chi_rec=None):
    tol = 1e-14 if precision == 0 else 1e-6
    bcs = [bc] * dim
    op = OProblem(dim, M, Euler(dim), (n0,) * dim, (lo,) * dim, (hi,) * dim, bcs, cfl=cfl)
    gp = ader.Problem(dim=dim, M=M, n=(n0,) * dim + (1,) * (3 - dim), lo=(lo,) * 3,
                      hi=(hi,) * 3, bc=tuple(ader.BC_PERIODIC if bc == "periodic"
                                             else ader.BC_TRANSMISSIVE for _ in range(3)),
                      precision=precision, picard_tol=tol, cfl=cfl)
    H = Hierarchy(op, r, L, Us, flags=flags, indicator_var=indicator_var, chi_ref=chi_ref,
                  chi_rec=chi_rec)
    A = ader.Amr(gp, r=r, max_level=L, indicator_var=indicator_var, chi_ref=chi_ref,
                 use_graph=use_graph, chi_rec=chi_rec)
    for l in range(L + 1):
        A.set_level(l, Us[l])
    if flags is not None:
        for l in range(L):
            A.set_flags(l, flags[l])
    A.build()
    return H, A


def _compare(H, A, tol=1e-11, tol_max=None):
    """Bit-exact status arrays; the active cells' averages within tol pooled
    relative L1 and tol_max (default tol) element by element,
    max |gpu - oracle| / max(1, |oracle|)."""
    num = den = 0.0
    worst = 0.0
    for l in range(H.L + 1):
        U, st = A.level(l)
        assert np.array_equal(st, H.status[l])
        act = st == 0
        num += np.abs(U[:, act] - H.U[l][:, act]).sum()
        den += np.abs(H.U[l][:, act]).sum()
        if act.any():
            worst = max(worst, max_rel(U[:, act], H.U[l][:, act]))
    err = num / den
    print(f"AMR parity: pooled L1 {err:.3e}, element-wise {worst:.3e}")
    assert err <= tol, err
    assert worst <= (tol if tol_max is None else tol_max), worst
    return err


def _patch_flags(n0, r):
    F0 = np.zeros((n0, n0), bool)
    F0[2:4, 2:4] = True
    F1 = np.zeros((n0 * r, n0 * r), bool)
    F1[7:9, 7:9] = True
    return [F0, F1]


def test_amr_patches_two_levels_parity(ader):
    say("AMR 2D 6^2 r=3 L=2 M=2, refined patches: 2 level-0 steps vs oracle")
    n0, r = 6, 3
    Us = _levels_from_fine(wl.perturbed_smooth_euler((n0 * 9, n0 * 9), 5), r, 2)
    H, A = _make(ader, 2, 2, n0, r, 2, Us, flags=_patch_flags(n0, r))
    for c_gpu, c_or in zip([A.counts(l) for l in range(3)], H.counts()):
        assert c_gpu == c_or
    for _ in range(2):
        amr_step(H, 0.0, 1.0)
        A.step(1.0)
    t, steps, _ = A.clock()
    assert steps == 2
    _compare(H, A)
    assert A.stats()["flags"] == 0


def test_amr_indicator_mesh_explosion(ader):
    say("AMR explosion 16^2 r=3 L=2 M=2 transmissive CFL 0.5, indicator on E: 2 steps")
    n0, r = 16, 3
    Us = [wl.explosion_2d(n0 * r ** l, seed=2) for l in range(3)]
    H, A = _make(ader, 2, 2, n0, r, 2, Us, bc="transmissive", lo=-1.0, hi=1.0,
                 indicator_var=3, cfl=0.5)
    assert H.counts()[2]["active"] > 0 and H.counts()[0]["active"] > 0
    for _ in range(2):
        amr_step(H, 0.0, 1.0)
        A.step(1.0)
    _compare(H, A)


@pytest.mark.parametrize("M", [1, 3])
def test_amr_degrees(ader, M):
    say(f"AMR 2D 6^2 r=3 L=1 M={M}: 2 level-0 steps vs oracle")
    n0, r = 6, 3
    Us = _levels_from_fine(wl.perturbed_smooth_euler((n0 * r, n0 * r), 7 + M), r, 1)
    F0 = np.zeros((n0, n0), bool)
    F0[1:3, 2:5] = True
    H, A = _make(ader, 2, M, n0, r, 1, Us, flags=[F0])
    for _ in range(2):
        amr_step(H, 0.0, 1.0)
        A.step(1.0)
    _compare(H, A)


def test_amr_3d_parity(ader):
    say("AMR 3D 4^3 r=2 L=1 M=2: 1 level-0 step vs oracle")
    n0, r = 4, 2
    Us = _levels_from_fine(wl.perturbed_smooth_euler((n0 * r,) * 3, 8), r, 1)
    F0 = np.zeros((n0,) * 3, bool)
    F0[1, 1, 1] = True
    H, A = _make(ader, 3, 2, n0, r, 1, Us, flags=[F0])
    amr_step(H, 0.0, 1.0)
    A.step(1.0)
    _compare(H, A)


_ORACLE_AFTER = {}


def _oracle_steps(key, H, steps):
    """The oracle hierarchy after 'steps' level-0 steps, computed once per
    case and shared by the fp64 and fp32-predictor variants of a test."""
    if key not in _ORACLE_AFTER:
        for _ in range(steps):
            amr_step(H, 0.0, 1.0)
        _ORACLE_AFTER[key] = H
    return _ORACLE_AFTER[key]


# fp32-predictor AMR bars (pooled, element-wise), about ten times the measured
# errors against the fp64 oracle: 3D r = 3 patch 2.3e-8 / 1.4e-7, blast
# 4.4e-9 / 3.2e-8, full-size explosion 3.0e-8 / 2.8e-7
MIXED_AMR = {"3d_r3": (2e-7, 1.5e-6), "blast": (5e-8, 3e-7), "explosion": (3e-7, 3e-6)}


@pytest.mark.parametrize("precision", [0, 1])
def test_amr_3d_r3_parity(ader, precision):
    """3D at the blast workload's refinement factor r = 3: a refined block
    of 2 x 2 x 2 level-0 cells, two level-0 steps (three level-1 substeps
    each), so that the projection at sub-cell offsets 0..2 and the face
    memories summed over r^2 children meet (Section 3.1.3, eq. memory.sum)."""
    say(f"AMR 3D 6^3 r=3 L=1 M=2 precision={precision}: 2 level-0 steps vs oracle")
    n0, r = 6, 3
    Us = _levels_from_fine(wl.perturbed_smooth_euler((n0 * r,) * 3, 14), r, 1)
    F0 = np.zeros((n0,) * 3, bool)
    F0[2:4, 2:4, 1:3] = True
    H, A = _make(ader, 3, 2, n0, r, 1, Us, flags=[F0], precision=precision)
    for c_gpu, c_or in zip([A.counts(l) for l in range(2)], H.counts()):
        assert c_gpu == c_or
    H = _oracle_steps("3d_r3", H, 2)
    for _ in range(2):
        A.step(1.0)
    if precision == 0:
        _compare(H, A)
    else:
        _compare(H, A, *MIXED_AMR["3d_r3"])
    assert A.stats()["flags"] == 0


@pytest.mark.parametrize("precision", [0, 1])
def test_amr_blast_indicator_mesh_r3(ader, precision):
    """The blast workload at a reduced level-0 mesh (8^3, r = 3, one level,
    M = 2, transmissive, CFL 0.5): mesh from the Loehner indicator on the
    energy, two level-0 steps."""
    say(f"AMR 3D blast 8^3 r=3 L=1 M=2 precision={precision}: 2 level-0 steps vs oracle")
    n0, r = 8, 3
    Us = [wl.blast_3d(n0 * r ** l, seed=3, nq=2) for l in range(2)]
    H, A = _make(ader, 3, 2, n0, r, 1, Us, bc="transmissive", lo=-1.0, hi=1.0,
                 indicator_var=4, cfl=0.5, precision=precision)
    assert H.counts()[1]["active"] > 0
    H = _oracle_steps("blast", H, 2)
    for _ in range(2):
        A.step(1.0)
    if precision == 0:
        _compare(H, A)
    else:
        _compare(H, A, *MIXED_AMR["blast"])
    assert A.stats()["flags"] == 0


@pytest.mark.parametrize("precision", [0, 1])
def test_amr_explosion_full_size_step(ader, precision):
    """The 2D explosion workload at its full size (level 0 100^2, r = 3, two
    levels, M = 2, transmissive, CFL 0.5, indicator on the energy): one
    level-0 step (three level-1 and nine level-2 substeps) against the
    oracle's AMR."""
    say(f"AMR explosion 100^2 r=3 L=2 M=2 precision={precision}: 1 level-0 step vs oracle")
    n0, r = 100, 3
    Us = [wl.explosion_2d(n0 * r ** l, seed=2) for l in range(3)]
    H, A = _make(ader, 2, 2, n0, r, 2, Us, bc="transmissive", lo=-1.0, hi=1.0,
                 indicator_var=3, cfl=0.5, precision=precision)
    assert H.counts()[2]["active"] > 20000
    H = _oracle_steps("explosion", H, 1)
    A.step(1.0)
    if precision == 0:
        _compare(H, A)
    else:
        _compare(H, A, *MIXED_AMR["explosion"])
    assert A.stats()["flags"] == 0


def test_amr_conservation_and_graph(ader):
    say("AMR conservation over 3 steps; graph replay equals direct launches")
    n0, r = 6, 3
    Us = _levels_from_fine(wl.perturbed_smooth_euler((n0 * 9, n0 * 9), 11), r, 2)
    res = []
    for use_graph in (True, False):
        H, A = _make(ader, 2, 2, n0, r, 2, Us, flags=_patch_flags(n0, r), use_graph=use_graph)
        tot0 = H.total()
        for _ in range(3):
            A.step(1.0)
        lv = [A.level(l) for l in range(3)]
        tot = 0.0
        for l, (U, st) in enumerate(lv):
            tot = tot + np.prod(H.dx(l)) * U[:, st == 0].sum(axis=1)
        assert np.all(np.abs(tot - tot0) <= 1e-12 * np.abs(tot0).max())
        res.append(lv)
    for (Ua, _), (Ub, _) in zip(*res):
        assert np.array_equal(np.nan_to_num(Ua, nan=7.0), np.nan_to_num(Ub, nan=7.0))


def test_amr_mixed_precision_error(ader):
    say("AMR fp32 predictor, 2 levels: error vs the fp64 oracle")
    n0, r = 6, 3
    Us = _levels_from_fine(wl.perturbed_smooth_euler((n0 * 9, n0 * 9), 12), r, 2)
    H, A = _make(ader, 2, 2, n0, r, 2, Us, flags=_patch_flags(n0, r), precision=1)
    for _ in range(2):
        amr_step(H, 0.0, 1.0)
        A.step(1.0)
    # about ten times the measured 5.3e-8 pooled
    err = _compare(H, A, tol=5e-7, tol_max=1e-5)
    print(f"fp32-predictor AMR relative L1 vs fp64 oracle: {err:.3e}")


@pytest.mark.parametrize("dim,precision", [(2, 1), (3, 0), (2, 0)])
def test_amr_tune_keeps_the_bits(ader, dim, precision):
    say(f"AMR autotuner ({dim}D, precision {precision}): tuned shapes give the same bits")
    n0, r = (6, 3) if dim == 2 else (4, 2)
    L = 2 if dim == 2 else 1
    Uf = wl.perturbed_smooth_euler((n0 * r ** L,) * dim, 13)
    Us = _levels_from_fine(Uf, r, L)
    if dim == 2:
        flags = _patch_flags(n0, r)
    else:
        F0 = np.zeros((n0,) * 3, bool)
        F0[1, 1:3, 1] = True
        flags = [F0]
    out = []
    for tune in (False, True):
        H, A = _make(ader, dim, 2, n0, r, L, Us, flags=flags, precision=precision)
        A.step(1.0)
        if tune:
            pb, fb, ms = A.tune(reps=2)
            assert pb in (128, 256, 512) and fb in (128, 256, 512)
            assert set(ms["flux"]) == {128, 256, 512} and ms["predict"]
            assert all(m > 0 for d in ms.values() for m in d.values())
        for _ in range(2):
            A.step(1.0)
        out.append(([A.level(l) for l in range(L + 1)], A.stats()))
    for (Ua, sa), (Ub, sb) in zip(out[0][0], out[1][0]):
        assert np.array_equal(sa, sb)
        assert np.array_equal(np.nan_to_num(Ua, nan=7.0), np.nan_to_num(Ub, nan=7.0))
    assert out[0][1] == out[1][1]       # statistics untouched by the tuning launches


@pytest.mark.parametrize("r,L,M", [(2, 3, 2), (4, 1, 3), (2, 2, 1)])
def test_amr_factors_and_depths(ader, r, L, M):
    say(f"AMR 2D r={r} L={L} M={M}: nested patches, 2 level-0 steps vs oracle, then a regrid")
    n0 = 8
    Us = _levels_from_fine(wl.perturbed_smooth_euler((n0 * r ** L,) * 2, 20 + r + L), r, L)
    flags = []
    for l in range(L):
        F = np.zeros((n0 * r ** l,) * 2, bool)
        lo, hi = (3 * r ** l, 5 * r ** l) if l == 0 else (4 * r ** l - 1, 4 * r ** l + 1)
        F[lo:hi, lo:hi] = True
        flags.append(F)
    H, A = _make(ader, 2, M, n0, r, L, Us, flags=flags)
    for c_gpu, c_or in zip([A.counts(l) for l in range(L + 1)], H.counts()):
        assert c_gpu == c_or
    for _ in range(2):
        amr_step(H, 0.0, 1.0)
        A.step(1.0)
    _compare(H, A)
    from oracle.amr import regrid
    G = [np.roll(f, 1, axis=0) for f in flags]     # move every patch by one cell
    for l, f in enumerate(G):
        A.set_flags(l, f)
    assert regrid(H, flags=G) == A.regrid()
    amr_step(H, 0.0, 1.0)
    A.step(1.0)
    _compare(H, A)
    assert A.stats()["flags"] == 0


@pytest.mark.parametrize("system,flux", [("mhd", "rusanov"), ("linadv", "rusanov"),
                                         ("euler", "osher")])
def test_amr_other_systems_and_fluxes(ader, system, flux):
    say(f"AMR 2D {system} ({flux}) r=3 L=1 M=2: 2 level-0 steps vs oracle, then a regrid")
    from gpu_helpers import make_pair
    from oracle.amr import Hierarchy, regrid
    n0, r, L = 8, 3, 1
    op, gp = make_pair(ader, 2, 2, (n0, n0), (0.0, 0.0), (1.0, 1.0), system=system, flux=flux)
    nf = n0 * r
    if system == "mhd":
        Uf = wl.orszag_tang(nf, seed=5)
    elif system == "linadv":
        Uf = wl.perturbed_smooth_euler((nf, nf), 9)[:1]
    else:
        Uf = wl.perturbed_smooth_euler((nf, nf), 9)
    Us = _levels_from_fine(Uf, r, L)
    F0 = np.zeros((n0, n0), bool)
    F0[3:5, 2:6] = True
    H = Hierarchy(op, r, L, Us, flags=[F0])
    A = ader.Amr(gp, r=r, max_level=L)
    for l in range(L + 1):
        A.set_level(l, Us[l])
    A.set_flags(0, F0)
    A.build()
    for _ in range(2):
        amr_step(H, 0.0, 1.0)
        A.step(1.0)
    _compare(H, A)
    G0 = np.roll(F0, 1, axis=1)
    A.set_flags(0, G0)
    assert regrid(H, flags=[G0]) == A.regrid()
    amr_step(H, 0.0, 1.0)
    A.step(1.0)
    _compare(H, A)
    assert A.stats()["flags"] == 0
