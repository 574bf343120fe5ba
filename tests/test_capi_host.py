"""Host-side checks of the C ABI: exports, argument validation, constants.

None of these calls launches a kernel or touches a GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.basis import basis

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ader.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1212_3585_amd import ader
    if not os.path.exists(ader._LIB_PATH):
        from paper_1212_3585_amd.build import build_library
        build_library()
    return ader.load_library()


@pytest.fixture(scope="module")
def ader_mod(lib):
    from paper_1212_3585_amd import ader
    return ader


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ader_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib, ader_mod):
    names = declared_functions()
    assert set(names) == set(ader_mod.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def _create(ader_mod, **kw):
    prob = ader_mod.Problem(**kw).to_c()
    plan = ctypes.c_void_p()
    st = ader_mod.load_library().ader_plan_create(ctypes.byref(prob), ctypes.byref(plan))
    return st, plan


@pytest.mark.parametrize("kw,status", [
    (dict(dim=1), -2), (dict(M=4), -2), (dict(M=-1), -2), (dict(system=7), -2),
    (dict(n=(0, 4, 1)), -1), (dict(cfl=0.0), -1), (dict(cfl=1.5), -1),
    (dict(gamma=1.0), -1), (dict(picard_tol=0.0), -1), (dict(picard_max=0), -1),
    (dict(hi=(0.0, 1.0, 1.0)), -1), (dict(bc=(0, 5, 0)), -1), (dict(precision=3), -1),
    (dict(lo=(float("nan"), 0.0, 0.0)), -1),
    (dict(dim=3, n=(1024, 1024, 257)), -2),      # beyond 2^28 cells
])
def test_plan_create_rejects_bad_problems(ader_mod, kw, status):
    st, plan = _create(ader_mod, **kw)
    assert st == status
    assert not plan.value
    assert len(ader_mod.load_library().ader_last_error()) > 0


def test_plan_basics_and_workspace(ader_mod):
    lib = ader_mod.load_library()
    for dim, M, system, nv in [(2, 3, 1, 4), (3, 2, 1, 5), (2, 1, 0, 1)]:
        st, plan = _create(ader_mod, dim=dim, M=M, system=system, n=(8, 6, 5))
        assert st == 0
        n = ctypes.c_int()
        assert lib.ader_plan_nvar(plan, ctypes.byref(n)) == 0 and n.value == nv
        b = ctypes.c_size_t()
        assert lib.ader_workspace_bytes(plan, ctypes.byref(b)) == 0
        C = 8 * 6 * (5 if dim == 3 else 1)
        # at least the predictor tensor of every cell
        assert b.value >= 8 * nv * (M + 1) ** (dim + 1) * C
        assert lib.ader_plan_destroy(plan) == 0
    assert lib.ader_plan_destroy(None) == 0


def test_compute_calls_validate_before_launching(ader_mod):
    lib = ader_mod.load_library()
    st, plan = _create(ader_mod, dim=2, M=2, n=(8, 8, 1))
    assert st == 0
    fake = ctypes.c_void_p(0x10000)
    ws = ctypes.c_void_p(0x20000)
    dt = ctypes.c_void_p(0x30000)
    # same input and output
    assert lib.ader_step(plan, fake, fake, 64, dt, ws, None) == -1
    # overlapping input and output
    assert lib.ader_step(plan, fake, ctypes.c_void_p(0x10000 + 8), 64, dt, ws, None) == -1
    # ld too small
    assert lib.ader_step(plan, fake, ctypes.c_void_p(0x90000), 63, dt, ws, None) == -1
    # misaligned / null workspace
    assert lib.ader_step(plan, fake, ctypes.c_void_p(0x90000), 64, dt,
                         ctypes.c_void_p(0x20008), None) == -4
    assert lib.ader_step(plan, fake, ctypes.c_void_p(0x90000), 64, dt, None, None) == -4
    # bad time interval
    assert lib.ader_compute_dt(plan, fake, 64, 1.0, 0.5, dt, ws, None) == -1
    assert lib.ader_debug_predict(plan, fake, -1, fake, dt, ws, None) == -1
    lib.ader_plan_destroy(plan)


def test_static_step_validates_before_launching(ader_mod):
    """ader_step_static checks its arguments and the static workspace's size
    before any HIP call."""
    lib = ader_mod.load_library()
    st, plan = _create(ader_mod, dim=2, M=2, n=(8, 8, 1))
    assert st == 0
    fake = ctypes.c_void_p(0x10000)
    dt = ctypes.c_void_p(0x30000)
    assert lib.ader_step_static(plan, fake, fake, 64, dt, None, None) == -1
    assert lib.ader_step_static(plan, fake, ctypes.c_void_p(0x10000 + 8), 64, dt, None,
                                None) == -1
    assert lib.ader_step_static(plan, fake, ctypes.c_void_p(0x90000), 63, dt, None, None) == -1
    assert lib.ader_step_static(plan, fake, ctypes.c_void_p(0x90000), 64, None, None,
                                None) == -1
    lib.ader_plan_destroy(plan)
    # 512^2 at M = 3 needs 512 MiB of traces: more than the static 64 MiB
    st, plan = _create(ader_mod, dim=2, M=3, n=(512, 512, 1))
    assert st == 0
    big = ctypes.c_void_p(0x100000000)
    assert lib.ader_step_static(plan, fake, big, 512 * 512, dt, None, None) == -4
    assert b"static workspace" in lib.ader_last_error()
    lib.ader_plan_destroy(plan)


@pytest.mark.parametrize("M", [0, 1, 2, 3])
def test_device_path_constants_agree_with_oracle(ader_mod, M):
    """The library's long-double generator and the oracle's exact polynomial
    algebra are separate routes to the same reference-element constants."""
    lib = ader_mod.load_library()
    st, plan = _create(ader_mod, dim=2, M=M, n=(4, 4, 1))
    assert st == 0
    n = M + 1
    arrs = [np.zeros(n), np.zeros(n), np.zeros(n * n), np.zeros(n * n)]
    assert lib.ader_debug_constants(plan, *[a.ctypes.data_as(ctypes.c_void_p)
                                            for a in arrs]) == 0
    b = basis(M)
    np.testing.assert_allclose(arrs[0], b.nodes, rtol=0, atol=2e-16)
    np.testing.assert_allclose(arrs[1], b.weights, rtol=0, atol=2e-16)
    np.testing.assert_allclose(arrs[2].reshape(n, n), b.dmat, rtol=0, atol=1e-13)
    A = np.linalg.solve(b.time_matrix(), np.diag(b.weights))
    np.testing.assert_allclose(arrs[3].reshape(n, n), A, rtol=0, atol=1e-14)
    lib.ader_plan_destroy(plan)


def test_step_level_validates_before_launching(ader_mod):
    lib = ader_mod.load_library()
    st, plan = _create(ader_mod, dim=2, M=2, n=(8, 8, 1))
    assert st == 0
    fake = ctypes.c_void_p(0x10000)
    out = ctypes.c_void_p(0x90000)
    ws = ctypes.c_void_p(0x20000)
    dt = ctypes.c_void_p(0x30000)
    V = ader_mod.CLevelView
    ok = dict(npred=4, pred_cells=0x40000, pred_patch=0x50000, nupd=2, upd=0x60000,
              upd_nbr=0x70000)

    def call(**over):
        kw = dict(ok, **over)
        v = V()
        v.dx[:] = kw.pop("dx", [0.1, 0.1, 1.0])
        for k, val in kw.items():
            setattr(v, k, val)
        return lib.ader_step_level(plan, ctypes.byref(v), fake, out, 64, dt, ws, None)
    assert call(nupd=5) == -1                 # more updated than predicted
    assert call(npred=-1) == -1
    assert call(pred_patch=None) == -1
    assert call(upd_nbr=None) == -1
    assert call(dx=[0.0, 0.1, 1.0]) == -1
    v = V()
    v.dx[:] = [0.1, 0.1, 1.0]
    assert lib.ader_step_level(plan, ctypes.byref(v), fake, fake, 64, dt, ws, None) == -1
    assert lib.ader_step_level(plan, None, fake, out, 64, dt, ws, None) == -1
    b = ctypes.c_size_t()
    assert lib.ader_level_workspace_bytes(plan, 1000, ctypes.byref(b)) == 0 and b.value > 0
    assert lib.ader_level_workspace_bytes(plan, -1, ctypes.byref(b)) == -1
    lib.ader_plan_destroy(plan)


def test_server_host_validation(ader_mod):
    """Server arguments are checked on the host before any device call."""
    lib = ader_mod.load_library()
    h = ctypes.c_void_p()
    for cfg in [(0, 4, 1, 1), (1 << 30, 0, 1, 1), (1 << 30, 5000, 1, 1),
                (1 << 30, 4, 0, 1), (1 << 30, 4, 17, 1), (1 << 30, 4, 1, 0), (1 << 30, 4, 1, 9)]:
        c = ader_mod.CServerConfig(*cfg)
        assert lib.ader_server_create(ctypes.byref(c), ctypes.byref(h)) == ader_mod.EINVAL
    b = ctypes.c_size_t()
    p3 = ader_mod.Problem(dim=3, M=2, n=(8, 8, 8)).to_c()
    assert lib.ader_server_footprint(ctypes.byref(p3), ctypes.byref(b)) == ader_mod.EUNSUPPORTED
    bad = ader_mod.Problem(dim=2, M=5, n=(8, 8, 1)).to_c()
    assert lib.ader_server_footprint(ctypes.byref(bad), ctypes.byref(b)) == ader_mod.EUNSUPPORTED
    # footprint: two fp64 state copies, a 1 KiB header, the CFL partials and
    # four face traces of nv * n^2 values per cell
    for M, prec, el in [(3, 0, 8), (2, 1, 4), (1, 0, 8)]:
        pr = ader_mod.Problem(dim=2, M=M, n=(64, 48, 1), precision=prec)
        assert lib.ader_server_footprint(ctypes.byref(pr.to_c()), ctypes.byref(b)) == 0
        n, C = M + 1, 64 * 48
        expect = 2 * 4 * C * 8 + 1024 + 1024 + 4 * 4 * n * n * C * el
        assert expect <= b.value <= expect + 4 * 256


def test_mhd_problem_validation(ader_mod):
    lib = ader_mod.load_library()
    h = ctypes.c_void_p()
    good = ader_mod.Problem(dim=2, M=2, system=ader_mod.SYS_MHD_GLM, gamma=5.0 / 3.0, ch=2.0,
                            n=(8, 8, 1))
    assert lib.ader_plan_create(ctypes.byref(good.to_c()), ctypes.byref(h)) == 0
    nv = ctypes.c_int()
    assert lib.ader_plan_nvar(h, ctypes.byref(nv)) == 0 and nv.value == 9
    lib.ader_plan_destroy(h)
    for ch in (0.0, -1.0, float("nan"), float("inf")):
        bad = ader_mod.Problem(dim=2, M=2, system=ader_mod.SYS_MHD_GLM, gamma=5.0 / 3.0, ch=ch,
                               n=(8, 8, 1))
        assert lib.ader_plan_create(ctypes.byref(bad.to_c()), ctypes.byref(h)) == ader_mod.EINVAL
    bad = ader_mod.Problem(dim=2, M=2, system=ader_mod.SYS_MHD_GLM, gamma=1.0, n=(8, 8, 1))
    assert lib.ader_plan_create(ctypes.byref(bad.to_c()), ctypes.byref(h)) == ader_mod.EINVAL
    bad = ader_mod.Problem(dim=2, M=2, system=3, n=(8, 8, 1))
    assert lib.ader_plan_create(ctypes.byref(bad.to_c()), ctypes.byref(h)) == ader_mod.EUNSUPPORTED


def test_orszag_tang_field_is_divergence_free():
    """The seeded Orszag-Tang family keeps B_x = B_x(y), B_y = B_y(x): the
    discrete divergence of the cell averages vanishes identically."""
    from paper_1212_3585_amd import workloads as wl
    U = wl.orszag_tang(16, seed=7)
    Bx, By = U[5], U[6]
    assert np.allclose(Bx, Bx[:1, :], atol=1e-14)   # independent of x
    assert np.allclose(By, By[:, :1], atol=1e-14)   # independent of y
    assert np.all(U[8] == 0) and np.all(U[3] == 0) and np.all(U[7] == 0)


def test_flux_selector_validation(ader_mod):
    lib = ader_mod.load_library()
    h = ctypes.c_void_p()
    ok = ader_mod.Problem(dim=2, M=2, n=(8, 8, 1), flux=ader_mod.FLUX_OSHER)
    assert lib.ader_plan_create(ctypes.byref(ok.to_c()), ctypes.byref(h)) == 0
    lib.ader_plan_destroy(h)
    bad = ader_mod.Problem(dim=2, M=2, n=(8, 8, 1), flux=2)
    assert lib.ader_plan_create(ctypes.byref(bad.to_c()), ctypes.byref(h)) == ader_mod.EINVAL
    mhd = ader_mod.Problem(dim=2, M=2, system=ader_mod.SYS_MHD_GLM, gamma=5 / 3, n=(8, 8, 1),
                           flux=ader_mod.FLUX_OSHER)
    assert lib.ader_plan_create(ctypes.byref(mhd.to_c()), ctypes.byref(h)) == ader_mod.EUNSUPPORTED


def test_tile_rows_validation(ader_mod):
    lib = ader_mod.load_library()
    for kw, good, bad in [
        (dict(dim=2, M=3, n=(32, 32, 1)), (0, 2, 4, 8, 16), (1, 3, 32)),
        (dict(dim=2, M=2, n=(32, 32, 1), system=ader_mod.SYS_MHD_GLM), (2, 4, 8), (16,)),
        (dict(dim=2, M=2, n=(32, 32, 1), system=ader_mod.SYS_MHD_GLM, precision=1),
         (2, 4, 8), (16,)),
    ]:
        st, plan = _create(ader_mod, **kw)
        assert st == 0
        for r in good:
            assert lib.ader_set_tile_rows(plan, r) == 0, (kw, r)
        for r in bad:
            assert lib.ader_set_tile_rows(plan, r) == -1, (kw, r)
        # reps out of range is refused before any launch
        assert lib.ader_tune(plan, None, 0, None, None, None, 0, None, None) == -1
        lib.ader_plan_destroy(plan)
    st, plan3 = _create(ader_mod, dim=3, M=2, n=(8, 8, 8))
    assert st == 0
    assert lib.ader_set_tile_rows(plan3, 8) == -2
    lib.ader_plan_destroy(plan3)
    assert lib.ader_set_tile_rows(None, 8) == -1


def test_amr_tune_needs_a_built_mesh(ader_mod):
    lib = ader_mod.load_library()
    assert lib.ader_amr_tune(None, 3, None, None, None) == -1
