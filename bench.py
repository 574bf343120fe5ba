"""Throughput benchmark of the ADER-WENO hot path on one MI355X.

Workload: 2D Euler, Kelvin-Helmholtz shear layer on the periodic unit square,
uniform 512 x 512 mesh, order 4 (M = 3), Rusanov flux, CFL 0.9 (seeded
synthetic initial data, paper_1212_3585_amd.workloads).  A step is one pass of
the whole hot path: CFL time step (device reduction), WENO reconstruction,
space-time predictor, face fluxes and update.  The state stays resident in
HBM; nothing crosses PCIe inside the timed region.

Prints ONE JSON line:
  value           fp64 path, cell-updates/s (active cells x steps / s)
  mixed           the fp32-predictor form on the same GPU: rate, speedup,
                  relative L1 against the fp64 oracle
  roofline        dominant kernel (the predictor): algorithmic flops per
                  launch / its average duration from HIP events recorded on
                  the launch stream, against the fp64 vector peak
  cpu_baseline    the CPU oracle timed on a bounded sample of the workload
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 512
M = 3
FP64_PEAK_TFLOPS = 78.6     # MI355X fp64 vector (256 CU x 2.4 GHz x 128 flop/clk)
FP32_PEAK_TFLOPS = 157.3    # MI355X fp32 vector (packed)
HBM_PEAK_GBS = 8000.0


def predictor_flops_per_cell_iteration(dim, M, nv, euler=True):
    """Algorithmic flops of one Picard iteration of one cell.

    per space-time node: physical fluxes (Euler: d^2 + 5 d + 3 flops, a
    division counted as one), scaling by dt/dx (d nv); per node and variable:
    the d spatial derivative products (2 d n), the time product (2 n) and the
    subtraction from w_hat (1).
    """
    n = M + 1
    nst = n ** (dim + 1)
    cflux = dim * dim + 5 * dim + 3 if euler else dim
    return nst * (cflux + dim * nv + nv * (2 * dim * n + 2 * n + 1))


def weno_flops_per_line(M):
    """One 1D WENO reconstruction (eqs. rec.x, sigmas, omegas, weno).

    per stencil: the n x n inverse (2 n^2); sigma as the sum of the squared
    Legendre coefficients of the derivatives alpha = 1..M, M (M + 1) / 2
    coefficients of n products each (2 n + 2 per coefficient); the weight
    lambda / (sigma + eps)^8 (5); then the sum and normalisation of the
    weights (2 per stencil) and the combination (2 n per stencil).
    """
    n = M + 1
    nst = 3 if M % 2 == 0 else 4
    nr = M * (M + 1) // 2
    return nst * (2 * n * n + nr * (2 * n + 2) + 5) + 2 * nst + 2 * n * nst


def predictor_flops_first_sweep(dim, M, nv, euler=True):
    """Algorithmic flops of a cell's first Picard sweep, which starts from
    q = w_hat at every time node: the physical fluxes, their dt/dx scaling
    and the spatial derivative products at the n^d spatial nodes only; then
    per space-time node and variable the product with the row sum of the
    time matrix and the subtraction from w_hat (2)."""
    n = M + 1
    cflux = dim * dim + 5 * dim + 3 if euler else dim
    return n ** dim * (cflux + dim * nv + nv * 2 * dim * n) + n ** (dim + 1) * nv * 2


def cell_kernel_flops(dim, M, nv, picard_sweeps_total, ncells):
    """Algorithmic flops of one launch of the fused cell kernel: WENO
    (nv (1 + n) lines per cell in 2D), the Picard sweeps counted on the
    device (every cell's first sweep at its reduced cost), and the four face
    traces (2 n flops per trace value)."""
    n = M + 1
    weno = ncells * nv * (1 + n) * weno_flops_per_line(M)
    picard = ((picard_sweeps_total - ncells) * predictor_flops_per_cell_iteration(dim, M, nv)
              + ncells * predictor_flops_first_sweep(dim, M, nv))
    traces = ncells * 2 * dim * nv * n ** dim * 2 * n
    return weno + picard + traces


# the sources the uniform 2D cell and face kernels are compiled from (their
# launcher, kernels, constants and the header they include)
CELL_KERNEL_SOURCES = ("impl2d.hip", "impl.hpp", "plan.hpp", "fused2d.hpp", "level.hpp",
                       "predict_mfma.hpp", "predict_wave.hpp", "kernels.hpp", "consts.hpp",
                       "consts.cpp",
                       "cell2d_launch.hpp", "cell2d_rows.hpp", "cell2d_rows2.hip",
                       "cell2d_rows4.hip", "cell2d_rows8.hip", "cell2d_rows16.hip")


def device_source_hash():
    """sha256 of the sources of the measured kernels: a traffic figure taken
    on other kernels than the ones built now is not reported."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1212_3585_amd", "csrc")
    h = hashlib.sha256()
    for name in CELL_KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(ROOT, "include", "ader.h"), "rb") as f:
        h.update(b"ader.h\0" + f.read())
    return h.hexdigest()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_cell2d_kh512_m3.json")
CLOCK_FILE = os.path.join(ROOT, "profiles", "clock_k_cell2d_kh512_m3.json")
NOMINAL_CLOCK_GHZ = 2.4


def recorded_traffic():
    """HBM bytes per launch of the fp64 cell kernel from the committed
    counter measurement, or None when the kernels have changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("device_source_sha256") != device_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def recorded_clock_ghz():
    """Shader clock measured during the fp64 cell kernel (GRBM_GUI_ACTIVE of
    one XCD over the dispatch's duration, from the committed counter run), or
    None when the kernels have changed since."""
    try:
        with open(CLOCK_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("device_source_sha256") != device_source_hash():
        return None
    return rec.get("measured_clock_ghz")


def traffic_probe():
    """Run under rocprofv3 --pmc: one step of each precision on the bench
    workload, then a 256 MiB device-to-device copy whose FETCH_SIZE and
    WRITE_SIZE calibrate the counters (known 256 MiB read + 256 MiB write)."""
    import torch
    from paper_1212_3585_amd import ader, workloads as wl
    ader.require_gpu()
    U0 = wl.kelvin_helmholtz(N)
    u0 = torch.tensor(wl.to_soa(U0), dtype=torch.float64, device="cuda")
    for precision, tol in ((ader.PREC_FP64, 1e-14), (ader.PREC_FP32_PREDICTOR, 1e-6)):
        s = ader.Solver(ader.Problem(dim=2, M=M, n=(N, N, 1), precision=precision,
                                     picard_tol=tol))
        b = torch.empty_like(u0)
        s.compute_dt(u0)
        s.tune(u0, reps=2)
        s.step(u0, b)
    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print("traffic probe done: copy of", src.numel() * 8, "bytes", flush=True)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


SERVE_SIZES = (32, 64, 128, 256, 512)
SERVE_ORDERS = (1, 2, 3)
SERVE_T_END = 0.5


def serving_requests(ader, wl, count, seed=4):
    """Seeded request mix of the serving workload: half 2D Euler
    Kelvin-Helmholtz solves (unit square, gamma 1.4), half GLM-MHD
    Orszag-Tang solves ([0, 2 pi]^2, gamma 5/3, c_h = 2, random phases and
    amplitudes), each with its own seed; meshes 32^2..512^2 and degrees
    M = 1..3 drawn uniformly; each to t = 0.5, fp64."""
    import numpy as np
    r = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for i in range(count):
        n = int(r.choice(SERVE_SIZES))
        M = int(r.choice(SERVE_ORDERS))
        if i % 2 == 0:
            prob = ader.Problem(dim=2, M=M, n=(n, n, 1), precision=ader.PREC_FP64,
                                picard_tol=1e-14)
            U0 = wl.kelvin_helmholtz(n, seed=100 + i)
        else:
            L = 2.0 * np.pi
            prob = ader.Problem(dim=2, M=M, system=ader.SYS_MHD_GLM, gamma=5.0 / 3.0, ch=2.0,
                                n=(n, n, 1), lo=(0.0, 0.0, 0.0), hi=(L, L, 1.0),
                                precision=ader.PREC_FP64, picard_tol=1e-14)
            U0 = wl.orszag_tang(n, seed=100 + i)
        reqs.append((prob, U0, SERVE_T_END))
    return reqs


def serve(ader, reqs, arrivals, hbm_bytes):
    """Run one request stream through a fresh server: request i is submitted
    at arrivals[i] seconds (None: all at once).  Returns per-request latency
    (submit to result in host memory), makespan and cell updates."""
    import numpy as np
    srv = ader.Server(hbm_bytes=hbm_bytes, max_slots=256, streams=4, rounds_ahead=2)
    ids = []
    t0 = time.monotonic()
    i = 0
    n = len(reqs)
    while True:
        now = time.monotonic() - t0
        while i < n and (arrivals is None or arrivals[i] <= now):
            ids.append(srv.submit(*reqs[i]))
            i += 1
        srv.progress(wait=(i == n))
        if i == n and srv.stats()["completed"] == n:
            break
    makespan = time.monotonic() - t0
    infos = [srv.info(rid) for rid in ids]
    st = srv.stats()
    srv.close()
    lat = np.array([f["done_s"] - f["submit_s"] for f in infos])
    cell_updates = sum(f["steps"] * p.n[0] * p.n[1] for f, (p, _, _) in zip(infos, reqs))
    bad = [f["state"] for f in infos if f["state"] != ader.REQ_DONE]
    return {"latency": lat, "makespan": makespan, "cell_updates": cell_updates,
            "failed": len(bad), "peak_resident": st["peak_resident"],
            "peak_bytes": st["peak_bytes_in_use"], "rounds": st["rounds"]}


def amr_leg(ader, label, dim, n0, r, L, M, ic, precision, steps, cfl=0.5, regrid_steps=0):
    """One AMR configuration: mesh built by the Loehner indicator on the
    energy (the density noise does not enter it), one-layer flag buffer,
    local time stepping, one recorded graph per level-0 step.  Rate =
    active-cell substeps per second over 'steps' level-0 steps on the static
    mesh; then 'regrid_steps' steps each followed by a regrid (refine above
    chi 0.2, recoarsen below 0.1), regrid time included in that rate."""
    import numpy as np
    tol = 1e-14 if precision == ader.PREC_FP64 else 1e-6
    prob = ader.Problem(dim=dim, M=M, n=(n0,) * dim + (1,) * (3 - dim), lo=(-1.0,) * 3,
                        hi=(1.0,) * 3, bc=(ader.BC_TRANSMISSIVE,) * 3, cfl=cfl,
                        precision=precision, picard_tol=tol)
    A = ader.Amr(prob, r=r, max_level=L, indicator_var=dim + 1, chi_ref=0.2, chi_rec=0.1,
                 eps=0.01, buffer=1, use_graph=True)
    for l in range(L + 1):
        A.set_level(l, ic(n0 * r ** l, l))
    t0 = time.perf_counter()
    A.build()
    build_s = time.perf_counter() - t0
    counts = [A.counts(l) for l in range(L + 1)]

    def totals():
        """Integral of each conserved variable over the active cells."""
        tot = 0.0
        for l in range(L + 1):
            U, stat = A.level(l)
            vol = (2.0 / (n0 * r ** l)) ** dim
            tot = tot + vol * U[:, stat == 0].sum(axis=1)
        return tot

    tot0 = totals()
    A.step(1e9)                      # warm-up (sets the level steps)
    pb, fb, tune_ms = A.tune(reps=3)  # launch shapes of the predictor and the face fluxes
    A.step(1e9)                      # records the graph with the tuned shapes
    A.clock()
    cu0 = A.stats()["cell_updates"]
    t0 = time.perf_counter()
    for _ in range(steps):
        A.step(1e9)
    t_sim, nsteps, dt0 = A.clock()
    el = time.perf_counter() - t0
    st = A.stats()
    cu = st["cell_updates"] - cu0
    out = {"workload": label, "precision": "fp64" if precision == ader.PREC_FP64 else
           "fp32 predictor / fp64", "levels": counts, "mesh_build_s": build_s,
           "level0_steps": steps, "cell_updates": cu, "seconds": el,
           "cell_updates_per_s": cu / el, "ms_per_level0_step": el / steps * 1e3,
           "t_reached": t_sim, "status_flags": st["flags"],
           "autotune": {"predict_block": pb, "flux_block": fb, "ms_per_launch": tune_ms}}
    if regrid_steps > 0:
        cu0 = st["cell_updates"]
        t_regrid, changed = 0.0, 0
        t0 = time.perf_counter()
        for _ in range(regrid_steps):
            A.step(1e9)
            A.clock()
            t1 = time.perf_counter()
            changed += A.regrid()
            t_regrid += time.perf_counter() - t1
        A.clock()
        el = time.perf_counter() - t0
        st = A.stats()
        cu = st["cell_updates"] - cu0
        out["with_regrid"] = {
            "level0_steps": regrid_steps, "regrids_that_changed_the_mesh": changed,
            "cell_updates": cu, "seconds": el, "cell_updates_per_s": cu / el,
            "regrid_ms_avg": t_regrid / regrid_steps * 1e3,
            "levels_after": [A.counts(l) for l in range(L + 1)], "status_flags": st["flags"]}
    # conservation over every step of the leg (no wave reaches the boundary
    # in this time): relative drift of each conserved variable's total
    tot1 = totals()
    scale = float(np.abs(tot0).max())
    out["conservation_max_rel_drift"] = float(np.abs(tot1 - tot0).max() / scale)
    A.close()
    return out


def amr_legs(ader, wl):
    """The paper-shaped AMR workloads: 2D explosion (level 0 100^2, r = 3,
    two levels, M = 2, fp32 predictor and fp64) and 3D blast (level 0 64^3,
    r = 3, one level, M = 2, fp64 and fp32 predictor), transmissive, CFL 0.5."""
    out = []
    expl = lambda n, l: wl.explosion_2d(n, seed=2)
    blast = lambda n, l: wl.blast_3d(n, seed=3, nq=4 if l == 0 else 2)
    for prec in (ader.PREC_FP32_PREDICTOR, ader.PREC_FP64):
        log(f"bench: AMR 2D explosion, precision {prec}")
        out.append(amr_leg(ader, "2D Euler explosion (rho, p) = (1, 1) inside r = 0.5, "
                           "(0.125, 0.1) outside, 1% density noise (seed 2), [-1,1]^2, "
                           "level 0 100^2, r = 3, 2 levels, M = 2",
                           2, 100, 3, 2, 2, expl, prec, steps=10, regrid_steps=10))
    for prec in (ader.PREC_FP64, ader.PREC_FP32_PREDICTOR):
        log(f"bench: AMR 3D blast, precision {prec}")
        out.append(amr_leg(ader, "3D Euler blast p = 1 inside r = 0.3, 0.1 outside, rho = 1 "
                           "with 1% noise (seed 3), [-1,1]^3, level 0 64^3, r = 3, 1 level, "
                           "M = 2", 3, 64, 3, 1, 2, blast, prec, steps=2, regrid_steps=2))
    return out


def vortex_leg(ader, wl, torch):
    """Isentropic vortex, 20x20, M = 2, periodic [0,10]^2, CFL 0.9, to t = 1:
    per-step latency (a step = CFL kernel + cell kernel + face kernel, with
    the host reading dt back) and the error against the exact solution, the
    initial state translated by (t, t)."""
    import numpy as np
    n, t_end = 20, 1.0
    prob = ader.Problem(dim=2, M=2, n=(n, n, 1), lo=(0, 0, 0), hi=(10, 10, 1), cfl=0.9)
    s = ader.Solver(prob)
    u0 = torch.tensor(wl.to_soa(wl.isentropic_vortex(n)), dtype=torch.float64, device="cuda")
    s.run(u0, t_end)                                   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, t, steps = s.run(u0, t_end)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    got = wl.from_soa(u.cpu().numpy(), (n, n))
    exact = wl.isentropic_vortex(n, t=t)
    flags, _ = s.read_status()
    return {"workload": "2D Euler isentropic vortex (eps 5), 20x20 on periodic [0,10]^2, M = 2, "
                        "Rusanov, CFL 0.9, to t = 1, fp64",
            "steps": steps, "t": t, "ms_per_step": wall / steps * 1e3,
            "l1_vs_exact": float(np.abs(got - exact).sum() / np.abs(exact).sum()),
            "l1_rho_vs_exact": float(np.abs(got[0] - exact[0]).sum() / np.abs(exact[0]).sum()),
            "status_flags": flags}


def serving_leg(ader, wl, count, hbm_bytes=16 << 30, seed=4):
    """Closed loop (all requests at t = 0) for the maximum rate, then Poisson
    arrivals (seed 5) at 0.5 and 0.9 of it: p50 / p99 latency and solves/s."""
    import numpy as np
    reqs = serving_requests(ader, wl, count, seed)
    log(f"bench: serving, {count} requests, closed loop")
    closed = serve(ader, reqs, None, hbm_bytes)
    mu = count / closed["makespan"]
    out = {
        "workload": f"{count} independent 2D solves (alternately Euler KH and GLM-MHD "
                    f"Orszag-Tang) to t = {SERVE_T_END}, meshes "
                    f"{SERVE_SIZES[0]}^2..{SERVE_SIZES[-1]}^2, M in {list(SERVE_ORDERS)}, fp64, "
                    f"drawn uniformly (PCG64 seed {seed}); server arena {hbm_bytes >> 30} GiB, "
                    "4 streams",
        "max_solves_per_s": mu,
        "closed_loop": {"makespan_s": closed["makespan"],
                        "cell_updates_per_s": closed["cell_updates"] / closed["makespan"],
                        "p50_latency_s": float(np.percentile(closed["latency"], 50)),
                        "p99_latency_s": float(np.percentile(closed["latency"], 99)),
                        "peak_resident": closed["peak_resident"],
                        "peak_arena_bytes": closed["peak_bytes"], "failed": closed["failed"]},
        "poisson": [],
    }
    r = np.random.Generator(np.random.PCG64(seed + 1))
    gaps = r.exponential(1.0, size=count)
    for frac in (0.5, 0.9):
        lam = frac * mu
        arrivals = np.cumsum(gaps) / lam
        log(f"bench: serving, Poisson arrivals at {lam:.2f} solves/s")
        res = serve(ader, reqs, arrivals, hbm_bytes)
        out["poisson"].append({
            "offered_solves_per_s": lam, "solves_per_s": count / res["makespan"],
            "cell_updates_per_s": res["cell_updates"] / res["makespan"],
            "p50_latency_s": float(np.percentile(res["latency"], 50)),
            "p99_latency_s": float(np.percentile(res["latency"], 99)),
            "peak_resident": res["peak_resident"], "failed": res["failed"]})
    return out


def time_form(ader, wl, torch, precision, tol, steps, warmup, u0):
    """Warm up, then time `steps` steps.  Every launch of this solver (warmup,
    timed steps, and the later check step) is bracketed by HIP events on its
    stream, so per-kernel averages cover the same launches a profiler sees."""
    prob = ader.Problem(dim=2, M=M, system=ader.SYS_EULER, gamma=1.4, n=(N, N, 1),
                        lo=(0, 0, 0), hi=(1, 1, 1), bc=(0, 0, 0), cfl=0.9,
                        precision=precision, picard_tol=tol, picard_max=64)
    s = ader.Solver(prob)
    # tile height of the cell kernel: timed on this state, fastest kept
    s.compute_dt(u0)
    rows, tune_ms = s.tune(u0, reps=5)
    s.profile_begin()
    a = u0.clone()
    b = torch.empty_like(a)
    for _ in range(warmup):
        s.compute_dt(a)
        s.step(a, b)
        a, b = b, a
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        s.compute_dt(a)
        s.step(a, b)
        a, b = b, a
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"ms": e0.elapsed_time(e1), "wall_s": wall, "solver": s, "tile_rows": rows,
            "tune_ms": tune_ms}


def finish_form(r):
    """Stop the stage events; totals and the Picard count over all launches."""
    s = r["solver"]
    r["stages"] = s.profile_end()
    r["flags"], r["iters"] = s.read_status()
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-rows", type=int, default=256,
                    help="mesh rows of the CPU-oracle sample (512 cells each)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="requests of the serving leg (0 skips it)")
    ap.add_argument("--no-amr", action="store_true", help="skip the AMR legs")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run the launches that the HBM counters calibrate")
    ap.add_argument("--amr-only", action="store_true",
                    help="only the AMR legs (for profiling them); prints {\"amr\": [...]}")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on exactly one GPU; --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)
    if args.traffic_probe:
        traffic_probe()
        return
    if args.amr_only:
        from paper_1212_3585_amd import ader, workloads as wl
        ader.require_gpu()
        print(json.dumps({"amr": amr_legs(ader, wl)}), flush=True)
        return
    import numpy as np
    import torch

    from paper_1212_3585_amd import ader, workloads as wl
    ader.require_gpu()

    log("bench: building initial data (KH 512^2)")
    U0 = wl.kelvin_helmholtz(N)
    u0 = torch.tensor(wl.to_soa(U0), dtype=torch.float64, device="cuda")
    ncells = N * N

    log("bench: fp64 timed run")
    r64 = time_form(ader, wl, torch, ader.PREC_FP64, 1e-14, args.steps, args.warmup, u0)
    log("bench: fp32-predictor timed run")
    r32 = time_form(ader, wl, torch, ader.PREC_FP32_PREDICTOR, 1e-6, args.steps,
                    args.warmup, u0)
    rate64 = ncells * args.steps / (r64["ms"] * 1e-3)
    rate32 = ncells * args.steps / (r32["ms"] * 1e-3)

    # one step of each form from the initial data, sampled against the oracle
    sample_rows = max(1, args.cpu_rows)
    cells = np.array([[i, j] for j in range(sample_rows) for i in range(N)])
    outs = {}
    for name, r in (("fp64", r64), ("fp32", r32)):
        s = r["solver"]
        b = torch.empty_like(u0)
        s.compute_dt(u0)
        s.step(u0, b)
        outs[name] = wl.from_soa(b.cpu().numpy(), (N, N))[:, cells[:, 0], cells[:, 1]]
        finish_form(r)

    # roofline of the dominant kernel (predictor) of the fp64 path
    pms, plaunch = r64["stages"]["predict"]
    flops_launch = cell_kernel_flops(2, M, 4, r64["iters"] / plaunch, ncells)
    avg_s = pms / plaunch * 1e-3
    achieved = flops_launch / avg_s / 1e12
    p32ms, p32l = r32["stages"]["predict"]
    ach32 = cell_kernel_flops(2, M, 4, r32["iters"] / p32l, ncells) / (p32ms / p32l * 1e-3) / 1e12

    cpu = None
    l1 = {"fp64": None, "fp32": None}
    if not args.no_cpu:
        import oracle
        from threadpoolctl import threadpool_limits
        prob = oracle.Problem(2, M, oracle.Euler(2), (N, N), (0.0, 0.0), (1.0, 1.0),
                              ["periodic", "periodic"])
        dt = oracle.cfl_dt(prob, U0)
        log(f"bench: CPU oracle on {len(cells)} cells (rows 0..{sample_rows - 1})")
        with threadpool_limits(1):
            t0 = time.perf_counter()
            ref, _ = oracle.step_cells(prob, U0, dt, cells)
            el = time.perf_counter() - t0
        cpu = {"value": len(cells) / el, "unit": "cell-updates/s", "cores": 1,
               "kind": "oracle",
               "sample": f"one step of rows 0..{sample_rows - 1} ({len(cells)} cells) of the "
                         f"512x512 M=3 KH workload, numpy fp64 single-threaded, "
                         f"{el:.1f} s"}
        # relative L1 pooled over the conserved variables
        for k in ("fp64", "fp32"):
            l1[k] = float(np.abs(outs[k] - ref).sum() / np.abs(ref).sum())

    log("bench: isentropic vortex 20^2 (latency, error against the exact solution)")
    vortex = vortex_leg(ader, wl, torch)
    serving = None
    if args.serve_requests > 0:
        serving = serving_leg(ader, wl, args.serve_requests)
    amr = None if args.no_amr else amr_legs(ader, wl)

    clock = recorded_clock_ghz()
    line = {
        "metric": "cell-updates/s (FP32-predictor vs FP64) at stated L1 err; "
                  "p50/p99 solve latency",
        "value": rate64,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D Euler Kelvin-Helmholtz, uniform 512x512, ADER-WENO "
                               "order 4 (M=3), Rusanov, CFL 0.9, periodic, seed 1",
                   "cells": ncells, "M": M, "parallelism": "single GPU"},
        "l1_vs_oracle_fp64": l1["fp64"],
        "status_flags": r64["flags"],
        "picard_iterations_per_cell": r64["iters"] / plaunch / ncells,
        "stage_avg_ms_per_launch": {k: v[0] / v[1]
                                    for k, v in r64["stages"].items() if v[1]},
        "mixed": {"value": rate32, "unit": "cell-updates/s", "dtype": "f32 predictor / f64",
                  "speedup_vs_fp64": rate32 / rate64,
                  "l1_vs_fp64_oracle": l1["fp32"],
                  "status_flags": r32["flags"],
                  "picard_iterations_per_cell": r32["iters"] / p32l / ncells,
                  "cell_kernel_tflops": ach32,
                  "cell_kernel_frac_of_fp32_peak": ach32 / FP32_PEAK_TFLOPS,
                  "tile_rows": r32["tile_rows"],
                  "autotune_ms_per_launch": r32["tune_ms"]},
        "autotune": {"what": "tile height of the fused cell kernel (4 x rows cells), "
                             "timed on the initial state, fastest kept",
                     "fp64_tile_rows": r64["tile_rows"],
                     "fp64_ms_per_launch": r64["tune_ms"]},
        "roofline": {"bound": "alu",
                     "kernel": f"k_cell2d<3,1,{r64['tile_rows']},double> "
                               "(WENO + Picard predictor + traces)",
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": recorded_traffic(),
                     "measured_clock_ghz": clock,
                     "frac_at_measured_clock": (None if clock is None else achieved / (
                         FP64_PEAK_TFLOPS * clock / NOMINAL_CLOCK_GHZ)),
                     "flops_per_launch": flops_launch,
                     "avg_launch_ms": avg_s * 1e3},
        "cpu_baseline": cpu,
        "vortex": vortex,
        "serving": serving,
        "amr": amr,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
