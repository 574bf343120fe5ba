"""Shared helpers of the GPU tests: problem construction and comparisons."""
import sys

import numpy as np

import oracle
from oracle import Euler, GLMMHD, LinearAdvection, Problem as OProblem
from paper_1212_3585_amd import workloads as wl

BCS = {"periodic": 0, "transmissive": 1}


def say(msg):
    """Name the case before a GPU step (survives a crash of the process)."""
    print(msg, flush=True)
    sys.stdout.flush()


def make_pair(ader, dim, M, n, lo, hi, bc="periodic", system="euler", adv=(1.0, 0.5, 0.25),
              precision=0, cfl=0.9, tol=1e-14, maxit=64, gamma=None, ch=2.0, flux="rusanov"):
    """(oracle problem, GPU problem) describing the same mesh and scheme.
    system: "euler" (gamma 1.4), "mhd" (GLM-MHD, gamma 5/3, cleaning speed ch)
    or "linadv"."""
    bcs = [bc] * dim if isinstance(bc, str) else list(bc)
    if gamma is None:
        gamma = 5.0 / 3.0 if system == "mhd" else 1.4
    sysobj = {"euler": lambda: Euler(dim, gamma), "mhd": lambda: GLMMHD(dim, gamma, ch),
              "linadv": lambda: LinearAdvection(dim, adv)}[system]()
    sys_id = {"euler": ader.SYS_EULER, "mhd": ader.SYS_MHD_GLM, "linadv": ader.SYS_LINADV}[system]
    op = OProblem(dim, M, sysobj, tuple(n), tuple(lo), tuple(hi), bcs, cfl=cfl,
                  tol=tol, max_iter=maxit, flux=flux)
    gp = ader.Problem(dim=dim, M=M, system=sys_id, ch=ch,
                      flux={"rusanov": ader.FLUX_RUSANOV, "osher": ader.FLUX_OSHER}[flux],
                      gamma=gamma, adv=tuple(adv), n=tuple(n) + (1,) * (3 - dim),
                      lo=tuple(lo) + (0.0,) * (3 - dim), hi=tuple(hi) + (1.0,) * (3 - dim),
                      bc=tuple(BCS[b] for b in bcs) + (0,) * (3 - dim), cfl=cfl,
                      precision=precision, picard_tol=tol, picard_max=maxit)
    return op, gp


def to_device(U, ld=None):
    import torch
    return torch.tensor(wl.to_soa(U, ld), dtype=torch.float64, device="cuda")


def from_device(u, shape):
    return wl.from_soa(u.cpu().numpy(), shape)


def rel_l1(a, b):
    """Relative L1 distance of two states, pooled over the conserved variables:
    sum_{v,cells} |a - b| / sum_{v,cells} |b|."""
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def max_rel(a, b):
    """Element-wise distance: max over entries of |a - b| / max(1, |b|)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float((np.abs(a - b) / np.maximum(1.0, np.abs(b))).max())


def check_parity(got, ref, tol=1e-11, tol_max=None, label="parity"):
    """Assert pooled relative L1 <= tol and element-wise max_rel <= tol_max
    (default tol); print both; return them."""
    l1, mx = rel_l1(got, ref), max_rel(got, ref)
    print(f"{label}: pooled L1 {l1:.3e}, element-wise {mx:.3e}")
    assert l1 <= tol, (l1, rel_l1_per_var(got, ref))
    assert mx <= (tol if tol_max is None else tol_max), mx
    return l1, mx


def rel_l1_per_var(a, b):
    """Per-variable relative L1 (informative: a variable near zero, such as the
    momentum of a gas at rest, makes its own ratio meaningless)."""
    return [float(np.abs(a[v] - b[v]).sum() / max(np.abs(b[v]).sum(), 1e-300))
            for v in range(a.shape[0])]


def oracle_wh_to_gpu_layout(w, dim):
    """oracle w[v, C, px, py(, pz)] -> flat [(cell * nv + v) * n^d + a]."""
    from oracle.predictor import spatial_flat
    wf = spatial_flat(w, dim)                 # [v, C, a]
    return np.ascontiguousarray(np.transpose(wf, (1, 0, 2))).ravel()


def gpu_qh_to_oracle_layout(qh, nv, C, nst):
    """flat [(cell * nv + v) * nst + i] -> [v, C, nst]."""
    return np.transpose(qh.reshape(C, nv, nst), (1, 0, 2))
