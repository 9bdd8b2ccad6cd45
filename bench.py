#!/usr/bin/env python3
"""Throughput of the DOLINC explicit residual on one MI355X.

A step is one SSP-RK3 step (three residual stages: gradients, reconstruction,
Riemann flux, face-to-cell accumulation and the stage update) over the whole
mesh, with the state resident in HBM.  The headline value is cell-updates per
second per Runge-Kutta stage of the FP32-mixed path; the FP64 path on the
same mesh is reported beside it.  One JSON line goes to stdout.
"""
from __future__ import annotations

import argparse
import atexit
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per RK stage (FP32 vs FP64) + achieved HBM GB/s, 3D Euler"
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_case(workload):
    from synth import configs
    if workload == "vortex3d":
        case = configs.vortex_3d(point_ic=True, scheme="USR3")
        desc = ("3-D Euler isentropic vortex, [0,10]^3 periodic, 64^3 jittered hexes x 6 Kuhn tets "
                f"({case.mesh.n_cells:,} cells, {case.mesh.n_faces:,} faces), USR3 DOLINC, Rusanov, SSP-RK3")
        return case, desc, dict(blend="none"), dict(u_ref="cell")
    if workload == "tgv3d":
        case = configs.taylor_green_3d()
        desc = ("3-D Euler Taylor-Green vortex Mach 0.1, [0,2pi]^3 periodic, 288^3 jittered hexes "
                f"({case.mesh.n_cells:,} cells, {case.mesh.n_faces:,} faces), USR5 DOLINC, HLLC, "
                "learned-indicator blend with Van Leer, SSP-RK3")
        return case, desc, dict(blend="learned"), dict(u_ref="cell")
    raise SystemExit(f"unknown workload {workload}")


# Cells per partition of the flux kernel.  FP32 keeps two flux shares per
# face entry in LDS (each side about its own cell) and runs 512-cell
# partitions with 512-thread workgroups, two per CU (flux kernel at 288^3,
# same box: 2.82 ms, against 2.87 ms on 256-cell and 3.27 ms on 1024-cell
# partitions).  FP64's 512-cell partitions measured 4 % slower than 256.
PART_CELLS = {"fp32": 512, "fp64": 256}
# schemes timed without the blend on the headline mesh, and the paper's own
# figures of the same kind (context: CPU times of an OpenFOAM implementation)
SCHEME_COST_SCHEMES = ("CD2", "USR3", "CSR4", "USR5", "CSR6", "ENO3", "WENO5")
SCHEME_COST_NOTE = ("time per step relative to CD2 on the same mesh, HLLC, no blend; the paper's CPU-time "
                    "increases over CD2 (1-D linear advection, OpenFOAM on 2x Xeon Platinum 9242): USR3 +16 %, "
                    "CSR4 +18 %, USR5 +29 %, CSR6 +29 %, WENO5 +44 %")


def indicator_weights():
    import numpy as np
    return np.load(os.path.join(ROOT, "paper_2404_08952_amd", "data", "indicator_weights.npy"))


def flux_kernel_bytes(nc, nf, nv, dim, el, scheme, blend=False):
    """Algorithmic bytes of one flux + update launch: every array it needs
    read once, its output written once (Un counted in 2 of 3 stages)."""
    ord_ = 0 if scheme in ("FOU", "CD2") else (1 if scheme in ("USR3", "CSR4") else 2)
    dcs = 3  # d; the coefficients are evaluated in the kernel from omega
    # second differentials arrive contracted with d, one value per face side
    per_cell = nv * el + (nv * dim * el if ord_ >= 1 or blend else 0) \
        + el + 4 + nv * el + (2.0 / 3.0) * nv * el + (4 if blend else 0)
    # second differentials: the two one-byte record positions and d.H.d of
    # both cells
    per_face = 8 + 4 * el + dcs * el + 4 + (2 + 2 * nv * el if ord_ >= 2 else 0)
    return nc * per_cell + nf * per_face, per_cell, per_face


def grad_features_bytes(nc, nrec, nv, dim, el):
    """Algorithmic bytes of the first-gradient + features kernel: U, 1/V and
    the face count per cell, the two face records (sigma w S + the other
    cell: 4 values; sigma d: 3) per record, G1 and the 24 bf16 features
    written."""
    return nc * (nv * el + el + 4 + nv * dim * el + 48) + nrec * 7 * el


def grad_bytes(nc, nrec, nv, dim, el):
    """The plain first-gradient kernel: U and 1/V per cell, the records'
    sigma w S and other cell (it needs no face vector), G1 written."""
    return nc * (nv * el + el + nv * dim * el) + nrec * 4 * el


def hface_bytes(nc, nrec, nv, dim, el):
    """Algorithmic bytes of the second-derivative kernel: the cell's G1 row,
    1/V and its face count per cell, the two face records (7 values) and
    d.H.d written per record."""
    return nc * (nv * dim * el + el + 4) + nrec * (7 * el + nv * el)


# Compulsory bytes per cell and stage of the Taylor-Green workload (USR5,
# hexahedra: 3 faces per cell): U in, U^n in, U out; per face two cell
# indices, S, omega and d, and the DOLINC coefficients of both sides (8
# doubles: the FP64 values the method precomputes).
COMPULSORY_BYTES = {"fp32": 3 * 20 + 3 * (8 + 4 * 7 + 64), "fp64": 3 * 40 + 3 * (8 + 8 * 7 + 64)}


def time_path(s, case, precision, extra, steps, warmup, params=None, windows=0, window_steps=34):
    import torch
    t0 = time.time()
    s.configure(**(params or case.params), precision=precision, **extra)
    if extra.get("blend") == "learned":
        s.mlp_set(indicator_weights())
    log(f"[bench] {precision}: precompute {time.time() - t0:.1f} s")
    U = s.to_internal(case.U0)
    torch.cuda.synchronize()
    for _ in range(warmup):
        s.rk_step(U, case.dt)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    s.timing(True)
    e0.record(stream)
    for _ in range(steps):
        s.rk_step(U, case.dt)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_k, n_k = s.timing(False)
    ms = e0.elapsed_time(e1)
    # further windows of >= 100 stages without per-kernel events (their
    # median backs the single timed window above)
    win = []
    for _ in range(windows):
        e0.record(stream)
        for _ in range(window_steps):
            s.rk_step(U, case.dt)
        e1.record(stream)
        torch.cuda.synchronize()
        win.append(e0.elapsed_time(e1) / window_steps)
    diag = s.diagnostics(U)
    out = dict(ms_total=ms, ms_per_step=ms / steps, kernel_ms=ms_k.tolist(), kernel_n=n_k.tolist(),
               stats=s.stats(), finite=bool(diag[-1] == 0), min_rho=float(diag[s.nv]), min_p=float(diag[s.nv + 1]))
    if win:
        out["windows"] = dict(steps_each=window_steps, stages_each=3 * window_steps, ms_per_step=win,
                              median_ms_per_step=float(sorted(win)[len(win) // 2]))
    del U
    torch.cuda.empty_cache()
    return out


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "stage_kernels_tgv288_usr5_hllc_learned.txt")


def measured_traffic(workload):
    """HBM bytes per launch of the stage kernels ({"fp32 k_flux": bytes, ...})
    from the committed rocprofv3 counter summary, or {} when it belongs to
    other sources."""
    if workload != "tgv3d":
        return {}
    from paper_2404_08952_amd import profiling
    got = profiling.read_summary(TRAFFIC_SUMMARY)
    if got is None or got[1] != profiling.source_hash():
        return {}
    return got[0]


def shock_tube_line(args):
    """Sod shock tube with zero-gradient ends through auxiliary cells:
    1024 x 64 x 64 hexes (4.2M cells, 8,192 boundary faces), WENO5 + local
    Lax-Friedrichs, FP32; throughput of the bounded path."""
    import numpy as np
    import torch
    from paper_2404_08952_amd import Solver
    from synth import fields
    from synth import mesh as M
    n = (1024, 64, 64)
    t0 = time.time()
    mesh = M.bounded(M.periodic_3d(*n, lengths=(1.0, 0.0625, 0.0625)), 0)
    xc = (np.arange(n[0]) + 0.5) / n[0]
    left = np.tile(xc < 0.5, n[1] * n[2])
    vel = np.zeros((mesh.n_cells, 3))
    U0 = fields.prim_to_cons(np.where(left, 1.0, 0.125), vel, np.where(left, 1.0, 0.1))
    s = Solver(mesh, pde="euler", scheme="WENO5", flux="rusanov", precision="fp32", u_ref="cell")
    log(f"[bench] shock tube {mesh.n_cells:,} cells: set-up {time.time() - t0:.1f} s")
    U = s.to_internal(U0)
    dt = 0.3 / n[0] / 2.5
    steps = max(1, min(args.steps, 5))
    s.rk_step(U, dt)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    s.timing(True)
    e0.record()
    for _ in range(steps):
        s.rk_step(U, dt)
    e1.record()
    torch.cuda.synchronize()
    ms_k, n_k = s.timing(False)
    ms = e0.elapsed_time(e1) / steps
    d = s.diagnostics(U)
    out = dict(workload=f"3-D Sod tube {n[0]}x{n[1]}x{n[2]} hexes, zero-gradient ends ({s.n_rows - mesh.n_cells:,} "
                        "auxiliary cells), WENO5 + local Lax-Friedrichs, FP32",
               value=mesh.n_cells * 3 / (ms * 1e-3), unit="cell-updates/s", ms_per_step=ms,
               flux_kernel_avg_ms=float(ms_k[3] / max(n_k[3], 1)), finite=bool(d[-1] == 0))
    log(f"[bench] shock tube: {ms:.3f} ms/step, kernels ms {ms_k.tolist()}")
    s.close()
    return out


def tgv_kinetic_energy_line(args):
    """Kinetic-energy history of the Taylor-Green vortex on the 2.0M-cell
    subset mesh (126^3 jittered hexes, same recipe): the FP32 path with the
    learned blend against the FP64 plain path (no blend), beside FP32 plain,
    FP64 learned and FP32 with the classical sensor; 100 SSP-RK3 steps at
    CFL 0.4, sampled every 10 steps."""
    import torch
    from paper_2404_08952_amd import Solver
    from synth import configs
    case = configs.taylor_green_3d(n=126)
    nsteps, every = 100, 10
    hist = {}
    theta = {}
    ref = dict(u_ref="cell")
    for label, prec, extra in (("fp64_plain", "fp64", dict(blend="none")),
                               ("fp32_plain", "fp32", dict(blend="none", **ref)),
                               ("fp64_learned", "fp64", dict(blend="learned")),
                               ("fp32_learned", "fp32", dict(blend="learned", **ref)),
                               ("fp32_classical", "fp32", dict(blend="classical", **ref))):
        s = Solver(case.mesh, **case.params, precision=prec, **extra)
        if extra["blend"] == "learned":
            s.mlp_set(indicator_weights())
        V = s.geometry()["V"][:case.mesh.n_cells]

        def ke(U):
            u = U[:case.mesh.n_cells].double()
            return float(((0.5 * (u[:, 1:4] ** 2).sum(1) / u[:, 0]) * V).sum() / V.sum())
        U = s.to_internal(case.U0)
        h = [ke(U)]
        for _ in range(nsteps // every):
            s.advance(U, case.dt, every)
            h.append(ke(U))
        hist[label] = h
        if extra["blend"] != "none":  # blend weights of the final state
            if extra["blend"] == "learned":
                th = s.mlp_forward(s.features(U, fp32=False)[1])[:case.mesh.n_cells]
            else:
                th = s.classical_theta(U)[:case.mesh.n_cells]
            theta[label] = dict(mean=float(th.mean()), frac_below_0_9=float((th < 0.9).double().mean()))
        s.close()
        del U
        torch.cuda.empty_cache()
    a64 = hist["fp64_plain"]
    out = dict(workload=f"Taylor-Green 126^3 ({case.mesh.n_cells:,} cells), {nsteps} steps, dt {case.dt:.4e}",
               t=[case.dt * every * k for k in range(len(a64))], kinetic_energy=hist, theta_final=theta,
               decay={k: h[0] - h[-1] for k, h in hist.items()},
               max_rel_difference_vs_fp64_plain={k: max(abs(x - y) / y for x, y in zip(h, a64))
                                                  for k, h in hist.items() if k != "fp64_plain"})
    log(f"[bench] TGV 126^3 kinetic energy decay over {nsteps} steps: " +
        ", ".join(f"{k} {v:.3e}" for k, v in out["decay"].items()) +
        "; max relative difference to FP64 plain: " +
        ", ".join(f"{k} {v:.2e}" for k, v in out["max_rel_difference_vs_fp64_plain"].items()) +
        f"; learned theta: {theta}")
    return out


def vortex_line(args):
    """The convected isentropic vortex on 64^3 jittered hexes split into 6
    Kuhn tetrahedra (1,572,864 cells), USR3 DOLINC, Rusanov, SSP-RK3 at CFL
    0.4 for 200 steps (the fourth-order CSR4 template of the recipe is
    linearly unstable on jittered tetrahedra), FP64 and FP32 from the same
    cell averages: throughput and the density error against the closed-form
    vortex (cell averages, one Gauss point per sub-tetrahedron).  The time
    step follows the cells' own geometry (below)."""
    import numpy as np
    import torch
    from paper_2404_08952_amd import Solver
    from synth import configs, fields
    t0 = time.time()
    case = configs.vortex_3d(scheme="USR3", quad_pts=1)
    steps, cfl = 200, 0.4
    # CFL on the cells' own geometry (the lattice rule of the recipe is ten
    # times larger on the jittered Kuhn slivers, where every scheme blows up)
    dt = geometric_dt(case, cfl, "euler")
    exact = fields.cell_averages(case.mesh, case.exact(steps * dt), n_pts=1)
    log(f"[bench] vortex 64^3 x 6 tets: set-up {time.time() - t0:.1f} s")
    out = dict(workload=f"isentropic vortex, {case.mesh.n_cells:,} jittered Kuhn tetrahedra, USR3, Rusanov, "
                        f"{steps} SSP-RK3 steps at CFL {cfl} on the cell geometry, dt {dt:.4e}")
    rho = {}
    for prec, extra in (("fp64", {}), ("fp32", dict(u_ref="cell"))):
        s = Solver(case.mesh, **case.params, precision=prec, part_cells=PART_CELLS[prec], **extra)
        U = s.to_internal(case.U0)
        s.rk_step(U, dt)
        U = s.to_internal(case.U0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s.advance(U, dt, steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        r = s.to_external(U)[:, 0].astype(np.float64)
        rho[prec] = r
        err = float(np.sqrt(np.mean((r - exact[:, 0]) ** 2)))
        out[prec] = dict(ms_per_step=ms, value=case.mesh.n_cells * 3 / (ms * 1e-3), unit="cell-updates/s",
                         rho_l2_error=err)
        log(f"[bench] vortex {prec}: {ms:.3f} ms/step, density L2 error {err:.4e}")
        s.close()
        del U
        torch.cuda.empty_cache()
    out["rho_fp32_vs_fp64_rel_l2"] = float(np.linalg.norm(rho["fp32"] - rho["fp64"]) / np.linalg.norm(rho["fp64"]))
    return out


def advance_logged(s, U, dt, steps, label, chunk=1000):
    """steps SSP-RK3 steps in chunks, a progress line per chunk; returns the
    mean ms per step (HIP events on the current stream around all chunks)."""
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        s.advance(U, dt, k)
        done += k
        if done < steps:
            torch.cuda.synchronize()
            log(f"[bench] {label}: {done} of {steps} steps")
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def shocks_line(args, n=100, paths=("fp32_learned", "fp64_classical"), t_end=0.1):
    """The Sod slab of the shock workload on n^3 jittered hexes, 30 % split
    into tetrahedra and prisms (200^3, the workload's size: 15.2M cells;
    100^3: 1.9M), USR3 + Rusanov with the positivity rule of the cell
    averages to t_end (time step on the cell geometry, CFL 0.2): the FP32
    path with the learned blend and the FP64 classical-sensor run (and, with
    --shocks-only, the FP32 classical-sensor run), each against the exact
    Riemann solution (density L1, position of the right shock), and the
    learned run against the FP64 classical one.  The time step follows the
    thinnest sliver of the mesh: 3,600 steps to t = 0.1 at 100^3, 50,044 at
    200^3 (the thinnest sliver there is 7x thinner), so the full-size line
    runs to an earlier time (--sod-t-end)."""
    import numpy as np
    import torch
    from paper_2404_08952_amd import Solver
    from synth import configs, fields
    t0 = time.time()
    case = configs.shocks_3d(n=n, problem="sod")
    # CFL 0.2 on the cell geometry (the lattice rule blows up on the
    # jittered slivers)
    case.dt, case.steps = geometric_dt(case, 0.2, "euler", t_end=t_end)
    x = fields.cell_points(case.mesh)[:, 0]
    t_end = case.dt * case.steps
    rho_ex = fields.sod_slab_exact(x, t_end)[0]
    rho_post = fields.riemann_exact((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), np.array([1.7]))[0][0]
    # a band after the right contact holding only the right shock (0.86 - 1.0 at t = 0.1)
    band = (x > 0.75 + 1.1 * t_end) & (x < 0.75 + 2.5 * t_end)
    log(f"[bench] shock slab {case.mesh.n_cells:,} cells: set-up {time.time() - t0:.1f} s")
    out = dict(workload=f"Sod slab, {case.mesh.n_cells:,} mixed cells ({n}^3 hexes, 30 % split), USR3, Rusanov, "
                        f"positivity rule, {case.steps} steps to t = {t_end:.3f}")
    rho = {}
    runs = {"fp64_classical": ("fp64", "classical"), "fp32_classical": ("fp32", "classical"),
            "fp32_learned": ("fp32", "learned")}
    for label in paths:
        prec, blend = runs[label]
        s = Solver(case.mesh, **case.params, precision=prec, blend=blend, positivity=True,
                   **(dict(u_ref="cell") if prec == "fp32" else {}))
        if blend == "learned":
            s.mlp_set(indicator_weights())
        U = s.to_internal(case.U0)
        ms = advance_logged(s, U, case.dt, case.steps, f"shock slab {label}")
        d = s.diagnostics(U)
        th = (s.mlp_forward(s.features(U, fp32=False)[1]) if blend == "learned" else s.classical_theta(U))
        frac = float((th[:case.mesh.n_cells] < 0.5).double().mean())
        u = s.to_external(U)
        V = s.geometry()["V"].cpu().numpy()[s.perm]
        s.close()
        r = u[:, 0].astype(np.float64)
        rho[label] = (r, V)
        l1 = float(np.sum(V * np.abs(r - rho_ex)) / V.sum())
        xs = float(np.sum(V[band] * (r[band] - rho_ex[band])) / (rho_post - 0.125) / V.sum())
        out[label] = dict(ms_per_step=ms, value=case.mesh.n_cells * 3 / (ms * 1e-3), unit="cell-updates/s",
                          rho_l1_vs_exact=l1, shock_position_error=xs, frac_theta_below_half=frac,
                          min_rho=float(d[5]), min_p=float(d[6]), nonfinite=int(d[-1]))
        log(f"[bench] shock slab {label}: {ms:.3f} ms/step, rho L1 {l1:.4e}, shock position error {xs:+.2e}, "
            f"theta < 0.5 in {100 * frac:.0f} % of cells")
    r64, V = rho["fp64_classical"]
    out["learned_vs_fp64_classical_l1"] = float(np.sum(V * np.abs(rho["fp32_learned"][0] - r64)) / V.sum())
    return out


def blast_line(args, n=100):
    """The spherical blast of the shock workload (rho 1 at rest, p 10 inside
    r < 0.2 about the centre, 0.1 outside) on n^3 jittered hexes with 30 %
    split (100^3: 1.9M cells), USR3 + Rusanov with the positivity rule of the
    cell averages to t = 0.05 (time step on the cell geometry, CFL 0.2): the
    FP32 path with the learned blend against the FP64 classical-sensor run
    and the FP64 run limited everywhere, each against a fine 1-D radial
    solution (4000 shells; the flow stays spherical inside the unit cube
    until t = 0.05).  Without the positivity rule every path loses
    positivity in a sliver cell near the initial sphere at any time step."""
    import numpy as np
    import torch
    from paper_2404_08952_amd import Solver
    from synth import configs, fields
    t0 = time.time()
    case = configs.shocks_3d(n=n, problem="blast")
    t_end = case.dt * case.steps
    case.dt, case.steps = geometric_dt(case, 0.2, "euler", t_end=t_end)
    t_end = case.dt * case.steps
    r = np.linalg.norm(fields.cell_points(case.mesh) - 0.5, axis=1)
    rho_ref = fields.blast_reference(t_end, n=4000)(r)[0]
    log(f"[bench] blast {case.mesh.n_cells:,} cells: set-up and radial reference {time.time() - t0:.1f} s")
    out = dict(workload=f"spherical blast, {case.mesh.n_cells:,} mixed cells ({n}^3 hexes, 30 % split), USR3, "
                        f"Rusanov, positivity rule, {case.steps} steps to t = {t_end:.3f}; reference: 1-D radial "
                        "Euler, 4000 shells")
    rho = {}
    for label, prec, blend in (("fp64_limited", "fp64", "theta"), ("fp64_classical", "fp64", "classical"),
                               ("fp32_learned", "fp32", "learned")):
        s = Solver(case.mesh, **case.params, precision=prec, blend=blend, positivity=True,
                   **(dict(u_ref="cell") if prec == "fp32" else {}))
        if blend == "learned":
            s.mlp_set(indicator_weights())
        if blend == "theta":
            s.set_theta(torch.zeros(case.mesh.n_cells, dtype=torch.float32, device=s.device))
        U = s.to_internal(case.U0)
        ms = advance_logged(s, U, case.dt, case.steps, f"blast {label}")
        d = s.diagnostics(U)
        frac = 1.0
        if blend != "theta":
            th = (s.mlp_forward(s.features(U, fp32=False)[1]) if blend == "learned" else s.classical_theta(U))
            frac = float((th[:case.mesh.n_cells] < 0.5).double().mean())
        u = s.to_external(U)
        V = s.geometry()["V"].cpu().numpy()[s.perm]
        s.close()
        rr = u[:, 0].astype(np.float64)
        rho[label] = (rr, V)
        l1 = float(np.sum(V * np.abs(rr - rho_ref)) / V.sum())
        out[label] = dict(ms_per_step=ms, rho_l1_vs_radial=l1, frac_theta_below_half=frac,
                          min_rho=float(d[5]), min_p=float(d[6]), nonfinite=int(d[-1]))
        log(f"[bench] blast {label}: {ms:.3f} ms/step, rho L1 {l1:.4e}, theta < 0.5 in {100 * frac:.0f} % of cells")
    r64, V = rho["fp64_classical"]
    out["learned_vs_fp64_classical_l1"] = float(np.sum(V * np.abs(rho["fp32_learned"][0] - r64)) / V.sum())
    return out


def ordering_line(args):
    """Cell-ordering ablation on the Taylor-Green workload at 160^3 (4.1M
    jittered hexes, the input order a seeded shuffle): FP32 USR5 + HLLC +
    learned-blend SSP-RK3 steps with the library's Hilbert renumbering, with
    reverse Cuthill-McKee, and with the input order kept; face entries per
    face (seam duplicates) and ms per step."""
    import torch
    from paper_2404_08952_amd import Solver
    from synth import configs
    t0 = time.time()
    case = configs.taylor_green_3d(n=160)
    nc, nf = case.mesh.n_cells, case.mesh.n_faces
    log(f"[bench] ordering ablation {nc:,} cells: set-up {time.time() - t0:.1f} s")
    out = dict(workload=f"Taylor-Green 160^3 ({nc:,} jittered hexes, input order shuffled), USR5, HLLC, learned "
                        "blend, FP32, SSP-RK3")
    for label, ren in (("hilbert", 2), ("rcm", 1), ("input_order", 0)):
        t1 = time.time()
        s = Solver(case.mesh, **case.params, precision="fp32", blend="learned", u_ref="cell", renumber=ren)
        setup = time.time() - t1
        s.mlp_set(indicator_weights())
        U = s.to_internal(case.U0)
        s.rk_step(U, case.dt)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        steps = 3
        e0.record()
        for _ in range(steps):
            s.rk_step(U, case.dt)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        st = s.stats()
        s.close()
        out[label] = dict(ms_per_step=ms, value=nc * 3 / (ms * 1e-3), unit="cell-updates/s",
                          entries_per_face=st["n_entries"] / nf, partitions=st["n_parts"],
                          max_partition_entries=st["max_entries"], create_s=setup)
        log(f"[bench] ordering {label}: {ms:.3f} ms/step, {st['n_entries'] / nf:.3f} entries per face, "
            f"create {setup:.1f} s")
    return out


def geometric_dt(case, cfl, pde, t_end=None):
    """CFL time step on the cells' own geometry, dt = cfl min_c 2 V_c /
    (lambda sum_f |S_f|) (h / dim on a square or cube); with t_end, the
    step count to reach it and the step that lands on it."""
    import math
    import numpy as np
    import torch
    from paper_2404_08952_amd import Solver
    from synth import fields
    g = Solver(case.mesh, **case.params, precision="fp64")
    geo = g.geometry()
    n = case.mesh.n_cells
    area = torch.linalg.norm(geo["S"], dim=1).cpu().numpy()
    two = case.mesh.neighbour >= 0
    ssum = np.bincount(case.mesh.owner, weights=area, minlength=n) + \
        np.bincount(case.mesh.neighbour[two], weights=area[two], minlength=n)
    V = geo["V"].cpu().numpy()[g.perm]
    g.close()
    dt = cfl * float(np.min(2.0 * V / ssum)) / fields.max_wave_speed(pde, case.U0)
    if t_end is None:
        return dt
    steps = int(math.ceil(t_end / dt - 1e-12))
    return t_end / steps, steps


def burgers_sweep_line(args):
    """2-D inviscid Burgers along (1, 1) on the mixed tri / quad / pentagon
    meshes of the recipe (half the quads split, 5 % pentagons, +-0.25 h
    jitter; the same meshes unjittered; regular all-triangle and all-quad
    meshes to 256^2), u0 = 0.5 + 0.25 sin 2 pi (x + y) to t = 0.05 (before the shock),
    USR3 and CSR4 with the Godunov flux at CFL 0.5 on the cell geometry
    (geometric_dt), FP64 and FP32 (each face side about its own cell): error
    against the exact solution's cell averages at 64^2 .. 512^2 and the
    observed orders, and the throughput at 256^2."""
    import numpy as np
    import torch
    from paper_2404_08952_amd import Solver
    from synth import configs, fields
    from synth import mesh as M
    kinds = ("jittered", "unjittered", "triangles", "quads")
    combos = [(k, sch, prec) for k in kinds for sch in ("USR3", "CSR4") for prec in ("fp64", "fp32")]
    res = {c: dict(cells=[], l2_error=[], finite=[], cell_updates_per_s_256=None) for c in combos}
    runs = [(k, n) for k in kinds for n in ((64, 128, 256, 512) if k in kinds[:2] else (64, 128, 256))]
    for kind, n in runs:
        case = configs.burgers_2d(n=n, jitter=0.25 if kind == "jittered" else 0.0)
        if kind in ("triangles", "quads"):  # the same problem on regular meshes of one cell type
            case.mesh = M.periodic_2d(n, n, split=1.0 if kind == "triangles" else 0.0, diagonal="main")
            case.U0 = fields.cell_averages(case.mesh, fields.burgers_diag(0.0), n_pts=4)
        dt, steps = geometric_dt(case, 0.5, "burgers", t_end=0.05)
        case.dt, case.steps = dt, steps
        ex = fields.cell_averages(case.mesh, case.exact(case.steps * case.dt), n_pts=4)[:, 0]
        for _k, scheme, prec in [c for c in combos if c[0] == kind]:
            # FP32 with each face side about its own cell
            s = Solver(case.mesh, **dict(case.params, scheme=scheme), precision=prec,
                       **(dict(u_ref="cell") if prec == "fp32" else {}))
            U = s.to_internal(case.U0)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            s.advance(U, case.dt, case.steps)
            e1.record()
            torch.cuda.synchronize()
            r = res[(kind, scheme, prec)]
            if n == 256:
                r["cell_updates_per_s_256"] = case.mesh.n_cells * 3 * case.steps / (e0.elapsed_time(e1) * 1e-3)
            u = s.to_external(U)[:, 0].astype(np.float64)
            V = s.geometry()["V"].cpu().numpy()[s.perm]
            s.close()
            ok = bool(np.isfinite(u).all())
            r["l2_error"].append(float(np.sqrt(np.sum(V * (u - ex) ** 2) / np.sum(V))) if ok else float("nan"))
            r["cells"].append(case.mesh.n_cells)
            r["finite"].append(ok)
    out = {}
    for (kind, scheme, prec), r in res.items():
        e = np.array(r["l2_error"])
        r["observed_order"] = [float(x) for x in np.log2(e[:-1] / e[1:])]
        key = f"{kind}_{scheme}_{prec}"
        out[key] = r
        log(f"[bench] Burgers 2-D {key}: L2 errors {['%.3e' % x for x in r['l2_error']]}, orders "
            f"{['%.2f' % x for x in r['observed_order']]}")
    return out


MLP_FWD_FLOP = 2 * (24 * 64 + 64 * 64 + 64 * 1)   # multiply-adds of 24 -> 64 -> 64 -> 1, per cell
BF16_PEAK_TFLOPS = 2500.0


def indicator_line(args):
    """The indicator network alone: inference (forward) and training (forward,
    backward, Adam) throughput on 5M synthetic bf16 feature rows, the size of
    the shock workload's training set; achieved FLOP/s against the dense BF16
    matrix-core peak (in the stage the same k_mlp_fwd runs on the solver's
    second stream)."""
    import torch
    from paper_2404_08952_amd import Solver
    from paper_2404_08952_amd import binding as B
    from synth import mesh as M
    n = 5_000_000
    s = Solver(M.periodic_3d(8, 8, 8), pde="euler", scheme="USR3", flux="rusanov", blend="learned")
    s.mlp_set(indicator_weights())
    gen = torch.Generator(device="cuda")
    gen.manual_seed(51)
    X = torch.zeros(n, B.FEATURE_STRIDE, dtype=torch.float32, device="cuda")
    X[:, :B.N_FEATURES] = torch.randn(n, B.N_FEATURES, generator=gen, device="cuda")
    Xb = X.to(torch.bfloat16).view(torch.int16)
    del X
    y = torch.rand(n, generator=gen, device="cuda")
    out = {}
    for kind, call, reps, flop in (("inference", lambda: s.mlp_forward(Xb), 20, MLP_FWD_FLOP),
                                   ("training", lambda: s.mlp_train_step(Xb, y, 1e-4), 10, 3 * MLP_FWD_FLOP)):
        call()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = flop * n / (ms * 1e-3) / 1e12
        out[kind] = dict(rows=n, ms=ms, rows_per_s=n / (ms * 1e-3), tflops=tf, mfma_frac=tf / BF16_PEAK_TFLOPS)
        log(f"[bench] indicator {kind}: {ms:.3f} ms for {n:,} rows, {tf:.1f} TFLOP/s")
    s.close()
    del Xb, y
    torch.cuda.empty_cache()
    return out


def copy_bandwidth():
    import torch
    n = 1 << 29  # 2 GiB of float32 per buffer
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    # y = -x: one read and one write stream with a kernel name of its own,
    # which also calibrates the HBM byte counters (paper_2404_08952_amd.profiling)
    for _ in range(2):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 10
    for _ in range(reps):
        torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbps


def cpu_baseline_leg(budget_s, workload, lattice):
    """The FP64 oracle, single-threaded, on a bounded sample of the workload:
    the same pipeline (for the Taylor-Green workload: features, indicator
    network, blended USR5 + HLLC residual) on the same generator's mesh at a
    smaller lattice -- by default the 126^3 (2.0M-cell) subset mesh of the
    Taylor-Green workload, or the vortex workload's full 64^3 mesh.  Stages
    run until the budget is spent (at these sizes: one stage)."""
    import numpy as np

    from oracle import geometry as OG
    from oracle import indicator as OI
    from oracle import scheme as OS
    from oracle import solver as SV
    from synth import configs
    t_set = time.perf_counter()
    if workload == "tgv3d":
        case = configs.taylor_green_3d(n=lattice)
        params = indicator_weights().astype(np.float64)
    else:
        case = configs.vortex_3d(n=lattice, point_ic=True, scheme="USR3")
        params = None
    geo = OG.geometry(case.mesh)
    U = case.U0
    t_set = time.perf_counter() - t_set

    def stage():
        th = None
        if params is not None:
            X = OI.features(case.mesh, geo, U, OS.gauss_linear(case.mesh, geo, U))
            th, _ = OI.forward(params, X)
        return SV.residual(case.mesh, geo, U, case.params, theta=th)
    n, t0 = 0, time.perf_counter()
    while True:
        stage()
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    lat = case.mesh.info["lattice"][0]
    return dict(value=case.mesh.n_cells * n / dt, unit="cell-updates/s", cores=1, kind="oracle",
                sample=(f"oracle residual stages (FP64 NumPy, same scheme and flux"
                        f"{', indicator features + network + blend' if params is not None else ''}) on the "
                        f"same workload's generator at a {lat}^3 lattice ({case.mesh.n_cells:,} cells), "
                        f"{n} stage(s) in {dt:.1f} s, one thread, run beside the GPU legs "
                        f"(mesh and geometry set-up {t_set:.0f} s, untimed)"),
                cpu=_cpu_model(), host_cpus=os.cpu_count(), stages=n, seconds=dt, lattice=lat)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def start_cpu_baseline(budget_s, workload, lattice):
    """The oracle leg in a child process of its own (one thread), started
    before the GPU legs so that its minutes overlap theirs."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               NUMEXPR_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--cpu-budget", str(budget_s),
           "--workload", workload, "--cpu-lattice", str(lattice)]
    proc = subprocess.Popen(cmd, env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
    # if a GPU leg fails, the child does not outlive the benchmark
    atexit.register(lambda: proc.poll() is None and proc.kill())
    return proc


def finish_cpu_baseline(proc, timeout_s=900):
    try:
        out, err = proc.communicate(timeout=timeout_s)
    except subprocess.TimeoutExpired:
        proc.kill()
        proc.communicate()
        log("[bench] CPU oracle baseline did not finish in time")
        return None
    if proc.returncode != 0:
        log(err[-2000:])
        return None
    return json.loads(out.strip().splitlines()[-1])


def cpu_lattice(args):
    return args.cpu_lattice or (126 if args.workload == "tgv3d" else 64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tgv3d", choices=["vortex3d", "tgv3d"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--cpu-lattice", type=int, default=0,
                    help="lattice of the oracle sample (default: 126 for the Taylor-Green workload, 64 for the vortex)")
    ap.add_argument("--cpu-baseline-only", action="store_true")
    ap.add_argument("--indicator-only", action="store_true",
                    help="only the indicator network's inference / training throughput (for counter runs)")
    ap.add_argument("--ke-only", action="store_true", help="only the Taylor-Green kinetic-energy comparison")
    ap.add_argument("--vortex-only", action="store_true", help="only the isentropic-vortex line")
    ap.add_argument("--burgers-only", action="store_true", help="only the 2-D Burgers refinement sweep")
    ap.add_argument("--shocks-only", action="store_true", help="only the shock-slab and spherical-blast lines")
    ap.add_argument("--sod-n", type=int, default=100, help="lattice of the Sod-slab line (200: the workload's size)")
    ap.add_argument("--sod-t-end", type=float, default=0.1, help="end time of the Sod-slab line")
    ap.add_argument("--blast-n", type=int, default=100, help="lattice of the spherical-blast line")
    ap.add_argument("--ordering-only", action="store_true", help="only the cell-ordering ablation")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the FP32 / FP64 headline paths (for profiler runs: per-kernel averages of one mesh)")
    args = ap.parse_args()

    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline_leg(args.cpu_budget, args.workload, cpu_lattice(args))))
        return
    if args.gpus != 1:
        raise SystemExit("this benchmark runs on one GPU only (no multi-GPU path is built); use --gpus 1")

    import torch

    from paper_2404_08952_amd import Solver
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.indicator_only:
        print(json.dumps(indicator_line(args)))
        return
    if args.ke_only:
        print(json.dumps(tgv_kinetic_energy_line(args)))
        return
    if args.vortex_only:
        print(json.dumps(vortex_line(args)))
        return
    if args.burgers_only:
        print(json.dumps(burgers_sweep_line(args)))
        return
    if args.ordering_only:
        print(json.dumps(ordering_line(args)))
        return
    if args.shocks_only:
        print(json.dumps(dict(shock_slab=shocks_line(args, n=args.sod_n, t_end=args.sod_t_end,
                                                     paths=("fp32_learned", "fp64_classical", "fp32_classical")),
                              spherical_blast=blast_line(args, n=args.blast_n))))
        return
    cpu_proc = None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline started beside the GPU legs ({cpu_lattice(args)}^3 lattice)")
        cpu_proc = start_cpu_baseline(args.cpu_budget, args.workload, cpu_lattice(args))
    dev = torch.cuda.get_device_name(0)
    t0 = time.time()
    case, desc, extra, fp32_extra = make_case(args.workload)
    log(f"[bench] {args.workload}: mesh + initial data {time.time() - t0:.1f} s")
    nc, nf = case.mesh.n_cells, case.mesh.n_faces
    nv, dim = 5, 3
    scheme = case.params["scheme"]
    blend = extra.get("blend", "none") != "none"
    res = {}
    # the non-oscillatory DOLINC schemes and CSR6 on the same mesh (FP32, no blend)
    nonlin = {}
    scheme_costs = {}
    extras = args.workload == "tgv3d" and not args.headline_only
    for prec in ("fp32", "fp64"):
        t0 = time.time()
        solver = Solver(case.mesh, **case.params, **extra, precision=prec, part_cells=PART_CELLS[prec])
        log(f"[bench] create (renumber, {PART_CELLS[prec]}-cell partitions, upload, FP64 geometry) "
            f"{time.time() - t0:.1f} s")
        ex = dict(extra, **(fp32_extra if prec == "fp32" else {}))
        res[prec] = time_path(solver, case, prec, ex, args.steps, args.warmup,
                              windows=0 if args.headline_only else 5)
        log(f"[bench] {prec}: {res[prec]['ms_per_step']:.3f} ms/step, kernels ms {res[prec]['kernel_ms']}")
        if extras:
            # every scheme on the same mesh without the blend: the cost of the
            # DOLINC schemes relative to CD2, the form of the paper's own speed
            # figures (its CPU-time increases over CD2)
            el_ = 4 if prec == "fp32" else 8
            for sch in SCHEME_COST_SCHEMES:
                r = time_path(solver, case, prec, dict(ex, blend="none"), max(1, min(args.steps, 5)), 1,
                              params=dict(case.params, scheme=sch))
                fb = flux_kernel_bytes(nc, nf, nv, dim, el_, sch)[0]
                fl = r["kernel_ms"][3] / max(r["kernel_n"][3], 1)
                row = dict(ms_per_step=r["ms_per_step"], value=nc * 3 / (r["ms_per_step"] * 1e-3),
                           flux_kernel_avg_ms=fl, flux_kernel_gbps=fb / (fl * 1e-3) / 1e9,
                           finite=r["finite"], min_rho=r["min_rho"], min_p=r["min_p"])
                scheme_costs.setdefault(prec, {})[sch] = row
                if prec == "fp32" and sch in ("WENO5", "ENO3", "CSR6"):
                    nonlin[sch] = row
                log(f"[bench] {prec} {sch} (no blend): {r['ms_per_step']:.3f} ms/step, kernels ms {r['kernel_ms']}")
            base = scheme_costs[prec]["CD2"]["ms_per_step"]
            for sch, row in scheme_costs[prec].items():
                row["time_vs_cd2"] = row["ms_per_step"] / base
        solver.close()
        del solver
    tube = shock_tube_line(args) if extras else None
    mlp = indicator_line(args) if extras else None
    ke = tgv_kinetic_energy_line(args) if extras else None
    vtx = vortex_line(args) if extras else None
    brg = burgers_sweep_line(args) if extras else None
    shk = shocks_line(args, n=args.sod_n, t_end=args.sod_t_end) if extras else None
    blast = blast_line(args, n=args.blast_n) if extras else None
    order = ordering_line(args) if extras else None
    gbps_copy = copy_bandwidth()
    log(f"[bench] streaming y = -x: {gbps_copy:.0f} GB/s")

    traffic = measured_traffic(args.workload)

    def summarize(prec):
        r = res[prec]
        el = 4 if prec == "fp32" else 8
        stages = 3 * args.steps
        cups = nc * stages / (r["ms_total"] * 1e-3)
        nrec = r["stats"]["n_slots"]
        fb, fpc, fpf = flux_kernel_bytes(nc, nf, nv, dim, el, scheme, blend)
        per = lambda k: r["kernel_ms"][k] / max(r["kernel_n"][k], 1)  # noqa: E731
        # kinds of the per-kernel events: 0 first gradient, 1 second
        # derivatives (d.H.d per face record), 2 sensor, or with the learned
        # blend the first gradient fused with the features, 3 flux + update
        kern = {}

        def add(name, kind, alg):
            if not r["kernel_n"][kind]:
                return
            ms = per(kind)
            gbps = alg / (ms * 1e-3) / 1e9
            t = traffic.get(f"{prec} {name}")
            kern[name] = dict(avg_ms=ms, alg_bytes=alg, gbps=gbps, frac=gbps / HBM_PEAK_GBPS,
                              traffic_bytes=t, traffic_over_alg=(t / alg if t else None),
                              # measured (counter) traffic over the live duration: the
                              # achieved HBM rate of the kernel, as a fraction of peak
                              traffic_gbps=(t / (ms * 1e-3) / 1e9 if t else None),
                              traffic_frac=(t / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS if t else None))
        add("k_flux", 3, fb)
        if blend:
            add("k_grad_features", 2, grad_features_bytes(nc, nrec, nv, dim, el))
        else:
            add("k_grad", 0, grad_bytes(nc, nrec, nv, dim, el))
        add("k_hface", 1, hface_bytes(nc, nrec, nv, dim, el))
        comp = COMPULSORY_BYTES[prec] * cups / 1e9
        return dict(value=cups, ms_per_step=r["ms_per_step"], ms_per_stage=r["ms_per_step"] / 3,
                    flux_kernel=dict(avg_ms=per(3), alg_bytes=fb, gbps=fb / (per(3) * 1e-3) / 1e9,
                                     bytes_per_cell=fpc, bytes_per_face=fpf),
                    stage_kernels=kern,
                    stage_effective=dict(compulsory_bytes_per_cell=COMPULSORY_BYTES[prec], gbps=comp,
                                         frac=comp / HBM_PEAK_GBPS,
                                         alg_bytes_per_stage=sum(k["alg_bytes"] for k in kern.values())),
                    stage_kernel_ms=sum(per(k) for k in range(4) if r["kernel_n"][k]),
                    finite=r["finite"], min_rho=r["min_rho"], min_p=r["min_p"], partitions=r["stats"],
                    windows=r.get("windows"))

    s32, s64 = summarize("fp32"), summarize("fp64")
    for prec, sm in (("fp32", s32), ("fp64", s64)):
        for name, k in sm["stage_kernels"].items():
            log(f"[bench] {prec} {name}: {k['avg_ms']:.3f} ms, {k['alg_bytes'] / 1e9:.3f} GB algorithmic, "
                f"{k['gbps']:.0f} GB/s = {k['frac']:.3f} of peak"
                + (f", counter traffic {k['traffic_bytes'] / 1e9:.3f} GB = {k['traffic_over_alg']:.2f} x algorithmic"
                   f" = {k['traffic_gbps']:.0f} GB/s = {k['traffic_frac']:.3f} of peak"
                   if k["traffic_bytes"] else ""))
        se = sm["stage_effective"]
        log(f"[bench] {prec} stage: {sm['ms_per_stage']:.3f} ms, compulsory {se['compulsory_bytes_per_cell']} B/cell "
            f"x {sm['value']:.3e} cell-updates/s = {se['gbps']:.0f} GB/s = {se['frac']:.3f} of peak")
    log("[bench] algorithmic bytes per launch: " +
        " ".join(f'"{p} {n}={k["alg_bytes"]:.6e}"' for p, sm in (("fp32", s32), ("fp64", s64))
                 for n, k in sm["stage_kernels"].items()))
    fk = s32["flux_kernel"]
    out = {
        "metric": METRIC,
        "value": s32["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": s32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "cells": nc, "faces": nf, "stages_per_step": 3,
                   "precision": ("FP32 bulk, each face side carried about its own cell (flux shares "
                                 "F.S - F(U_c).S); geometry and face weights precomputed in FP64 and stored in FP32, "
                                 "the DOLINC coefficients evaluated from the weights in FP64 in the flux kernel"),
                   "partition_cells": PART_CELLS["fp32"]},
        "roofline": {"bound": "hbm", "achieved": fk["gbps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": fk["gbps"] / HBM_PEAK_GBPS, "traffic": traffic.get("fp32 k_flux"),
                     "kernel": "k_flux (reconstruction + blend + Riemann flux + segmented accumulation + RK update)",
                     "alg_bytes_per_launch": fk["alg_bytes"], "avg_launch_ms": fk["avg_ms"]},
        "fp64": {"value": s64["value"], "ms_per_step": s64["ms_per_step"], "dtype": "f64",
                 "flux_kernel_gbps": s64["flux_kernel"]["gbps"],
                 "flux_kernel_frac": s64["flux_kernel"]["gbps"] / HBM_PEAK_GBPS},
        "stage_kernels_fp32": s32["stage_kernels"],
        "stage_kernels_fp64": s64["stage_kernels"],
        "stage_effective_bandwidth": {"fp32": s32["stage_effective"], "fp64": s64["stage_effective"]},
        "fp32_detail": s32,
        "fp64_detail": s64,
        "fp32_over_fp64": s32["value"] / s64["value"],
        "other_schemes_fp32": {k: dict(v, unit="cell-updates/s", scheme=k, flux="hllc", blend="none")
                               for k, v in nonlin.items()},
        "scheme_costs": dict(scheme_costs, note=SCHEME_COST_NOTE) if scheme_costs else None,
        "bounded_fp32": tube,
        "indicator_network": mlp,
        "tgv_kinetic_energy": ke,
        "vortex_closed_form": vtx,
        "burgers_2d_sweep": brg,
        "shock_slab": shk,
        "spherical_blast": blast,
        "cell_ordering": order,
        "device": dev,
        "copy_gbps": gbps_copy,
    }
    if cpu_proc is not None:
        log("[bench] waiting for the CPU oracle baseline ...")
        out["cpu_baseline"] = finish_cpu_baseline(cpu_proc)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
