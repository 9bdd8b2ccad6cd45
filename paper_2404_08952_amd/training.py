"""Label generation and GPU training of the learned blending indicator.

Labels come from the method itself: a classical smoothness indicator
evaluated on a fine-mesh solution of the method.  For each 3-D problem
(Sod and Lax slabs in the three axis directions and the spherical blast on
the shock workload's mesh recipe, the Taylor-Green vortex at Mach 0.1 and
0.3, smooth density waves) a coarse run on the jittered workload mesh and a
fine run on an unjittered hexahedral lattice twice as fine advance side by
side (classical-sensor blend and the positivity rule of the cell averages,
FP64).  At snapshots, every coarse cell gets the label

    theta* = min over the 4 x 4 x 4 fine cells around its centre of the
             classical sensor's theta on the fine solution (the sensor's
             beta weighted by the size of the jump, see
             _fine_theta_block),

so a coarse cell is marked for limiting when a discontinuity lies within
its stencil in the resolved flow, and smooth otherwise, whatever the
coarse mesh's jitter does to its own difference quotients; its features are
those of the coarse state.  Cells labelled smooth are subsampled to balance
the set.  (The first, 1-D generator, least-squares blend weights against a
4x finer classical-sensor run on unjittered slabs, is kept for the quick
training of the gain test.)  Features come from the library's feature
kernel; training runs the library's bf16 matrix-core forward/backward and
Adam kernels.  Everything runs through the C ABI.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import binding

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "data", "indicator_weights.npy")


def _synth():
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth  # seeded input generators (meshes, initial data)
    return synth


def _slab(synth, n, axis, L=1.0):
    dims = [2, 2, 2]
    dims[axis] = n
    lengths = [0.1, 0.1, 0.1]
    lengths[axis] = L
    return synth.periodic_3d(dims[0], dims[1], dims[2], lengths=tuple(lengths))


def _shock_tube(synth, left, right, axis):
    def f(x):
        s = x[:, axis]
        inside = np.abs(s - 0.5) < 0.25
        rho = np.where(inside, left[0], right[0])
        u = np.where(inside, left[1], right[1])
        p = np.where(inside, left[2], right[2])
        vel = np.zeros((x.shape[0], 3))
        vel[:, axis] = np.where(s < 0.5, -u, u) if left[1] != 0.0 else u
        return synth.fields.prim_to_cons(rho, vel, p)
    return f


def _wave(synth, amp, k, axis):
    def f(x):
        s = x[:, axis]
        rho = 1.0 + amp * np.sin(2 * np.pi * k * s)
        vel = np.zeros((x.shape[0], 3))
        vel[:, axis] = 1.0
        return synth.fields.prim_to_cons(rho, vel, np.ones_like(s))
    return f


def _labels(sol_hi, sol_lim, U, Uref_faces, owner, neigh, n_cells, scale):
    """theta* per cell from exported face states (caller face order)."""
    UHL, UHR, _ = sol_hi.face_states(U)
    ULL, ULR, _ = sol_lim.face_states(U)
    UHL, UHR = UHL.cpu().numpy(), UHR.cpu().numpy()
    ULL, ULR = ULL.cpu().numpy(), ULR.cpu().numpy()
    num = np.zeros(n_cells)
    den = np.zeros(n_cells)
    for (H, Lm, cells) in ((UHL, ULL, owner), (UHR, ULR, neigh)):
        a = (H - Lm) / scale
        b = (Uref_faces - Lm) / scale
        np.add.at(num, cells, np.sum(a * b, 1))
        np.add.at(den, cells, np.sum(a * a, 1))
    tiny = 1e-12
    return np.where(den > tiny, np.clip(num / np.maximum(den, tiny), 0.0, 1.0), 1.0)


def _face_positions(mesh):
    cnt = np.diff(mesh.face_ptr)
    pos = np.zeros((mesh.n_faces, 3))
    idx = np.repeat(np.arange(mesh.n_faces), cnt)
    for a in range(3):
        pos[:, a] = np.bincount(idx, weights=mesh.nodes[mesh.face_nodes, a], minlength=mesh.n_faces) / cnt
    return pos


def slab_samples(n, axis, ic, t_end, snaps, cfl=0.4, refine=4, scheme="USR3"):
    """Samples (Xbf16 rows, labels) from one 1-D problem at resolution n."""
    synth = _synth()
    coarse = _slab(synth, n, axis)
    fine = _slab(synth, refine * n, axis)
    kw = dict(pde="euler", scheme=scheme, flux="rusanov", gamma=1.4)
    run_c = binding.Solver(coarse, blend="classical", **kw)
    run_f = binding.Solver(fine, blend="classical", **kw)
    hi = binding.Solver(coarse, blend="none", **kw)
    lim = binding.Solver(coarse, blend="theta", **kw)
    import torch
    lim.set_theta(torch.zeros(coarse.n_cells, dtype=torch.float32, device=lim.device))
    pts_c = synth.fields.cell_points(coarse)
    pts_f = synth.fields.cell_points(fine)
    Uc = run_c.to_internal(ic(pts_c))
    Uf = run_f.to_internal(ic(pts_f))
    lam = 2.0 * synth.fields.max_wave_speed("euler", ic(pts_c))  # waves speed up behind shocks
    dt = cfl * (1.0 / n) / (3 * lam)
    steps = int(np.ceil(t_end / dt))
    dt = t_end / steps
    snap_at = set(np.linspace(0, steps, snaps + 1).astype(int)[1:].tolist())
    # fine x-faces that coincide with coarse faces along the slab axis
    fpos_c = _face_positions(coarse)[:, axis]
    xf_f = pts_f[:, axis]
    order_f = np.argsort(xf_f, kind="stable")
    col_f = np.empty(fine.n_cells, dtype=np.int64)
    col_f[order_f] = np.arange(fine.n_cells) // 4
    normal = np.abs(run_c.geometry()["S"].cpu().numpy()[:, axis]) > 0
    Xs, ys = [], []
    for k in range(1, steps + 1):
        run_c.rk_step(Uc, dt)
        for _ in range(refine):
            run_f.rk_step(Uf, dt / refine)
        if k not in snap_at:
            continue
        Uf_h = run_f.to_external(Uf)
        colmean = np.zeros((refine * n, 5))
        for v in range(5):
            colmean[:, v] = np.bincount(col_f, weights=Uf_h[:, v], minlength=refine * n) / 4.0
        # reference state at each coarse face: mean of the two fine columns
        # on either side of it (faces normal to the slab axis), else the
        # mean of the fine columns inside the coarse column
        ref = np.zeros((coarse.n_faces, 5))
        j = np.rint(fpos_c * refine * n).astype(np.int64) % (refine * n)
        ref[normal] = 0.5 * (colmean[j[normal] - 1] + colmean[j[normal]])
        own_x = pts_c[coarse.owner[~normal], axis]
        jc = np.floor(own_x * n).astype(np.int64) % n
        ref[~normal] = colmean.reshape(n, refine, 5).mean(1)[jc]
        scale = np.maximum(np.abs(Uf_h).max(0), 1e-3)
        Ucur = run_c.to_external(Uc)
        Ui = hi.to_internal(Ucur)
        y = _labels(hi, lim, Ui, ref, coarse.owner, coarse.neighbour, coarse.n_cells, scale)
        _X32, Xb = hi.features(Ui, fp32=False)
        Xb = Xb.cpu().numpy()[hi.perm]
        # the four cells of a slab column are copies: keep one per column
        keep = np.unique(np.floor(pts_c[:, axis] * n).astype(np.int64) % n, return_index=True)[1]
        Xs.append(Xb[keep])
        ys.append(y[keep])
    for s in (run_c, run_f, hi, lim):
        s.close()
    return np.concatenate(Xs), np.concatenate(ys)


def vortex_samples(n=24, jitter=0.2, seed=21):
    """Smooth 3-D vortex cells labelled against the closed-form face values."""
    synth = _synth()
    case = synth.configs.vortex_3d(n=n, jitter=jitter, seed=seed, point_ic=True, scheme="USR3")
    mesh = case.mesh
    kw = dict(pde="euler", scheme="USR3", flux="rusanov", gamma=1.4)
    hi = binding.Solver(mesh, blend="none", **kw)
    lim = binding.Solver(mesh, blend="theta", **kw)
    import torch
    lim.set_theta(torch.zeros(mesh.n_cells, dtype=torch.float32, device=lim.device))
    Ui = hi.to_internal(case.U0)
    ref = case.exact(0.0)(hi.geometry()["xf"].cpu().numpy())
    scale = np.maximum(np.abs(case.U0).max(0), 1e-3)
    y = _labels(hi, lim, Ui, ref, mesh.owner, mesh.neighbour, mesh.n_cells, scale)
    _X32, Xb = hi.features(Ui, fp32=False)
    X = Xb.cpu().numpy()[hi.perm]
    hi.close()
    lim.close()
    return X, y


def build_dataset(seed=34, quick=False):
    sod = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    lax = ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571))
    synth = _synth()
    rng = np.random.default_rng(seed)
    Xs, ys = [], []
    res = (64, 128) if quick else (64, 128, 256)
    for n in res:
        for axis in range(3):
            for (L, R), t in ((sod, 0.1), (lax, 0.08)):
                X, y = slab_samples(n, axis, _shock_tube(synth, L, R, axis), t, 6 if quick else 12)
                Xs.append(X); ys.append(y)
            for _ in range(1 if quick else 2):
                amp = float(rng.uniform(0.05, 0.4))
                k = int(rng.integers(1, 4))
                X, y = slab_samples(n, axis, _wave(synth, amp, k, axis), 0.2, 4 if quick else 8)
                Xs.append(X); ys.append(y)
    X, y = vortex_samples(n=16 if quick else 24)
    Xs.append(X); ys.append(y)
    return np.concatenate(Xs), np.concatenate(ys).astype(np.float32)


# ---------------------------------------------------------------- 3-D labels
JUMP_TOL = 0.05  # relative jump of rho or p between lattice neighbours that counts as a discontinuity


def _fine_theta_block(Uf, xf_cells, nfine, gamma=1.4, tol=JUMP_TOL, reach=1):
    """Smoothness label on the fine lattice [nz, ny, nx] and its 4 x 4 x 4
    running minimum (periodic), indexed by the fine lattice cell.

    The classical sensor on a uniform lattice, beta = |2 q_i - q_(i-1) -
    q_(i+1)| / (|q_i - q_(i-1)| + |q_(i+1) - q_i|) per axis, for q = rho and
    p, is weighted by the size of the larger of the two jumps relative to
    JUMP_TOL |q_i| (capped at 1): a ratio of differences alone also reads
    the extrema of smooth fields and grid-scale ripples of tiny amplitude
    (the acoustic noise of a low-Mach flow) as discontinuities.
    theta = clip((0.9 - max beta_w) / 0.3, 0, 1)."""
    idx = np.floor(xf_cells * nfine).astype(np.int64) % nfine
    rho = Uf[:, 0]
    p = (gamma - 1.0) * (Uf[:, 4] - 0.5 * np.sum(Uf[:, 1:4] ** 2, 1) / rho)
    bmax = np.zeros((nfine, nfine, nfine))
    for q in (rho, p):
        g = np.empty((nfine, nfine, nfine))
        g[idx[:, 2], idx[:, 1], idx[:, 0]] = q
        for ax in range(3):
            a, c = np.roll(g, 1, axis=2 - ax), np.roll(g, -1, axis=2 - ax)
            dl, dr = np.abs(g - a), np.abs(c - g)
            beta = np.abs(2.0 * g - a - c) / (dl + dr + 1e-12 * np.abs(g) + 1e-300)
            w = np.minimum(1.0, np.maximum(dl, dr) / (tol * np.abs(g) + 1e-300))
            bmax = np.maximum(bmax, beta * w)
    out = np.clip((0.9 - bmax) / 0.3, 0.0, 1.0)
    for ax in range(3):
        m = out.copy()
        for sh in range(-reach, reach + 2):
            m = np.minimum(m, np.roll(out, -sh, axis=ax))
        out = m
    return out  # out[i] = min over i-reach .. i+reach+1 in every axis


def field_samples(problem, n, snaps, seed, refine=2, cfl=0.2, keep_smooth=0.25, rng=None, tol=JUMP_TOL, reach=1):
    """(X bf16 rows, labels) from one 3-D problem: coarse cells of the
    jittered workload mesh labelled by the classical sensor on the fine
    unjittered solution (see the module docstring)."""
    import torch
    synth = _synth()
    rng = rng or np.random.default_rng(seed)
    fields = synth.fields
    L = 1.0
    if problem.startswith("tgv"):
        mach = 0.1 if problem == "tgv_m01" else 0.3
        L = 2 * np.pi
        coarse = synth.periodic_3d(n, lengths=(L, L, L), jitter=0.2, seed=seed)
        fine = synth.periodic_3d(refine * n, lengths=(L, L, L))
        ic = fields.taylor_green(mach)
        t_end = 1.0
    else:
        coarse = synth.periodic_3d(n, jitter=0.2, seed=seed,
                                   kinds=synth.mesh.mixed_kinds(n, split_frac=0.3, seed=seed + 1))
        fine = synth.periodic_3d(refine * n)
        if problem.startswith("sod") or problem.startswith("lax"):
            axis = "xyz".index(problem[-1])
            sod = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
            lax = ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571))
            left, right = sod if problem.startswith("sod") else lax
            ic = _shock_tube(synth, left, right, axis)
            t_end = 0.1 if problem.startswith("sod") else 0.08
        elif problem == "blast":
            ic = fields.blast()
            t_end = 0.05
        elif problem.startswith("wave"):
            axis = "xyz".index(problem[-1])
            amp = float(rng.uniform(0.05, 0.4))
            k = int(rng.integers(1, 4))
            ic = _wave(synth, amp, k, axis)
            t_end = 0.2
        else:
            raise ValueError(problem)
    kw = dict(pde="euler", scheme="USR3", flux="rusanov", gamma=1.4, positivity=True)
    run_c = binding.Solver(coarse, blend="classical", **kw)
    run_f = binding.Solver(fine, blend="classical", **kw)
    hi = binding.Solver(coarse, blend="none", pde="euler", scheme="USR3", flux="rusanov", gamma=1.4)
    pts_c = fields.cell_points(coarse)
    pts_f = fields.cell_points(fine)
    U0c, U0f = ic(pts_c), ic(pts_f)
    Uc = run_c.to_internal(U0c)
    Uf = run_f.to_internal(U0f)
    lam = 2.0 * fields.max_wave_speed("euler", U0c)  # waves speed up behind shocks

    def dt_of(solver, mesh):
        geo = solver.geometry()
        area = torch.linalg.norm(geo["S"], dim=1).cpu().numpy()
        ssum = np.bincount(mesh.owner, weights=area, minlength=mesh.n_cells) + \
            np.bincount(mesh.neighbour, weights=area, minlength=mesh.n_cells)
        V = geo["V"].cpu().numpy()[solver.perm]
        return cfl * float(np.min(2.0 * V / ssum)) / lam
    dt_c, dt_f = dt_of(run_c, coarse), dt_of(run_f, fine)
    xc_frac = np.mod(pts_c / L, 1.0)
    xf_frac = np.mod(pts_f / L, 1.0)
    nfine = refine * n
    ci = np.floor(xc_frac * nfine).astype(np.int64) % nfine
    Xs, ys = [], []
    t = 0.0
    for k in range(1, snaps + 1):
        t_next = t_end * k / snaps
        for solver, U, dt0 in ((run_c, Uc, dt_c), (run_f, Uf, dt_f)):
            m = int(np.ceil((t_next - t) / dt0 - 1e-12))
            solver.advance(U, (t_next - t) / m, m)
        t = t_next
        blk = _fine_theta_block(run_f.to_external(Uf), xf_frac, nfine, tol=tol, reach=reach)
        y = blk[ci[:, 2], ci[:, 1], ci[:, 0]]
        Ucur = run_c.to_external(Uc)
        Ui = hi.to_internal(Ucur)
        _X32, Xb = hi.features(Ui, fp32=False)
        X = Xb.cpu().numpy()[hi.perm]
        smooth = y >= 0.99
        keep = ~smooth | (rng.random(y.size) < keep_smooth)
        Xs.append(X[keep])
        ys.append(y[keep])
    for sv in (run_c, run_f, hi):
        sv.close()
    return np.concatenate(Xs), np.concatenate(ys)


PROBLEMS_3D = ("sod_x", "sod_y", "sod_z", "lax_x", "lax_y", "lax_z", "blast", "tgv_m01", "tgv_m03",
               "wave_x", "wave_y", "wave_z")


def build_dataset_3d(n=48, snaps=10, seed=34, problems=PROBLEMS_3D, log=None, tol=JUMP_TOL, reach=1):
    """The 3-D labelled set: every problem of PROBLEMS_3D at coarse lattice n."""
    rng = np.random.default_rng(seed)
    Xs, ys = [], []
    for i, prob in enumerate(problems):
        t0 = time.time()
        X, y = field_samples(prob, n, snaps, seed + 10 * i, rng=rng, tol=tol, reach=reach)
        Xs.append(X)
        ys.append(y)
        if log:
            log(f"[train] {prob}: {X.shape[0]:,} samples, label mean {y.mean():.3f}, "
                f"{np.mean(y < 0.5):.3f} below 1/2, {time.time() - t0:.1f} s")
    return np.concatenate(Xs), np.concatenate(ys).astype(np.float32)


def train(X, y, steps=3000, batch=4096, lr=1e-3, seed=34, holder=None):
    """Train the network on (X bf16 rows [n][32] uint16, y) with the GPU kernels."""
    import torch
    synth = _synth()
    own = holder is None
    if own:
        holder = binding.Solver(synth.periodic_3d(2), pde="euler", scheme="USR3", flux="rusanov",
                                blend="learned")
    rng = np.random.default_rng(seed)
    p0 = xavier(seed)
    holder.mlp_set(p0)
    Xd = torch.from_numpy(np.ascontiguousarray(X).view(np.int16)).to(holder.device)
    yd = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(holder.device)
    n = X.shape[0]
    losses = []
    for k in range(steps):
        idx = torch.from_numpy(rng.integers(0, n, size=min(batch, n))).to(holder.device)
        loss = holder.mlp_train_step(Xd[idx].contiguous(), yd[idx].contiguous(), lr)
        if k % 100 == 0 or k == steps - 1:
            losses.append((k, float(loss.item())))
    params = holder.mlp_get()
    if own:
        holder.close()
    return params, losses


def xavier(seed):
    """Seeded Xavier-uniform weights and zero biases, packed."""
    rng = np.random.default_rng(seed)

    def u(fo, fi):
        a = np.sqrt(6.0 / (fi + fo))
        return rng.uniform(-a, a, size=(fo, fi))
    return np.concatenate([u(64, 24).ravel(), np.zeros(64), u(64, 64).ravel(), np.zeros(64), u(1, 64)[0],
                           [0.0]]).astype(np.float32)


def main(quick=False, out=WEIGHTS, n=48, snaps=10, steps=20000, batch=16384):
    t0 = time.time()
    if quick:
        X, y = build_dataset(quick=True)
    else:
        X, y = build_dataset_3d(n=n, snaps=snaps, log=lambda m: print(m, flush=True))
    t1 = time.time()
    params, losses = train(X, y, steps=1500 if quick else steps, batch=4096 if quick else batch)
    t2 = time.time()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    np.save(out, params)
    info = dict(samples=int(X.shape[0]), label_mean=float(y.mean()), label_lt_half=float(np.mean(y < 0.5)),
                data_s=t1 - t0, train_s=t2 - t1, losses=losses)
    with open(os.path.splitext(out)[0] + ".json", "w") as f:
        json.dump(info, f, indent=1)
    print(json.dumps(info))
    return params


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--n", type=int, default=48)
    ap.add_argument("--snaps", type=int, default=10)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=16384)
    a = ap.parse_args()
    main(quick=a.quick, out=a.out, n=a.n, snaps=a.snaps, steps=a.steps, batch=a.batch)
