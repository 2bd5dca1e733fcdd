"""Evaluation runs of the two extensions on the GPU (synthetic workloads).

  python -m paper_2607_06045_amd.evaluate mixed [--steps 200]
      shear layer on the 59,392-leaf band mesh (N = 3) with dynamic AMR from
      the modal indicator every 5 steps: the FP64 run chooses the refine /
      coarsen flags, the mixed-precision run replays them, so both share every
      mesh; reports per-variable relative L1 and max errors of the mixed state
      against the FP64 state, bound violations, mass change and wall times

  python -m paper_2607_06045_amd.evaluate learned [--steps 100]
      trains the indicator network on the GPU from (features, modal indicator)
      pairs of seeded blasts and shear layers, then runs the 22,156-leaf blast
      with dynamic AMR every 5 steps twice, with the modal indicator and with
      the network; reports the refine / keep / coarsen agreement of the two
      indicators on the learned run's states, the element counts over time,
      the L1 density difference of the two runs (base-cell means) and wall times

  python -m paper_2607_06045_amd.evaluate scale [--steps 500]
      four-quadrant states on the 246,736-leaf mesh (N = 4) with dynamic AMR
      every 5 steps: the plain FP64 method with the modal indicator against
      the mixed-precision method with the learned indicator; reports
      throughput (with and without the adaptation time), element counts,
      sampled bound violations and the L1 density difference of the two runs

  python -m paper_2607_06045_amd.evaluate cfl [--t-end 3.0] [--n 128] [--amr]
      the Sedov blast of Sec. 3.4 ([-2, 2]^2, rho = 1, p0 = 1e-5, e = 1 in
      r0 = 0.21875, N = 3) on a uniform n x n mesh (the finest level of the
      paper's adaptive mesh) to t-end, twice: local bounds from bar states
      with the IDP time step at CFL 0.95, and local bounds from the low-order
      solution with the low-order time step at CFL 0.4; reports the number of
      steps, wall time, the smallest and largest dt, mean limiting factors and
      bound violations of each run; with --amr a 16 x 16 root grid adapts
      every 5 steps between 16 and n elements per direction, as in the paper

  python -m paper_2607_06045_amd.evaluate dmr [--level 4] [--t-end 0.2] [--amr]
      the double Mach reflection of Sec. 3.5 on [0, 3.25] x [0, 1] (16 x 5
      root cells, uniform at the given level, N = 4, bar-state local limiting,
      IDP time step at CFL 0.9): characteristic boundaries on x-, x+ and y+
      against the exact moving incident shock (the post-shock state where
      x < 1/6 + (y + 20 t)/sqrt(3), updated before every step), characteristic
      inflow on y- for x < 1/6 and a slip wall beyond; reports steps, time,
      violations, the smallest density and pressure, and the incident shock's
      position on the upper side against its exact value; with --amr the mesh
      starts two levels coarser and the modal indicator adapts it every 5
      steps up to the given level (the exterior states follow every new mesh)

  python -m paper_2607_06045_amd.evaluate jet [--level 8] [--t-end 0.0015] [--amr] [--mixed]
      the Mach-2000 jet of Sec. 3.6 on [-0.5, 0.5]^2 (gamma = 5/3, N = 3,
      Chandrashekar volume flux, combined limiting, IDP time step at CFL 0.9,
      uniform at the given level): characteristic inflow on x- with the jet
      state for |y| <= 0.05 and the ambient state elsewhere, characteristic
      x+, periodic in y; reports steps, time, violations and the smallest
      density and pressure, and how far the jet head has come; with --amr the
      mesh adapts every 5 steps between level 2 and the given level (the
      paper: 2..9) and the inflow band is set again on every new mesh

Prints one JSON object.  All inputs are seeded and synthetic.
"""
import argparse
import json
import sys
import time

import numpy as np


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _solver(P, spec, N=3, precision=None):
    s = P.Solver(N, precision=P.FP64 if precision is None else precision)
    s.set_mesh(*spec.args())
    return s


def base_means(s, u, w, base_level, nx0, ny0):
    """Area-weighted means of every variable on the cells of the base level
    (each leaf lies in one base cell), [4, ny0 2^base, nx0 2^base]."""
    lv, ix, iy = s.mesh()
    shift = lv.astype(np.int64) - base_level
    if (shift < 0).any():
        raise ValueError("leaf coarser than the base level")
    bx, by = ix >> shift, iy >> shift
    W = np.outer(w, w) / 4.0
    leaf_mean = (u * W).sum(axis=(2, 3))  # [E, 4]
    area = 0.25 ** shift.astype(np.float64)  # in base-cell units
    nxb, nyb = nx0 << base_level, ny0 << base_level
    out = np.zeros((4, nyb, nxb))
    for v in range(4):
        np.add.at(out[v], (by, bx), leaf_mean[:, v] * area)
    return out


def adapt_run(P, spec, u_fn, steps, every, ctrl, indicator, precision=None, replay=None,
              record=None, on_adapt=None, zs_eps=1e-10):
    """Run with dynamic AMR.  indicator(s) -> per-leaf float array; ctrl is
    (base, med, med_threshold, max, max_threshold); replay: list of flag arrays
    to apply instead of the indicator's; record: list that receives the flags."""
    import torch
    s = _solver(P, spec, precision=precision)
    x, y = s.node_coords()
    s.upload(u_fn(x, y))
    counts, viol, k = [], 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        if it % every == 0:
            if replay is not None:
                flags = replay[k]
            else:
                lv, _, _ = s.mesh()
                flags = P.amr_flags(indicator(s), lv, *ctrl)
            if on_adapt is not None:
                on_adapt(s, flags)
            if record is not None:
                record.append(flags.copy())
            k += 1
            s.refine_coarsen(flags, zs_eps=zs_eps)
            counts.append(s.E)
            if k % 5 == 1:
                log(f"  step {it}: {s.E} leaves")
        st = s.step(0.5)
        viol += st["violations"]
    torch.cuda.synchronize()
    return s, {"wall_s": time.perf_counter() - t0, "elements": counts, "violations": int(viol)}


def run_mixed(steps):
    import paper_2607_06045_amd as P
    from workloads import states
    from workloads.meshes import workload_mesh
    spec = workload_mesh("shear59k")
    # levels relative to the 128 x 128 root grid (absolute levels 7 to 10)
    ctrl = (0, 1, 0.01, 3, 0.1)
    w = P.host_tables(3)["w"]
    flags = []

    def ind(s):
        return s.indicator(P.IND_HENNEMANN)

    def mass(s, absolute=False):
        """sum_i m_i u_i per variable (or of |u_i|)"""
        lv, _, _ = s.mesh()
        u = s.download()
        if absolute:
            u = np.abs(u)
        W = np.outer(w, w) / 4.0
        h2 = (2.0 / (128 << lv.astype(np.int64))) ** 2
        return ((u * W).sum(axis=(2, 3)) * h2[:, None]).sum(axis=0)

    u_fn = lambda x, y: states.workload_state("shear59k", x, y)  # noqa: E731
    log("FP64 run")
    s64, r64 = adapt_run(P, spec, u_fn, steps, 5, ctrl, ind, record=flags)
    log("mixed run")
    smx, rmx = adapt_run(P, spec, u_fn, steps, 5, ctrl, ind, precision=P.MIXED, replay=flags)
    a, b = s64.download(), smx.download()
    m0 = _solver(P, spec)
    x, y = m0.node_coords()
    m0.upload(u_fn(x, y))
    mass0, abs0 = mass(m0), mass(m0, True)
    rel_l1 = np.abs(b - a).sum(axis=(0, 2, 3)) / np.abs(a).sum(axis=(0, 2, 3))
    rel_max = np.abs(b - a).max(axis=(0, 2, 3)) / np.abs(a).max(axis=(0, 2, 3))
    return {"case": "shear layer, 59,392-leaf band mesh, N=3, dynamic AMR every 5 steps (levels 7-10), "
                    "mixed run replays the FP64 run's flags", "steps": steps,
            "rel_l1_per_variable": rel_l1.tolist(), "rel_max_per_variable": rel_max.tolist(),
            "violations": {"fp64": r64["violations"], "mixed": rmx["violations"]},
            # |change of sum m u| / sum m |u|, per variable
            "conservation_defect": {"fp64": (np.abs(mass(s64) - mass0) / abs0).tolist(),
                                    "mixed": (np.abs(mass(smx) - mass0) / abs0).tolist()},
            "elements_final": s64.E, "elements_max": max(r64["elements"]),
            "wall_s": {"fp64": r64["wall_s"], "mixed": rmx["wall_s"]}}


def training_data(P, blasts=3, shears=2, snaps=6, every=5, seed=0):
    """(features, modal indicator) pairs on the GPU from seeded plain runs."""
    import torch
    from workloads import states
    from workloads.meshes import workload_mesh
    from workloads.rng import uniform
    X, Y = [], []
    log("training data")
    for k in range(blasts):
        r = uniform(1000 + seed * 97 + k, np.arange(4, dtype=np.uint64))
        E0, sig = 0.5 + 1.5 * r[0], 0.04 + 0.04 * r[1]
        xc, yc = -0.2 + 0.4 * r[2], -0.2 + 0.4 * r[3]
        s = _solver(P, workload_mesh("blast22k"))
        x, y = s.node_coords()
        s.upload(states.sedov_gaussian(x, y, E0=E0, sigma=sig, xc=xc, yc=yc))
        for i in range(snaps * every):
            if i % every == 0:
                X.append(s.features(device=True))
                Y.append(s.indicator(P.IND_HENNEMANN, device=True))
            s.step(0.5, stats=False)
    for k in range(shears):
        r = uniform(2000 + seed * 89 + k, np.arange(2, dtype=np.uint64))
        s = _solver(P, workload_mesh("shear59k"))
        x, y = s.node_coords()
        s.upload(states.shear_layer(x, y, seed=300 + k, amp=0.05 + 0.1 * r[1]))
        for i in range(snaps * every):
            if i % every == 0:
                X.append(s.features(device=True))
                Y.append(s.indicator(P.IND_HENNEMANN, device=True))
            s.step(0.5, stats=False)
    return torch.cat(X), torch.cat(Y)


def he_uniform(seed):
    """He-uniform weights and zero biases, in the library's parameter order
    W1[64][16], b1, W2[64][64], b2, W3[64], b3."""
    rng = np.random.default_rng(seed)

    def weights(shape, fan_in):
        lim = np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, shape).ravel()

    parts = [weights((64, 16), 16), np.zeros(64), weights((64, 64), 64), np.zeros(64),
             weights((64,), 64), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def fit(P, X, Y, iters, batch=8192, lr=2e-3, seed=11):
    """Adam on the GPU with the library's kernels; returns the context."""
    import torch
    net = P.Solver(3)
    net.mlp_set_weights(he_uniform(seed))
    g = torch.Generator(device="cuda").manual_seed(seed)
    for _ in range(iters):
        idx = torch.randint(0, X.shape[0], (batch,), device="cuda", generator=g)
        net.mlp_train_step(X[idx], Y[idx], lr)
    return net


def run_learned(steps, iters=3000, blasts=3, shears=2, snaps=6):
    import torch
    import paper_2607_06045_amd as P
    from workloads import states
    from workloads.meshes import workload_mesh
    t0 = time.perf_counter()
    X, Y = training_data(P, blasts, shears, snaps)
    n = X.shape[0]
    perm = torch.randperm(n, generator=torch.Generator().manual_seed(0)).cuda()
    ntr = int(0.9 * n)
    Xtr, Ytr, Xva, Yva = X[perm[:ntr]], Y[perm[:ntr]], X[perm[ntr:]], Y[perm[ntr:]]
    t_data = time.perf_counter() - t0
    log(f"training on {ntr} samples")
    t0 = time.perf_counter()
    net = fit(P, Xtr, Ytr, iters)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    w = net.mlp_get_weights()
    val_mse = ((net.mlp_forward(Xva) - Yva) ** 2).mean().item()
    val_var = ((Yva - Yva.mean()) ** 2).mean().item()

    spec = workload_mesh("blast22k")
    # levels relative to the 64 x 64 root grid (absolute levels 6 to 9)
    ctrl = (0, 2, 0.01, 3, 0.1)
    u_fn = lambda x, y: states.workload_state("blast22k", x, y)  # noqa: E731

    def plain(s):
        return s.indicator(P.IND_HENNEMANN)

    agree = {"n": 0, "same": 0, "refine_recall": [0, 0], "coarsen_recall": [0, 0]}

    def learned(s):
        if not getattr(s, "_w", False):
            s.mlp_set_weights(w)
            s._w = True
        return s.indicator(P.IND_MLP)

    def compare(s, flags):
        lv, _, _ = s.mesh()
        fp = P.amr_flags(plain(s), lv, *ctrl)
        agree["n"] += len(fp)
        agree["same"] += int((fp == flags).sum())
        for key, val in (("refine_recall", 1), ("coarsen_recall", -1)):
            agree[key][0] += int(((fp == val) & (flags == val)).sum())
            agree[key][1] += int((fp == val).sum())

    log("plain-indicator run")
    s_p, r_p = adapt_run(P, spec, u_fn, steps, 5, ctrl, plain)
    log("learned-indicator run")
    s_l, r_l = adapt_run(P, spec, u_fn, steps, 5, ctrl, learned, on_adapt=compare)
    wts = P.host_tables(3)["w"]
    mp = base_means(s_p, s_p.download(), wts, 0, spec.nx0, spec.ny0)[0]
    ml = base_means(s_l, s_l.download(), wts, 0, spec.nx0, spec.ny0)[0]
    # indicator cost on the final state of the plain run
    s_p.mlp_set_weights(w)
    for kind in (P.IND_HENNEMANN, P.IND_MLP):
        s_p.indicator(kind, device=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_ind = {}
    for name, kind in (("modal", P.IND_HENNEMANN), ("network", P.IND_MLP)):
        ev0.record()
        for _ in range(20):
            s_p.indicator(kind, device=True)
        ev1.record()
        torch.cuda.synchronize()
        t_ind[name] = ev0.elapsed_time(ev1) / 20
    return {"case": "Sedov blast, 22,156-leaf start mesh, N=3, dynamic AMR every 5 steps (levels 6-9)",
            "steps": steps,
            "training": {"samples": n, "train": ntr, "iters": iters, "batch": 8192,
                         "data_s": t_data, "train_s": t_train, "val_mse": val_mse,
                         "val_target_variance": val_var},
            "agreement": agree["same"] / max(agree["n"], 1),
            "refine_recall": agree["refine_recall"][0] / max(agree["refine_recall"][1], 1),
            "coarsen_recall": agree["coarsen_recall"][0] / max(agree["coarsen_recall"][1], 1),
            "elements": {"plain": r_p["elements"], "learned": r_l["elements"]},
            "violations": {"plain": r_p["violations"], "learned": r_l["violations"]},
            "l1_density_base_cells": float(np.abs(mp - ml).mean()),
            "l1_density_scale": float(np.abs(mp).mean()),
            "wall_s": {"plain": r_p["wall_s"], "learned": r_l["wall_s"]},
            "indicator_ms": t_ind}


def run_scale(steps, iters=2000, seeds=2, snaps=3):
    """Four-quadrant states on the 246,736-leaf mesh, N = 4, dynamic AMR every 5
    steps up to level 2: the plain FP64 method with the modal indicator against
    the mixed-precision method with the learned indicator (trained on the GPU
    from N = 4 (features, modal indicator) pairs of other seeds)."""
    import torch
    import paper_2607_06045_amd as P
    from workloads import states
    from workloads.meshes import workload_mesh
    spec = workload_mesh("quadrants247k")
    N, n = 4, 5
    ctrl = (0, 1, 0.01, 2, 0.1)  # levels relative to the 256 x 256 root grid
    # training data: seeds other than the evaluated state's
    X, Y = [], []
    t0 = time.perf_counter()
    for k in range(seeds):
        s = _solver(P, spec, N)
        x, y = s.node_coords()
        s.upload(states.quadrants(x, y, seed=100 + k))
        for i in range(snaps * 5):
            if i % 5 == 0:
                X.append(s.features(device=True))
                Y.append(s.indicator(P.IND_HENNEMANN, device=True))
            s.step(0.5, stats=False)
        s.close()
    X, Y = torch.cat(X), torch.cat(Y)
    t_data = time.perf_counter() - t0
    log(f"training on {X.shape[0]} samples")
    t0 = time.perf_counter()
    net = fit(P, X, Y, iters)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    w = net.mlp_get_weights()
    u_fn = lambda x, y: states.workload_state("quadrants247k", x, y)  # noqa: E731

    def plain(s):
        return s.indicator(P.IND_HENNEMANN)

    def learned(s):
        if not getattr(s, "_w", False):
            s.mlp_set_weights(w)
            s._w = True
        return s.indicator(P.IND_MLP)

    def adapt_run_n4(indicator, precision):
        s = P.Solver(N, precision=precision)
        s.set_mesh(*spec.args())
        x, y = s.node_coords()
        s.upload(u_fn(x, y))
        counts, viol, dof_updates, t_adapt = [], 0, 0, 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(steps):
            if it % 5 == 0:
                # steps are queued asynchronously: the adaptation interval
                # starts when the queued steps have finished
                torch.cuda.synchronize()
                ta = time.perf_counter()
                lv, _, _ = s.mesh()
                s.refine_coarsen(P.amr_flags(indicator(s), lv, *ctrl))
                torch.cuda.synchronize()
                t_adapt += time.perf_counter() - ta
                counts.append(s.E)
                if it % 100 == 0:
                    log(f"  step {it}: {s.E} leaves")
            st = s.step(0.5, stats=(it % 25 == 0))
            if st:
                viol += st["violations"]
            dof_updates += 3 * s.E * n * n
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return s, {"wall_s": wall, "adapt_s": t_adapt, "dof_updates_per_s": dof_updates / wall,
                   "dof_updates_per_s_steps_only": dof_updates / (wall - t_adapt),
                   "elements_first_last_max": [counts[0], counts[-1], max(counts)],
                   "violations_sampled": int(viol)}

    log("plain FP64 run, modal indicator")
    s_p, r_p = adapt_run_n4(plain, P.FP64)
    log("mixed-precision run, learned indicator")
    s_l, r_l = adapt_run_n4(learned, P.MIXED)
    wts = P.host_tables(N)["w"]
    mp = base_means(s_p, s_p.download(), wts, 0, spec.nx0, spec.ny0)[0]
    ml = base_means(s_l, s_l.download(), wts, 0, spec.nx0, spec.ny0)[0]
    return {"case": "four quadrant states (seed 5), 246,736-leaf start mesh, N=4, dynamic AMR every "
                    "5 steps (levels 8-10)", "steps": steps,
            "training": {"samples": int(X.shape[0]), "iters": iters, "data_s": t_data,
                         "train_s": t_train},
            "plain_fp64": r_p, "mixed_learned": r_l,
            "l1_density_base_cells": float(np.abs(mp - ml).mean()),
            "l1_density_scale": float(np.abs(mp).mean())}


def run_cfl(t_end=3.0, n=128, amr=False, every=5):
    import torch

    import paper_2607_06045_amd as P
    from workloads import states
    from workloads.meshes import uniform_mesh

    # with AMR: a 16 x 16 root grid adapted by the modal indicator between 16
    # and n elements per direction (the paper: 16 to 128), every `every` steps
    top = max(0, int(round(np.log2(n / 16))))
    ctrl = (0, max(0, top - 1), 0.01, top, 0.1)
    spec = uniform_mesh(16, 16, -2.0, -2.0, 4.0, 4.0) if amr else uniform_mesh(n, n, -2.0, -2.0, 4.0, 4.0)
    out = {"mesh": (f"adaptive 16^2..{16 << top}^2 on [-2,2]^2, every {every} steps, N=3" if amr
                    else f"uniform {n}x{n} on [-2,2]^2, N=3"), "t_end": t_end}
    for name, lim, mode, cfl in (("bar_state_bounds_idp_cfl_0.95", P.LIMIT_LOCAL, P.DT_IDP, 0.95),
                                 ("low_order_bounds_lo_cfl_0.4", P.LIMIT_LOCAL_LOWORDER, P.DT_LOWORDER, 0.4)):
        s = P.Solver(3, limiter=lim, dt_mode=mode)
        s.set_mesh(*spec.args())
        x, y = s.node_coords()
        s.upload(states.sedov_tophat(x, y))
        if amr:  # refine the initial disc, taking the exact state each time
            for _ in range(top):
                s.refine_coarsen(P.amr_flags(s.indicator(), s.mesh()[0], *ctrl))
                x, y = s.node_coords()
                s.upload(states.sedov_tophat(x, y))
        leaves = [s.E]
        t, k, viol, inad = 0.0, 0, 0, 0
        a_vol, a_mort, dts = 0.0, 0.0, []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while t < t_end * (1 - 1e-14):
            if amr and k > 0 and k % every == 0:
                s.refine_coarsen(P.amr_flags(s.indicator(), s.mesh()[0], *ctrl))
                leaves.append(s.E)
            dt = min(s.max_dt(cfl), t_end - t)
            st = s.step_dt(dt)
            t += dt
            k += 1
            dts.append(dt)
            viol += st["violations"]
            inad += st["fv_inadmissible"]
            a_vol += st["alpha_vol_mean"]
            a_mort += st["alpha_mort_mean"]
            if k % 1000 == 0:
                log(f"{name}: step {k} t={t:.4f}")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = {"steps": k, "wall_s": wall, "ms_per_step": 1e3 * wall / k,
                     "dt_min": min(dts), "dt_max": max(dts), "violations": viol,
                     "fv_inadmissible": inad, "alpha_vol_mean": a_vol / k, "alpha_mort_mean": a_mort / k,
                     "leaves_min": min(leaves), "leaves_max": max(leaves)}
        log(f"{name}: {out[name]}")
    b_, l_ = out["bar_state_bounds_idp_cfl_0.95"], out["low_order_bounds_lo_cfl_0.4"]
    out["step_ratio"] = b_["steps"] / l_["steps"]
    out["time_ratio"] = b_["wall_s"] / l_["wall_s"]
    out["paper"] = {"steps_bar_state": 6523, "steps_low_order": 2357, "time_ratio": "about 4"}
    return out


def _boundary_xy(s, x, y):
    """Coordinates of the solver's boundary nodes (numbering of boundary_nodes)."""
    N = s.N
    bn = s.boundary_nodes()
    e, f, k = bn[:, 0], bn[:, 1], bn[:, 2]
    a = np.where(f == 0, 0, np.where(f == 1, N, k))
    b = np.where(f == 2, 0, np.where(f == 3, N, k))
    return x[e, b, a], y[e, b, a], f


def _cons(r, v1, v2, p, g):
    return np.array([r, r * v1, r * v2, p / (g - 1.0) + 0.5 * r * (v1 * v1 + v2 * v2)])


def run_dmr(level=4, t_end=0.2, amr=False, every=5):
    import torch

    import paper_2607_06045_amd as P
    from workloads.meshes import MeshSpec

    g, N = 1.4, 4
    # with AMR: start two levels coarser; the modal indicator refines up to
    # the given level (controller levels relative to the 16 x 5 root grid)
    ctrl = (level - 2, level - 1, 0.01, level, 0.1)
    start = level - 2 if amr else level
    nx, ny = 16 << start, 5 << start
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    spec = MeshSpec(np.full(nx * ny, start, np.int8), ii.ravel().astype(np.int32),
                    jj.ravel().astype(np.int32), 0.0, 0.0, 3.25, 1.0, 16, 5)
    post = _cons(8.0, 8.25 * np.cos(np.pi / 6), -8.25 * np.sin(np.pi / 6), 116.5, g)
    pre = _cons(1.4, 0.0, 0.0, 1.0, g)
    CH = P.BC_CHARACTERISTIC
    s = P.Solver(N, gamma=g, limiter=P.LIMIT_LOCAL, bc=[CH] * 4,
                 ext=np.stack([post, pre, post, pre]))
    s.set_mesh(*spec.args())

    def initial(x, y):
        left = x < 1.0 / 6.0 + y / np.sqrt(3.0)
        return np.ascontiguousarray(np.where(left[:, None], post[None, :, None, None],
                                             pre[None, :, None, None]))

    x, y = s.node_coords()
    s.upload(initial(x, y))
    if amr:  # refine the initial discontinuity, taking the exact state each time
        for _ in range(3):
            s.refine_coarsen(P.amr_flags(s.indicator(), s.mesh()[0], *ctrl))
            x, y = s.node_coords()
            s.upload(initial(x, y))
    bx, by, bf = _boundary_xy(s, x, y)
    leaves = [s.E]

    def exterior(t):
        kind = np.full(len(bx), CH, np.int8)
        kind[(bf == 2) & (bx >= 1.0 / 6.0)] = P.BC_WALL
        shocked = bx < 1.0 / 6.0 + (by + 20.0 * t) / np.sqrt(3.0)
        ext = np.where(shocked[:, None], post[None, :], pre[None, :])
        ext[bf == 2] = post  # the characteristic part of y- is post-shock
        return kind, np.ascontiguousarray(ext)

    t, k, viol = 0.0, 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while t < t_end * (1 - 1e-14):
        if amr and k > 0 and k % every == 0:
            s.refine_coarsen(P.amr_flags(s.indicator(), s.mesh()[0], *ctrl))
            x, y = s.node_coords()
            bx, by, bf = _boundary_xy(s, x, y)
            leaves.append(s.E)
        s.set_boundary_states(*exterior(t))
        dt = min(s.max_dt(0.9), t_end - t)
        st = s.step_dt(dt)
        viol += st["violations"]
        t += dt
        k += 1
        if k % 500 == 0:
            log(f"dmr: step {k} t={t:.4f}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    u = s.download()
    rho = u[:, 0]
    p = (g - 1) * (u[:, 3] - 0.5 * (u[:, 1] ** 2 + u[:, 2] ** 2) / u[:, 0])
    # incident shock on the upper side: where the top row of nodes crosses the
    # mean of the two densities, against 1/6 + (1 + 20 t)/sqrt(3)
    top = np.abs(y - 1.0) < 1e-12
    xs, rs = x[top], rho[top]
    o = np.argsort(xs)
    xs, rs = xs[o], rs[o]
    mid = 0.5 * (8.0 + 1.4)
    cross = xs[np.nonzero((rs[:-1] >= mid) & (rs[1:] < mid))[0]]
    exact = 1.0 / 6.0 + (1.0 + 20.0 * t_end) / np.sqrt(3.0)
    mesh = (f"adaptive, levels {ctrl[0]}..{ctrl[3]} of the 16x5 root grid (finest {16 << level}x{5 << level}),"
            f" adapted every {every} steps, N={N}" if amr else f"uniform {nx}x{ny}, N={N}")
    return {"mesh": mesh, "elements": s.E, "leaves_min": min(leaves), "leaves_max": max(leaves),
            "t_end": t_end, "steps": k,
            "wall_s": wall, "ms_per_step": 1e3 * wall / k, "violations": viol,
            "rho_min": float(rho.min()), "p_min": float(p.min()), "rho_max": float(rho.max()),
            "top_shock_x": [float(c) for c in cross], "top_shock_x_exact": exact,
            "hx": 3.25 / (16 << level)}


def run_jet(level=8, t_end=0.0015, amr=False, every=5, base=2, mixed=False):
    import torch

    import paper_2607_06045_amd as P
    from workloads.meshes import uniform_mesh

    g, N = 5.0 / 3.0, 3
    # with AMR: levels base..level of a single root cell (the paper: 2..9), the
    # modal indicator every `every` steps
    ctrl = (base, level - 1, 0.01, level, 0.1)
    n = 1 << (base if amr else level)
    spec = uniform_mesh(n, n, -0.5, -0.5, 1.0, 1.0)
    if amr:  # one root cell refined uniformly to the base level
        from workloads.meshes import MeshSpec
        ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        spec = MeshSpec(np.full(n * n, base, np.int8), ii.ravel().astype(np.int32),
                        jj.ravel().astype(np.int32), -0.5, -0.5, 1.0, 1.0, 1, 1)
    amb = _cons(0.5, 0.0, 0.0, 0.4127, g)
    jet = _cons(5.0, 800.0, 0.0, 0.4127, g)
    CH = P.BC_CHARACTERISTIC
    s = P.Solver(N, gamma=g, limiter=P.LIMIT_COMBINED, volume_flux=P.FLUX_CHANDRASHEKAR,
                 precision=P.MIXED if mixed else P.FP64,
                 bc=[CH, CH, P.BC_PERIODIC, P.BC_PERIODIC], ext=np.stack([amb, amb, amb, amb]))
    s.set_mesh(*spec.args())
    x, y = s.node_coords()
    s.upload(np.ascontiguousarray(np.broadcast_to(amb[None, :, None, None], (s.E, 4, N + 1, N + 1))))

    def inflow():
        xx, yy = s.node_coords()
        bx, by, bf = _boundary_xy(s, xx, yy)
        ext = np.tile(amb, (len(bx), 1))
        ext[(bf == 0) & (np.abs(by) <= 0.05)] = jet
        s.set_boundary_states(np.full(len(bx), CH, np.int8), ext)

    if amr:  # resolve the inflow band at the finest level before the first step
        for _ in range(level - base):
            lv, ix, iy = s.mesh()
            h = 1.0 / (1 << lv.astype(np.int64))
            yc = -0.5 + (iy + 0.5) * h
            near = (ix == 0) & (np.abs(yc) < 0.05 + h)
            s.refine_coarsen(np.where(near & (lv < level), 1, 0).astype(np.int8))
        x, y = s.node_coords()
        s.upload(np.ascontiguousarray(np.broadcast_to(amb[None, :, None, None], (s.E, 4, N + 1, N + 1))))
    inflow()
    leaves = [s.E]
    t, k, viol, inad = 0.0, 0, 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while t < t_end * (1 - 1e-14):
        if amr and k % every == 0:
            s.refine_coarsen(P.amr_flags(s.indicator(), s.mesh()[0], *ctrl))
            inflow()
            leaves.append(s.E)
        dt = min(s.max_dt(0.9), t_end - t)
        st = s.step_dt(dt)
        viol += st["violations"]
        inad += st["fv_inadmissible"]
        t += dt
        k += 1
        if k % 500 == 0:
            log(f"jet: step {k} t={t:.6f}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    u = s.download()
    rho = u[:, 0]
    p = (g - 1) * (u[:, 3] - 0.5 * (u[:, 1] ** 2 + u[:, 2] ** 2) / u[:, 0])
    v1 = u[:, 1] / rho
    fast = v1 > 400.0  # jet material
    x, y = s.node_coords()
    mesh = (f"adaptive, levels {base}..{level} (finest {1 << level}^2), adapted every {every} steps, N={N}"
            if amr else f"uniform {n}x{n}, N={N}")
    return {"mesh": mesh, "elements": s.E, "leaves_min": min(leaves), "leaves_max": max(leaves),
            "t_end": t_end, "steps": k,
            "wall_s": wall, "ms_per_step": 1e3 * wall / k, "violations": viol,
            "fv_inadmissible": inad, "rho_min": float(rho.min()), "p_min": float(p.min()),
            "rho_max": float(rho.max()), "jet_head_x": float(x[fast].max()) if fast.any() else None,
            "dofs": s.E * (N + 1) ** 2}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["mixed", "learned", "scale", "cfl", "dmr", "jet"])
    ap.add_argument("--level", type=int, default=None)
    ap.add_argument("--amr", action="store_true")
    ap.add_argument("--mixed", action="store_true")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--t-end", type=float, default=None)
    ap.add_argument("--n", type=int, default=128)
    a = ap.parse_args(argv)
    if a.mode == "cfl":
        out = run_cfl(3.0 if a.t_end is None else a.t_end, a.n, a.amr)
    elif a.mode == "dmr":
        out = run_dmr(4 if a.level is None else a.level, 0.2 if a.t_end is None else a.t_end, a.amr)
    elif a.mode == "jet":
        out = run_jet(8 if a.level is None else a.level, 0.0015 if a.t_end is None else a.t_end, a.amr,
                      mixed=a.mixed)
    elif a.mode == "mixed":
        out = run_mixed(a.steps or 200)
    elif a.mode == "scale":
        out = run_scale(a.steps or 500, iters=a.iters)
    else:
        out = run_learned(a.steps or 100, iters=a.iters)
    print(json.dumps(out, default=float), flush=True)


if __name__ == "__main__":
    sys.exit(main())
