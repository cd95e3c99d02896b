"""Benchmark of the dynamic cutoff method hot path on one MI355X.

One step = one pass of the whole per-step path on one synthetic system
(velocity-Verlet kick + drift, interface detection on the density grid,
cutoff-limited distance sweep, cutoff assignment, cell binning, the
dynamic-cutoff LJ force/energy evaluation, final kick), run through the
library's dcm_step with re-detection every step.  Inputs are resident in HBM
before the timed region starts.

Printed (one JSON line): pair interactions per second over the whole step,
force evaluations per second, the pair kernel's achieved rate against the
VALU roofline (HIP events around every pair launch inside the timed region),
the FP64 path's figures on the same workload, and the FP64 CPU oracle timed
on a bounded sample of the same workload.  Context beside them: the same
step with re-detection every 10 steps, the 64-system batched form, Verlet
lists against the cell walk, and the symmetric rule with and without
Newton's third law.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# algorithmic work per interacting ordered pair (force + energy), FMA = 2:
# separation 3, r^2 5, 1/r^2 1, (1/r^2)^3 2, force factor 4, force 6, energy 3
FLOP_PER_PAIR_FE = 24
VALU_PEAK_FP64 = 78.6            # MI355X vector FP64 (also its unpacked FP32 rate)
VALU_PEAK_FP32 = 157.3           # MI355X vector FP32 (packed)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="slab_large")
    p.add_argument("--prec", default="fp32_mixed", choices=["fp32_mixed", "fp64"])
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison leg")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--no-batched", action="store_true", help="skip the 64-system batched leg")
    p.add_argument("--no-list", action="store_true", help="skip the Verlet-list leg")
    p.add_argument("--no-n3", action="store_true", help="skip the Newton's-third-law leg")
    p.add_argument("--no-table1", action="store_true",
                   help="skip the Table 1 analogue (DCM vs static cutoff, 1.2M-particle slab)")
    p.add_argument("--no-curved", action="store_true",
                   help="skip the droplet and cylinder legs (FP32-mixed and FP64)")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--table1", action="store_true",
                   help="only run the DCM-versus-static-cutoff timing of the paper's Table 1 "
                        "settings on the 1.2M-particle planar slab and print that as the line")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run a plain device copy of MIB MiB five times (the reference "
                        "kernel for scaling the HBM traffic counters) and exit")
    return p.parse_args()


def run_leg(s, prec, steps, warmup, dev, redetect=1):
    import torch

    import paper_1701_05242_amd as dcm

    f64 = dict(dtype=torch.float64, device=dev)
    pos = [torch.tensor(a, **f64) for a in (s.x, s.y, s.z)]
    vel = [torch.tensor(a, **f64) for a in (s.vx, s.vy, s.vz)]
    frc = [torch.zeros(s.n, **f64) for _ in range(3)]
    rc = torch.zeros(s.n, **f64)
    grid = dcm.make_grid(s.box, s.h)
    rule = dcm.make_rule(*s.rule)
    rcg = dcm.rc_grid_for(rule, grid)
    lj = dcm.make_lj()
    ctx = dcm.dcm_create()
    try:
        dcm.dcm_step(ctx, *pos, *vel, *frc, s.box, lj, rule, grid, rcg, 0.005, 0, prec=prec, rc=rc)
        cell_len = dcm.dcm_cell_dims(ctx)[1]  # the step's tuned cell edge
        if warmup:
            dcm.dcm_step(ctx, *pos, *vel, *frc, s.box, lj, rule, grid, rcg, 0.005, warmup,
                         prec=prec, redetect_every=redetect, rc=rc)
        if dcm.dcm_sync_status(ctx) != dcm.DCM_OK:
            raise RuntimeError(dcm.dcm_last_error(ctx))

        def count_pairs():
            npairs = torch.zeros(1, dtype=torch.uint64, device=dev)
            e = torch.zeros(1, **f64)
            dcm.dcm_build_cells(ctx, *pos, rc, s.box, 0.0, prec, rc_bound=s.rule[1])
            dcm.dcm_forces(ctx, lj, *frc, prec=prec, ev_flags=dcm.DCM_EV_COUNTS | dcm.DCM_EV_ENERGY,
                           energy=e, npairs=npairs)
            torch.cuda.synchronize()
            return int(npairs.cpu().numpy()[0])

        pairs_before = count_pairs()
        fams = ("pair", "cells", "detect", "sweep", "cutoffs", "verlet")
        # the timed steps: HIP events around the pair kernel's launches only
        dcm.dcm_set_profiling(ctx, True)
        dcm.dcm_set_profiling_only(ctx, "pair")
        for fam in fams:
            dcm.dcm_kernel_time(ctx, fam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dcm.dcm_step(ctx, *pos, *vel, *frc, s.box, lj, rule, grid, rcg, 0.005, steps,
                     prec=prec, redetect_every=redetect, step0=warmup, rc=rc)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pair_timed = dcm.dcm_kernel_time(ctx, "pair")
        status = dcm.dcm_sync_status(ctx)
        if status != dcm.DCM_OK:
            raise RuntimeError(f"device status {status}: {dcm.dcm_last_error(ctx)}")
        pairs_after = count_pairs()
        # the same number of further steps, untimed, with every stage's events
        # (the stage split)
        dcm.dcm_set_profiling_only(ctx, None)
        dcm.dcm_step(ctx, *pos, *vel, *frc, s.box, lj, rule, grid, rcg, 0.005, steps,
                     prec=prec, redetect_every=redetect, step0=warmup + steps, rc=rc)
        fam_ms = {fam: dcm.dcm_kernel_time(ctx, fam) for fam in fams}
        dcm.dcm_set_profiling(ctx, False)
        status = dcm.dcm_sync_status(ctx)
        if status != dcm.DCM_OK:
            raise RuntimeError(f"device status {status}: {dcm.dcm_last_error(ctx)}")
        # the cell walk's work at the step's cell edge (a pair-count pass)
        npairs = torch.zeros(1, dtype=torch.uint64, device=dev)
        dcm.dcm_build_cells(ctx, *pos, rc, s.box, min(cell_len) * (1.0 - 1e-12), prec,
                            rc_bound=s.rule[1])
        dcm.dcm_forces(ctx, lj, *frc, prec=prec, ev_flags=dcm.DCM_EV_COUNTS, npairs=npairs)
        cand, rows = dcm.dcm_walk_stats(ctx)
        walk_pairs = max(int(npairs.cpu().numpy()[0]), 1)
        walk = {"candidates_per_pair": cand / walk_pairs, "rows_per_particle": rows / s.n,
                "candidates": cand, "rows": rows, "pairs": walk_pairs}
    finally:
        dcm.dcm_destroy(ctx)
    wall = t1 - t0
    pairs = 0.5 * (pairs_before + pairs_after)
    pair_ms, pair_launches = pair_timed
    avg_pair_s = pair_ms / max(pair_launches, 1) / 1e3
    return dict(wall=wall, ms_per_step=wall / steps * 1e3, pairs_per_step=pairs, cell_len=cell_len,
                pair_rate=pairs * steps / wall, force_evals=steps / wall,
                avg_pair_ms=avg_pair_s * 1e3,
                pair_kernel_tflops=pairs * FLOP_PER_PAIR_FE / avg_pair_s / 1e12,
                pair_launches=pair_launches,
                stage_ms={k: v[0] / max(v[1], 1) for k, v in fam_ms.items()},
                stage_launches={k: v[1] for k, v in fam_ms.items()}, walk=walk)


# (rc_min, rc_max) settings of the paper's Table 1 and the speedups it prints
# (DCM over a static cutoff rc = rc_max, planar system, Section 4.2)
TABLE1 = ((3.0, 7.0, 2.31), (3.0, 8.0, 2.66), (3.5, 8.0, 2.38), (3.0, 9.0, 2.42), (3.5, 9.0, 2.23))


def table1_leg(steps, warmup, dev, prec):
    """Seconds per velocity-Verlet step of the planar slab under DCM (cutoff
    ramp rc_max -> rc_min over 5 sigma from the interface, re-detection every
    10 steps) and under a static cutoff rc_max for every particle (no
    detection inside the timed steps), for each Table 1 setting."""
    import torch

    import paper_1701_05242_amd as dcm
    import workloads

    s = workloads.make("slab_table1")
    f64 = dict(dtype=torch.float64, device=dev)
    grid = dcm.make_grid(s.box, s.h)
    lj = dcm.make_lj()

    def run(rule_t, every):
        pos = [torch.tensor(a, **f64) for a in (s.x, s.y, s.z)]
        vel = [torch.tensor(a, **f64) for a in (s.vx, s.vy, s.vz)]
        frc = [torch.zeros(s.n, **f64) for _ in range(3)]
        rc = torch.zeros(s.n, **f64)
        rule = dcm.make_rule(*rule_t)
        rcg = dcm.rc_grid_for(rule, grid)
        ctx = dcm.dcm_create()
        try:
            dcm.dcm_step(ctx, *pos, *vel, *frc, s.box, lj, rule, grid, rcg, 0.005, 0, prec=prec,
                         rc=rc)
            dcm.dcm_step(ctx, *pos, *vel, *frc, s.box, lj, rule, grid, rcg, 0.005, warmup,
                         prec=prec, redetect_every=every, rc=rc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dcm.dcm_step(ctx, *pos, *vel, *frc, s.box, lj, rule, grid, rcg, 0.005, steps,
                         prec=prec, redetect_every=every, step0=warmup, rc=rc)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            npairs = torch.zeros(1, dtype=torch.uint64, device=dev)
            dcm.dcm_build_cells(ctx, *pos, rc, s.box, 0.5 * rule_t[0], prec, rc_bound=rule_t[1])
            dcm.dcm_forces(ctx, lj, *frc, prec=prec, ev_flags=dcm.DCM_EV_COUNTS, npairs=npairs)
            if dcm.dcm_sync_status(ctx) != dcm.DCM_OK:
                raise RuntimeError(dcm.dcm_last_error(ctx))
            pairs = int(npairs.cpu().numpy()[0])
        finally:
            dcm.dcm_destroy(ctx)
        return (t1 - t0) / steps * 1e3, pairs

    rows = []
    for rmin, rmax, paper in TABLE1:
        dcm_ms, dcm_pairs = run((rmin, rmax, 5.0), 10)
        static_ms, static_pairs = run((rmax, rmax, 5.0), 1 << 30)
        rows.append(dict(setting=f"{rmin}/{rmax}", dcm_ms_per_step=dcm_ms,
                         static_ms_per_step=static_ms, speedup=static_ms / dcm_ms,
                         paper_speedup=paper, dcm_pairs=dcm_pairs, static_pairs=static_pairs,
                         pair_ratio=static_pairs / dcm_pairs))
        print(f"[bench] table1 {json.dumps(rows[-1])}", file=sys.stderr, flush=True)
    return dict(experiment="Table 1 analogue: DCM vs static rc = rc_max, planar slab",
                workload=f"slab_table1: 120x120x250 LJ slab, N={s.n}, liquid 75 <= z < 175",
                steps=steps, warmup=warmup, precision="fp32_mixed" if prec else "fp64",
                redetect_every=10, rows=rows)


def curved_leg(steps, warmup, dev):
    """The curved-interface workloads (a droplet of radius 30 and a cylinder of
    radius 25): the full DCM step with re-detection every step, FP32-mixed and
    FP64."""
    import workloads

    out = {}
    for name in ("droplet", "cylinder"):
        s = workloads.make(name)
        legs = {}
        for tag, prec in (("fp32_mixed", 1), ("fp64", 0)):
            r = run_leg(s, prec, steps, warmup, dev)
            legs[tag] = {"ms_per_step": r["ms_per_step"], "pair_rate": r["pair_rate"],
                         "pair_kernel_ms": r["avg_pair_ms"], "tuned_cell_edge": r["cell_len"]}
        legs["n_particles"] = s.n
        legs["pairs_per_step"] = r["pairs_per_step"]
        legs["fp32_mixed_speedup_per_step"] = (legs["fp64"]["ms_per_step"] /
                                               legs["fp32_mixed"]["ms_per_step"])
        out[name] = legs
        print(f"[bench] curved {name} {json.dumps(legs)}", file=sys.stderr, flush=True)
    return out


def batched_leg(steps, dev):
    """64 independent slabs (2,000-200,000 particles, rc_max 4-8): cells +
    forces for all of them as one replayed graph around one persistent pair
    launch (FP32-mixed, tuned cell edge), against the same work as 64
    sequential single-system FP64 calls.  Cutoffs come from the library's own
    detection / sweep / assignment steps, run once before timing."""
    import torch

    import paper_1701_05242_amd as dcm
    import workloads

    f64 = dict(dtype=torch.float64, device=dev)
    systems = workloads.batched_systems()
    lj = dcm.make_lj()
    ctx = dcm.dcm_create()
    try:
        batch = []
        for s in systems:
            x, y, z = (torch.tensor(a, **f64) for a in (s.x, s.y, s.z))
            rc = torch.zeros(s.n, **f64)
            grid = dcm.make_grid(s.box, s.h)
            nv = dcm.grid_voxels(grid)
            seg = torch.zeros(nv, dtype=torch.uint8, device=dev)
            iface = torch.zeros(nv, dtype=torch.uint8, device=dev)
            dist = torch.zeros(nv, **f64)
            rule = dcm.make_rule(*s.rule)
            dcm.dcm_detect_interface(ctx, x, y, z, s.box, grid, seg, iface)
            dcm.dcm_sweep_distance(ctx, seg, iface, grid, dcm.rc_grid_for(rule, grid), 128, dist)
            dcm.dcm_assign_cutoffs(ctx, x, y, z, s.box, grid, dist, rule, rc)
            batch.append(dict(x=x, y=y, z=z, rc=rc, fx=torch.zeros(s.n, **f64),
                              fy=torch.zeros(s.n, **f64), fz=torch.zeros(s.n, **f64),
                              energy=torch.zeros(1, **f64),
                              npairs=torch.zeros(1, dtype=torch.uint64, device=dev),
                              box=s.box, cell_edge=0.0, rc_bound=s.rule[1]))
        if dcm.dcm_sync_status(ctx) != dcm.DCM_OK:
            raise RuntimeError(dcm.dcm_last_error(ctx))
        ev = dcm.DCM_EV_ENERGY | dcm.DCM_EV_COUNTS

        def timed(fn, reps):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps

        arr = dcm.make_systems(batch)

        def batched(prec, graph):
            return lambda: dcm.dcm_forces_batched(ctx, arr, lj, prec=prec, ev_flags=ev,
                                                  use_graph=graph)

        def check():
            if dcm.dcm_sync_status(ctx) != dcm.DCM_OK:
                raise RuntimeError(dcm.dcm_last_error(ctx))
            return sum(int(d["npairs"].cpu().numpy()[0]) for d in batch)

        graph_s = timed(batched(dcm.DCM_FP32_MIXED, True), steps)
        pairs = check()
        edge = dcm.dcm_batched_edge(ctx)
        queues = dcm.dcm_batched_queues(ctx)
        lists = dcm.dcm_batched_row_lists(ctx)
        # each work-queue layout forced (the edge re-tuned under it)
        layout_s = {}
        for q in (1, 8):
            dcm.dcm_set_batched_queues(ctx, q)
            layout_s[q] = timed(batched(dcm.DCM_FP32_MIXED, True), steps)
            check()
        dcm.dcm_set_batched_queues(ctx, 0)
        # the same batch without the recorded graph, and in FP64 with it
        eager_s = timed(batched(dcm.DCM_FP32_MIXED, False), steps)
        check()
        graph64_s = timed(batched(dcm.DCM_FP64, True), steps)
        check()

        def sequential(prec):
            def run():
                for s, d in zip(systems, batch):
                    dcm.dcm_build_cells(ctx, d["x"], d["y"], d["z"], d["rc"], s.box, edge,
                                        prec, rc_bound=s.rule[1])
                    dcm.dcm_forces(ctx, lj, d["fx"], d["fy"], d["fz"], prec=prec,
                                   ev_flags=ev, energy=d["energy"], npairs=d["npairs"])
            return run

        seq_s = timed(sequential(dcm.DCM_FP64), max(2, steps // 4))
        seq_pairs = check()
        seq32_s = timed(sequential(dcm.DCM_FP32_MIXED), max(2, steps // 4))
        check()
    finally:
        dcm.dcm_destroy(ctx)
    n_total = sum(s.n for s in systems)
    leg = lambda sec, p: {"ms": sec * 1e3, "pair_rate": p / sec}
    return {"workload": f"{len(systems)} slabs, N 2e3-2e5 log-uniform (total {n_total}), "
                        "rc_max U[4,8], cells + forces per evaluation",
            "n_particles": n_total, "pairs": pairs, "tuned_cell_edge": edge,
            "tuned_queues": queues,
            "tuned_row_lists": lists,
            "graph_fp32_mixed": leg(graph_s, pairs),
            "graph_fp32_mixed_one_queue": leg(layout_s[1], pairs),
            "graph_fp32_mixed_queue_per_xcd": leg(layout_s[8], pairs),
            "eager_batched_fp32_mixed": leg(eager_s, pairs),
            "graph_fp64": leg(graph64_s, pairs),
            "sequential_fp32_mixed": leg(seq32_s, pairs),
            "sequential_fp64": leg(seq_s, seq_pairs),
            "attribution": {"batching (sequential / eager batched, FP32-mixed)": seq32_s / eager_s,
                            "graph (eager / graph, FP32-mixed)": eager_s / graph_s,
                            "precision (FP64 / FP32-mixed, graph)": graph64_s / graph_s,
                            "total (sequential FP64 / graph FP32-mixed)": seq_s / graph_s}}


def list_leg(s, dev, reps=5, skin=0.3):
    """Verlet lists (Algorithms 2.2-2.3) against the cell walk on the same
    cells: per precision, the average pair-kernel time of dcm_forces and of
    dcm_forces_list with skins 0 and `skin`, the list build and a list update
    (HIP events of the library's "pair" and "list" families).  Cutoffs come
    from one detection / sweep / assignment pass before timing."""
    import torch

    import paper_1701_05242_amd as dcm

    f64 = dict(dtype=torch.float64, device=dev)
    x, y, z = (torch.tensor(a, **f64) for a in (s.x, s.y, s.z))
    grid = dcm.make_grid(s.box, s.h)
    rule = dcm.make_rule(*s.rule)
    nv = dcm.grid_voxels(grid)
    seg = torch.zeros(nv, dtype=torch.uint8, device=dev)
    iface = torch.zeros_like(seg)
    dist = torch.zeros(nv, **f64)
    rc = torch.zeros(s.n, **f64)
    F = [torch.zeros(s.n, **f64) for _ in range(3)]
    e = torch.zeros(1, **f64)
    lj = dcm.make_lj()
    ctx = dcm.dcm_create()
    out = {"workload": s.name, "cell_edge": 1.25}
    try:
        dcm.dcm_detect_interface(ctx, x, y, z, s.box, grid, seg, iface)
        dcm.dcm_sweep_distance(ctx, seg, iface, grid, dcm.rc_grid_for(rule, grid), 64, dist)
        dcm.dcm_assign_cutoffs(ctx, x, y, z, s.box, grid, dist, rule, rc)

        def avg(fam, fn, n):
            dcm.dcm_set_profiling(ctx, True)
            dcm.dcm_kernel_time(ctx, fam)
            for _ in range(n):
                fn()
            ms, k = dcm.dcm_kernel_time(ctx, fam)
            dcm.dcm_set_profiling(ctx, False)
            return ms / max(k, 1)

        forces = lambda p: dcm.dcm_forces(ctx, lj, *F, prec=p, ev_flags=dcm.DCM_EV_ENERGY,
                                          energy=e)
        forces_list = lambda p: dcm.dcm_forces_list(ctx, lj, *F, prec=p,
                                                    ev_flags=dcm.DCM_EV_ENERGY, energy=e)
        for name, p in (("fp64", dcm.DCM_FP64), ("fp32_mixed", dcm.DCM_FP32_MIXED)):
            dcm.dcm_build_cells(ctx, x, y, z, rc, s.box, 1.25, p, rc_bound=s.rule[1])
            leg = {"cell_walk_ms": avg("pair", lambda: forces(p), reps)}
            for sk in (0.0, skin):
                leg[f"skin_{sk:g}"] = {
                    "build_ms": avg("list", lambda: dcm.dcm_build_list(ctx, sk), 2),
                    "forces_ms": avg("pair", lambda: forces_list(p), reps)}
            leg["update_ms"] = avg("list", lambda: dcm.dcm_update_list(ctx, x, y, z, rc), 2)
            out[name] = leg
        if dcm.dcm_sync_status(ctx) != dcm.DCM_OK:
            raise RuntimeError(dcm.dcm_last_error(ctx))
    finally:
        dcm.dcm_destroy(ctx)
    return out


def n3_leg(s, dev, reps=3):
    """The symmetric rule (r_ij <= max(rc_i, rc_j)) in FP64 on the same cells:
    the plain traversal (every particle searches the largest cutoff) against
    the Newton's-third-law form (each pair once, from the endpoint with the
    larger cutoff, reactions added with atomics), and the own-cutoff rule
    for reference.  Per form: average pair-kernel time ("pair" events) and
    wall time of the whole dcm_forces call; pairs counted once per call."""
    import torch

    import paper_1701_05242_amd as dcm

    f64 = dict(dtype=torch.float64, device=dev)
    x, y, z = (torch.tensor(a, **f64) for a in (s.x, s.y, s.z))
    grid = dcm.make_grid(s.box, s.h)
    rule = dcm.make_rule(*s.rule)
    nv = dcm.grid_voxels(grid)
    seg = torch.zeros(nv, dtype=torch.uint8, device=dev)
    iface = torch.zeros_like(seg)
    dist = torch.zeros(nv, **f64)
    rc = torch.zeros(s.n, **f64)
    F = [torch.zeros(s.n, **f64) for _ in range(3)]
    e = torch.zeros(1, **f64)
    npairs = torch.zeros(1, dtype=torch.uint64, device=dev)
    lj = dcm.make_lj()
    ctx = dcm.dcm_create()
    out = {"workload": s.name, "precision": "fp64", "cell_edge": 1.25}
    try:
        dcm.dcm_detect_interface(ctx, x, y, z, s.box, grid, seg, iface)
        dcm.dcm_sweep_distance(ctx, seg, iface, grid, dcm.rc_grid_for(rule, grid), 64, dist)
        dcm.dcm_assign_cutoffs(ctx, x, y, z, s.box, grid, dist, rule, rc)
        dcm.dcm_build_cells(ctx, x, y, z, rc, s.box, 1.25, dcm.DCM_FP64, rc_bound=s.rule[1])
        for name, pr in (("own", dcm.DCM_PAIR_OWN), ("max", dcm.DCM_PAIR_MAX),
                         ("max_n3", dcm.DCM_PAIR_MAX_N3)):
            call = lambda: dcm.dcm_forces(ctx, lj, *F, pair_rule=pr,
                                          ev_flags=dcm.DCM_EV_ENERGY | dcm.DCM_EV_COUNTS,
                                          energy=e, npairs=npairs)
            call()
            torch.cuda.synchronize()
            dcm.dcm_set_profiling(ctx, True)
            dcm.dcm_kernel_time(ctx, "pair")
            t0 = time.perf_counter()
            for _ in range(reps):
                call()
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / reps
            ms, k = dcm.dcm_kernel_time(ctx, "pair")
            dcm.dcm_set_profiling(ctx, False)
            out[name] = {"pair_kernel_ms": ms / max(k, 1), "call_ms": wall * 1e3,
                         "pairs": int(npairs.cpu().numpy()[0])}
        if dcm.dcm_sync_status(ctx) != dcm.DCM_OK:
            raise RuntimeError(dcm.dcm_last_error(ctx))
    finally:
        dcm.dcm_destroy(ctx)
    return out


def cpu_baseline(s, seconds):
    """The oracle's O(N) per-particle sums on a seeded sample of particles at
    all host threads (the reported CPU baseline) and at one thread, and the
    CPU cell-list DCM of the paper (Algorithms 2.2-2.3, OpenMP dynamic,20):
    the whole system at all threads, a seeded sample at one thread.  Every leg
    runs on the oracle's own cutoffs."""
    import numpy as np

    import oracle
    import workloads

    oracle.build(force=False)
    threads = oracle.num_threads()
    det = oracle.detect_interface(s.x, s.y, s.z, s.box, s.h)
    rcg = oracle.rc_grid_for(s.rule, det["hv"])
    D, _ = oracle.fsm(det["nv"], det["hv"], det["seg"], det["iface"], rcg)
    rc = oracle.cutoffs(oracle.particle_distance(s.x, s.y, s.z, s.box, det["nv"], D), s.rule)

    def oracle_leg(budget, seed):
        # a probe large enough that thread start-up does not dominate its time
        probe = workloads.sample_indices(s.n, 512, seed=7)
        t0 = time.perf_counter()
        oracle.forces(s.x, s.y, s.z, rc, s.box, idx=probe)
        per_i = (time.perf_counter() - t0) / len(probe)
        k = int(max(64, min(s.n, budget / max(per_i, 1e-9))))
        idx = workloads.sample_indices(s.n, k, seed=seed)
        t0 = time.perf_counter()
        out = oracle.forces(s.x, s.y, s.z, rc, s.box, idx=idx)
        dt = time.perf_counter() - t0
        pairs = int(np.sum(out["nnbr"]))
        return k, pairs, dt

    k, pairs, dt = oracle_leg(seconds, 8)
    main = dict(value=pairs / dt, unit="pair-interactions/s", cores=threads, kind="oracle",
                sample=f"O(N^2) oracle force sums for {k} seeded particles of {s.name} "
                       f"(all {s.n} j each), {pairs} interacting pairs in {dt:.1f} s")
    detail = {}
    edge = float(s.rule[0])  # small bins: the smallest cutoff (Section 2.3)
    g = oracle.cpu_cells_forces(s.x, s.y, s.z, rc, s.box, edge)
    detail["cell_list_all_threads"] = dict(
        threads=threads, pair_rate=g["pairs"] / (g["t_build"] + g["t_force"]),
        force_evals_per_s=1.0 / (g["t_build"] + g["t_force"]), list_build_s=g["t_build"],
        force_loop_s=g["t_force"], pairs=g["pairs"],
        sample=f"whole system ({s.n} particles), bins of {edge:g} sigma")
    oracle.set_threads(1)
    try:
        k1, pairs1, dt1 = oracle_leg(max(2.0, seconds / 3.0), 9)
        detail["oracle_1_thread"] = dict(
            threads=1, pair_rate=pairs1 / dt1,
            sample=f"{k1} seeded particles (all {s.n} j each), {pairs1} pairs in {dt1:.1f} s")
        m = min(s.n, max(1000, int(0.04 * s.n)))
        idx = workloads.sample_indices(s.n, m, seed=10)
        g1 = oracle.cpu_cells_forces(s.x, s.y, s.z, rc, s.box, edge, idx=idx)
        t1 = g1["t_build"] + g1["t_force"]
        detail["cell_list_1_thread"] = dict(
            threads=1, pair_rate=g1["pairs"] / t1, list_build_s=g1["t_build"],
            force_loop_s=g1["t_force"], pairs=g1["pairs"],
            sample=f"{m} seeded particles' lists and forces, bins of {edge:g} sigma")
    finally:
        oracle.set_threads(threads)
    return main, detail


def copy_calibration(mib):
    """Five launches of torch's plain device copy of a known number of bytes."""
    import torch

    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 5}), flush=True)


PAIR_SOURCES = ("k_pair.hip", "dcm_device.hpp", "dcm_internal.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pair_slab_large_traffic.txt")


def pair_source_digest():
    import hashlib

    h = hashlib.sha256()
    for name in PAIR_SOURCES:
        with open(os.path.join(ROOT, "paper_1701_05242_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, prec_name):
    """HBM bytes per pair launch from the committed counter summary, or None.

    The summary holds FETCH_SIZE and WRITE_SIZE per dispatch of the pair
    kernel, each scaled by the same counter's reading for a plain copy of
    known size.  It applies only while the pair kernel's sources hash to the
    digest recorded with the counters, and only to the workload and precision
    they were taken on.
    """
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(" "))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if (kv.get("source_sha256") != pair_source_digest() or kv.get("workload") != workload
            or kv.get("precision") != prec_name):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the path is single-GPU by design", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1701_05242_amd as dcm
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prec = dcm.DCM_FP32_MIXED if args.prec == "fp32_mixed" else dcm.DCM_FP64
    if args.table1:
        print(json.dumps(table1_leg(args.steps, args.warmup, dev, prec)), flush=True)
        return
    s = workloads.make(args.workload)
    print(f"[bench] {s.name} n={s.n} box={s.box} rule={s.rule}", file=sys.stderr, flush=True)
    main_leg = run_leg(s, prec, args.steps, args.warmup, dev)
    print(f"[bench] main leg {json.dumps(main_leg)}", file=sys.stderr, flush=True)
    fp64_leg = None
    if not args.no_fp64 and prec != dcm.DCM_FP64:
        fp64_leg = run_leg(s, dcm.DCM_FP64, max(3, args.steps // 4), 1, dev)
        print(f"[bench] fp64 leg {json.dumps(fp64_leg)}", file=sys.stderr, flush=True)
    every10 = None
    if not args.no_fp64:
        every10 = run_leg(s, prec, args.steps, args.warmup, dev, redetect=10)
        print(f"[bench] re-detect every 10 {json.dumps(every10)}", file=sys.stderr, flush=True)
    batched = None
    if not args.no_batched:
        batched = batched_leg(args.steps, dev)
        print(f"[bench] batched {json.dumps(batched)}", file=sys.stderr, flush=True)
    vlist = None
    if not args.no_list:
        vlist = list_leg(s, dev)
        print(f"[bench] verlet list {json.dumps(vlist)}", file=sys.stderr, flush=True)
    n3 = None
    if not args.no_n3:
        n3 = n3_leg(s, dev)
        print(f"[bench] newton3 {json.dumps(n3)}", file=sys.stderr, flush=True)
    curved = None
    if not args.no_curved:
        curved = curved_leg(max(5, args.steps // 2), 2, dev)
    table1 = None
    if not args.no_table1:
        table1 = table1_leg(max(5, args.steps // 2), 2, dev, prec)
    cpu = cpu_detail = None
    if not args.no_cpu:
        cpu, cpu_detail = cpu_baseline(s, args.cpu_seconds)
        print(f"[bench] cpu {json.dumps(cpu)} {json.dumps(cpu_detail)}", file=sys.stderr,
              flush=True)
    achieved = main_leg["pair_kernel_tflops"]
    # the vector peak of the arithmetic the pair kernel computes in
    peak = VALU_PEAK_FP32 if prec == dcm.DCM_FP32_MIXED else VALU_PEAK_FP64
    line = {
        "metric": "DCM pair-interactions/s & force evals/s, FP32-mixed vs FP64, at rel err <=1e-5",
        "value": main_leg["pair_rate"],
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+f64" if prec == dcm.DCM_FP32_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": f"{s.name}: {s.box[0]:g}x{s.box[1]:g}x{s.box[2]:g} LJ slab, "
                               f"N={s.n}, rc {s.rule[0]:g}-{s.rule[1]:g}, full DCM step "
                               "(re-detect every step)",
                   "n_particles": s.n, "pairs_per_step": main_leg["pairs_per_step"],
                   "precision": args.prec, "tuned_cell_edge": main_leg["cell_len"]},
        "force_evals_per_s": main_leg["force_evals"],
        "stage_ms": main_leg["stage_ms"],
        "walk": main_leg["walk"],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic(s.name, args.prec)},
        "roofline_note": (f"pair kernel, {FLOP_PER_PAIR_FE} flop per interacting pair "
                          f"(force + energy), {main_leg['pairs_per_step']:.4g} pairs per launch, "
                          f"avg {main_leg['avg_pair_ms']:.3f} ms over "
                          f"{main_leg['pair_launches']} launches; against the {VALU_PEAK_FP64} "
                          f"TFLOP/s unpacked rate (the reachable one: packed FP32 is not "
                          f"used): {achieved / VALU_PEAK_FP64:.3f}"),
        "fp64": None if fp64_leg is None else {
            "value": fp64_leg["pair_rate"], "ms_per_step": fp64_leg["ms_per_step"],
            "force_evals_per_s": fp64_leg["force_evals"],
            "pair_kernel_ms": fp64_leg["avg_pair_ms"],
            "pair_kernel_tflops": fp64_leg["pair_kernel_tflops"]},
        "redetect_every_10": None if every10 is None else {
            "value": every10["pair_rate"], "ms_per_step": every10["ms_per_step"],
            "force_evals_per_s": every10["force_evals"]},
        "batched": batched,
        "verlet_list": vlist,
        "newton3": n3,
        "curved": curved,
        "table1": table1,
        "cpu_baseline": cpu,
        "cpu_baselines": cpu_detail,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
