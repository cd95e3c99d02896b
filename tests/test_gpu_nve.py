"""Velocity-Verlet NVE runs of the ~99k-particle slab (54 x 54 x 120 sigma,
40-sigma liquid slab): 100 steps at dt = 0.005 with re-detection every 10
steps, FP64 and FP32-mixed.

The oracle only ever sees the generator's inputs: the step-0 forces of both
precisions are checked against it.  Later checkpoints (steps 10, 50, 100)
compare the FP32-mixed forces with the FP64 GPU path evaluated at the same
positions -- the FP64 path is itself pinned to the oracle at 1e-12 -- and the
energy drift of the two precisions is compared step by step.  Under the
own-cutoff rule the forces are not the gradient of one energy, so the drift is
reported, not required to vanish."""
import json

import numpy as np
import pytest
import torch

import oracle
import paper_1701_05242_amd as dcm
import workloads
from gpu_util import DEV, F64, Ctx, dev, force_errors, host

pytestmark = pytest.mark.gpu

DT, EVERY = 0.005, 10
CHECKPOINTS = (10, 50, 100)


def run(s, prec):
    """Trajectory of one precision: forces, cutoffs and positions at each
    checkpoint, and the (potential, kinetic) energy after every step."""
    grid = dcm.make_grid(s.box, s.h)
    rule = dcm.make_rule(*s.rule)
    rcg = dcm.rc_grid_for(rule, grid)
    lj = dcm.make_lj()
    pos = [dev(a) for a in (s.x, s.y, s.z)]
    vel = [dev(a) for a in (s.vx, s.vy, s.vz)]
    f = [torch.zeros(s.n, **F64) for _ in range(3)]
    rc = torch.zeros(s.n, **F64)
    series = []
    snaps = {}
    with Ctx() as ctx:
        dcm.dcm_step(ctx, *pos, *vel, *f, s.box, lj, rule, grid, rcg, DT, 0, prec=prec, rc=rc)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
        snaps[0] = dict(F=np.stack([host(t) for t in f], 1), rc=host(rc),
                        x=[host(t) for t in pos])
        done = 0
        for stop in CHECKPOINTS:
            k = stop - done
            es = torch.zeros(2 * k, **F64)
            dcm.dcm_step(ctx, *pos, *vel, *f, s.box, lj, rule, grid, rcg, DT, k, prec=prec,
                         redetect_every=EVERY, step0=done, energy_series=es, rc=rc)
            assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
            series.append(host(es).reshape(k, 2))
            snaps[stop] = dict(F=np.stack([host(t) for t in f], 1), rc=host(rc),
                               x=[host(t) for t in pos])
            done = stop
    return snaps, np.concatenate(series)


def fp64_forces_at(s, x, rc):
    """FP64 GPU forces at given positions and cutoffs."""
    fx, fy, fz = (torch.zeros(s.n, **F64) for _ in range(3))
    with Ctx() as ctx:
        dcm.dcm_build_cells(ctx, *(dev(a) for a in x), dev(rc), s.box, 0.0, dcm.DCM_FP64,
                            rc_bound=s.rule[1])
        dcm.dcm_forces(ctx, dcm.make_lj(), fx, fy, fz, prec=dcm.DCM_FP64)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
    return np.stack([host(fx), host(fy), host(fz)], 1)


def test_config1_nve_fp32_mixed_vs_fp64():
    print("[gpu] config-1 NVE, 100 steps, FP64 and FP32-mixed", flush=True)
    s = workloads.make("slab_medium")
    s64, e64 = run(s, dcm.DCM_FP64)
    s32, e32 = run(s, dcm.DCM_FP32_MIXED)
    report = {"workload": f"{s.name} N={s.n}", "dt": DT, "redetect_every": EVERY}
    # step 0 against the oracle (its own cutoffs, generator positions)
    det = oracle.detect_interface(s.x, s.y, s.z, s.box, s.h)
    rcg = oracle.rc_grid_for(s.rule, det["hv"])
    D, _ = oracle.fsm(det["nv"], det["hv"], det["seg"], det["iface"], rcg)
    rc0 = oracle.cutoffs(oracle.particle_distance(s.x, s.y, s.z, s.box, det["nv"], D), s.rule)
    idx = workloads.sample_indices(s.n, 2048, seed=99)
    ref = oracle.forces(s.x, s.y, s.z, rc0, s.box, idx=idx)
    R0 = np.stack([ref["fx"], ref["fy"], ref["fz"]], 1)
    for tag, snaps, tol in (("fp64", s64, 1e-12), ("fp32_mixed", s32, 1e-5)):
        emax, erms = force_errors(snaps[0]["F"][idx], R0)
        report[f"step0_{tag}_vs_oracle"] = {"err_max": emax, "err_rms": erms}
        assert emax <= tol and erms <= tol, (tag, emax, erms)
    # later checkpoints: FP32-mixed against FP64 at the FP32-mixed positions
    for st in CHECKPOINTS:
        F64ref = fp64_forces_at(s, s32[st]["x"], s32[st]["rc"])
        emax, erms = force_errors(s32[st]["F"], F64ref)
        report[f"step{st}_fp32_mixed_vs_fp64"] = {"err_max": emax, "err_rms": erms}
        assert emax <= 1e-5 and erms <= 1e-5, (st, emax, erms)
    # energy: total = potential + kinetic after every step
    t64, t32 = e64.sum(1), e32.sum(1)
    e0 = t64[0]
    drift64 = (t64 - e0) / abs(e0)
    drift32 = (t32 - e0) / abs(e0)
    report["energy_drift_fp64"] = float(drift64[-1])
    report["energy_drift_fp32_mixed"] = float(drift32[-1])
    report["max_abs_drift_difference"] = float(np.max(np.abs(drift32 - drift64)))
    print("[gpu] NVE report " + json.dumps(report), flush=True)
    assert np.all(np.isfinite(t64)) and np.all(np.isfinite(t32))
    # the two precisions follow the same energy history
    assert report["max_abs_drift_difference"] <= 1e-5
