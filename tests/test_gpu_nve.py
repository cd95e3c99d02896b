"""Velocity-Verlet NVE runs of the ~99k-particle slab (54 x 54 x 120 sigma,
40-sigma liquid slab): 100 steps at dt = 0.005 with re-detection every 10
steps, FP64 and FP32-mixed.

The oracle only ever sees positions: the generator's at step 0, and at each
later checkpoint (steps 10, 50, 100) the FP32-mixed trajectory's own
positions, from which it redoes the whole path -- interface detection,
distances, cutoffs and force sums on a seeded sample -- so the checkpoint
errors measure the precision of the FP32-mixed forces, not the divergence of
two trajectories.  The FP32-mixed forces are also compared with the FP64 GPU
path at the same positions on every particle, and the energy drift of the two
precisions is compared step by step.  Under the own-cutoff rule the forces
are not the gradient of one energy, so the drift is reported, not required to
vanish."""
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
    # later checkpoints: the oracle's whole path at the FP32-mixed positions
    # (the field was re-detected at each checkpoint's own positions, since
    # every checkpoint is a multiple of the re-detection interval)
    for st in CHECKPOINTS:
        x = s32[st]["x"]
        det = oracle.detect_interface(*x, s.box, s.h)
        D, _ = oracle.fsm(det["nv"], det["hv"], det["seg"], det["iface"], rcg)
        rc_o = oracle.cutoffs(oracle.particle_distance(*x, s.box, det["nv"], D), s.rule)
        np.testing.assert_allclose(s32[st]["rc"], rc_o, rtol=1e-12, atol=0)
        idx = workloads.sample_indices(s.n, 2048, seed=100 + st)
        ref = oracle.forces(*x, rc_o, s.box, idx=idx)
        R = np.stack([ref["fx"], ref["fy"], ref["fz"]], 1)
        emax, erms, efloor = force_errors(s32[st]["F"][idx], R, detail=True)
        report[f"step{st}_fp32_mixed_vs_oracle"] = {"err_max": emax, "err_rms": erms,
                                                    "floored": efloor}
        assert emax <= 1e-5 and erms <= 1e-5, (st, emax, erms)
        # and every particle against the FP64 GPU path at the same positions
        F64ref = fp64_forces_at(s, x, s32[st]["rc"])
        emax, erms = force_errors(s32[st]["F"], F64ref)
        report[f"step{st}_fp32_mixed_vs_fp64_all"] = {"err_max": emax, "err_rms": erms}
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
