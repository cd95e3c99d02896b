"""Rule DCM_PAIR_MAX_N3: the symmetric rule evaluated once per pair with
Newton's third law (Section 2.4 and its footnotes on the trade-off), through
the C ABI.

Its reference is the oracle's rule MAX (r_ij <= max(rc_i, rc_j)): neighbour
counts bit for bit, forces, energy and virial within the precision's bar.
Against the GPU's own rule MAX: identical counts, forces and sums within
FP64 rounding (the reactions are summed with atomics, in no fixed order), and
a net force that vanishes.  Inputs: the seeded workloads with the oracle's
DCM cutoffs, and a seeded tiny box in which every axis wraps."""
import functools

import numpy as np
import pytest
import torch

import oracle
import paper_1701_05242_amd as dcm
import workloads
from gpu_util import DEV, F64, Ctx, dev, force_errors, gpu_forces, host, rel

pytestmark = pytest.mark.gpu

N3 = dcm.DCM_PAIR_MAX_N3


@functools.lru_cache(maxsize=None)
def ref_rc(name):
    s = workloads.make(name)
    det = oracle.detect_interface(s.x, s.y, s.z, s.box, s.h)
    rcg = oracle.rc_grid_for(s.rule, det["hv"])
    D, _ = oracle.fsm(det["nv"], det["hv"], det["seg"], det["iface"], rcg)
    delta = oracle.particle_distance(s.x, s.y, s.z, s.box, det["nv"], D)
    return oracle.cutoffs(delta, s.rule)


@functools.lru_cache(maxsize=None)
def ref_max(name):
    s = workloads.make(name)
    return oracle.forces(s.x, s.y, s.z, ref_rc(name), s.box, rule=dcm.DCM_PAIR_MAX)


def ref_F(r):
    return np.stack([r["fx"], r["fy"], r["fz"]], 1)


@pytest.mark.parametrize("name", ["slab_small", "slab_medium"])
@pytest.mark.parametrize("prec", [dcm.DCM_FP64, dcm.DCM_FP32_MIXED])
def test_n3_matches_the_oracle_max_rule(name, prec):
    print(f"[gpu] N3 forces {name} prec={prec}", flush=True)
    s = workloads.make(name)
    ref = ref_max(name)
    got = gpu_forces(s, ref_rc(name), prec=prec, rule=N3)
    assert got["status"] == dcm.DCM_OK
    np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
    assert got["npairs"] == int(ref["nnbr"].sum())
    tol = 1e-12 if prec == dcm.DCM_FP64 else 1e-5
    emax, erms = force_errors(got["F"], ref_F(ref))
    print(f"[gpu]   err_max={emax:.3e} err_rms={erms:.3e}", flush=True)
    assert emax <= tol and erms <= tol
    assert abs(got["E"] - ref["E"]) <= tol * abs(ref["E"])
    assert rel(got["W"], ref["W"]) <= tol


@pytest.mark.parametrize("edge", [0.0, 1.3, 2.9])
def test_n3_against_the_plain_max_rule(edge):
    s = workloads.make("slab_medium")
    rc = ref_rc("slab_medium")
    a = gpu_forces(s, rc, rule=dcm.DCM_PAIR_MAX, edge=edge)
    b = gpu_forces(s, rc, rule=N3, edge=edge)
    np.testing.assert_array_equal(a["nnbr"], b["nnbr"])
    assert a["npairs"] == b["npairs"]
    # the same FP64 pair terms summed in another order (reactions arrive by
    # atomics): the worst particle, whose force is ~60 F_rms, differs by a few
    # ulps of its own force, i.e. ~3e-13 F_rms -- within the FP64 bar
    emax, erms = force_errors(b["F"], a["F"])
    assert emax <= 1e-12 and erms <= 1e-13
    assert abs(a["E"] - b["E"]) <= 1e-13 * abs(a["E"])
    assert rel(b["W"], a["W"]) <= 1e-13
    # Newton's third law: the reactions cancel the actions
    F = b["F"]
    assert np.linalg.norm(F.sum(0)) <= 1e-12 * np.abs(F).sum()
    # energy, virial and counts come from fixed-order sums
    again = gpu_forces(s, rc, rule=N3, edge=edge)
    assert again["E"] == b["E"]
    np.testing.assert_array_equal(again["W"], b["W"])
    np.testing.assert_array_equal(again["nnbr"], b["nnbr"])


def test_n3_tiny_box_every_axis_wraps():
    rng = np.random.default_rng(11)
    box = (7.0, 7.5, 8.0)
    L = np.asarray(box)
    pts = []
    while len(pts) < 150:
        p = rng.uniform(0, 1, 3) * L
        if all(np.sum(((p - q) - L * np.rint((p - q) / L)) ** 2) > 0.81 for q in pts):
            pts.append(p)
    pts = np.asarray(pts)
    s = workloads.System("tiny", pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy(),
                         *(np.zeros(150) for _ in range(3)), box)
    # equal cutoffs exercise the tie between endpoints
    rc = np.where(rng.uniform(0, 1, 150) < 0.3, 2.5, rng.uniform(1.0, 3.45, 150))
    ref = oracle.forces(s.x, s.y, s.z, rc, box, rule=dcm.DCM_PAIR_MAX)
    for prec, tol in ((dcm.DCM_FP64, 1e-12), (dcm.DCM_FP32_MIXED, 1e-5)):
        for edge in (0.5, 1.0, 3.4):
            got = gpu_forces(s, rc, prec=prec, rule=N3, edge=edge)
            np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
            emax, _ = force_errors(got["F"], ref_F(ref))
            assert emax <= tol


def test_n3_in_dcm_step():
    s = workloads.make("slab_small")
    grid = dcm.make_grid(s.box, s.h)
    rule = dcm.make_rule(*s.rule)
    out = {}
    for pr in (dcm.DCM_PAIR_MAX, N3):
        pos = [dev(a) for a in (s.x, s.y, s.z)]
        vel = [dev(a) for a in (s.vx, s.vy, s.vz)]
        frc = [torch.zeros(s.n, **F64) for _ in range(3)]
        with Ctx() as ctx:
            dcm.dcm_step(ctx, *pos, *vel, *frc, s.box, dcm.make_lj(), rule, grid,
                         dcm.rc_grid_for(rule, grid), 0.005, 0, pair_rule=pr)
            dcm.dcm_step(ctx, *pos, *vel, *frc, s.box, dcm.make_lj(), rule, grid,
                         dcm.rc_grid_for(rule, grid), 0.005, 3, pair_rule=pr, redetect_every=2)
            assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
        out[pr] = np.stack([host(t) for t in pos + frc], 1)
    # three steps apart only by rounding
    assert np.max(np.abs(out[N3] - out[dcm.DCM_PAIR_MAX])) <= 1e-9


def test_n3_is_single_system_only():
    s = workloads.make("slab_small")
    rc = dev(ref_rc("slab_small"))
    d = dict(x=dev(s.x), y=dev(s.y), z=dev(s.z), rc=rc, fx=torch.zeros(s.n, **F64),
             fy=torch.zeros(s.n, **F64), fz=torch.zeros(s.n, **F64), box=s.box, cell_edge=1.3,
             rc_bound=s.rule[1])
    with Ctx() as ctx:
        with pytest.raises(dcm.DcmError):
            dcm.dcm_forces_batched(ctx, dcm.make_systems([d]), dcm.make_lj(), pair_rule=N3)
        with pytest.raises(dcm.DcmError):
            dcm.dcm_build_cells(ctx, d["x"], d["y"], d["z"], rc, s.box, 1.3, dcm.DCM_FP64,
                                rc_bound=s.rule[1])
            dcm.dcm_forces(ctx, dcm.make_lj(), d["fx"], d["fy"], d["fz"], pair_rule=3)


def test_n3_empty_system():
    z0 = torch.zeros(0, **F64)
    e = torch.zeros(1, **F64)
    with Ctx() as ctx:
        dcm.dcm_build_cells(ctx, z0, z0, z0, z0, (10.0, 10.0, 10.0), 1.0, dcm.DCM_FP64,
                            rc_bound=3.0)
        dcm.dcm_forces(ctx, dcm.make_lj(), z0, z0, z0, pair_rule=N3,
                       ev_flags=dcm.DCM_EV_ENERGY, energy=e)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
    assert float(host(e)[0]) == 0.0
