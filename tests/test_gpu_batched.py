"""Parity of the batched form (dcm_forces_batched) with the FP64 oracle and
with the single-system entry points.

Every system of a batch must get what dcm_build_cells + dcm_forces give it
alone -- bit for bit at the same cell edge -- and the oracle's O(N^2) sums
within the precision's tolerance (1e-12 FP64, 1e-5 FP32-mixed), with exact
neighbour counts.  The cutoffs fed to the GPU come from the oracle's own
interface/distance/cutoff steps or from the seeded generator, never from the
HIP path."""
import ctypes
import functools

import numpy as np
import pytest
import torch

import oracle
import paper_1701_05242_amd as dcm
import workloads
from gpu_util import DEV, F64, Ctx, dev, force_errors, gpu_forces, host, rel

pytestmark = pytest.mark.gpu

EV_ALL = dcm.DCM_EV_ENERGY | dcm.DCM_EV_VIRIAL | dcm.DCM_EV_COUNTS
TUNE_EDGES = (1.0, 1.15, 1.3, 1.5, 1.75)


@functools.lru_cache(maxsize=None)
def small_batch():
    return tuple(workloads.batched_systems(count=6, n_min=1500, n_max=12000))


@functools.lru_cache(maxsize=None)
def full_batch():
    return tuple(workloads.batched_systems())


@functools.lru_cache(maxsize=None)
def oracle_rc(kind, b):
    """DCM cutoffs of batch system b from the oracle's steps (Sections 2.1-2.2)."""
    s = (small_batch() if kind == "small" else full_batch())[b]
    det = oracle.detect_interface(s.x, s.y, s.z, s.box, s.h)
    rcg = oracle.rc_grid_for(s.rule, det["hv"])
    D, _ = oracle.fsm(det["nv"], det["hv"], det["seg"], det["iface"], rcg)
    return oracle.cutoffs(oracle.particle_distance(s.x, s.y, s.z, s.box, det["nv"], D), s.rule)


@functools.lru_cache(maxsize=None)
def oracle_forces(kind, b, rule):
    s = small_batch()[b]
    return oracle.forces(s.x, s.y, s.z, oracle_rc(kind, b), s.box, rule=rule)


def device_batch(systems, rcs, edge=0.0, bounds=None):
    out = []
    for k, (s, rc) in enumerate(zip(systems, rcs)):
        n = s.n
        out.append(dict(
            x=dev(s.x), y=dev(s.y), z=dev(s.z), rc=dev(rc),
            fx=torch.zeros(n, **F64), fy=torch.zeros(n, **F64), fz=torch.zeros(n, **F64),
            nnbr=torch.zeros(n, dtype=torch.int32, device=DEV),
            energy=torch.zeros(1, **F64), virial=torch.zeros(6, **F64),
            npairs=torch.zeros(1, dtype=torch.uint64, device=DEV),
            box=s.box, cell_edge=edge,
            rc_bound=(s.rule[1] if bounds is None else bounds[k])))
    return out


def results(d):
    F = np.stack([host(d["fx"]), host(d["fy"]), host(d["fz"])], 1)
    return dict(F=F, nnbr=host(d["nnbr"]), E=float(host(d["energy"])[0]), W=host(d["virial"]),
                npairs=int(host(d["npairs"])[0]))


def clear_outputs(batch):
    for d in batch:
        for k in ("fx", "fy", "fz", "nnbr", "energy", "virial", "npairs"):
            d[k].zero_()


@pytest.mark.parametrize("prec", [dcm.DCM_FP64, dcm.DCM_FP32_MIXED])
@pytest.mark.parametrize("rule", [dcm.DCM_PAIR_OWN, dcm.DCM_PAIR_MAX])
def test_batched_matches_oracle(rule, prec):
    print(f"[gpu] batched vs oracle rule={rule} prec={prec}", flush=True)
    systems = small_batch()
    rcs = [oracle_rc("small", b) for b in range(len(systems))]
    batch = device_batch(systems, rcs, edge=1.25)
    with Ctx() as ctx:
        dcm.dcm_forces_batched(ctx, batch, dcm.make_lj(), pair_rule=rule, prec=prec,
                               ev_flags=EV_ALL)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
    tol = 1e-12 if prec == dcm.DCM_FP64 else 1e-5
    for b, d in enumerate(batch):
        got = results(d)
        ref = oracle_forces("small", b, rule)
        R = np.stack([ref["fx"], ref["fy"], ref["fz"]], 1)
        np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
        assert got["npairs"] == int(ref["nnbr"].sum())
        emax, erms = force_errors(got["F"], R)
        assert emax <= tol and erms <= tol, (b, emax, erms)
        assert abs(got["E"] - ref["E"]) <= tol * abs(ref["E"])
        assert rel(got["W"], ref["W"]) <= tol


@pytest.mark.parametrize("lists", [14, 16])
def test_batched_row_lists_match_oracle(lists):
    """The compact-record batched kernel with each row-list size forced: the
    oracle's counts bit for bit, forces, energy and virial within 1e-5."""
    print(f"[gpu] batched row lists {lists}", flush=True)
    systems = small_batch()
    rcs = [oracle_rc("small", b) for b in range(len(systems))]
    batch = device_batch(systems, rcs, edge=1.25)
    with Ctx() as ctx:
        dcm.dcm_set_batched_row_lists(ctx, lists)
        dcm.dcm_forces_batched(ctx, batch, dcm.make_lj(), prec=dcm.DCM_FP32_MIXED,
                               ev_flags=EV_ALL)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
        assert dcm.dcm_batched_row_lists(ctx) == lists
    for b, d in enumerate(batch):
        got = results(d)
        ref = oracle_forces("small", b, dcm.DCM_PAIR_OWN)
        R = np.stack([ref["fx"], ref["fy"], ref["fz"]], 1)
        np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
        emax, erms = force_errors(got["F"], R)
        assert emax <= 1e-5 and erms <= 1e-5, (b, emax, erms)
        assert abs(got["E"] - ref["E"]) <= 1e-5 * abs(ref["E"])
        assert rel(got["W"], ref["W"]) <= 1e-5


@pytest.mark.parametrize("queues", [1, 8])
@pytest.mark.parametrize("prec", [dcm.DCM_FP64, dcm.DCM_FP32_MIXED])
@pytest.mark.parametrize("rule", [dcm.DCM_PAIR_OWN, dcm.DCM_PAIR_MAX])
def test_batched_bitwise_equals_single_system(rule, prec, queues):
    """Same cell edge => the batch reproduces every single-system result
    exactly (forces, counts, energy and virial sums), whichever work-queue
    layout drains it."""
    print(f"[gpu] batched vs single rule={rule} prec={prec} queues={queues}", flush=True)
    systems = small_batch()
    rcs = [workloads.uniform_cutoffs(s.n, s.rule[0], s.rule[1], seed=900 + b)
           for b, s in enumerate(systems)]
    batch = device_batch(systems, rcs, edge=1.1)
    with Ctx() as ctx:
        dcm.dcm_set_batched_queues(ctx, queues)
        dcm.dcm_forces_batched(ctx, batch, dcm.make_lj(), pair_rule=rule, prec=prec,
                               ev_flags=EV_ALL)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
        assert dcm.dcm_batched_queues(ctx) == queues
    for b, (s, rc, d) in enumerate(zip(systems, rcs, batch)):
        got = results(d)
        one = gpu_forces(s, rc, prec=prec, rule=rule, edge=1.1, rc_bound=s.rule[1])
        assert one["status"] == dcm.DCM_OK
        np.testing.assert_array_equal(got["F"], one["F"])
        np.testing.assert_array_equal(got["nnbr"], one["nnbr"])
        assert got["npairs"] == one["npairs"]
        assert got["E"] == one["E"]
        np.testing.assert_array_equal(got["W"], one["W"])


def test_batched_tuner_and_graph_replays():
    """Tuned edge + recorded graph: the first call tunes and records, every
    replay (with eager work and position updates between replays) equals an
    eager run of the same plan bit for bit, and the tuned result still meets
    the oracle."""
    print("[gpu] batched tuner + graph replays", flush=True)
    systems = small_batch()
    rcs = [oracle_rc("small", b) for b in range(len(systems))]
    batch = device_batch(systems, rcs, edge=0.0)
    prec = dcm.DCM_FP32_MIXED
    lj = dcm.make_lj()
    with Ctx() as ctx:
        arr = dcm.dcm_forces_batched(ctx, batch, lj, prec=prec, ev_flags=EV_ALL, use_graph=True)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
        edge = dcm.dcm_batched_edge(ctx)
        assert edge in TUNE_EDGES
        queues = dcm.dcm_batched_queues(ctx)
        assert queues in (1, 8)
        lists = dcm.dcm_batched_row_lists(ctx)
        assert lists in (14, 16)
        first = [results(d) for d in batch]
        for b, got in enumerate(first):
            ref = oracle_forces("small", b, dcm.DCM_PAIR_OWN)
            R = np.stack([ref["fx"], ref["fy"], ref["fz"]], 1)
            np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
            emax, erms = force_errors(got["F"], R)
            assert emax <= 1e-5 and erms <= 1e-5, (b, emax, erms)
        for rep in range(4):
            if rep:
                # move every particle a little (eager torch work between replays)
                for d in batch:
                    d["x"].add_(0.02 * torch.sin(d["y"] + rep))
                    d["z"].sub_(0.02 * torch.cos(d["x"] - rep))
            clear_outputs(batch)
            dcm.dcm_forces_batched(ctx, arr, lj, prec=prec, ev_flags=EV_ALL, use_graph=True)
            assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
            replay = [results(d) for d in batch]
            clear_outputs(batch)
            dcm.dcm_forces_batched(ctx, arr, lj, prec=prec, ev_flags=EV_ALL, use_graph=False)
            assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
            eager = [results(d) for d in batch]
            assert dcm.dcm_batched_edge(ctx) == edge
            assert dcm.dcm_batched_queues(ctx) == queues
            assert dcm.dcm_batched_row_lists(ctx) == lists
            for b, (g, e) in enumerate(zip(replay, eager)):
                np.testing.assert_array_equal(g["F"], e["F"])
                np.testing.assert_array_equal(g["nnbr"], e["nnbr"])
                assert g["E"] == e["E"] and g["npairs"] == e["npairs"], (rep, b)
                np.testing.assert_array_equal(g["W"], e["W"])


def test_batched_full_size_sampled():
    """64 systems of 2,000-200,000 particles (sum about 2.5 M), FP32-mixed,
    tuned edge, recorded graph: sampled particles against the oracle."""
    print("[gpu] batched full size", flush=True)
    systems = full_batch()
    rcs = [oracle_rc("full", b) for b in range(len(systems))]
    batch = device_batch(systems, rcs, edge=0.0)
    with Ctx() as ctx:
        dcm.dcm_forces_batched(ctx, batch, dcm.make_lj(), prec=dcm.DCM_FP32_MIXED,
                               ev_flags=EV_ALL, use_graph=True)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
    worst = 0.0
    for b, (s, rc, d) in enumerate(zip(systems, rcs, batch)):
        got = results(d)
        idx = workloads.sample_indices(s.n, 24, seed=4000 + b)
        ref = oracle.forces(s.x, s.y, s.z, rc, s.box, idx=idx)
        R = np.stack([ref["fx"], ref["fy"], ref["fz"]], 1)
        np.testing.assert_array_equal(got["nnbr"][idx], ref["nnbr"])
        assert got["npairs"] == int(got["nnbr"].astype(np.int64).sum())
        emax, _ = force_errors(got["F"][idx], R)
        worst = max(worst, emax)
        assert np.isfinite(got["E"]) and np.all(np.isfinite(got["W"]))
    assert worst <= 1e-5, worst


def test_batched_full_size_fp32_mixed_every_particle():
    """The 64-system batch in the benchmark's form (FP32-mixed, tuned edge,
    recorded graph) against the FP64 batch at the same edge, every particle
    of every system: force errors in units of each system's RMS force,
    identical neighbour counts, energy and virial within 1e-5."""
    print("[gpu] batched full size, FP32-mixed vs FP64 on every particle", flush=True)
    systems = full_batch()
    rcs = [oracle_rc("full", b) for b in range(len(systems))]
    b32 = device_batch(systems, rcs, edge=0.0)
    with Ctx() as ctx:
        dcm.dcm_forces_batched(ctx, b32, dcm.make_lj(), prec=dcm.DCM_FP32_MIXED,
                               ev_flags=EV_ALL, use_graph=True)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
        edge = dcm.dcm_batched_edge(ctx)
    b64 = device_batch(systems, rcs, edge=edge)
    with Ctx() as ctx:
        dcm.dcm_forces_batched(ctx, b64, dcm.make_lj(), prec=dcm.DCM_FP64, ev_flags=EV_ALL)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
    worst = [0.0, 0.0, 0.0]
    for b, (d32, d64) in enumerate(zip(b32, b64)):
        g32, g64 = results(d32), results(d64)
        np.testing.assert_array_equal(g32["nnbr"], g64["nnbr"])
        assert g32["npairs"] == g64["npairs"]
        errs = force_errors(g32["F"], g64["F"], detail=True)
        worst = [max(w, e) for w, e in zip(worst, errs)]
        assert max(errs) <= 1e-5, (b, errs)
        assert abs(g32["E"] - g64["E"]) <= 1e-5 * abs(g64["E"]), b
        assert rel(g32["W"], g64["W"]) <= 1e-5, b
    print(f"[gpu]   worst system: err_max={worst[0]:.3e} err_rms={worst[1]:.3e} "
          f"floored={worst[2]:.3e}", flush=True)


def test_batched_edge_cases():
    """Empty batch; empty, one- and two-particle systems next to a normal one;
    a cutoff above its system's bound; invalid descriptors."""
    print("[gpu] batched edge cases", flush=True)
    lj = dcm.make_lj()
    s = small_batch()[2]
    rng = np.random.default_rng(np.random.PCG64(77))
    tiny = []
    for n in (0, 1, 2, 5):
        pos = rng.uniform(0.0, 6.0, size=(3, n))
        tiny.append(workloads.System(name=f"tiny{n}", x=pos[0], y=pos[1], z=pos[2],
                                     vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n),
                                     box=(6.0, 6.0, 6.0), rule=(1.5, 2.9, 1.0)))
    systems = [tiny[0], s, tiny[1], tiny[2], tiny[3]]
    rcs = [workloads.uniform_cutoffs(t.n, t.rule[0], t.rule[1], seed=50 + k)
           for k, t in enumerate(systems)]
    with Ctx() as ctx:
        dcm.dcm_forces_batched(ctx, [], lj)
        batch = device_batch(systems, rcs, edge=0.0)
        dcm.dcm_forces_batched(ctx, batch, lj, ev_flags=EV_ALL)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
        for t, rc, d in zip(systems, rcs, batch):
            got = results(d)
            ref = oracle.forces(t.x, t.y, t.z, rc, t.box)
            np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
            assert got["npairs"] == int(ref["nnbr"].sum())
            if t.n:
                R = np.stack([ref["fx"], ref["fy"], ref["fz"]], 1)
                if np.any(R != 0.0):
                    emax, _ = force_errors(got["F"], R)
                    assert emax <= 1e-12
                else:
                    assert np.all(got["F"] == 0.0)
            else:
                assert got["E"] == 0.0 and got["npairs"] == 0
        # a cutoff above the declared bound is clamped and flagged
        bad = device_batch([s], [np.full(s.n, 5.0)], edge=1.25, bounds=[4.0])
        dcm.dcm_forces_batched(ctx, bad, lj)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_ERR_RANGE
        # invalid descriptors are refused before anything is enqueued
        arr = dcm.make_systems(device_batch([s], [rcs[1]], edge=1.25))
        arr[0].x = None
        with pytest.raises(dcm.DcmError) as err:
            dcm.dcm_forces_batched(ctx, arr, lj)
        assert err.value.code == dcm.DCM_ERR_INVALID
        arr = dcm.make_systems(device_batch([s], [rcs[1]], edge=1.25))
        arr[0].energy = None
        with pytest.raises(dcm.DcmError) as err:
            dcm.dcm_forces_batched(ctx, arr, lj, ev_flags=dcm.DCM_EV_ENERGY)
        assert err.value.code == dcm.DCM_ERR_INVALID
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK


@pytest.mark.parametrize("prec", [dcm.DCM_FP64, dcm.DCM_FP32_MIXED])
def test_batched_evaluation_flags_do_not_change_results(prec):
    """As for single systems: each system's forces do not depend on which
    outputs are asked for, and each output is the same bit for bit whichever
    others come with it (the compact-record kernel counts pairs only when
    asked)."""
    systems = small_batch()
    rcs = [oracle_rc("small", b) for b in range(len(systems))]
    E, V, C = dcm.DCM_EV_ENERGY, dcm.DCM_EV_VIRIAL, dcm.DCM_EV_COUNTS
    out = {}
    for flags in (0, E, E | C, EV_ALL):
        batch = device_batch(systems, rcs, edge=1.25)
        with Ctx() as ctx:
            dcm.dcm_forces_batched(ctx, batch, dcm.make_lj(), prec=prec, ev_flags=flags)
            assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
        out[flags] = [results(d) for d in batch]
    for flags, res in out.items():
        for r, full in zip(res, out[EV_ALL]):
            np.testing.assert_array_equal(r["F"], full["F"])
            if flags & E:
                assert r["E"] == full["E"]
            if flags & C:
                np.testing.assert_array_equal(r["nnbr"], full["nnbr"])
                assert r["npairs"] == full["npairs"] == int(full["nnbr"].sum())
