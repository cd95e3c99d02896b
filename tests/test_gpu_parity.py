"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Integer work (voxel counts, phase map, interface, threshold, cells, neighbour
counts) must match bit for bit.  FP64 results must agree within 1e-12
relative (forces normalised by the oracle's RMS force); FP32-mixed within
1e-5.  Each stage is fed the oracle's own input for that stage, so that an
upstream rounding difference cannot perturb a downstream decision; the
end-to-end tests then chain the whole path."""
import functools

import numpy as np
import pytest
import torch

import oracle
import paper_1701_05242_amd as dcm
import workloads
from gpu_util import DEV, F64, Ctx, dev, force_errors, gpu_forces, host, rel

pytestmark = pytest.mark.gpu

SMALL = ["slab_small", "slab_medium"]
GRIDS = ["slab_small", "slab_medium", "droplet", "cylinder", "slab_large"]


@functools.lru_cache(maxsize=None)
def ref_detect(name):
    s = workloads.make(name)
    det = oracle.detect_interface(s.x, s.y, s.z, s.box, s.h)
    rcg = oracle.rc_grid_for(s.rule, det["hv"])
    D, passes = oracle.fsm(det["nv"], det["hv"], det["seg"], det["iface"], rcg)
    delta = oracle.particle_distance(s.x, s.y, s.z, s.box, det["nv"], D)
    rc = oracle.cutoffs(delta, s.rule)
    return dict(det, D=D, fsm_passes=passes, rc_grid=rcg, delta=delta, rc=rc)


@functools.lru_cache(maxsize=None)
def ref_forces(name, rule, idx_step=1):
    s = workloads.make(name)
    r = ref_detect(name)
    idx = None if idx_step == 1 else np.arange(0, s.n, idx_step)
    return oracle.forces(s.x, s.y, s.z, r["rc"], s.box, rule=rule, idx=idx)


def _ref_F(f):
    return np.stack([f["fx"], f["fy"], f["fz"]], 1)


# ------------------------------------------------------------------ grid

@pytest.mark.parametrize("name", GRIDS)
def test_detect_interface_bit_exact(name):
    print(f"[gpu] detect {name}", flush=True)
    s = workloads.make(name)
    ref = ref_detect(name)
    grid = dcm.make_grid(s.box, s.h)
    nv = dcm.grid_voxels(grid)
    assert list(grid.n) == list(ref["nv"])
    counts = torch.zeros(nv, dtype=torch.uint32, device=DEV)
    seg = torch.zeros(nv, dtype=torch.uint8, device=DEV)
    iface = torch.zeros(nv, dtype=torch.uint8, device=DEV)
    thr = torch.zeros(1, dtype=torch.int32, device=DEV)
    with Ctx() as ctx:
        dcm.dcm_detect_interface(ctx, dev(s.x), dev(s.y), dev(s.z), s.box, grid, seg, iface,
                                 counts=counts, threshold_out=thr)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
    np.testing.assert_array_equal(host(counts), ref["counts"])
    assert int(host(thr)[0]) == ref["threshold"]
    np.testing.assert_array_equal(host(seg), ref["seg"])
    np.testing.assert_array_equal(host(iface), ref["iface"])


def test_detect_fixed_split_and_degenerate_flag():
    s = workloads.make("slab_small")
    grid = dcm.make_grid(s.box, s.h)
    nv = dcm.grid_voxels(grid)
    seg = torch.zeros(nv, dtype=torch.uint8, device=DEV)
    iface = torch.zeros(nv, dtype=torch.uint8, device=DEV)
    ref = oracle.detect_interface(s.x, s.y, s.z, s.box, s.h, split=9.5)
    with Ctx() as ctx:
        dcm.dcm_detect_interface(ctx, dev(s.x), dev(s.y), dev(s.z), s.box, grid, seg, iface,
                                 split=9.5)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
    np.testing.assert_array_equal(host(seg), ref["seg"])
    np.testing.assert_array_equal(host(iface), ref["iface"])
    # only the liquid slab: one phase, flagged, everything high density
    liq = s.z < 40.0
    liq &= s.z >= 20.0
    x, y, z = s.x[liq], s.y[liq], s.z[liq] - 20.0
    box = (13.4, 13.4, 20.0)
    g2 = dcm.make_grid(box, 1.0)
    nv2 = dcm.grid_voxels(g2)
    seg = torch.zeros(nv2, dtype=torch.uint8, device=DEV)
    iface = torch.zeros(nv2, dtype=torch.uint8, device=DEV)
    ref = oracle.detect_interface(x, y, z, box, 1.0)
    assert ref["degenerate"]
    with Ctx() as ctx:
        dcm.dcm_detect_interface(ctx, dev(x), dev(y), dev(z), box, g2, seg, iface)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_ERR_DEGENERATE
    np.testing.assert_array_equal(host(seg), ref["seg"])
    assert host(iface).sum() == 0


def thin_layer_system(box, seed):
    """A dense layer (density 0.8, z in [0.3, 0.6) of the box) in a gas of
    density 0.05, uniform random positions."""
    rng = np.random.default_rng(seed)
    L = np.asarray(box, dtype=float)
    dense = rng.uniform(0, 1, (int(0.8 * 0.3 * L.prod()), 3)) * [L[0], L[1], 0.3 * L[2]]
    dense[:, 2] += 0.3 * L[2]
    gas = rng.uniform(0, 1, (int(0.05 * L.prod()), 3)) * L
    P = np.concatenate([dense, gas])
    return P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy()


# (1, 70, 9) and (70, 2, 33) voxels: the 27-window wraps onto the same voxels;
# (130, 6, 65): x not a multiple of the 64-voxel column, z a partial chunk
@pytest.mark.parametrize("box", [(3.0, 5.0, 40.0), (1.2, 70.0, 9.0), (70.0, 2.4, 33.0),
                                 (130.0, 6.0, 65.0)])
def test_detect_on_thin_and_ragged_grids(box):
    print(f"[gpu] detect on a thin or ragged grid {box}", flush=True)
    x, y, z = thin_layer_system(box, int(sum(box) * 10))
    ref = oracle.detect_interface(x, y, z, box, 1.0)
    grid = dcm.make_grid(box, 1.0)
    nv = dcm.grid_voxels(grid)
    assert list(grid.n) == list(ref["nv"])
    counts = torch.zeros(nv, dtype=torch.uint32, device=DEV)
    seg = torch.zeros(nv, dtype=torch.uint8, device=DEV)
    iface = torch.zeros(nv, dtype=torch.uint8, device=DEV)
    thr = torch.zeros(1, dtype=torch.int32, device=DEV)
    with Ctx() as ctx:
        dcm.dcm_detect_interface(ctx, dev(x), dev(y), dev(z), box, grid, seg, iface,
                                 counts=counts, threshold_out=thr)
        code = dcm.dcm_sync_status(ctx)
    assert code == (dcm.DCM_ERR_DEGENERATE if ref["degenerate"] else dcm.DCM_OK)
    np.testing.assert_array_equal(host(counts), ref["counts"])
    assert int(host(thr)[0]) == ref["threshold"]
    np.testing.assert_array_equal(host(seg), ref["seg"])
    np.testing.assert_array_equal(host(iface), ref["iface"])


@pytest.mark.parametrize("name", GRIDS)
def test_sweep_distance_matches_fsm(name):
    print(f"[gpu] sweep {name}", flush=True)
    s = workloads.make(name)
    ref = ref_detect(name)
    grid = dcm.make_grid(s.box, s.h)
    nv = dcm.grid_voxels(grid)
    dist = torch.zeros(nv, **F64)
    waves = torch.zeros(1, dtype=torch.int32, device=DEV)
    with Ctx() as ctx:
        dcm.dcm_sweep_distance(ctx, dev(ref["seg"], torch.uint8), dev(ref["iface"], torch.uint8),
                               grid, ref["rc_grid"], 200, dist, waves_out=waves)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
    D = host(dist)
    assert np.max(np.abs(D - ref["D"])) <= 1e-12 * ref["rc_grid"]
    assert int(host(waves)[0]) >= 2


def test_sweep_wave_limit_is_reported():
    s = workloads.make("slab_small")
    ref = ref_detect("slab_small")
    grid = dcm.make_grid(s.box, s.h)
    dist = torch.zeros(dcm.grid_voxels(grid), **F64)
    with Ctx() as ctx:
        dcm.dcm_sweep_distance(ctx, dev(ref["seg"], torch.uint8), dev(ref["iface"], torch.uint8),
                               grid, ref["rc_grid"], 2, dist)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_ERR_NOT_CONVERGED


@pytest.mark.parametrize("name", GRIDS)
def test_assign_cutoffs_bit_exact(name):
    s = workloads.make(name)
    ref = ref_detect(name)
    grid = dcm.make_grid(s.box, s.h)
    delta = torch.zeros(s.n, **F64)
    rc = torch.zeros(s.n, **F64)
    with Ctx() as ctx:
        dcm.dcm_assign_cutoffs(ctx, dev(s.x), dev(s.y), dev(s.z), s.box, grid, dev(ref["D"]),
                               dcm.make_rule(*s.rule), rc, delta=delta)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
    np.testing.assert_array_equal(host(delta), ref["delta"])
    np.testing.assert_array_equal(host(rc), ref["rc"])


# ------------------------------------------------------------------ cells

@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("edge", [0.9, 1.3, 2.5, 6.1])
def test_build_cells_bit_exact(name, edge):
    s = workloads.make(name)
    ref = ref_detect(name)
    nc = oracle.cell_dims(s.box, edge)
    ref_of, ref_start = oracle.cells(s.x, s.y, s.z, s.box, nc)
    cell_of = torch.zeros(s.n, dtype=torch.int32, device=DEV)
    start = torch.zeros(int(np.prod(nc)) + 1, dtype=torch.int32, device=DEV)
    with Ctx() as ctx:
        dcm.dcm_build_cells(ctx, dev(s.x), dev(s.y), dev(s.z), dev(ref["rc"]), s.box, edge,
                            dcm.DCM_FP64, cell_of=cell_of, cell_start=start)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
        dims, _ = dcm.dcm_cell_dims(ctx)
    assert dims == list(nc)
    np.testing.assert_array_equal(host(cell_of), ref_of)
    np.testing.assert_array_equal(host(start), ref_start)


# ------------------------------------------------------------------ forces

@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("rule", [dcm.DCM_PAIR_OWN, dcm.DCM_PAIR_MAX])
@pytest.mark.parametrize("prec", [dcm.DCM_FP64, dcm.DCM_FP32_MIXED])
def test_forces_match_oracle(name, rule, prec):
    print(f"[gpu] forces {name} rule={rule} prec={prec}", flush=True)
    s = workloads.make(name)
    ref = ref_forces(name, rule)
    got = gpu_forces(s, ref_detect(name)["rc"], prec=prec, rule=rule)
    assert got["status"] == dcm.DCM_OK
    np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
    assert got["npairs"] == int(ref["nnbr"].sum())
    tol = 1e-12 if prec == dcm.DCM_FP64 else 1e-5
    emax, erms, efloor = force_errors(got["F"], _ref_F(ref), detail=True)
    print(f"[gpu]   err_max={emax:.3e} err_rms={erms:.3e} floored={efloor:.3e}", flush=True)
    assert emax <= tol and erms <= tol and efloor <= tol
    assert abs(got["E"] - ref["E"]) <= tol * abs(ref["E"])
    assert rel(got["W"], ref["W"]) <= tol


def corner_blob(shift=0.0):
    """A dense cube of 1,000 particles (jittered unit lattice) centred on the
    corner of a 40-sigma periodic box: every particle lies within the ghost
    halo of all three axes, so each has seven periodic images -- far more
    than a uniform-density estimate of the ghost count allows."""
    rng = np.random.default_rng(np.random.PCG64(2024))
    g = np.arange(10) - 4.5
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pts = pts + rng.uniform(-0.1, 0.1, pts.shape) + shift
    pts = np.mod(pts, 40.0)
    n = len(pts)
    z0 = np.zeros(n)
    return workloads.System(name="corner_blob", x=pts[:, 0].copy(), y=pts[:, 1].copy(),
                            z=pts[:, 2].copy(), vx=z0, vy=z0, vz=z0, box=(40.0, 40.0, 40.0),
                            rule=(3.0, 3.0, 1.0))


@pytest.mark.parametrize("prec", [dcm.DCM_FP64, dcm.DCM_FP32_MIXED])
def test_ghost_images_of_a_dense_corner(prec):
    """The ghost-image buffer is sized from the build's exact image count
    (about 8 N here), both on a context's first build and on a later build of
    the same geometry after the particles moved: no overflow, forces and
    counts as the oracle's."""
    print(f"[gpu] dense periodic corner prec={prec}", flush=True)
    tol = 1e-12 if prec == dcm.DCM_FP64 else 1e-5
    lj = dcm.make_lj()
    with Ctx() as ctx:
        for shift in (0.0, 0.3):
            s = corner_blob(shift)
            rc = np.full(s.n, 3.0)
            fx, fy, fz = (torch.zeros(s.n, **F64) for _ in range(3))
            nn = torch.zeros(s.n, dtype=torch.int32, device=DEV)
            dcm.dcm_build_cells(ctx, dev(s.x), dev(s.y), dev(s.z), dev(rc), s.box, 1.25, prec,
                                rc_bound=3.0)
            dcm.dcm_forces(ctx, lj, fx, fy, fz, prec=prec, ev_flags=dcm.DCM_EV_COUNTS, nnbr=nn)
            assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
            ref = oracle.forces(s.x, s.y, s.z, rc, s.box)
            np.testing.assert_array_equal(host(nn), ref["nnbr"])
            F = np.stack([host(fx), host(fy), host(fz)], 1)
            emax, erms = force_errors(F, _ref_F(ref))
            assert emax <= tol and erms <= tol, (shift, emax, erms)


def crowded_centres():
    """Dilute gas (density 0.05) holding a few tight clusters: a centre with
    eight neighbours at the corners of a cube, all 0.95-1.05 sigma away (more
    close pairs in reach than the compact-record queue holds), plus a pair
    at 0.9 sigma."""
    rng = np.random.default_rng(np.random.PCG64(31))
    L = 18.0
    pts = [rng.uniform(0.0, L, (int(0.05 * L ** 3), 3))]
    corners = np.array([[a, b, c] for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)], float)
    for centre in ((4.0, 4.0, 4.0), (13.0, 5.0, 11.0), (9.0, 14.0, 6.0)):
        c = np.asarray(centre)
        r = rng.uniform(0.95, 1.05, (8, 1))
        pts.append(c[None, :])
        pts.append(c + corners / np.sqrt(3.0) * r)
    pts.append(np.array([[15.0, 15.0, 15.0], [15.9, 15.0, 15.0]]))
    pts = np.concatenate(pts)
    # keep the gas away from the clusters (at least 1.2 sigma)
    clusters = pts[int(0.05 * L ** 3):]
    gas = pts[:int(0.05 * L ** 3)]
    d = gas[:, None, :] - clusters[None, :, :]
    d -= L * np.rint(d / L)
    gas = gas[np.min(np.linalg.norm(d, axis=2), axis=1) > 1.2]
    keep = []
    for p in gas:  # and from each other (at least 0.9 sigma)
        if keep:
            e = np.asarray(keep) - p
            e -= L * np.rint(e / L)
            if np.min(np.linalg.norm(e, axis=1)) < 0.9:
                continue
        keep.append(p)
    pts = np.mod(np.concatenate([np.asarray(keep), clusters]), L)
    n = len(pts)
    z0 = np.zeros(n)
    return workloads.System(name="crowded", x=pts[:, 0].copy(), y=pts[:, 1].copy(),
                            z=pts[:, 2].copy(), vx=z0, vy=z0, vz=z0, box=(L, L, L),
                            rule=(2.5, 6.0, 5.0))


@pytest.mark.parametrize("edge", [0.9, 1.25, 2.0])
def test_fp32_mixed_many_close_pairs(edge):
    """Particles with more close pairs than the compact-record kernel queues
    (they start over on the FP64 records) next to ordinary ones: counts bit
    for bit and forces within the FP32-mixed bar against the oracle."""
    print(f"[gpu] crowded close pairs edge={edge}", flush=True)
    s = crowded_centres()
    rc = workloads.uniform_cutoffs(s.n, 2.5, 6.0, seed=37)
    got = gpu_forces(s, rc, prec=dcm.DCM_FP32_MIXED, edge=edge, rc_bound=6.0)
    assert got["status"] == dcm.DCM_OK
    ref = oracle.forces(s.x, s.y, s.z, rc, s.box)
    np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
    emax, erms, efloor = force_errors(got["F"], _ref_F(ref), detail=True)
    assert emax <= 1e-5 and erms <= 1e-5 and efloor <= 1e-5, (emax, erms)
    assert abs(got["E"] - ref["E"]) <= 1e-5 * abs(ref["E"])
    assert rel(got["W"], ref["W"]) <= 1e-5


@pytest.mark.parametrize("edge", [0.9, 1.3, 2.0])
def test_walk_stats_bracket_the_candidates(edge):
    """dcm_walk_stats after a pair-count pass: every interacting pair is among
    the candidates the walk tested, and no candidate lies outside the particle's
    box of half-width r_c + one cell edge (the rows reach one cell past the
    search sphere at most; brute force over that box with a periodic KD-tree).
    Both precisions walk the same rows and candidates: the compact records
    change only the arithmetic.  Each particle visits at least one row."""
    from scipy.spatial import cKDTree
    print(f"[gpu] walk stats edge={edge}", flush=True)
    s = workloads.make("slab_medium")
    rc = ref_detect("slab_medium")["rc"]
    g64 = gpu_forces(s, rc, prec=dcm.DCM_FP64, edge=edge, rc_bound=s.rule[1])
    g32 = gpu_forces(s, rc, prec=dcm.DCM_FP32_MIXED, edge=edge, rc_bound=s.rule[1])
    assert g64["status"] == dcm.DCM_OK and g32["status"] == dcm.DCM_OK
    cand, rows = g64["walk"]
    assert g32["walk"] == g64["walk"]
    assert cand >= g64["npairs"] and rows >= s.n
    length = max(g64["dims"][1])
    pts = np.mod(np.stack([s.x, s.y, s.z], 1), np.array(s.box))
    tree = cKDTree(pts, boxsize=np.array(s.box))
    # (1e-3: above the walk's 4e-6 (R + len) row-selection guard)
    box = tree.query_ball_point(pts, rc + length + 1e-3, p=np.inf, return_length=True)
    assert cand <= int(np.sum(box)) - s.n
    print(f"[gpu]   candidates/pair {cand / g64['npairs']:.3f}, rows/particle {rows / s.n:.1f}, "
          f"box bound/pair {(np.sum(box) - s.n) / g64['npairs']:.3f}", flush=True)


@pytest.mark.parametrize("prec", [dcm.DCM_FP64, dcm.DCM_FP32_MIXED])
def test_tuned_cell_edge(prec):
    """cell_edge < 0: the edge is one of the tuner's candidates (fractions of
    the smallest cutoff, at most 2 sigma for FP32-mixed), the same on a second
    context, and the forces are the oracle's."""
    print(f"[gpu] tuned cell edge prec={prec}", flush=True)
    s = workloads.make("slab_medium")
    rc = ref_detect("slab_medium")["rc"]
    r_ref = float(np.min(rc))
    top = min(L / np.ceil(L / 2.0) for L in s.box) if prec == dcm.DCM_FP32_MIXED else 1e9
    cands = sorted({min(f * r_ref, top) for f in (1.0 / 3.0, 0.4, 0.5, 0.6, 0.7, 0.8)})
    got = gpu_forces(s, rc, prec=prec, edge=-1.0, rc_bound=s.rule[1])
    again = gpu_forces(s, rc, prec=prec, edge=-1.0, rc_bound=s.rule[1])
    dims = got["dims"]
    edge_used = [s.box[a] / dims[0][a] for a in range(3)]
    assert any(all(int(np.floor(s.box[a] / c)) == dims[0][a] for a in range(3)) for c in cands), \
        (dims, cands, edge_used)
    assert again["dims"][0] == dims[0]
    np.testing.assert_array_equal(again["F"], got["F"])
    ref = ref_forces("slab_medium", dcm.DCM_PAIR_OWN)
    np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
    tol = 1e-12 if prec == dcm.DCM_FP64 else 1e-5
    emax, erms = force_errors(got["F"], _ref_F(ref))
    assert emax <= tol and erms <= tol


# 7.0: one cell across x and y (13.4 sigma), so the halo of two cells is
# wider than the grid and the ghost rows wrap the box more than once
@pytest.mark.parametrize("edge", [0.0, 0.7, 1.9, 3.3, 7.0])
def test_forces_independent_of_cell_edge_and_deterministic(edge):
    s = workloads.make("slab_small")
    rc = ref_detect("slab_small")["rc"]
    base = gpu_forces(s, rc, edge=1.3)
    got = gpu_forces(s, rc, edge=edge)
    np.testing.assert_array_equal(got["nnbr"], base["nnbr"])
    emax, _ = force_errors(got["F"], base["F"])
    assert emax <= 1e-13
    again = gpu_forces(s, rc, edge=edge)
    np.testing.assert_array_equal(again["F"], got["F"])
    assert again["E"] == got["E"]


@pytest.mark.parametrize("prec", [dcm.DCM_FP64, dcm.DCM_FP32_MIXED])
def test_evaluation_flags_do_not_change_results(prec):
    """Pair counts, energy and virial are optional outputs: the compact-record
    kernel counts pairs only when asked, and an energy-only call reduces only
    the energy.  Forces must not depend on which outputs are asked for, and
    each output must be the same bit for bit whichever others come with it."""
    s = workloads.make("slab_medium")
    rc = ref_detect("slab_medium")["rc"]
    x, y, z, r = dev(s.x), dev(s.y), dev(s.z), dev(rc)
    E, V, C = dcm.DCM_EV_ENERGY, dcm.DCM_EV_VIRIAL, dcm.DCM_EV_COUNTS
    out = {}
    with Ctx() as ctx:
        # 1.25-sigma cells: FP32-mixed runs the compact-record kernel
        dcm.dcm_build_cells(ctx, x, y, z, r, s.box, 1.25, prec, rc_bound=s.rule[1])
        for flags in (0, E, E | V, E | C, V | C, E | V | C):
            f = [torch.zeros(s.n, **F64) for _ in range(3)]
            e = torch.zeros(1, **F64)
            w = torch.zeros(6, **F64)
            nn = torch.zeros(s.n, dtype=torch.int32, device=DEV)
            npairs = torch.zeros(1, dtype=torch.uint64, device=DEV)
            dcm.dcm_forces(ctx, dcm.make_lj(), *f, prec=prec, ev_flags=flags, energy=e, virial=w,
                           nnbr=nn, npairs=npairs)
            assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
            out[flags] = (np.stack([host(t) for t in f], 1), float(host(e)[0]), host(w),
                          host(nn), int(host(npairs)[0]))
    full = out[E | V | C]
    for flags, (F, e, w, nn, npairs) in out.items():
        np.testing.assert_array_equal(F, full[0])
        if flags & E:
            assert e == full[1]
        if flags & V:
            np.testing.assert_array_equal(w, full[2])
        if flags & C:
            np.testing.assert_array_equal(nn, full[3])
            assert npairs == full[4] == int(full[3].sum())


def test_tiny_box_every_axis_wraps():
    """A box smaller than the cutoff stencil: every cell is visited once and the
    minimum image is taken per pair."""
    rng = np.random.default_rng(5)
    box = (7.0, 7.5, 8.0)
    pts = []
    while len(pts) < 150:
        p = rng.uniform(0, 1, 3) * np.asarray(box)
        if all(np.sum(((p - q) - np.asarray(box) * np.rint((p - q) / np.asarray(box))) ** 2) > 0.81
               for q in pts):
            pts.append(p)
    pts = np.asarray(pts)
    s = workloads.System("tiny", pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy(),
                         *(np.zeros(150) for _ in range(3)), box)
    rc = rng.uniform(1.0, 3.45, 150)
    for rule in (dcm.DCM_PAIR_OWN, dcm.DCM_PAIR_MAX):
        ref = oracle.forces(s.x, s.y, s.z, rc, box, rule=rule)
        for edge in (0.5, 1.0, 3.4):
            got = gpu_forces(s, rc, rule=rule, edge=edge)
            np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
            emax, _ = force_errors(got["F"], _ref_F(ref))
            assert emax <= 1e-12


def cutoff_boundary_system(seed):
    """Centres on a grid (spacing 10) with cutoffs in [2.5, 3.5], each with two
    partners at distance rc_i (1 -/+ eps) for eps from 1e-13 to 1e-5 (partner
    cutoff 0.5, so only the centre's decision counts).  The smallest eps lie
    inside the undecidable band of the FP32-mixed compact records and must be
    settled by the exact pass; the largest are decided from the records."""
    rng = np.random.default_rng(seed)
    box = (60.0, 60.0, 60.0)
    g = np.arange(6) * 10.0 + 5.0
    C = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    C = C + rng.uniform(-0.5, 0.5, C.shape)
    m = len(C)
    rcc = rng.uniform(2.5, 3.5, m)
    eps = np.array([1e-13, 1e-11, 1e-9, 1e-7, 1e-5])[rng.integers(0, 5, m)]
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    # the two partners on opposite sides of their centre
    P = [C] + [C + (sign * rcc * (1.0 + sign * eps))[:, None] * u for sign in (-1.0, 1.0)]
    X = np.concatenate(P)
    rc = np.concatenate([rcc, np.full(2 * m, 0.5)])
    sysm = workloads.System("boundary", X[:, 0].copy(), X[:, 1].copy(), X[:, 2].copy(),
                            *(np.zeros(len(X)) for _ in range(3)), box)
    return sysm, rc


def test_fp32_mixed_pairs_at_the_cutoff():
    print("[gpu] FP32-mixed pairs within 1e-13..1e-5 of the cutoff", flush=True)
    s, rc = cutoff_boundary_system(11)
    ref = oracle.forces(s.x, s.y, s.z, rc, s.box)
    m = s.n // 3
    # each centre sees exactly its inner partner
    assert np.all(ref["nnbr"][:m] == 1) and np.all(ref["nnbr"][m:] == 0)
    for edge in (0.9, 1.25, 3.6):
        got = gpu_forces(s, rc, prec=dcm.DCM_FP32_MIXED, edge=edge, rc_bound=3.5)
        assert got["status"] == dcm.DCM_OK
        np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
        emax, erms = force_errors(got["F"], _ref_F(ref))
        assert emax <= 1e-5 and erms <= 1e-5, (edge, emax, erms)
    # the batched form: two such systems in one pass
    s2, rc2 = cutoff_boundary_system(12)
    ref2 = oracle.forces(s2.x, s2.y, s2.z, rc2, s2.box)
    batch = []
    for t, r in ((s, rc), (s2, rc2)):
        batch.append(dict(
            x=dev(t.x), y=dev(t.y), z=dev(t.z), rc=dev(r),
            fx=torch.zeros(t.n, **F64), fy=torch.zeros(t.n, **F64), fz=torch.zeros(t.n, **F64),
            nnbr=torch.zeros(t.n, dtype=torch.int32, device=DEV),
            energy=torch.zeros(1, **F64), virial=torch.zeros(6, **F64),
            npairs=torch.zeros(1, dtype=torch.uint64, device=DEV),
            box=t.box, cell_edge=1.25, rc_bound=3.5))
    with Ctx() as ctx:
        dcm.dcm_forces_batched(ctx, batch, dcm.make_lj(), prec=dcm.DCM_FP32_MIXED,
                               ev_flags=dcm.DCM_EV_COUNTS)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
    for d, r in zip(batch, (ref, ref2)):
        np.testing.assert_array_equal(host(d["nnbr"]), r["nnbr"])
        F = np.stack([host(d["fx"]), host(d["fy"]), host(d["fz"])], 1)
        emax, erms = force_errors(F, _ref_F(r))
        assert emax <= 1e-5 and erms <= 1e-5


def dense_rod_system(seed):
    """A 120 x 80 x 40 sigma rod of the workloads' liquid (FCC at density 0.8,
    each site jittered by U(-0.05, 0.05)) filling two rows of 40-sigma cells of
    a 120^3 box, cutoff 8."""
    rng = np.random.default_rng(seed)
    ext = np.array([120.0, 80.0, 40.0])
    n = np.rint(ext / (4.0 / 0.8) ** (1.0 / 3.0)).astype(int)
    a = ext / n
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]) + 0.25
    c = np.stack(np.meshgrid(*(np.arange(k) for k in n), indexing="ij"), -1).reshape(-1, 1, 3)
    P = ((c + basis[None]) * a).reshape(-1, 3)
    P += rng.uniform(-0.05, 0.05, P.shape)
    z0 = np.zeros(len(P))
    s = workloads.System("rod", P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy(), z0, z0, z0,
                         (120.0, 120.0, 120.0))
    return s, np.full(s.n, 8.0)


def test_forty_sigma_cells_and_rows_of_100k_candidates():
    """Cells 40 sigma wide: a lane near both a y and an x cell boundary scans
    the other cell row of the rod across two x cells, ~100 K candidates in one
    row.  Compact FP32 records would be too coarse at this cell size, so
    FP32-mixed forces read the FP64 records and must still meet 1e-5."""
    print("[gpu] dense rod in 40-sigma cells", flush=True)
    s, rc = dense_rod_system(21)
    cell = 40.0
    # the other row's particles in two x cells number more than 65535
    other = (s.y >= cell) & (s.x < 2 * cell)
    assert other.sum() > 65535
    to_xb = np.abs(((s.x + cell / 2) % cell) - cell / 2)
    near = np.flatnonzero((to_xb < 7.0) & (s.y > cell - 7.0) & (s.y < cell))[::97]
    idx = np.unique(np.concatenate([workloads.sample_indices(s.n, 128, seed=21), near]))
    ref = oracle.forces(s.x, s.y, s.z, rc, s.box, idx=idx)
    full = {}
    for prec, tol in ((dcm.DCM_FP64, 1e-12), (dcm.DCM_FP32_MIXED, 1e-5)):
        got = gpu_forces(s, rc, prec=prec, edge=40.0, rc_bound=8.0)
        assert got["status"] == dcm.DCM_OK
        assert got["dims"][0] == [3, 3, 3]
        full[prec] = got
        np.testing.assert_array_equal(got["nnbr"][idx], ref["nnbr"])
        emax, erms = force_errors(got["F"][idx], _ref_F(ref))
        print(f"[gpu]   prec={prec} err_max={emax:.3e} err_rms={erms:.3e}", flush=True)
        assert emax <= tol and erms <= tol, (prec, emax, erms)
    np.testing.assert_array_equal(full[dcm.DCM_FP32_MIXED]["nnbr"], full[dcm.DCM_FP64]["nnbr"])


@pytest.mark.parametrize("f", [0.34, 1.7])
def test_lj_parameters_scale(f):
    """The small slab scaled by f (box, positions, cutoffs) with sigma = f and
    epsilon = 0.7: the oracle with the same parameters, and the reduced-unit
    law F(f x; eps, sigma = f) = (eps / f) F(x; 1, 1) (Eq. 3 depends on r only
    through r / sigma)."""
    base = workloads.make("slab_small")
    rc = ref_detect("slab_small")["rc"]
    s = workloads.System("scaled", base.x * f, base.y * f, base.z * f, base.vx, base.vy, base.vz,
                         tuple(L * f for L in base.box))
    eps = 0.7
    ref = oracle.forces(s.x, s.y, s.z, rc * f, s.box, eps=eps, sigma=f)
    unit = oracle.forces(base.x, base.y, base.z, rc, base.box)
    np.testing.assert_array_equal(ref["nnbr"], unit["nnbr"])
    emax, _ = force_errors(_ref_F(ref), _ref_F(unit) * (eps / f))
    assert emax <= 1e-12
    for prec, tol in ((dcm.DCM_FP64, 1e-12), (dcm.DCM_FP32_MIXED, 1e-5)):
        got = gpu_forces(s, rc * f, prec=prec, edge=1.25 * f, eps=eps, sigma=f,
                         rc_bound=float(np.max(rc)) * f)
        assert got["status"] == dcm.DCM_OK
        np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
        emax, erms = force_errors(got["F"], _ref_F(ref))
        assert emax <= tol and erms <= tol, (prec, emax, erms)
        assert abs(got["E"] - ref["E"]) <= tol * abs(ref["E"])
        assert rel(got["W"], ref["W"]) <= tol


def test_static_cutoff_reduces_to_eq3_and_balances():
    s = workloads.make("slab_small")
    rc = np.full(s.n, 3.0)
    a = gpu_forces(s, rc, rule=dcm.DCM_PAIR_OWN)
    b = gpu_forces(s, rc, rule=dcm.DCM_PAIR_MAX)
    np.testing.assert_array_equal(a["nnbr"], b["nnbr"])
    emax, _ = force_errors(a["F"], b["F"])
    assert emax <= 1e-14
    tot = np.abs(a["F"]).sum()
    assert np.all(np.abs(a["F"].sum(0)) <= 1e-12 * tot)


def test_cutoff_above_bound_is_flagged():
    s = workloads.make("slab_small")
    rc = ref_detect("slab_small")["rc"]
    got = gpu_forces(s, rc, rc_bound=5.0)
    assert got["status"] == dcm.DCM_ERR_RANGE
    ok = gpu_forces(s, np.minimum(rc, 5.0), rc_bound=5.0)
    assert ok["status"] == dcm.DCM_OK
    # without a bound the ghost halo covers half the box: same forces
    free = gpu_forces(s, rc, rc_bound=0.0)
    ref = gpu_forces(s, rc)
    np.testing.assert_array_equal(free["nnbr"], ref["nnbr"])
    assert force_errors(free["F"], ref["F"])[0] <= 1e-13


def test_empty_system():
    s = workloads.System("empty", *(np.zeros(0) for _ in range(6)), (10.0, 10.0, 10.0))
    got = gpu_forces(s, np.zeros(0))
    assert got["status"] == dcm.DCM_OK
    assert got["E"] == 0.0 and got["npairs"] == 0


def test_nonfinite_positions_are_flagged():
    s = workloads.make("slab_small")
    x = s.x.copy()
    x[17] = np.nan
    bad = workloads.System("bad", x, s.y, s.z, s.vx, s.vy, s.vz, s.box)
    got = gpu_forces(bad, np.full(s.n, 2.5))
    assert got["status"] == dcm.DCM_ERR_NONFINITE


# ------------------------------------------------------------ end to end

@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("prec", [dcm.DCM_FP64, dcm.DCM_FP32_MIXED])
def test_pipeline_end_to_end(name, prec):
    print(f"[gpu] pipeline {name} prec={prec}", flush=True)
    s = workloads.make(name)
    ref_d = ref_detect(name)
    ref = ref_forces(name, dcm.DCM_PAIR_OWN)
    grid = dcm.make_grid(s.box, s.h)
    rule = dcm.make_rule(*s.rule)
    f = [torch.zeros(s.n, **F64) for _ in range(3)]
    v = [dev(a) for a in (s.vx, s.vy, s.vz)]
    rc = torch.zeros(s.n, **F64)
    delta = torch.zeros(s.n, **F64)
    with Ctx() as ctx:
        dcm.dcm_step(ctx, dev(s.x), dev(s.y), dev(s.z), *v, *f, s.box, dcm.make_lj(), rule, grid,
                     dcm.rc_grid_for(rule, grid), dt=0.005, nsteps=0, prec=prec, rc=rc,
                     delta=delta)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
    assert dcm.rc_grid_for(rule, grid) == ref_d["rc_grid"]
    # distances come from a floating-point fixed point whose last bit may
    # depend on the update order: FP64 tolerance, not bit equality
    np.testing.assert_allclose(host(delta), ref_d["delta"], rtol=0, atol=1e-12 * ref_d["rc_grid"])
    np.testing.assert_allclose(host(rc), ref_d["rc"], rtol=1e-12, atol=0)
    F = np.stack([host(t) for t in f], 1)
    emax, erms = force_errors(F, _ref_F(ref))
    tol = 1e-12 if prec == dcm.DCM_FP64 else 1e-5
    assert emax <= tol and erms <= tol


def test_verlet_trajectory_tracks_oracle():
    """20 FP64 steps with re-detection every 5 steps, against the same
    schedule run entirely on the oracle."""
    s = workloads.make("slab_small")
    dt, nsteps, every = 0.005, 20, 5
    grid = dcm.make_grid(s.box, s.h)
    rule = dcm.make_rule(*s.rule)
    rcg = dcm.rc_grid_for(rule, grid)
    pos = [dev(a) for a in (s.x, s.y, s.z)]
    vel = [dev(a) for a in (s.vx, s.vy, s.vz)]
    f = [torch.zeros(s.n, **F64) for _ in range(3)]
    es = torch.zeros(2 * nsteps, **F64)
    with Ctx() as ctx:
        dcm.dcm_step(ctx, *pos, *vel, *f, s.box, dcm.make_lj(), rule, grid, rcg, dt, 0)
        dcm.dcm_step(ctx, *pos, *vel, *f, s.box, dcm.make_lj(), rule, grid, rcg, dt, nsteps,
                     redetect_every=every, energy_series=es)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
    # oracle schedule
    x, v = (s.x, s.y, s.z), (s.vx, s.vy, s.vz)
    p = oracle.pipeline(*x, s.box, s.h, s.rule)
    D = p["D"]
    F = (p["forces"]["fx"], p["forces"]["fy"], p["forces"]["fz"])
    epot = []
    for st in range(nsteps):
        v = oracle.kick(v, F, dt)
        x = oracle.drift(x, v, dt, s.box)
        if (st + 1) % every == 0:
            det = oracle.detect_interface(*x, s.box, s.h)
            D, _ = oracle.fsm(det["nv"], det["hv"], det["seg"], det["iface"], rcg)
        rc = oracle.cutoffs(oracle.particle_distance(*x, s.box, p["nv"], D), s.rule)
        fo = oracle.forces(*x, rc, s.box)
        F = (fo["fx"], fo["fy"], fo["fz"])
        v = oracle.kick(v, F, dt)
        epot.append(fo["E"])
    L = np.asarray(s.box)
    for a in range(3):
        d = host(pos[a]) - x[a]
        d -= L[a] * np.rint(d / L[a])
        assert np.max(np.abs(d)) < 1e-9
    np.testing.assert_allclose(host(es)[0::2], epot, rtol=1e-9)
    ke = 0.5 * sum(np.sum(c * c) for c in v)
    assert host(es)[-1] == pytest.approx(ke, rel=1e-9)


@pytest.mark.parametrize("prec", [dcm.DCM_FP64, dcm.DCM_FP32_MIXED])
def test_step_without_energy_series_repeats_the_recorded_run(prec):
    """Without an energy series dcm_step fuses the closing and opening kicks
    (and, before a detection step, the density binning) and keeps fewer
    fields in step between its reorderings; with one it runs every kick and
    the binning on its own.  Both perform the same arithmetic, so 20 steps
    (reorderings after steps 1, 8 and 16) must give the same state bit for
    bit: positions, velocities, forces, cutoffs and distances."""
    print(f"[gpu] dcm_step with and without an energy series prec={prec}", flush=True)
    s = workloads.make("slab_small")
    grid = dcm.make_grid(s.box, s.h)
    rule = dcm.make_rule(*s.rule)
    rcg = dcm.rc_grid_for(rule, grid)
    out = []
    for series in (True, False):
        st = [dev(a) for a in (s.x, s.y, s.z, s.vx, s.vy, s.vz)]
        st += [torch.zeros(s.n, **F64) for _ in range(5)]  # forces, delta, rc
        es = torch.zeros(40, **F64) if series else None
        with Ctx() as ctx:
            dcm.dcm_step(ctx, *st[:9], s.box, dcm.make_lj(), rule, grid, rcg, 0.005, 20,
                         prec=prec, redetect_every=3, energy_series=es, delta=st[9], rc=st[10])
            assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
        out.append(np.stack([host(t) for t in st], 1))
    np.testing.assert_array_equal(out[0], out[1])


def step_forces(s, prec, want_edge=False):
    """dcm_step with nsteps = 0 (detection, distances, cutoffs, cells of its
    tuned edge, forces) from the generator's positions: forces and cutoffs
    (and the cell edge it used, one of its candidates f r_c^min,
    f in 1/3, 0.4, 1/2, 0.6, 0.7, 0.8, identified by the cell counts; FP64
    steps only, whose candidates are not capped)."""
    grid = dcm.make_grid(s.box, s.h)
    rule = dcm.make_rule(*s.rule)
    f = [torch.zeros(s.n, **F64) for _ in range(3)]
    v = [dev(a) for a in (s.vx, s.vy, s.vz)]
    rc = torch.zeros(s.n, **F64)
    with Ctx() as ctx:
        dcm.dcm_step(ctx, dev(s.x), dev(s.y), dev(s.z), *v, *f, s.box, dcm.make_lj(), rule, grid,
                     dcm.dcm_rc_grid(rule, grid), dt=0.005, nsteps=0, prec=prec, rc=rc)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
        nc, _ = dcm.dcm_cell_dims(ctx)
    out = (np.stack([host(t) for t in f], 1), host(rc))
    if not want_edge:
        return out
    assert prec == dcm.DCM_FP64
    cands = [fr * s.rule[0] for fr in (1.0 / 3.0, 0.4, 0.5, 0.6, 0.7, 0.8)]
    edge = [e for e in cands if all(int(np.floor(L / e)) == k for L, k in zip(s.box, nc))]
    assert edge, (nc, cands)
    return out + (edge[0],)


def test_large_slab_parity_and_full_population_accuracy():
    """The large slab (2.6 M particles) in the benchmark's configuration.
    Cutoffs against the oracle's (FP64 distance fixed point: 1e-12); the FP64
    forces, and the FP32-mixed ones, against the oracle's per-particle sums on
    a seeded sample that includes the particles nearest the interfaces (where
    cutoffs are largest), neighbour counts bit for bit; then the FP32-mixed
    forces against the FP64 GPU path on every particle, with identical
    neighbour counts everywhere."""
    name = "slab_large"
    print("[gpu] large slab parity and full-population accuracy", flush=True)
    s = workloads.make(name)
    ref_d = ref_detect(name)
    F32, rc32 = step_forces(s, dcm.DCM_FP32_MIXED)
    F64s, rc64, edge64 = step_forces(s, dcm.DCM_FP64, want_edge=True)
    np.testing.assert_allclose(rc64, ref_d["rc"], rtol=1e-12, atol=0)
    np.testing.assert_array_equal(rc32, rc64)
    idx = workloads.sample_indices(s.n, 1536, seed=4242)
    near = np.argsort(np.minimum(np.abs(s.z - 140.0), np.abs(s.z - 260.0)))[:512]
    idx = np.unique(np.concatenate([idx, near]))
    ref = oracle.forces(s.x, s.y, s.z, rc64, s.box, idx=idx)
    R = _ref_F(ref)
    for tag, F, tol in (("fp64", F64s, 1e-12), ("fp32_mixed", F32, 1e-5)):
        emax, erms, efloor = force_errors(F[idx], R, detail=True)
        print(f"[gpu]   {tag} vs oracle (sample {len(idx)}): err_max={emax:.3e} "
              f"err_rms={erms:.3e} floored={efloor:.3e}", flush=True)
        assert emax <= tol and erms <= tol and efloor <= tol, tag
    emax, erms, efloor = force_errors(F32, F64s, detail=True)
    print(f"[gpu]   fp32_mixed vs fp64, all {s.n}: err_max={emax:.3e} err_rms={erms:.3e} "
          f"floored={efloor:.3e}", flush=True)
    assert emax <= 1e-5 and erms <= 1e-5 and efloor <= 1e-5
    # neighbour counts: both precisions at the FP64 step's cells, every
    # particle; dcm_forces there gives the step's FP64 forces bit for bit
    c32 = gpu_forces(s, rc64, prec=dcm.DCM_FP32_MIXED, edge=edge64, rc_bound=s.rule[1])
    c64 = gpu_forces(s, rc64, prec=dcm.DCM_FP64, edge=edge64, rc_bound=s.rule[1])
    np.testing.assert_array_equal(c64["nnbr"][idx], ref["nnbr"])
    np.testing.assert_array_equal(c32["nnbr"], c64["nnbr"])
    assert c32["npairs"] == c64["npairs"] == int(c64["nnbr"].astype(np.int64).sum())
    assert abs(c32["E"] - c64["E"]) <= 1e-5 * abs(c64["E"])
    assert rel(c32["W"], c64["W"]) <= 1e-5
    np.testing.assert_array_equal(c64["F"], F64s)


@pytest.mark.parametrize("name", ["droplet", "cylinder"])
def test_curved_interface_full_population_accuracy(name):
    """FP32-mixed against FP64 forces on every particle of the droplet and
    the cylinder (dcm_step's configuration), neighbour counts identical."""
    print(f"[gpu] curved {name} full-population accuracy", flush=True)
    s = workloads.make(name)
    F32, rc32 = step_forces(s, dcm.DCM_FP32_MIXED)
    F64s, rc64 = step_forces(s, dcm.DCM_FP64)
    np.testing.assert_array_equal(rc32, rc64)
    emax, erms, efloor = force_errors(F32, F64s, detail=True)
    print(f"[gpu]   {name} fp32_mixed vs fp64, all {s.n}: err_max={emax:.3e} "
          f"err_rms={erms:.3e} floored={efloor:.3e}", flush=True)
    assert emax <= 1e-5 and erms <= 1e-5 and efloor <= 1e-5
    c32 = gpu_forces(s, rc64, prec=dcm.DCM_FP32_MIXED, edge=1.25, rc_bound=s.rule[1])
    c64 = gpu_forces(s, rc64, prec=dcm.DCM_FP64, edge=1.25, rc_bound=s.rule[1])
    np.testing.assert_array_equal(c32["nnbr"], c64["nnbr"])
    assert abs(c32["E"] - c64["E"]) <= 1e-5 * abs(c64["E"])
    assert rel(c32["W"], c64["W"]) <= 1e-5


@pytest.mark.parametrize("prec", [dcm.DCM_FP64, dcm.DCM_FP32_MIXED])
@pytest.mark.parametrize("name", ["droplet", "cylinder"])
def test_curved_interface_forces_sampled(name, prec):
    """Curved interfaces (sphere, cylinder): the whole path from positions
    through dcm_step's force evaluation, against the oracle's cutoffs and
    per-particle sums on a seeded sample that includes the particles nearest
    the interface (largest cutoffs)."""
    print(f"[gpu] curved {name} prec={prec}", flush=True)
    s = workloads.make(name)
    ref_d = ref_detect(name)
    grid = dcm.make_grid(s.box, s.h)
    rule = dcm.make_rule(*s.rule)
    f = [torch.zeros(s.n, **F64) for _ in range(3)]
    v = [dev(a) for a in (s.vx, s.vy, s.vz)]
    rc = torch.zeros(s.n, **F64)
    with Ctx() as ctx:
        dcm.dcm_step(ctx, dev(s.x), dev(s.y), dev(s.z), *v, *f, s.box, dcm.make_lj(), rule, grid,
                     dcm.rc_grid_for(rule, grid), dt=0.005, nsteps=0, prec=prec, rc=rc)
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
    np.testing.assert_allclose(host(rc), ref_d["rc"], rtol=1e-12, atol=0)
    idx = workloads.sample_indices(s.n, 1024, seed=5151)
    near = np.argsort(np.abs(ref_d["delta"] - 0.5))[:256]
    idx = np.unique(np.concatenate([idx, near]))
    ref = oracle.forces(s.x, s.y, s.z, ref_d["rc"], s.box, idx=idx)
    F = np.stack([host(t) for t in f], 1)[idx]
    emax, erms = force_errors(F, _ref_F(ref))
    tol = 1e-12 if prec == dcm.DCM_FP64 else 1e-5
    print(f"[gpu]   {name} prec={prec} err_max={emax:.3e} err_rms={erms:.3e}", flush=True)
    assert emax <= tol and erms <= tol
