"""dcm_detect_interface_noalloc (scratch in a static per-GPU array, no device
allocation) against dcm_detect_interface on the same inputs: counts, phase
map, interface and threshold bit for bit, on two calls in a row, the second
on a smaller grid (the array keeps the first call's contents), and the
size limit refused before anything is enqueued."""
import numpy as np
import pytest
import torch

import paper_1701_05242_amd as dcm
import workloads
from gpu_util import DEV, Ctx, dev, host

pytestmark = pytest.mark.gpu


def detect(ctx, fn, s, with_counts):
    grid = dcm.make_grid(s.box, s.h)
    nv = dcm.grid_voxels(grid)
    counts = torch.full((nv,), 7, dtype=torch.uint32, device=DEV) if with_counts else None
    seg = torch.full((nv,), 3, dtype=torch.uint8, device=DEV)
    iface = torch.full((nv,), 3, dtype=torch.uint8, device=DEV)
    thr = torch.full((1,), -5, dtype=torch.int32, device=DEV)
    fn(ctx, dev(s.x), dev(s.y), dev(s.z), s.box, grid, seg, iface, counts=counts,
       threshold_out=thr)
    status = dcm.dcm_sync_status(ctx)
    out = dict(seg=host(seg), iface=host(iface), thr=int(host(thr)[0]), status=status)
    if with_counts:
        out["counts"] = host(counts)
    return out


@pytest.mark.parametrize("with_counts", [True, False])
def test_noalloc_detection_matches_the_allocating_call(with_counts):
    print(f"[gpu] no-alloc detection, caller counts={with_counts}", flush=True)
    # larger grid first, then a smaller one: the static scratch keeps the
    # first call's contents, which the second must not see
    systems = [workloads.make("slab_medium"), workloads.make("slab_small")]
    with Ctx() as ctx:
        for s in systems:
            a = detect(ctx, dcm.dcm_detect_interface_noalloc, s, with_counts)
            b = detect(ctx, dcm.dcm_detect_interface, s, with_counts)
            assert a["status"] == b["status"] == dcm.DCM_OK, s.name
            for k in ("seg", "iface") + (("counts",) if with_counts else ()):
                np.testing.assert_array_equal(a[k], b[k], err_msg=f"{s.name} {k}")
            assert a["thr"] == b["thr"]
            assert a["seg"].sum() > 0 and a["iface"].sum() > 0


def test_noalloc_detection_refuses_a_grid_beyond_its_scratch():
    print("[gpu] no-alloc detection size limit", flush=True)
    s = workloads.make("slab_small")
    big = (160.0, 160.0, 400.0)  # 10.24 M voxels at h = 1
    grid = dcm.make_grid(big, 1.0)
    nv = dcm.grid_voxels(grid)
    seg = torch.zeros(nv, dtype=torch.uint8, device=DEV)
    iface = torch.zeros(nv, dtype=torch.uint8, device=DEV)
    with Ctx() as ctx:
        with pytest.raises(dcm.DcmError) as err:
            dcm.dcm_detect_interface_noalloc(ctx, dev(s.x), dev(s.y), dev(s.z), big, grid, seg,
                                             iface)
        assert err.value.code == dcm.DCM_ERR_RANGE
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK
