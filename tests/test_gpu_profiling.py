"""Kernel-family timers through the C ABI: every family while profiling,
only the named one under dcm_set_profiling_only, none when profiling is off
(the bench times its steps with events on the pair kernel alone)."""
import numpy as np
import pytest
import torch

import paper_1701_05242_amd as dcm
import workloads
from gpu_util import F64, Ctx, dev

pytestmark = pytest.mark.gpu


def test_profiling_only_one_family():
    print("[gpu] profiling families", flush=True)
    s = workloads.make("slab_small")
    x, y, z = dev(s.x), dev(s.y), dev(s.z)
    rc = torch.full((s.n,), 3.0, **F64)
    f = [torch.zeros(s.n, **F64) for _ in range(3)]
    with Ctx() as ctx:
        def run():
            dcm.dcm_build_cells(ctx, x, y, z, rc, s.box, 1.5, dcm.DCM_FP32_MIXED, rc_bound=3.0)
            dcm.dcm_forces(ctx, dcm.make_lj(), *f, prec=dcm.DCM_FP32_MIXED)

        def launches():
            return {fam: dcm.dcm_kernel_time(ctx, fam) for fam in ("cells", "pair")}

        dcm.dcm_set_profiling(ctx, True)
        run()
        t = launches()
        assert t["cells"][1] == 1 and t["pair"][1] == 1, t
        dcm.dcm_set_profiling_only(ctx, "pair")
        run()
        t = launches()
        assert t["cells"][1] == 0 and t["pair"][1] == 1 and t["pair"][0] > 0.0, t
        dcm.dcm_set_profiling_only(ctx, None)
        run()
        t = launches()
        assert t["cells"][1] == 1 and t["pair"][1] == 1, t
        dcm.dcm_set_profiling(ctx, False)
        run()
        t = launches()
        assert t["cells"][1] == 0 and t["pair"][1] == 0, t
        assert dcm.dcm_sync_status(ctx) == dcm.DCM_OK, dcm.dcm_last_error(ctx)
    assert np.all(np.isfinite(f[0].cpu().numpy()))
