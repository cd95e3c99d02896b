"""Shared helpers of the GPU parity tests: device copies of a workload and
the error measures the parity bar is written in."""
import numpy as np
import torch

import paper_1701_05242_amd as dcm

DEV = torch.device("cuda:0")
F64 = dict(dtype=torch.float64, device=DEV)


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    if t.dtype in (torch.uint32, torch.uint64):
        return t.cpu().numpy()
    return t.detach().cpu().numpy()


def force_errors(F, R, detail=False):
    """Force errors against the reference R, in units of the RMS force.

    err_max = max_i |F_i - R_i| / F_rms: the error of the worst particle in
    units of the typical force, F_rms = RMS_i |R_i|.
    err_rms = RMS_i |F_i - R_i| / F_rms.
    Both are what the parity bar (1e-12 FP64, 1e-5 FP32-mixed) is written
    in.  With detail=True also the floored per-particle relative error
    max_i |F_i - R_i| / max(|R_i|, F_rms), which never exceeds err_max (it
    forgives particles whose own force is large)."""
    frms = np.sqrt(np.mean(np.sum(R * R, 1)))
    d = np.linalg.norm(F - R, axis=1)
    out = (float(d.max() / frms), float(np.sqrt(np.mean(d * d)) / frms))
    if detail:
        scale = np.maximum(np.linalg.norm(R, axis=1), frms)
        return out + (float(np.max(d / scale)),)
    return out


def rel(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


class Ctx:
    """A library context bound to torch's current stream."""

    def __init__(self):
        self.h = dcm.dcm_create()

    def __enter__(self):
        return self.h

    def __exit__(self, *exc):
        dcm.dcm_destroy(self.h)
        return False


def gpu_forces(s, rc, prec=dcm.DCM_FP64, rule=dcm.DCM_PAIR_OWN, edge=0.0, eps=1.0, sigma=1.0,
               idx=None, rc_bound=None):
    """Cells + forces on the GPU from the given cutoffs; returns host arrays.
    rc_bound defaults to the largest given cutoff."""
    if rc_bound is None:
        rc_bound = float(np.max(rc)) if len(rc) else 0.0
    x, y, z, r = dev(s.x), dev(s.y), dev(s.z), dev(rc)
    n = s.n
    fx, fy, fz = (torch.zeros(n, **F64) for _ in range(3))
    e = torch.zeros(1, **F64)
    w = torch.zeros(6, **F64)
    nn = torch.zeros(n, dtype=torch.int32, device=DEV)
    npairs = torch.zeros(1, dtype=torch.uint64, device=DEV)
    with Ctx() as ctx:
        dcm.dcm_build_cells(ctx, x, y, z, r, s.box, edge, prec, rc_bound=rc_bound)
        dcm.dcm_forces(ctx, dcm.make_lj(eps, sigma), fx, fy, fz, pair_rule=rule, prec=prec,
                       ev_flags=dcm.DCM_EV_ENERGY | dcm.DCM_EV_VIRIAL | dcm.DCM_EV_COUNTS,
                       energy=e, virial=w, nnbr=nn, npairs=npairs)
        code = dcm.dcm_sync_status(ctx)
        dims = dcm.dcm_cell_dims(ctx)
        walk = dcm.dcm_walk_stats(ctx)
    F = np.stack([host(fx), host(fy), host(fz)], 1)
    out = dict(F=F, E=float(host(e)[0]), W=host(w), nnbr=host(nn),
               npairs=int(host(npairs)[0]), status=code, dims=dims, walk=walk)
    if idx is not None:
        out["F"] = out["F"][idx]
        out["nnbr"] = out["nnbr"][idx]
    return out
