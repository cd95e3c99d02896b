"""Python binding of libdcm.so, the gfx950 dynamic cutoff method library.

The functions here carry the names of the C ABI in ``include/dcm.h`` and only
marshal arguments: torch tensors supply device memory (``data_ptr()``) and the
HIP stream; every step of the method runs in the library's HIP kernels.  There
is no fallback: if ``libdcm.so`` is missing or fails to load, importing the
binding's entry points raises.

Array arguments must be contiguous CUDA/HIP tensors of the dtype the C ABI
names (float64 for positions, forces, distances and cutoffs; uint8 for the
phase map and interface mask; uint32 for voxel counts; int32 for cell data).
Scalar outputs (energy, virial, pair count, threshold, wave count) are
device tensors too.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdcm.so")

DCM_OK = 0
DCM_ERR_INVALID = 1
DCM_ERR_RANGE = 2
DCM_ERR_NOT_CONVERGED = 3
DCM_ERR_DEGENERATE = 4
DCM_ERR_NONFINITE = 5
DCM_ERR_HIP = 6
DCM_ERR_NOMEM = 7
STATUS_NAMES = {0: "DCM_OK", 1: "DCM_ERR_INVALID", 2: "DCM_ERR_RANGE",
                3: "DCM_ERR_NOT_CONVERGED", 4: "DCM_ERR_DEGENERATE",
                5: "DCM_ERR_NONFINITE", 6: "DCM_ERR_HIP", 7: "DCM_ERR_NOMEM"}

DCM_FP64 = 0
DCM_FP32_MIXED = 1
DCM_PAIR_OWN = 0
DCM_PAIR_MAX = 1
DCM_PAIR_MAX_N3 = 2
DCM_EV_ENERGY = 1
DCM_EV_VIRIAL = 2
DCM_EV_COUNTS = 4


class dcm_box(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3)]


class dcm_lj(ctypes.Structure):
    _fields_ = [("epsilon", ctypes.c_double), ("sigma", ctypes.c_double)]


class dcm_rule(ctypes.Structure):
    _fields_ = [("rc_min", ctypes.c_double), ("rc_max", ctypes.c_double),
                ("ramp", ctypes.c_double)]


class dcm_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3)]


class dcm_detect_opts(ctypes.Structure):
    _fields_ = [("split", ctypes.c_double), ("nu", ctypes.c_double),
                ("min_volume", ctypes.c_int64)]


class dcm_system(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("rc", ctypes.c_void_p), ("fx", ctypes.c_void_p), ("fy", ctypes.c_void_p),
                ("fz", ctypes.c_void_p), ("nnbr", ctypes.c_void_p),
                ("energy", ctypes.c_void_p), ("virial", ctypes.c_void_p),
                ("npairs", ctypes.c_void_p), ("n", ctypes.c_int64), ("box", dcm_box),
                ("cell_edge", ctypes.c_double), ("rc_bound", ctypes.c_double)]


class DcmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_F64 = ctypes.c_double
_INT = ctypes.c_int

# name -> argument types (every entry point returns dcm_status, an int32)
SIGNATURES = {
    "dcm_create": [ctypes.POINTER(_P), _P],
    "dcm_destroy": [_P],
    "dcm_set_stream": [_P, _P],
    "dcm_sync_status": [_P],
    "dcm_last_error": [_P],
    "dcm_make_grid": [dcm_box, _F64, ctypes.POINTER(dcm_grid)],
    "dcm_detect_interface": [_P, _P, _P, _P, _I64, dcm_box, dcm_grid, _F64, _P, _P, _P, _P],
    "dcm_rc_grid": [dcm_rule, dcm_grid, ctypes.POINTER(_F64)],
    "dcm_detect_interface_noalloc": [_P, _P, _P, _P, _I64, dcm_box, dcm_grid, _F64, _P, _P, _P,
                                     _P],
    "dcm_detect_interface_opts": [_P, _P, _P, _P, _I64, dcm_box, dcm_grid,
                                  ctypes.POINTER(dcm_detect_opts), _P, _P, _P, _P],
    "dcm_sweep_distance": [_P, _P, _P, dcm_grid, _F64, _I32, _P, _P],
    "dcm_assign_cutoffs": [_P, _P, _P, _P, _I64, dcm_box, dcm_grid, _P, dcm_rule, _P, _P],
    "dcm_build_cells": [_P, _P, _P, _P, _P, _I64, dcm_box, _F64, _F64, _INT, _P, _P],
    "dcm_cell_dims": [_P, ctypes.POINTER(_I32), ctypes.POINTER(_F64)],
    "dcm_forces": [_P, dcm_lj, _INT, _INT, _INT, _P, _P, _P, _P, _P, _P, _P],
    "dcm_build_list": [_P, _F64],
    "dcm_update_list": [_P, _P, _P, _P, _P, _I64, ctypes.POINTER(_F64), ctypes.POINTER(_F64),
                        ctypes.POINTER(_I32)],
    "dcm_forces_list": [_P, dcm_lj, _INT, _INT, _P, _P, _P, _P, _P, _P, _P],
    "dcm_step": [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I64, _F64, dcm_box, dcm_lj, dcm_rule,
                 dcm_grid, _F64, _INT, _INT, _F64, _I32, _I32, _I64, _P, _P, _P],
    "dcm_forces_batched": [_P, _I32, _P, dcm_lj, _INT, _INT, _INT, _INT],
    "dcm_batched_edge": [_P, ctypes.POINTER(_F64)],
    "dcm_batched_queues": [_P, ctypes.POINTER(ctypes.c_int32)],
    "dcm_batched_row_lists": [_P, ctypes.POINTER(ctypes.c_int32)],
    "dcm_set_batched_row_lists": [_P, ctypes.c_int32],
    "dcm_set_batched_queues": [_P, ctypes.c_int32],
    "dcm_walk_stats": [_P, ctypes.POINTER(ctypes.c_uint64)],
    "dcm_set_profiling": [_P, _INT],
    "dcm_set_profiling_only": [_P, ctypes.c_char_p],
    "dcm_kernel_time": [_P, ctypes.c_char_p, ctypes.POINTER(_F64), ctypes.POINTER(_I64)],
}

_lib = None


def load_library() -> ctypes.CDLL:
    """Load libdcm.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_1701_05242_amd/build.py` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "dcm_last_error" else ctypes.c_int32
    _lib = lib
    return lib


# ------------------------------------------------------------ marshalling

def _box(box: Sequence[float]) -> dcm_box:
    b = dcm_box()
    for a in range(3):
        b.L[a] = float(box[a])
    return b


def _ptr(t: Optional[torch.Tensor], dtype: torch.dtype, name: str, numel: Optional[int] = None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _check(ctx, code: int):
    if code != DCM_OK:
        msg = load_library().dcm_last_error(ctx).decode() if ctx else ""
        raise DcmError(code, msg)


def make_grid(box: Sequence[float], h: float) -> dcm_grid:
    g = dcm_grid()
    code = load_library().dcm_make_grid(_box(box), float(h), ctypes.byref(g))
    _check(None, code)
    return g


def make_rule(rc_min: float, rc_max: float, ramp: float) -> dcm_rule:
    return dcm_rule(float(rc_min), float(rc_max), float(ramp))


def make_lj(epsilon: float = 1.0, sigma: float = 1.0) -> dcm_lj:
    return dcm_lj(float(epsilon), float(sigma))


def grid_voxels(grid: dcm_grid) -> int:
    return int(grid.n[0]) * int(grid.n[1]) * int(grid.n[2])


# ------------------------------------------------------------ entry points

def dcm_create(stream=None) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(None, load_library().dcm_create(ctypes.byref(ctx), _stream_handle(stream)))
    return ctx


def dcm_destroy(ctx) -> None:
    _check(None, load_library().dcm_destroy(ctx))


def dcm_set_stream(ctx, stream=None) -> None:
    _check(ctx, load_library().dcm_set_stream(ctx, _stream_handle(stream)))


def dcm_sync_status(ctx) -> int:
    """Synchronise; return (not raise) the sticky device status code."""
    return int(load_library().dcm_sync_status(ctx))


def dcm_last_error(ctx) -> str:
    return load_library().dcm_last_error(ctx).decode()


def dcm_detect_interface(ctx, x, y, z, box, grid: dcm_grid, seg, iface, split: float = 0.0,
                         counts=None, threshold_out=None) -> None:
    n = x.numel()
    nv = grid_voxels(grid)
    f64 = torch.float64
    code = load_library().dcm_detect_interface(
        ctx, _ptr(x, f64, "x", n), _ptr(y, f64, "y", n), _ptr(z, f64, "z", n), n, _box(box),
        grid, float(split), _ptr(counts, torch.uint32, "counts", nv),
        _ptr(seg, torch.uint8, "seg", nv), _ptr(iface, torch.uint8, "iface", nv),
        _ptr(threshold_out, torch.int32, "threshold_out", 1))
    _check(ctx, code)


def dcm_detect_interface_noalloc(ctx, x, y, z, box, grid: dcm_grid, seg, iface,
                                 split: float = 0.0, counts=None, threshold_out=None) -> None:
    n = x.numel()
    nv = grid_voxels(grid)
    f64 = torch.float64
    code = load_library().dcm_detect_interface_noalloc(
        ctx, _ptr(x, f64, "x", n), _ptr(y, f64, "y", n), _ptr(z, f64, "z", n), n, _box(box),
        grid, float(split), _ptr(counts, torch.uint32, "counts", nv),
        _ptr(seg, torch.uint8, "seg", nv), _ptr(iface, torch.uint8, "iface", nv),
        _ptr(threshold_out, torch.int32, "threshold_out", 1))
    _check(ctx, code)


def dcm_detect_interface_opts(ctx, x, y, z, box, grid: dcm_grid, seg, iface, split: float = 0.0,
                              nu: float = -1.0, min_volume: int = 0, counts=None,
                              threshold_out=None) -> None:
    n = x.numel()
    nv = grid_voxels(grid)
    f64 = torch.float64
    opts = dcm_detect_opts(float(split), float(nu), int(min_volume))
    code = load_library().dcm_detect_interface_opts(
        ctx, _ptr(x, f64, "x", n), _ptr(y, f64, "y", n), _ptr(z, f64, "z", n), n, _box(box), grid,
        ctypes.byref(opts), _ptr(counts, torch.uint32, "counts", nv),
        _ptr(seg, torch.uint8, "seg", nv), _ptr(iface, torch.uint8, "iface", nv),
        _ptr(threshold_out, torch.int32, "threshold_out", 1))
    _check(ctx, code)


def dcm_sweep_distance(ctx, seg, iface, grid: dcm_grid, rc_grid: float, max_waves: int, dist,
                       waves_out=None) -> None:
    nv = grid_voxels(grid)
    code = load_library().dcm_sweep_distance(
        ctx, _ptr(seg, torch.uint8, "seg", nv), _ptr(iface, torch.uint8, "iface", nv), grid,
        float(rc_grid), int(max_waves), _ptr(dist, torch.float64, "dist", nv),
        _ptr(waves_out, torch.int32, "waves_out", 1))
    _check(ctx, code)


def dcm_assign_cutoffs(ctx, x, y, z, box, grid: dcm_grid, dist, rule: dcm_rule, rc,
                       delta=None) -> None:
    n = x.numel()
    f64 = torch.float64
    code = load_library().dcm_assign_cutoffs(
        ctx, _ptr(x, f64, "x", n), _ptr(y, f64, "y", n), _ptr(z, f64, "z", n), n, _box(box),
        grid, _ptr(dist, f64, "dist", grid_voxels(grid)), rule, _ptr(delta, f64, "delta", n),
        _ptr(rc, f64, "rc", n))
    _check(ctx, code)


def dcm_build_cells(ctx, x, y, z, rc, box, cell_edge: float = 0.0, prec: int = DCM_FP64,
                    cell_of=None, cell_start=None, rc_bound: float = 0.0) -> None:
    n = x.numel()
    f64 = torch.float64
    code = load_library().dcm_build_cells(
        ctx, _ptr(x, f64, "x", n), _ptr(y, f64, "y", n), _ptr(z, f64, "z", n),
        _ptr(rc, f64, "rc", n), n, _box(box), float(cell_edge), float(rc_bound), int(prec),
        _ptr(cell_of, torch.int32, "cell_of", n), _ptr(cell_start, torch.int32, "cell_start"))
    _check(ctx, code)


def dcm_walk_stats(ctx):
    """(candidates tested, cell rows visited) of the last DCM_EV_COUNTS forces call."""
    st = (ctypes.c_uint64 * 2)()
    _check(ctx, load_library().dcm_walk_stats(ctx, st))
    return int(st[0]), int(st[1])


def dcm_cell_dims(ctx):
    nc = (ctypes.c_int32 * 3)()
    ln = (ctypes.c_double * 3)()
    _check(ctx, load_library().dcm_cell_dims(ctx, nc, ln))
    return [int(v) for v in nc], [float(v) for v in ln]


def dcm_forces(ctx, lj: dcm_lj, fx, fy, fz, pair_rule: int = DCM_PAIR_OWN,
               prec: int = DCM_FP64, ev_flags: int = 0, energy=None, virial=None, nnbr=None,
               npairs=None) -> None:
    n = fx.numel()
    f64 = torch.float64
    code = load_library().dcm_forces(
        ctx, lj, int(pair_rule), int(prec), int(ev_flags), _ptr(fx, f64, "fx", n),
        _ptr(fy, f64, "fy", n), _ptr(fz, f64, "fz", n), _ptr(energy, f64, "energy", 1),
        _ptr(virial, f64, "virial", 6), _ptr(nnbr, torch.int32, "nnbr", n),
        _ptr(npairs, torch.uint64, "npairs", 1))
    _check(ctx, code)


def dcm_build_list(ctx, skin: float) -> None:
    _check(ctx, load_library().dcm_build_list(ctx, float(skin)))


def dcm_update_list(ctx, x, y, z, rc):
    """New positions and cutoffs for the list of the current cell build.
    Returns (valid, max_disp, min_slack)."""
    n = x.numel()
    f64 = torch.float64
    d, sl, v = _F64(0.0), _F64(0.0), _I32(0)
    code = load_library().dcm_update_list(
        ctx, _ptr(x, f64, "x", n), _ptr(y, f64, "y", n), _ptr(z, f64, "z", n),
        _ptr(rc, f64, "rc", n), n, ctypes.byref(d), ctypes.byref(sl), ctypes.byref(v))
    _check(ctx, code)
    return bool(v.value), d.value, sl.value


def dcm_forces_list(ctx, lj: dcm_lj, fx, fy, fz, prec: int = DCM_FP64, ev_flags: int = 0,
                    energy=None, virial=None, nnbr=None, npairs=None) -> None:
    n = fx.numel()
    f64 = torch.float64
    code = load_library().dcm_forces_list(
        ctx, lj, int(prec), int(ev_flags), _ptr(fx, f64, "fx", n), _ptr(fy, f64, "fy", n),
        _ptr(fz, f64, "fz", n), _ptr(energy, f64, "energy", 1), _ptr(virial, f64, "virial", 6),
        _ptr(nnbr, torch.int32, "nnbr", n), _ptr(npairs, torch.uint64, "npairs", 1))
    _check(ctx, code)


def dcm_step(ctx, x, y, z, vx, vy, vz, fx, fy, fz, box, lj: dcm_lj, rule: dcm_rule,
             grid: dcm_grid, rc_grid: float, dt: float, nsteps: int, mass: float = 1.0,
             pair_rule: int = DCM_PAIR_OWN, prec: int = DCM_FP64, redetect_every: int = 1,
             step0: int = 0, energy_series=None, delta=None, rc=None) -> None:
    n = x.numel()
    f64 = torch.float64
    code = load_library().dcm_step(
        ctx, _ptr(x, f64, "x", n), _ptr(y, f64, "y", n), _ptr(z, f64, "z", n),
        _ptr(vx, f64, "vx", n), _ptr(vy, f64, "vy", n), _ptr(vz, f64, "vz", n),
        _ptr(fx, f64, "fx", n), _ptr(fy, f64, "fy", n), _ptr(fz, f64, "fz", n), n, float(mass),
        _box(box), lj, rule, grid, float(rc_grid), int(pair_rule), int(prec), float(dt),
        int(nsteps), int(redetect_every), int(step0),
        _ptr(energy_series, f64, "energy_series", 2 * max(int(nsteps), 0)),
        _ptr(delta, f64, "delta", n), _ptr(rc, f64, "rc", n))
    _check(ctx, code)


def make_systems(systems) -> "ctypes.Array":
    """Descriptor array for dcm_forces_batched from a sequence of dicts with
    keys x, y, z, rc, fx, fy, fz (float64 [n] device tensors), box, and
    optionally nnbr (int32 [n]), energy (float64 [1]), virial (float64 [6]),
    npairs (uint64 [1]), cell_edge and rc_bound (floats, default 0).  Keep the
    tensors alive while the array is in use."""
    arr = (dcm_system * max(len(systems), 1))()
    f64 = torch.float64
    for b, d in enumerate(systems):
        n = d["x"].numel()
        s = arr[b]
        for k in ("x", "y", "z", "rc", "fx", "fy", "fz"):
            p = _ptr(d[k], f64, f"systems[{b}].{k}", n)
            setattr(s, k, p.value if p is not None else None)
        for k, dt, m in (("nnbr", torch.int32, n), ("energy", f64, 1), ("virial", f64, 6),
                         ("npairs", torch.uint64, 1)):
            p = _ptr(d.get(k), dt, f"systems[{b}].{k}", m)
            setattr(s, k, p.value if p is not None else None)
        s.n = n
        s.box = _box(d["box"])
        s.cell_edge = float(d.get("cell_edge", 0.0))
        s.rc_bound = float(d.get("rc_bound", 0.0))
    return arr


def dcm_forces_batched(ctx, systems, lj: dcm_lj, pair_rule: int = DCM_PAIR_OWN,
                       prec: int = DCM_FP64, ev_flags: int = 0, use_graph: bool = False):
    """systems: a sequence of dicts (see make_systems) or a descriptor array
    made by make_systems (reuse it to replay a recorded graph)."""
    if isinstance(systems, ctypes.Array):
        arr, nsys = systems, len(systems)
    else:
        arr, nsys = make_systems(systems), len(systems)
    code = load_library().dcm_forces_batched(
        ctx, int(nsys), ctypes.cast(arr, ctypes.c_void_p), lj, int(pair_rule), int(prec),
        int(ev_flags), 1 if use_graph else 0)
    _check(ctx, code)
    return arr


def dcm_batched_queues(ctx) -> int:
    """Work-queue layout (1 or 8) of the last batch, 0 before any."""
    q = ctypes.c_int32(0)
    _check(ctx, load_library().dcm_batched_queues(ctx, ctypes.byref(q)))
    return int(q.value)


def dcm_batched_row_lists(ctx) -> int:
    """Row-list entries per lane (14 or 16) of the last batch's pair kernel, 0 before any."""
    q = ctypes.c_int32(0)
    _check(ctx, load_library().dcm_batched_row_lists(ctx, ctypes.byref(q)))
    return int(q.value)


def dcm_set_batched_row_lists(ctx, entries: int) -> None:
    """Row-list entries of later batches: 0 (tuned), 14 or 16."""
    _check(ctx, load_library().dcm_set_batched_row_lists(ctx, int(entries)))


def dcm_set_batched_queues(ctx, queues: int) -> None:
    """Work-queue layout of later batches: 0 (tuned), 1 or 8."""
    _check(ctx, load_library().dcm_set_batched_queues(ctx, int(queues)))


def dcm_batched_edge(ctx) -> float:
    e = ctypes.c_double()
    _check(ctx, load_library().dcm_batched_edge(ctx, ctypes.byref(e)))
    return float(e.value)


def dcm_set_profiling(ctx, enable: bool) -> None:
    _check(ctx, load_library().dcm_set_profiling(ctx, 1 if enable else 0))


def dcm_set_profiling_only(ctx, family=None) -> None:
    """Time only this kernel family while profiling (None: every family)."""
    _check(ctx, load_library().dcm_set_profiling_only(ctx, family.encode() if family else None))


def dcm_kernel_time(ctx, family: str):
    """(total_ms, launches) of a kernel family since the last query."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(ctx, load_library().dcm_kernel_time(ctx, family.encode(), ctypes.byref(ms),
                                               ctypes.byref(cnt)))
    return float(ms.value), int(cnt.value)


def dcm_rc_grid(rule: dcm_rule, grid: dcm_grid) -> float:
    """Distance up to which the sweep propagates (the library's dcm_rc_grid)."""
    out = ctypes.c_double()
    _check(None, load_library().dcm_rc_grid(rule, grid, ctypes.byref(out)))
    return float(out.value)


rc_grid_for = dcm_rc_grid
