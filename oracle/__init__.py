"""FP64 CPU oracle for the dynamic cutoff method -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and it shares no code
with that path.

The arithmetic lives in ``dcm_oracle.c`` (plain C, FP64, no fused
multiply-add, Neumaier-compensated sums); this module compiles it with gcc
and wraps each step with numpy arrays.  Each wrapper names the part of the
paper it follows:

* ``voxel_counts`` / ``gray27`` / ``otsu`` / ``majority`` / ``interface`` --
  interface detection, Section 2.1 (Fig. 4, Eq. 4);
* ``fsm`` -- box-interface distances, Section 2.2 (Algorithm 2.1);
* ``particle_distance`` / ``cutoffs`` -- trilinear distance and cutoff
  assignment, Section 2.2;
* ``cells`` -- linked cells, Section 2.3;
* ``forces`` -- Eqs. 2-3 and Algorithm 2.3 as an O(N^2) minimum-image sum;
* ``kick`` / ``drift`` -- velocity Verlet, Fig. 3 box 5;
* ``cpu_cells_forces`` -- the CPU cell-list baseline (``cpu_cells.c``:
  Algorithms 2.2-2.3 with OpenMP dynamic scheduling, Section 2.4), timed by
  the benchmark for context and checked against ``forces``.

Every function here is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` against closed forms, invariants and brute force.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dcm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_CELLS_SRC = os.path.join(_HERE, "cpu_cells.c")
_CELLS_PATH = os.path.join(_HERE, "libcpucells.so")
_CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-msse4.1",
           "-fPIC", "-shared", "-std=c99", "-Wall"]

MAJORITY_MAX_PASSES = 16
FSM_MAX_PASSES = 64

_lib = None


def build(force: bool = True) -> str:
    """Compile dcm_oracle.c into liboracle.so and the CPU cell-list baseline
    cpu_cells.c into libcpucells.so next to them (gcc)."""
    for src, path in ((_SRC, _LIB_PATH), (_CELLS_SRC, _CELLS_PATH)):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, src, "-lm"])
            os.replace(tmp, path)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sig = {
        "orc_num_threads": (ctypes.c_int, []),
        "orc_set_threads": (None, [ctypes.c_int]),
        "orc_wrap": (None, [i64, P, P, P, P]),
        "orc_grid_dims": (None, [P, f64, P, P]),
        "orc_voxel_counts": (None, [i64, P, P, P, P, P, P]),
        "orc_gray27": (None, [P, P, P]),
        "orc_otsu": (ctypes.c_int, [i64, P, P, P, P]),
        "orc_majority": (ctypes.c_int, [P, P, ctypes.c_int]),
        "orc_potts": (ctypes.c_int, [P, P, f64, f64, f64, P, ctypes.c_int]),
        "orc_bubble_filter": (i64, [P, P, i64, P]),
        "orc_interface": (None, [P, P, P]),
        "orc_godunov": (f64, [f64, f64, f64, f64, f64, f64]),
        "orc_fsm": (ctypes.c_int, [P, P, P, P, f64, ctypes.c_int, P]),
        "orc_particle_distance": (None, [i64, P, P, P, P, P, P, P]),
        "orc_cutoffs": (None, [i64, P, f64, f64, f64, P]),
        "orc_cell_dims": (None, [P, f64, P]),
        "orc_cells": (None, [i64, P, P, P, P, P, P, P]),
        "orc_forces": (None, [i64, P, P, P, P, P, f64, f64, ctypes.c_int, P, i64,
                              P, P, P, P, P, P]),
        "orc_kick": (None, [i64, P, P, P, P, P, P, f64, f64]),
        "orc_drift": (None, [i64, P, P, P, P, P, P, f64, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _box(box) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(3))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


# -------------------------------------------------------------------- steps

def wrap(x, y, z, box):
    x, y, z = _f64(x).copy(), _f64(y).copy(), _f64(z).copy()
    _load().orc_wrap(x.size, _p(x), _p(y), _p(z), _p(_box(box)))
    return x, y, z


def grid_dims(box, h: float):
    nv = np.zeros(3, np.int32)
    hv = np.zeros(3, np.float64)
    _load().orc_grid_dims(_p(_box(box)), float(h), _p(nv), _p(hv))
    return nv, hv


def voxel_counts(x, y, z, box, nv) -> np.ndarray:
    x, y, z = _f64(x), _f64(y), _f64(z)
    nv = np.ascontiguousarray(nv, dtype=np.int32)
    counts = np.zeros(int(np.prod(nv)), np.uint32)
    _load().orc_voxel_counts(x.size, _p(x), _p(y), _p(z), _p(_box(box)), _p(nv), _p(counts))
    return counts


def gray27(nv, counts) -> np.ndarray:
    nv = np.ascontiguousarray(nv, dtype=np.int32)
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    g = np.zeros_like(counts)
    _load().orc_gray27(_p(nv), _p(counts), _p(g))
    return g


def otsu(g):
    """(T*, c0, c1, degenerate) of the two-phase split {g >= T*} / {g < T*}."""
    g = np.ascontiguousarray(g, dtype=np.uint32)
    t = np.zeros(1, np.int32)
    c = np.zeros(2, np.float64)
    deg = _load().orc_otsu(g.size, _p(g), _p(t), _p(c[0:1]), _p(c[1:2]))
    return int(t[0]), float(c[0]), float(c[1]), bool(deg)


def majority(nv, s, max_passes: int = MAJORITY_MAX_PASSES):
    nv = np.ascontiguousarray(nv, dtype=np.int32)
    s = np.ascontiguousarray(s, dtype=np.uint8).copy()
    passes = _load().orc_majority(_p(nv), _p(s), int(max_passes))
    return s, int(passes)


def potts(nv, g, c0: float, c1: float, nu: float, s, max_passes: int = MAJORITY_MAX_PASSES):
    """Length-term regularisation of the two-phase split (Section 2.1): synchronous
    iterated conditional modes on sum (g - c_s)^2 + nu * (26-neighbour pairs in
    different phases), means held fixed.  Returns (s, passes)."""
    nv = np.ascontiguousarray(nv, dtype=np.int32)
    g = np.ascontiguousarray(g, dtype=np.uint32)
    s = np.array(s, dtype=np.uint8, copy=True)
    passes = _load().orc_potts(_p(nv), _p(g), float(c0), float(c1), float(nu), _p(s),
                               int(max_passes))
    return s, int(passes)


def bubble_filter(nv, s, min_volume: int):
    """Section 2.1's bubble filter: every periodic 6-connected component of either
    phase with fewer than min_volume voxels takes the other phase.  Returns
    (s, label, flipped): label = smallest voxel index of each voxel's component
    in the input map."""
    nv = np.ascontiguousarray(nv, dtype=np.int32)
    s = np.array(s, dtype=np.uint8, copy=True)
    label = np.zeros(s.size, np.int32)
    flipped = _load().orc_bubble_filter(_p(nv), _p(s), int(min_volume), _p(label))
    return s, label, int(flipped)


def interface(nv, s) -> np.ndarray:
    nv = np.ascontiguousarray(nv, dtype=np.int32)
    s = np.ascontiguousarray(s, dtype=np.uint8)
    f = np.zeros_like(s)
    _load().orc_interface(_p(nv), _p(s), _p(f))
    return f


def godunov(ax, ay, az, hx, hy, hz) -> float:
    return float(_load().orc_godunov(float(ax), float(ay), float(az),
                                     float(hx), float(hy), float(hz)))


def fsm(nv, hv, s, iface, rc_grid: float, max_passes: int = FSM_MAX_PASSES):
    """(D, passes); passes == -1 means not converged within max_passes."""
    nv = np.ascontiguousarray(nv, dtype=np.int32)
    hv = _f64(hv)
    s = np.ascontiguousarray(s, dtype=np.uint8)
    iface = np.ascontiguousarray(iface, dtype=np.uint8)
    D = np.zeros(s.size, np.float64)
    passes = _load().orc_fsm(_p(nv), _p(hv), _p(s), _p(iface), float(rc_grid),
                             int(max_passes), _p(D))
    return D, int(passes)


def particle_distance(x, y, z, box, nv, D) -> np.ndarray:
    x, y, z = _f64(x), _f64(y), _f64(z)
    nv = np.ascontiguousarray(nv, dtype=np.int32)
    D = _f64(D)
    out = np.zeros(x.size, np.float64)
    _load().orc_particle_distance(x.size, _p(x), _p(y), _p(z), _p(_box(box)), _p(nv),
                                  _p(D), _p(out))
    return out


def cutoffs(delta, rule) -> np.ndarray:
    rc_min, rc_max, ramp = (float(v) for v in rule)
    delta = _f64(delta)
    rc = np.zeros_like(delta)
    _load().orc_cutoffs(delta.size, _p(delta), rc_min, rc_max, ramp, _p(rc))
    return rc


def cell_dims(box, edge: float) -> np.ndarray:
    nc = np.zeros(3, np.int32)
    _load().orc_cell_dims(_p(_box(box)), float(edge), _p(nc))
    return nc


def cells(x, y, z, box, nc):
    """(cell_of[N], cell_start[n_cells + 1]) for the given cell grid."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    nc = np.ascontiguousarray(nc, dtype=np.int32)
    cell_of = np.zeros(x.size, np.int32)
    start = np.zeros(int(np.prod(nc)) + 1, np.int32)
    _load().orc_cells(x.size, _p(x), _p(y), _p(z), _p(_box(box)), _p(nc), _p(cell_of),
                      _p(start))
    return cell_of, start


RULE_OWN = 0   # Algorithm 2.3: j acts on i iff r < rc_i
RULE_MAX = 1   # symmetric: iff r <= max(rc_i, rc_j)


def forces(x, y, z, rc, box, eps: float = 1.0, sigma: float = 1.0, rule: int = RULE_OWN,
           idx: Optional[Sequence[int]] = None) -> dict:
    """O(N^2) minimum-image DCM pair sum for the listed i (all when idx is None).

    Returns fx, fy, fz, nnbr (per listed i) and E, W (6: xx yy zz xy xz yz)
    summed over the listed i.
    """
    x, y, z, rc = _f64(x), _f64(y), _f64(z), _f64(rc)
    n = x.size
    if idx is None:
        m, pidx = n, None
    else:
        idx_arr = np.ascontiguousarray(idx, dtype=np.int64)
        m, pidx = idx_arr.size, _p(idx_arr)
    fx, fy, fz = (np.zeros(m, np.float64) for _ in range(3))
    nn = np.zeros(m, np.int32)
    e = np.zeros(1, np.float64)
    w = np.zeros(6, np.float64)
    _load().orc_forces(n, _p(x), _p(y), _p(z), _p(rc), _p(_box(box)), float(eps),
                       float(sigma), int(rule), pidx, m, _p(fx), _p(fy), _p(fz), _p(nn),
                       _p(e), _p(w))
    return dict(fx=fx, fy=fy, fz=fz, nnbr=nn, E=float(e[0]), W=w)


_cells_lib = None


def cpu_cells_forces(x, y, z, rc, box, bin_edge: float, eps: float = 1.0, sigma: float = 1.0,
                     idx: Optional[Sequence[int]] = None) -> dict:
    """CPU cell-list baseline (cpu_cells.c): Algorithm 2.2's per-step list on
    bins of edge >= bin_edge (the smallest cutoff: small bins, Section 2.3),
    then Algorithm 2.3's force loop, both OpenMP dynamic,20 (Section 2.4).
    Returns fx, fy, fz, nnbr (per listed i), E (half the listed i's pair
    energies), pairs, and the seconds of the list build and of the force
    loop.  Throughput context for the benchmark, checked against forces()."""
    global _cells_lib
    if _cells_lib is None:
        if not os.path.exists(_CELLS_PATH):
            build(force=True)
        lib = ctypes.CDLL(_CELLS_PATH)
        P = ctypes.c_void_p
        lib.cpu_cells_forces.restype = ctypes.c_int64
        lib.cpu_cells_forces.argtypes = [ctypes.c_int64, P, P, P, P, P, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, P, ctypes.c_int64,
                                         P, P, P, P, P, P, P]
        _cells_lib = lib
    x, y, z, rc = _f64(x), _f64(y), _f64(z), _f64(rc)
    n = x.size
    if idx is None:
        m, pidx = n, None
    else:
        idx_arr = np.ascontiguousarray(idx, dtype=np.int64)
        m, pidx = idx_arr.size, _p(idx_arr)
    fx, fy, fz = (np.zeros(m, np.float64) for _ in range(3))
    nn = np.zeros(m, np.int32)
    out = np.zeros(3, np.float64)
    pairs = _cells_lib.cpu_cells_forces(n, _p(x), _p(y), _p(z), _p(rc), _p(_box(box)),
                                        float(bin_edge), float(eps), float(sigma), pidx, m,
                                        _p(fx), _p(fy), _p(fz), _p(nn), _p(out[0:]),
                                        _p(out[1:]), _p(out[2:]))
    if pairs < 0:
        raise MemoryError("cpu_cells_forces: out of memory")
    return dict(fx=fx, fy=fy, fz=fz, nnbr=nn, E=float(out[0]), pairs=int(pairs),
                t_build=float(out[1]), t_force=float(out[2]))


def kick(v, f, dt: float, mass: float = 1.0):
    vx, vy, vz = (_f64(a).copy() for a in v)
    fx, fy, fz = (_f64(a) for a in f)
    _load().orc_kick(vx.size, _p(vx), _p(vy), _p(vz), _p(fx), _p(fy), _p(fz), float(dt),
                     float(mass))
    return vx, vy, vz


def drift(x, v, dt: float, box):
    xx, yy, zz = (_f64(a).copy() for a in x)
    vx, vy, vz = (_f64(a) for a in v)
    _load().orc_drift(xx.size, _p(xx), _p(yy), _p(zz), _p(vx), _p(vy), _p(vz), float(dt),
                      _p(_box(box)))
    return xx, yy, zz


# ------------------------------------------------------------ the pipeline

def rc_grid_for(rule, hv) -> float:
    """reading: distances are propagated up to ramp + 3 max(h); beyond ramp the
    cutoff is rc_min anyway (Section 2.2, footnote 4)."""
    return float(rule[2]) + 3.0 * float(np.max(hv))


def detect_interface(x, y, z, box, h: float, split: float = 0.0, nu: float = -1.0,
                     min_volume: int = 0) -> dict:
    """Section 2.1: bin -> gray value -> two-phase split -> regularise -> bubble
    filter -> interface.

    split <= 0 picks the threshold by the two-phase (2-means) criterion;
    split > 0 uses s = [g >= split].  A single-phase volume (degenerate) is
    classified as all high-density (no interface).  nu < 0 regularises with
    the majority vote, nu >= 0 with the length term of weight nu (needs the
    two-phase split; skipped for a single phase).  min_volume > 0 removes
    smaller components of either phase.
    """
    nv, hv = grid_dims(box, h)
    counts = voxel_counts(x, y, z, box, nv)
    g = gray27(nv, counts)
    degenerate = False
    if split > 0:
        t = int(np.ceil(split))
        s0 = (g >= split).astype(np.uint8)
        c0 = c1 = 0.0
    else:
        t, c0, c1, degenerate = otsu(g)
        if degenerate:
            s0 = np.ones(g.size, np.uint8)
        else:
            s0 = (g >= t).astype(np.uint8)
    if nu < 0:
        s, passes = majority(nv, s0)
    elif degenerate:
        s, passes = s0.copy(), 1
    else:
        if split > 0:
            raise ValueError("a length-term weight needs the two-phase split (split <= 0)")
        s, passes = potts(nv, g, c0, c1, nu, s0)
    flipped = 0
    if min_volume > 0:
        s, _, flipped = bubble_filter(nv, s, min_volume)
    f = interface(nv, s)
    return dict(nv=nv, hv=hv, counts=counts, g=g, threshold=t, c0=c0, c1=c1,
                degenerate=degenerate, s0=s0, seg=s, passes=passes, iface=f, flipped=flipped)


def pipeline(x, y, z, box, h: float, rule, eps=1.0, sigma=1.0, pair_rule=RULE_OWN,
             idx=None, split: float = 0.0) -> dict:
    """Interface -> distances -> cutoffs -> forces, all on the oracle."""
    det = detect_interface(x, y, z, box, h, split)
    rcg = rc_grid_for(rule, det["hv"])
    D, fpasses = fsm(det["nv"], det["hv"], det["seg"], det["iface"], rcg)
    delta = particle_distance(x, y, z, box, det["nv"], D)
    rc = cutoffs(delta, rule)
    out = dict(det, D=D, fsm_passes=fpasses, rc_grid=rcg, delta=delta, rc=rc)
    out["forces"] = forces(x, y, z, rc, box, eps, sigma, pair_rule, idx)
    return out
