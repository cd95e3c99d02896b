"""Seeded synthetic inputs for the dynamic cutoff method (DCM) hot path.

This module only *constructs* particle systems.  It holds none of the
method's arithmetic (no binning, no segmentation, no distances, no cutoffs,
no forces), so that both the FP64 oracle and the HIP library can consume the
same inputs without sharing any code.

The systems stand in for the interfacial Lennard-Jones liquid/vapour systems
the paper simulates (Section 3, Fig. 5: a planar slab and a non-planar,
cylindrical interface; Section 4.1: a planar system of 19,200 particles).
The paper ships no input files, so every system here is generated from a
recipe:

* liquid: an FCC lattice at reduced density 0.8 that tiles the box in the
  periodic directions and fits the slab thickness exactly (so the effective
  liquid/vapour planes sit at the nominal slab faces), each coordinate
  jittered uniformly by +-0.05 sigma;
* vapour: a Poisson number (mean 0.02 x vapour volume) of uniform points,
  rejected when closer than ``VAPOUR_MIN_DIST`` to any other particle (an LJ
  vapour has no overlapping pairs);
* velocities: Maxwell-Boltzmann at T* = 0.7 (mass 1), centre-of-mass
  momentum removed.

Every random number comes from numpy's PCG64 seeded per system, so the same
call always returns the same system.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import List, Optional, Tuple

import numpy as np
from scipy.spatial import cKDTree

SEED_BASE = 170105242
RHO_LIQUID = 0.8
RHO_VAPOUR = 0.02
TEMPERATURE = 0.7
JITTER = 0.05
VAPOUR_MIN_DIST = 0.85


@dataclasses.dataclass
class System:
    """One periodic particle system plus the DCM parameters it is run with.

    Coordinates are float64 arrays already inside [0, L_a).  ``rule`` is
    (rc_min, rc_max, ramp): the cutoff falls linearly from rc_max at the
    interface to rc_min at distance >= ramp (Section 2.2).  ``h`` is the
    density-grid voxel edge (Section 2.1, footnote 2).
    """

    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    box: Tuple[float, float, float]
    h: float = 1.0
    rule: Tuple[float, float, float] = (2.5, 6.0, 5.0)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def positions(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)


# --------------------------------------------------------------------------
# lattice and vapour construction
# --------------------------------------------------------------------------

_FCC_BASIS = np.array(
    [[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]]
)


def _fcc_sites(ncell: Tuple[int, int, int], a: Tuple[float, float, float],
               origin: Tuple[float, float, float]) -> np.ndarray:
    """FCC sites of an ncell lattice with per-axis spacing a, shifted by +a/4."""
    ix, iy, iz = np.meshgrid(np.arange(ncell[0]), np.arange(ncell[1]),
                             np.arange(ncell[2]), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    pts = (cells[:, None, :] + _FCC_BASIS[None, :, :] + 0.25).reshape(-1, 3)
    pts *= np.asarray(a)[None, :]
    pts += np.asarray(origin)[None, :]
    return pts


def _jitter(rng: np.random.Generator, pts: np.ndarray) -> np.ndarray:
    return pts + rng.uniform(-JITTER, JITTER, size=pts.shape)


def _vapour(rng: np.random.Generator, box: np.ndarray, liquid: np.ndarray,
            volume: float, sample_region) -> np.ndarray:
    """Poisson(RHO_VAPOUR*volume) uniform points from ``sample_region``.

    ``sample_region(rng, k)`` returns k uniform candidate points of the vapour
    region.  Candidates closer than VAPOUR_MIN_DIST (periodic) to the liquid
    or to an already accepted vapour point are redrawn.
    """
    target = int(rng.poisson(RHO_VAPOUR * volume))
    if target == 0:
        return np.zeros((0, 3))
    liq_tree = cKDTree(liquid, boxsize=box) if len(liquid) else None
    accepted = np.zeros((0, 3))
    while len(accepted) < target:
        need = target - len(accepted)
        cand = sample_region(rng, need + need // 4 + 8)
        cand = np.minimum(cand, np.nextafter(box, 0.0))
        ok = np.ones(len(cand), dtype=bool)
        if liq_tree is not None:
            d, _ = liq_tree.query(cand, k=1)
            ok &= d >= VAPOUR_MIN_DIST
        if len(accepted):
            d, _ = cKDTree(accepted, boxsize=box).query(cand, k=1)
            ok &= d >= VAPOUR_MIN_DIST
        cand = cand[ok]
        if len(cand) > 1:
            pairs = cKDTree(cand, boxsize=box).query_pairs(VAPOUR_MIN_DIST,
                                                           output_type="ndarray")
            if len(pairs):
                drop = np.zeros(len(cand), dtype=bool)
                drop[np.max(pairs, axis=1)] = True
                cand = cand[~drop]
        accepted = np.concatenate([accepted, cand[:need]], axis=0)
    return accepted


def _velocities(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(0.0, math.sqrt(TEMPERATURE), size=(n, 3))
    if n:
        v -= v.mean(axis=0, keepdims=True)
    return v


def _finish(name, rng, pts, box, h, rule, meta) -> System:
    box = tuple(float(b) for b in box)
    if not np.all((pts >= 0.0) & (pts < np.asarray(box))):
        raise AssertionError("generator produced a coordinate outside [0, L)")
    v = _velocities(rng, len(pts))
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    return System(name, pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy(),
                  v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy(),
                  box, h, tuple(rule), meta)


# --------------------------------------------------------------------------
# the three geometries
# --------------------------------------------------------------------------

def slab(name: str, box, z_lo: float, thickness: float, seed: int,
         h: float = 1.0, rule=(2.5, 6.0, 5.0)) -> System:
    """Planar liquid slab occupying z_lo <= z < z_lo + thickness."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    box = np.asarray(box, dtype=np.float64)
    a0 = (4.0 / RHO_LIQUID) ** (1.0 / 3.0)
    nx = max(1, int(round(box[0] / a0)))
    ny = max(1, int(round(box[1] / a0)))
    ax, ay = box[0] / nx, box[1] / ny
    nz = max(1, int(round(thickness / (4.0 / (RHO_LIQUID * ax * ay)))))
    az = thickness / nz
    liquid = _jitter(rng, _fcc_sites((nx, ny, nz), (ax, ay, az), (0.0, 0.0, z_lo)))
    z_hi = z_lo + thickness
    gap = box[2] - thickness

    def region(r, k):
        p = r.uniform(0.0, 1.0, size=(k, 3)) * np.array([box[0], box[1], gap])
        p[:, 2] = np.where(p[:, 2] < z_lo, p[:, 2], p[:, 2] + thickness)
        return p

    vap = _vapour(rng, box, liquid, box[0] * box[1] * gap, region)
    pts = np.concatenate([liquid, vap], axis=0)
    meta = dict(kind="slab", z_lo=z_lo, z_hi=z_hi, lattice=(nx, ny, nz),
                n_liquid=len(liquid), n_vapour=len(vap),
                rho_eff=len(liquid) / (box[0] * box[1] * thickness), seed=seed)
    return _finish(name, rng, pts, box, h, rule, meta)


def _clipped_lattice(rng, box, inside) -> np.ndarray:
    a0 = (4.0 / RHO_LIQUID) ** (1.0 / 3.0)
    n = [max(1, int(round(b / a0))) for b in box]
    a = [b / k for b, k in zip(box, n)]
    sites = _fcc_sites(tuple(n), tuple(a), (0.0, 0.0, 0.0))
    sites = sites[inside(sites)]
    return _jitter(rng, sites)


def droplet(name: str, box, radius: float, seed: int, h: float = 1.0,
            rule=(2.5, 8.0, 5.0)) -> System:
    """Spherical liquid droplet of the given radius centred in the box."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    box = np.asarray(box, dtype=np.float64)
    c = box / 2.0

    def inside(p):
        return np.sum((p - c) ** 2, axis=1) < radius * radius

    liquid = _clipped_lattice(rng, box, inside)

    def region(r, k):
        out = np.zeros((0, 3))
        while len(out) < k:
            p = r.uniform(0.0, 1.0, size=(2 * k, 3)) * box
            out = np.concatenate([out, p[~inside(p)]], axis=0)
        return out[:k]

    vol = float(np.prod(box)) - 4.0 / 3.0 * math.pi * radius ** 3
    vap = _vapour(rng, box, liquid, vol, region)
    pts = np.concatenate([liquid, vap], axis=0)
    meta = dict(kind="droplet", radius=radius, centre=tuple(c), n_liquid=len(liquid),
                n_vapour=len(vap), seed=seed)
    return _finish(name, rng, pts, box, h, rule, meta)


def cylinder(name: str, box, radius: float, seed: int, h: float = 1.0,
             rule=(2.5, 8.0, 5.0)) -> System:
    """Liquid cylinder of the given radius along x through the box centre."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    box = np.asarray(box, dtype=np.float64)
    cy, cz = box[1] / 2.0, box[2] / 2.0

    def inside(p):
        return (p[:, 1] - cy) ** 2 + (p[:, 2] - cz) ** 2 < radius * radius

    liquid = _clipped_lattice(rng, box, inside)

    def region(r, k):
        out = np.zeros((0, 3))
        while len(out) < k:
            p = r.uniform(0.0, 1.0, size=(2 * k, 3)) * box
            out = np.concatenate([out, p[~inside(p)]], axis=0)
        return out[:k]

    vol = float(np.prod(box)) - math.pi * radius ** 2 * box[0]
    vap = _vapour(rng, box, liquid, vol, region)
    pts = np.concatenate([liquid, vap], axis=0)
    meta = dict(kind="cylinder", radius=radius, axis="x", n_liquid=len(liquid),
                n_vapour=len(vap), seed=seed)
    return _finish(name, rng, pts, box, h, rule, meta)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

WORKLOADS = {
    # small slab: 13.4 x 13.4 x 60, liquid for 20 <= z < 40, ~3k particles
    "slab_small": dict(kind="slab", box=(13.4, 13.4, 60.0), z_lo=20.0, thickness=20.0,
                       rule=(2.5, 6.0, 5.0), index=0),
    # medium slab: 54 x 54 x 120, liquid for 40 <= z < 80, ~99k particles
    "slab_medium": dict(kind="slab", box=(54.0, 54.0, 120.0), z_lo=40.0, thickness=40.0,
                        rule=(2.5, 6.0, 5.0), index=1),
    # large slab: 160 x 160 x 400, liquid for 140 <= z < 260, ~2.6M particles
    "slab_large": dict(kind="slab", box=(160.0, 160.0, 400.0), z_lo=140.0,
                       thickness=120.0, rule=(2.5, 8.0, 5.0), index=2),
    # planar slab of the paper's accuracy experiment (about 19,200 particles):
    # 26.8 x 26.8 x 90, liquid for 28.5 <= z < 61.5, ~19.8k particles
    "slab_fig6": dict(kind="slab", box=(26.8, 26.8, 90.0), z_lo=28.5, thickness=33.0,
                      rule=(3.0, 8.0, 5.0), index=5),
    # planar slab of the paper's DCM-versus-static timing (1024 cores x 1200
    # particles): 120 x 120 x 250, liquid for 75 <= z < 175, ~1.2M particles
    "slab_table1": dict(kind="slab", box=(120.0, 120.0, 250.0), z_lo=75.0, thickness=100.0,
                        rule=(3.0, 8.0, 5.0), index=6),
    # droplet of radius 30 in a 120^3 box, ~123k particles
    "droplet": dict(kind="droplet", box=(120.0, 120.0, 120.0), radius=30.0,
                    rule=(2.5, 8.0, 5.0), index=3),
    # cylinder of radius 25 along x in a 200 x 100 x 100 box, ~346k particles
    "cylinder": dict(kind="cylinder", box=(200.0, 100.0, 100.0), radius=25.0,
                     rule=(2.5, 8.0, 5.0), index=3, seed_offset=100),
}


@functools.lru_cache(maxsize=8)
def make(name: str, seed: Optional[int] = None) -> System:
    """Build a named workload (cached per process; treat the arrays as read-only)."""
    spec = WORKLOADS[name]
    if seed is None:
        seed = SEED_BASE + spec["index"] + spec.get("seed_offset", 0)
    if spec["kind"] == "slab":
        return slab(name, spec["box"], spec["z_lo"], spec["thickness"], seed,
                    rule=spec["rule"])
    if spec["kind"] == "droplet":
        return droplet(name, spec["box"], spec["radius"], seed, rule=spec["rule"])
    return cylinder(name, spec["box"], spec["radius"], seed, rule=spec["rule"])


def batched_systems(count: int = 64, n_min: float = 2000.0, n_max: float = 200000.0,
                    seed_base: int = SEED_BASE + 1000) -> List[System]:
    """Independent slabs of log-uniform size and uniform rc_max in [4, 8].

    Each system b uses its own PCG64 stream (seed_base + b).  The box keeps
    the small slab's aspect ratio (60 / 13.4) where it can; every edge is at
    least 2 rc_max + 0.5 so the minimum image stays valid; the liquid fills
    the middle third of L_z.
    """
    rho_mean = RHO_LIQUID / 3.0 + 2.0 * RHO_VAPOUR / 3.0
    aspect = 60.0 / 13.4
    out = []
    for b in range(count):
        rng = np.random.default_rng(np.random.PCG64(seed_base + b))
        n_target = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        rc_max = float(rng.uniform(4.0, 8.0))
        lmin = 2.0 * rc_max + 0.5
        lxy = max(lmin, (n_target / (rho_mean * aspect)) ** (1.0 / 3.0))
        lz = max(lmin, n_target / (rho_mean * lxy * lxy))
        s = slab(f"batch{b:02d}", (lxy, lxy, lz), lz / 3.0, lz / 3.0,
                 seed_base + b + 500, rule=(2.5, rc_max, 5.0))
        s.meta["n_target"] = n_target
        out.append(s)
    return out


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """Seeded sorted sample of k distinct particle indices out of n."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


def uniform_cutoffs(n: int, rc_min: float, rc_max: float, seed: int) -> np.ndarray:
    """Seeded per-particle cutoffs drawn uniformly from [rc_min, rc_max): an
    input that exercises very different cutoffs between neighbours."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    return rng.uniform(rc_min, rc_max, size=n)
