"""Pins for the FP64 oracle: each test ties an oracle step to something other
than the oracle itself -- a closed form, a printed/analytic value under
tests/golden/, a finite-difference derivative, an invariant, or a brute-force
enumeration -- chosen so that a plausible slip (wrong sign, dropped term,
swapped index, < vs <=) fails at least one of them.  CPU only."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


def _random_gas(n, box, seed, dmin=0.9):
    """Random points with a minimum separation (no LJ overlaps)."""
    rng = np.random.default_rng(seed)
    pts = []
    box = np.asarray(box, float)
    while len(pts) < n:
        p = rng.uniform(0, 1, 3) * box
        ok = True
        for q in pts:
            d = p - q
            d -= box * np.round(d / box)
            if d @ d < dmin * dmin:
                ok = False
                break
        if ok:
            pts.append(p)
    pts = np.array(pts)
    return pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy()


# ------------------------------------------------------------------ LJ pair

@pytest.mark.parametrize("eps,sigma", [(1.0, 1.0), (1.3, 1.1)])
def test_lj_closed_form_points(orc, eps, sigma):
    for r_s, u_e, f_s in _golden("lj_points.txt"):
        r = float(r_s) * sigma
        box = (50.0, 50.0, 50.0)
        x = np.array([10.0, 10.0 + r])
        y = np.array([5.0, 5.0])
        z = np.array([7.0, 7.0])
        rc = np.full(2, 3.0 * sigma)
        out = orc.forces(x, y, z, rc, box, eps, sigma, orc.RULE_OWN)
        # two ordered pairs, each carrying half the pair energy
        assert out["E"] == pytest.approx(float(u_e) * eps, abs=1e-13)
        # force on particle 0 points away from particle 1 when repulsive
        assert out["fx"][0] == pytest.approx(-float(f_s) * eps / sigma, abs=1e-12)
        assert out["fx"][1] == pytest.approx(float(f_s) * eps / sigma, abs=1e-12)
        assert out["fy"][0] == 0.0 and out["fz"][0] == 0.0
        assert list(out["nnbr"]) == [1, 1]


def test_cutoff_is_strict_for_own_rule_and_inclusive_for_max(orc):
    # Algorithm 2.3 tests |r_ij| < rc[i]; the symmetric rule uses <=.
    box = (40.0, 40.0, 40.0)
    x = np.array([1.0, 3.0])
    y = np.zeros(2) + 1.0
    z = np.zeros(2) + 1.0
    rc = np.array([2.0, 2.0])
    own = orc.forces(x, y, z, rc, box, rule=orc.RULE_OWN)
    mx = orc.forces(x, y, z, rc, box, rule=orc.RULE_MAX)
    assert list(own["nnbr"]) == [0, 0]
    assert list(mx["nnbr"]) == [1, 1]


def test_forces_are_minus_energy_gradient(orc):
    """F_i = -dE/dx_i by central differences (static cutoff, rule MAX)."""
    box = (9.0, 10.0, 11.0)
    x, y, z = _random_gas(60, box, seed=3)
    rc = np.full(x.size, 2.5)
    base = orc.forces(x, y, z, rc, box, 1.2, 1.05, orc.RULE_MAX)
    h = 1e-6
    for i in (0, 7, 31):
        for axis, arr in enumerate((x, y, z)):
            a = arr.copy()
            a[i] += h
            args = [x, y, z]
            args[axis] = a
            ep = orc.forces(*args, rc, box, 1.2, 1.05, orc.RULE_MAX)["E"]
            a[i] -= 2 * h
            em = orc.forces(*args, rc, box, 1.2, 1.05, orc.RULE_MAX)["E"]
            num = -(ep - em) / (2 * h)
            ana = base[("fx", "fy", "fz")[axis]][i]
            assert num == pytest.approx(ana, rel=1e-6, abs=1e-6)


def test_virial_diagonal_is_minus_box_scaling_derivative(orc):
    """W_aa = -dE/dlambda_a for the affine stretch x_a -> lambda x_a, L_a -> lambda L_a."""
    box = np.array([9.0, 10.0, 11.0])
    x, y, z = _random_gas(60, box, seed=5)
    rc = np.full(x.size, 2.5)
    W = orc.forces(x, y, z, rc, box, rule=orc.RULE_MAX)["W"]
    h = 1e-6
    for a in range(3):
        vals = []
        for lam in (1 + h, 1 - h):
            pos = [x.copy(), y.copy(), z.copy()]
            pos[a] = pos[a] * lam
            b = box.copy()
            b[a] *= lam
            vals.append(orc.forces(*pos, rc, b, rule=orc.RULE_MAX)["E"])
        dEdl = (vals[0] - vals[1]) / (2 * h)
        assert -dEdl == pytest.approx(W[a], rel=1e-6)


def test_rotation_covariance_of_force_and_virial(orc):
    """An isolated cluster rotated by R: F' = R F, W' = R W R^T, E' = E."""
    box = (200.0, 200.0, 200.0)
    cx, cy, cz = _random_gas(40, (7.0, 7.0, 7.0), seed=11)
    pts = np.stack([cx, cy, cz], 1) + 90.0
    rc = np.full(40, 30.0)
    ang = 0.7
    R = np.array([[math.cos(ang), -math.sin(ang), 0.0], [math.sin(ang), math.cos(ang), 0.0],
                  [0.0, 0.0, 1.0]])
    R = R @ np.array([[1.0, 0.0, 0.0], [0.0, math.cos(0.4), -math.sin(0.4)],
                      [0.0, math.sin(0.4), math.cos(0.4)]])
    c = pts.mean(0)
    rot = (pts - c) @ R.T + c
    a = orc.forces(pts[:, 0], pts[:, 1], pts[:, 2], rc, box)
    b = orc.forces(rot[:, 0], rot[:, 1], rot[:, 2], rc, box)

    def sym(w):
        return np.array([[w[0], w[3], w[4]], [w[3], w[1], w[5]], [w[4], w[5], w[2]]])

    assert b["E"] == pytest.approx(a["E"], rel=1e-12)
    Fa = np.stack([a["fx"], a["fy"], a["fz"]], 1)
    Fb = np.stack([b["fx"], b["fy"], b["fz"]], 1)
    np.testing.assert_allclose(Fb, Fa @ R.T, rtol=1e-9, atol=1e-9 * np.abs(Fa).max())
    np.testing.assert_allclose(sym(b["W"]), R @ sym(a["W"]) @ R.T, rtol=1e-9,
                               atol=1e-9 * np.abs(a["W"]).max())


def test_newton3_and_static_cutoff_reduction(orc):
    """Uniform rc: both rules are Eq. 3 (identical), and sum_i F_i = 0."""
    s = workloads.make("slab_small")
    rc = np.full(s.n, 3.0)
    own = orc.forces(s.x, s.y, s.z, rc, s.box, rule=orc.RULE_OWN)
    mx = orc.forces(s.x, s.y, s.z, rc, s.box, rule=orc.RULE_MAX)
    for k in ("fx", "fy", "fz", "nnbr"):
        np.testing.assert_array_equal(own[k], mx[k])
    assert own["E"] == mx["E"]
    total = sum(np.abs(own[k]).sum() for k in ("fx", "fy", "fz"))
    for k in ("fx", "fy", "fz"):
        assert abs(own[k].sum()) <= 1e-13 * total
    # the symmetric rule also balances with per-particle cutoffs
    rng = np.random.default_rng(1)
    rcv = rng.uniform(2.5, 6.0, s.n)
    mx = orc.forces(s.x, s.y, s.z, rcv, s.box, rule=orc.RULE_MAX)
    total = sum(np.abs(mx[k]).sum() for k in ("fx", "fy", "fz"))
    for k in ("fx", "fy", "fz"):
        assert abs(mx[k].sum()) <= 1e-13 * total


def test_own_rule_imbalance_identity(orc):
    """Algorithm 2.3 drops Newton-3: sum_i F_i equals the sum of the pair forces
    f_ij over ordered pairs that i sees but j does not (rc_j <= r < rc_i)."""
    box = (12.0, 12.0, 12.0)
    x, y, z = _random_gas(150, box, seed=21)
    rng = np.random.default_rng(2)
    rc = rng.uniform(2.0, 5.5, x.size)
    out = orc.forces(x, y, z, rc, box, rule=orc.RULE_OWN)
    L = np.asarray(box)
    expect = np.zeros(3)
    for i in range(x.size):
        for j in range(x.size):
            if i == j:
                continue
            d = np.array([x[i] - x[j], y[i] - y[j], z[i] - z[j]])
            d -= L * np.rint(d / L)
            r = math.sqrt(d @ d)
            if rc[j] <= r < rc[i]:
                # the pair force from an isolated two-particle oracle call
                two = orc.forces(np.array([x[i], x[j]]), np.array([y[i], y[j]]),
                                 np.array([z[i], z[j]]), np.array([rc[i], 0.0]), box)
                expect += np.array([two["fx"][0], two["fy"][0], two["fz"][0]])
    got = np.array([out["fx"].sum(), out["fy"].sum(), out["fz"].sum()])
    scale = sum(np.abs(out[k]).sum() for k in ("fx", "fy", "fz"))
    np.testing.assert_allclose(got, expect, atol=1e-12 * scale)


def test_translation_and_permutation_invariance(orc):
    """Minimum image: a rigid periodic shift or a relabelling changes nothing."""
    s = workloads.make("slab_small")
    rng = np.random.default_rng(4)
    rc = rng.uniform(2.5, 6.0, s.n)
    idx = np.arange(0, s.n, 37)
    a = orc.forces(s.x, s.y, s.z, rc, s.box, idx=idx)
    L = np.asarray(s.box)
    sh = np.array([5.3, -2.9, 31.7])
    xs, ys, zs = orc.wrap(s.x + sh[0], s.y + sh[1], s.z + sh[2], s.box)
    b = orc.forces(xs, ys, zs, rc, s.box, idx=idx)
    np.testing.assert_array_equal(a["nnbr"], b["nnbr"])
    for k in ("fx", "fy", "fz"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-9, atol=1e-9)
    perm = rng.permutation(s.n)
    inv = np.argsort(perm)
    c = orc.forces(s.x[perm], s.y[perm], s.z[perm], rc[perm], s.box, idx=inv[idx])
    np.testing.assert_array_equal(a["nnbr"], c["nnbr"])
    for k in ("fx", "fy", "fz"):
        np.testing.assert_allclose(c[k], a[k], rtol=1e-12, atol=1e-12)
    assert L.shape == (3,)


def test_forces_scale_with_sigma_and_epsilon(orc):
    """Eq. 3 depends on r only through r / sigma: scaling positions, box and
    cutoffs by f with sigma = f multiplies forces by eps / f, the energy by
    eps and the virial by eps, and keeps every neighbour count."""
    s = workloads.make("slab_small")
    rng = np.random.default_rng(12)
    rc = rng.uniform(2.5, 6.0, s.n)
    idx = np.arange(0, s.n, 29)
    a = orc.forces(s.x, s.y, s.z, rc, s.box, idx=idx)
    for f, eps in ((0.34, 0.7), (1.7, 2.5)):
        b = orc.forces(s.x * f, s.y * f, s.z * f, rc * f, tuple(L * f for L in s.box), eps=eps,
                       sigma=f, idx=idx)
        np.testing.assert_array_equal(a["nnbr"], b["nnbr"])
        scale = max(np.max(np.abs(a[k])) for k in ("fx", "fy", "fz"))
        for k in ("fx", "fy", "fz"):
            np.testing.assert_allclose(b[k], a[k] * (eps / f), rtol=0, atol=1e-12 * scale * eps / f)
        assert b["E"] == pytest.approx(a["E"] * eps, rel=1e-12)
        np.testing.assert_allclose(b["W"], np.asarray(a["W"]) * eps, rtol=1e-11, atol=1e-12)


def test_large_cutoff_converges_to_full_sum(orc):
    """Eq. 2 vs Eq. 3: with rc beyond the half-diagonal every minimum image
    pair is included, and the truncation error shrinks as rc grows."""
    box = (8.0, 8.0, 8.0)
    x, y, z = _random_gas(70, box, seed=8)
    full = orc.forces(x, y, z, np.full(70, 7.0), box, rule=orc.RULE_MAX)
    assert np.all(full["nnbr"] == 69)
    errs = []
    for R in (2.0, 2.8, 3.6):
        o = orc.forces(x, y, z, np.full(70, R), box, rule=orc.RULE_MAX)
        errs.append(np.sqrt(np.mean((o["fx"] - full["fx"]) ** 2 + (o["fy"] - full["fy"]) ** 2
                                    + (o["fz"] - full["fz"]) ** 2)))
    assert errs[0] > errs[1] > errs[2]


# ------------------------------------------------------- grid / segmentation

def test_voxel_and_cell_binning(orc):
    s = workloads.make("slab_small")
    nv, hv = orc.grid_dims(s.box, 1.0)
    assert list(nv) == [13, 13, 60]
    np.testing.assert_allclose(hv, [13.4 / 13, 13.4 / 13, 1.0])
    counts = orc.voxel_counts(s.x, s.y, s.z, s.box, nv)
    assert counts.sum() == s.n
    for edge in (1.3, 2.5, 6.7):
        nc = orc.cell_dims(s.box, edge)
        cell_of, start = orc.cells(s.x, s.y, s.z, s.box, nc)
        np.testing.assert_array_equal(np.diff(start), np.bincount(cell_of, minlength=nc.prod()))
        cx = cell_of % nc[0]
        cy = (cell_of // nc[0]) % nc[1]
        cz = cell_of // (nc[0] * nc[1])
        for c, p, L, k in ((cx, s.x, 13.4, nc[0]), (cy, s.y, 13.4, nc[1]), (cz, s.z, 60.0, nc[2])):
            w = L / k
            assert np.all(p >= c * w - 1e-12) and np.all(p < (c + 1) * w + 1e-12)


def test_gray_majority_interface_match_direct_stencils(orc):
    rng = np.random.default_rng(0)
    for shape in [(5, 4, 6), (1, 3, 7), (2, 2, 2), (9, 8, 7)]:
        nx, ny, nz = shape
        nv = np.array(shape, np.int32)
        counts = rng.integers(0, 5, size=nz * ny * nx).astype(np.uint32)
        c3 = counts.reshape(nz, ny, nx).astype(np.int64)
        box27 = sum(np.roll(np.roll(np.roll(c3, dz, 0), dy, 1), dx, 2)
                    for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1))
        np.testing.assert_array_equal(orc.gray27(nv, counts), box27.ravel())
        s0 = (rng.random(nz * ny * nx) < 0.5).astype(np.uint8)
        one, passes = orc.majority(nv, s0, max_passes=1)
        s3 = s0.reshape(nz, ny, nx).astype(np.int64)
        m27 = sum(np.roll(np.roll(np.roll(s3, dz, 0), dy, 1), dx, 2)
                  for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1))
        np.testing.assert_array_equal(one, (m27 >= 14).astype(np.uint8).ravel())
        # iterate to the end and check the stopping rule holds
        fin, passes = orc.majority(nv, s0)
        again, _ = orc.majority(nv, fin, max_passes=1)
        twice, _ = orc.majority(nv, again, max_passes=1)
        assert passes <= 16
        if passes < 16:
            assert np.array_equal(again, fin) or np.array_equal(twice, fin)
        f = orc.interface(nv, fin)
        t3 = fin.reshape(nz, ny, nx)
        nb0 = np.zeros_like(t3, dtype=bool)
        for ax in range(3):
            for sh in (-1, 1):
                nb0 |= np.roll(t3, sh, ax) == 0
        np.testing.assert_array_equal(f, ((t3 == 1) & nb0).astype(np.uint8).ravel())


def test_otsu_matches_exhaustive_enumeration(orc):
    """The two-phase split minimises the within-class sum of squares; compare
    with an exact (rational) enumeration of every threshold."""
    rng = np.random.default_rng(7)
    for trial in range(6):
        a = rng.integers(0, 4, size=200)
        b = rng.integers(10 + trial, 30, size=int(rng.integers(20, 150)))
        g = np.concatenate([a, b]).astype(np.uint32)
        rng.shuffle(g)
        best, best_t = None, None
        for t in range(1, int(g.max()) + 1):
            lo, hi = g[g < t].astype(int), g[g >= t].astype(int)
            if len(lo) == 0 or len(hi) == 0:
                continue
            ss = Fraction(0)
            for part in (lo, hi):
                m = Fraction(int(part.sum()), len(part))
                ss += sum((Fraction(int(v)) - m) ** 2 for v in part)
            if best is None or ss < best:
                best, best_t = ss, t
        t, c0, c1, deg = orc.otsu(g)
        assert t == best_t
        assert not deg
        assert c0 == pytest.approx(g[g < t].mean()) and c1 == pytest.approx(g[g >= t].mean())
    # a single value has no split; a low-contrast field is one phase
    assert orc.otsu(np.full(50, 7, np.uint32))[3]
    assert orc.otsu(rng.integers(20, 24, size=300).astype(np.uint32))[3]


def test_slab_segmentation_gives_analytic_planes(orc):
    for name, lo, hi in _golden("slab_layers.txt"):
        s = workloads.make(name)
        det = orc.detect_interface(s.x, s.y, s.z, s.box, s.h)
        nv = det["nv"]
        seg = det["seg"].reshape(nv[2], nv[1], nv[0])
        f = det["iface"].reshape(nv[2], nv[1], nv[0])
        lo, hi = int(lo), int(hi)
        expect = np.zeros(nv[2], bool)
        expect[lo:hi + 1] = True
        assert np.all(seg[expect] == 1) and np.all(seg[~expect] == 0)
        layers = np.where(f.any(axis=(1, 2)))[0]
        assert list(layers) == [lo, hi]
        assert np.all(f[lo] == 1) and np.all(f[hi] == 1)
        assert not det["degenerate"]


def test_length_term_limits_and_flip_threshold(orc):
    """The length-term regulariser against what fixes it independently: with no
    length term the two-phase split is already optimal for fixed means (the
    global 2-means split assigns every value to its nearer mean); with no data
    term (c0 = c1) the pass is the 27-window majority vote; an isolated voxel
    flips exactly when the length penalty exceeds its data-term gain."""
    for name in ("slab_small", "slab_fig6"):
        s = workloads.make(name)
        det = orc.detect_interface(s.x, s.y, s.z, s.box, s.h)
        seg, passes = orc.potts(det["nv"], det["g"], det["c0"], det["c1"], 0.0, det["s0"])
        assert passes == 1
        np.testing.assert_array_equal(seg, det["s0"])
    rng = np.random.default_rng(3)
    for shape in [(5, 4, 6), (9, 8, 7), (2, 3, 11)]:
        nv = np.array(shape, np.int32)
        n = int(np.prod(shape))
        g = rng.integers(0, 40, size=n).astype(np.uint32)
        s0 = (rng.random(n) < 0.5).astype(np.uint8)
        a, pa = orc.potts(nv, g, 12.5, 12.5, 0.7, s0)
        b, pb = orc.majority(nv, s0)
        np.testing.assert_array_equal(a, b)
        assert pa == pb
    # one voxel with g = c1 among voxels with g = c0: the data term favours it
    # by (c1 - c0)^2 = 100, the length term charges 26 nu
    nv = np.array((5, 5, 5), np.int32)
    g = np.zeros(125, np.uint32)
    s0 = np.zeros(125, np.uint8)
    g[62] = 10
    s0[62] = 1
    kept, _ = orc.potts(nv, g, 0.0, 10.0, 3.8, s0, max_passes=1)
    gone, _ = orc.potts(nv, g, 0.0, 10.0, 3.9, s0, max_passes=1)
    assert kept[62] == 1 and kept.sum() == 1
    assert gone.sum() == 0


def test_bubble_filter_matches_scipy_components(orc):
    """Connected components from scipy.ndimage.label (6-connected) on maps
    framed by a low-density layer, where periodic and open boundaries give the
    same components; plus one component that exists only through the periodic
    wrap."""
    ndimage = pytest.importorskip("scipy.ndimage")
    six = ndimage.generate_binary_structure(3, 1)
    rng = np.random.default_rng(11)
    for shape in [(12, 10, 9), (7, 15, 6)]:
        nz, ny, nx = shape[2], shape[1], shape[0]
        inner = (rng.random((nz - 2, ny - 2, nx - 2)) < 0.55).astype(np.uint8)
        s3 = np.zeros((nz, ny, nx), np.uint8)
        s3[1:-1, 1:-1, 1:-1] = inner
        s = s3.ravel()
        nv = np.array((nx, ny, nz), np.int32)
        comps = []
        for phase in (0, 1):
            lab, k = ndimage.label(s3 == phase, structure=six)
            for c in range(1, k + 1):
                comps.append(np.flatnonzero(lab.ravel() == c))
        for min_volume in (1, 3, 8, 30):
            expect = s.copy()
            want_label = np.empty(s.size, np.int64)
            for idx in comps:
                want_label[idx] = idx.min()
                if idx.size < min_volume:
                    expect[idx] = 1 - expect[idx]
            got, label, flipped = orc.bubble_filter(nv, s, min_volume)
            np.testing.assert_array_equal(got, expect)
            np.testing.assert_array_equal(label, want_label)
            assert flipped == int(np.sum(got != s))
    # a high-density pair joined only across the periodic x boundary
    nv = np.array((8, 5, 5), np.int32)
    s3 = np.zeros((5, 5, 8), np.uint8)
    s3[2, 2, 0] = s3[2, 2, 7] = 1
    s = s3.ravel()
    got, label, _ = orc.bubble_filter(nv, s, 2)
    np.testing.assert_array_equal(got, s)
    v0, v7 = (2 * 5 + 2) * 8 + 0, (2 * 5 + 2) * 8 + 7
    assert label[v0] == label[v7] == v0
    got, _, flipped = orc.bubble_filter(nv, s, 3)
    assert flipped == 2 and got.sum() == 0


# ------------------------------------------------------------ distances

def test_godunov_closed_forms(orc):
    inf = math.inf
    assert orc.godunov(2.0, inf, inf, 1.0, 1.0, 1.0) == 3.0
    assert orc.godunov(0.0, 5.0, 5.0, 1.0, 1.0, 1.0) == 1.0
    assert orc.godunov(1.0, 1.0, inf, 1.0, 1.0, 1.0) == pytest.approx(1 + 1 / math.sqrt(2), abs=1e-15)
    assert orc.godunov(1.0, 1.0, 1.0, 1.0, 1.0, 1.0) == pytest.approx(1 + 1 / math.sqrt(3), abs=1e-15)
    hx, hy = 0.7, 1.3
    e = hx * hy / math.sqrt(hx * hx + hy * hy)
    assert orc.godunov(4.0, 4.0, inf, hx, hy, 1.0) == pytest.approx(4.0 + e, abs=1e-14)
    # symmetric in the axis order
    assert orc.godunov(1.0, 1.4, 2.0, 1.0, 0.9, 1.1) == orc.godunov(1.4, 2.0, 1.0, 0.9, 1.1, 1.0)
    assert orc.godunov(inf, inf, inf, 1, 1, 1) == inf


def test_fsm_point_source_closed_forms(orc):
    n = 11
    nv = np.array([n, n, n], np.int32)
    s = np.ones(n ** 3, np.uint8)
    iface = np.zeros(n ** 3, np.uint8)
    c = 5
    iface[(c * n + c) * n + c] = 1
    D, passes = orc.fsm(nv, [1.0, 1.0, 1.0], s, iface, rc_grid=100.0)
    assert passes > 0
    D3 = D.reshape(n, n, n)
    for i, j, k, d in _golden("godunov_point_source.txt"):
        i, j, k = int(i), int(j), int(k)
        for (a, b, cc) in {(i, j, k), (j, k, i), (k, i, j)}:
            assert D3[c + cc, c + b, c + a] == pytest.approx(float(d), abs=1e-12)
            assert D3[c - cc, c - b, c - a] == pytest.approx(float(d), abs=1e-12)


def test_fsm_is_order_independent_and_cap_is_exact(orc):
    """Jacobi iteration of the same local solve reaches the oracle's
    Gauss-Seidel fixed point (the CFSM result equals the FSM within rc_grid),
    and capping at rc_grid only clips values above it."""
    rng = np.random.default_rng(9)
    n = (9, 8, 7)
    nv = np.array(n, np.int32)
    hv = np.array([0.9, 1.1, 1.0])
    s = (rng.random(np.prod(n)) < 0.85).astype(np.uint8)
    iface = orc.interface(nv, s)
    Dgs, _ = orc.fsm(nv, hv, s, iface, rc_grid=50.0)
    # Jacobi sweeps in the test, reusing only the local Godunov solve
    D = np.where((s == 0) | (iface == 1), 0.0, np.inf).reshape(n[2], n[1], n[0])
    src = ((s == 0) | (iface == 1)).reshape(n[2], n[1], n[0])
    for _ in range(200):
        new = D.copy()
        for k in range(n[2]):
            for j in range(n[1]):
                for i in range(n[0]):
                    if src[k, j, i]:
                        continue
                    ax = min(D[k, j, (i - 1) % n[0]], D[k, j, (i + 1) % n[0]])
                    ay = min(D[k, (j - 1) % n[1], i], D[k, (j + 1) % n[1], i])
                    az = min(D[(k - 1) % n[2], j, i], D[(k + 1) % n[2], j, i])
                    new[k, j, i] = min(D[k, j, i], orc.godunov(ax, ay, az, *hv))
        if np.array_equal(new, D):
            break
        D = new
    np.testing.assert_allclose(D.ravel(), Dgs, rtol=0, atol=1e-12)
    cap = 1.7
    Dc, _ = orc.fsm(nv, hv, s, iface, rc_grid=cap)
    np.testing.assert_allclose(Dc, np.minimum(Dgs, cap), rtol=0, atol=1e-12)


def test_fsm_slab_is_exact_and_droplet_near_euclidean(orc):
    s = workloads.make("slab_small")
    det = orc.detect_interface(s.x, s.y, s.z, s.box, s.h)
    nv, hv = det["nv"], det["hv"]
    rcg = orc.rc_grid_for(s.rule, hv)
    D, passes = orc.fsm(nv, hv, det["seg"], det["iface"], rcg)
    assert passes > 0
    D3 = D.reshape(nv[2], nv[1], nv[0])
    for k in range(nv[2]):
        dist = min(abs(k - 20), abs(k - 39)) if 20 <= k <= 39 else 0
        assert np.all(D3[k] == min(float(dist), rcg))
    # a sphere of radius 6 voxels: within h of the brute-force distance to the
    # nearest interface voxel centre
    n = 24
    nv = np.array([n, n, n], np.int32)
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r = np.sqrt((ii - 11.3) ** 2 + (jj - 12.1) ** 2 + (kk - 11.8) ** 2)
    seg = (r < 6.0).astype(np.uint8).ravel()
    iface = orc.interface(nv, seg)
    D, _ = orc.fsm(nv, [1.0, 1.0, 1.0], seg, iface, rc_grid=100.0)
    centres = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1)[iface == 1]
    inside = np.where((seg == 1) & (iface == 0))[0]
    pts = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1)[inside]
    dbf = np.sqrt(((pts[:, None, :] - centres[None, :, :]) ** 2).sum(-1)).min(1)
    assert np.all(np.abs(D[inside] - dbf) <= 1.0)


def test_trilinear_distance_and_cutoff_rule(orc):
    box = (6.0, 5.0, 8.0)
    nv, hv = orc.grid_dims(box, 1.0)
    # a field linear in z between voxel centres: D(k) = 0.5*k + 1
    kz = np.arange(nv[2])
    D = np.broadcast_to((0.5 * kz + 1.0)[:, None, None], (nv[2], nv[1], nv[0])).ravel().copy()
    rng = np.random.default_rng(3)
    z = rng.uniform(0.5, 7.5, 200)     # between the first and last centre
    x = rng.uniform(0, 6.0, 200)
    y = rng.uniform(0, 5.0, 200)
    delta = orc.particle_distance(x, y, z, box, nv, D)
    np.testing.assert_allclose(delta, 0.5 * (z - 0.5) + 1.0, atol=1e-13)
    # at voxel centres the interpolant returns the voxel value
    Dr = rng.uniform(0, 3, nv.prod())
    ci = rng.integers(0, nv[0], 50)
    cj = rng.integers(0, nv[1], 50)
    ck = rng.integers(0, nv[2], 50)
    dc = orc.particle_distance((ci + 0.5) * hv[0], (cj + 0.5) * hv[1], (ck + 0.5) * hv[2],
                               box, nv, Dr)
    np.testing.assert_allclose(dc, Dr[(ck * nv[1] + cj) * nv[0] + ci], atol=1e-14)
    # periodic: z = 0.25 lies a quarter voxel past the last layer's centre
    # (at z = -0.5 across the boundary) and 3/4 of the way to the first's
    d0 = orc.particle_distance(np.array([1.0]), np.array([1.0]), np.array([0.25]), box, nv, D)
    assert d0[0] == pytest.approx(0.25 * (0.5 * 7 + 1.0) + 0.75 * 1.0, abs=1e-14)
    rc = orc.cutoffs(np.array([0.0, 2.5, 5.0, 9.0]), (2.5, 6.0, 5.0))
    np.testing.assert_allclose(rc, [6.0, 4.25, 2.5, 2.5])


def test_slab_particle_cutoffs(orc):
    s = workloads.make("slab_small")
    out = orc.pipeline(s.x, s.y, s.z, s.box, s.h, s.rule, idx=np.arange(0, s.n, 50))
    # vapour particles sit at distance 0 and get rc_max
    vap = (s.z < 19.5) | (s.z > 40.5)
    assert np.all(out["delta"][vap] == 0.0)
    assert np.all(out["rc"][vap] == 6.0)
    # deep liquid particles get rc_min; in between delta is the distance from the
    # interface layer centre (analytic for the planar slab)
    mid = (s.z > 21.0) & (s.z < 24.0)
    np.testing.assert_allclose(out["delta"][mid], s.z[mid] - 20.5, atol=1e-12)
    deep = (s.z > 27.0) & (s.z < 33.0)
    assert np.all(out["rc"][deep] == 2.5)


# ---------------------------------------------------------------- Verlet

def test_verlet_time_reversible(orc):
    box = (9.0, 9.0, 9.0)
    x, y, z = _random_gas(50, box, seed=12, dmin=1.0)
    rng = np.random.default_rng(5)
    v = [rng.normal(0, 0.5, 50) for _ in range(3)]
    rc = np.full(50, 2.5)
    dt = 0.002

    def force(p):
        o = orc.forces(*p, rc, box, rule=orc.RULE_MAX)
        return (o["fx"], o["fy"], o["fz"])

    p0 = (x, y, z)
    p, vv = p0, v
    f = force(p)
    for sgn in (1, -1):
        if sgn < 0:
            vv = tuple(-a for a in vv)
        for _ in range(40):
            vv = orc.kick(vv, f, dt)
            p = orc.drift(p, vv, dt, box)
            f = force(p)
            vv = orc.kick(vv, f, dt)
    L = np.asarray(box)
    for a in range(3):
        d = p[a] - p0[a]
        d -= L[a] * np.rint(d / L[a])
        assert np.max(np.abs(d)) < 1e-9
    # with no force, drift is exact free flight
    xx = orc.drift((np.array([1.0]), np.array([2.0]), np.array([3.0])),
                   (np.array([0.5]), np.array([-1.0]), np.array([40.0])), 0.25, box)
    np.testing.assert_allclose([xx[0][0], xx[1][0], xx[2][0]], [1.125, 1.75, 4.0])


def test_wrap_range(orc):
    L = (3.0, 4.0, 5.0)
    x = np.array([-1e-17, 3.0, 6.5, -3.0, 2.9999999999999996])
    y = np.array([0.0, 4.0, -8.0, 7.99, 1.0])
    z = np.array([5.0, -0.1, 10.0, 1e-300, 4.9])
    wx, wy, wz = orc.wrap(x, y, z, L)
    for w, l in ((wx, 3.0), (wy, 4.0), (wz, 5.0)):
        assert np.all((w >= 0) & (w < l))
    assert wx[1] == 0.0 and wx[2] == 0.5 and wy[2] == 0.0
