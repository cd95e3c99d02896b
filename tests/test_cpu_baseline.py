"""The CPU cell-list baseline (Algorithms 2.2-2.3 with OpenMP dynamic
scheduling) that the benchmark times for context gives the O(N^2) oracle's
pairs and forces: neighbour counts equal, forces within summation order."""
import numpy as np
import pytest

import workloads


def _F(d):
    return np.stack([d["fx"], d["fy"], d["fz"]], 1)


@pytest.mark.parametrize("edge", [2.5, 1.0, 6.0])
def test_cell_list_baseline_matches_the_oracle_on_the_small_slab(orc, edge):
    s = workloads.make("slab_small")
    p = orc.pipeline(s.x, s.y, s.z, s.box, s.h, s.rule)
    rc = p["rc"]
    ref = orc.forces(s.x, s.y, s.z, rc, s.box)
    got = orc.cpu_cells_forces(s.x, s.y, s.z, rc, s.box, edge)
    np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
    assert got["pairs"] == int(ref["nnbr"].sum())
    R = _F(ref)
    frms = np.sqrt(np.mean(np.sum(R * R, 1)))
    assert np.max(np.linalg.norm(_F(got) - R, axis=1)) <= 1e-12 * frms
    assert got["E"] == pytest.approx(ref["E"], rel=1e-12)


def test_cell_list_baseline_on_a_subset_and_a_small_box(orc):
    """Listed particles only (their sums over all j), in a box where the
    cutoff reaches round the periodic bins (4.9 sigma in 10 sigma)."""
    rng = np.random.default_rng(np.random.PCG64(5))
    n = 700
    L = (10.0, 11.0, 10.5)
    pos = rng.uniform(0, 1, (n, 3)) * L
    rc = rng.uniform(1.0, 4.9, n)
    idx = rng.choice(n, 97, replace=False)
    ref = orc.forces(pos[:, 0], pos[:, 1], pos[:, 2], rc, L, idx=idx)
    got = orc.cpu_cells_forces(pos[:, 0], pos[:, 1], pos[:, 2], rc, L, 2.4, idx=idx)
    np.testing.assert_array_equal(got["nnbr"], ref["nnbr"])
    R = _F(ref)
    scale = np.max(np.linalg.norm(R, axis=1))
    assert np.max(np.linalg.norm(_F(got) - R, axis=1)) <= 1e-12 * scale
