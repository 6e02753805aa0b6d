"""Seeded workload generators: determinism, geometry rules, probe sets, and the
paper's Table 1 lattice-velocity convention."""
import json
import math
import os

import numpy as np
import pytest

from paper_2508_18202_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_vector():
    # published test vector of splitmix64 for seed 1234567
    r = inputs.SplitMix64(1234567)
    assert [r.next() for _ in range(5)] == [6457827717110365317, 3203168211198807973,
                                            9817491932198370423, 4593380528125082431,
                                            16408922859458223821]


def test_geometry_hashes_are_stable():
    with open(os.path.join(GOLDEN, "geometry_hashes.json")) as fh:
        want = json.load(fh)
    ws = [inputs.small_block(), inputs.urban_les(), inputs.adjoint_case(), inputs.assimilation_case(), inputs.cylinder_gpc()] + inputs.uneven_cases()
    for w in ws:
        assert inputs.mask_hash(inputs.solid_mask(w)) == want[w.name], w.name


@pytest.mark.parametrize("w,F,nb", [(inputs.urban_les(), 16, 24), (inputs.adjoint_case(), 10, 12),
                                   (inputs.assimilation_case(), 16, 60)])
def test_building_array_rules(w, F, nb):
    m = inputs.solid_mask(w)
    assert m.shape == (w.nz, w.ny, w.nx)
    foot = m[0]
    # connected footprints: count squares by scanning rows of the ground plane
    from scipy.ndimage import label
    lab, n = label(foot)
    assert n == nb
    for k in range(1, n + 1):
        ys, xs = np.nonzero(lab == k)
        assert xs.max() - xs.min() + 1 == F and ys.max() - ys.min() + 1 == F
        h = m[:, ys[0], xs[0]].sum()
        assert 8 <= h <= min(40, w.nz - 8)
        assert (m[:h, ys[0], xs[0]] == 1).all()
    # buildings stay away from the inflow/outflow faces and the sky
    assert not m[:, :, : w.nx // 8].any() and not m[:, :, (3 * w.nx) // 4:].any()
    assert not m[w.nz - 8:].any()


def test_uneven_case_footprints():
    for w in inputs.uneven_cases()[::16]:
        from scipy.ndimage import label
        lab, n = label(inputs.solid_mask(w)[0])
        assert n == 24
        F = {128: 8, 192: 12, 256: 16}[w.nx]
        assert (lab == 1).sum() == F * F


def test_small_block_geometry():
    m = inputs.solid_mask(inputs.small_block())
    assert m.sum() == 6 * 6 * 8 and m[0:8, 5:11, 10:16].all()


def test_probe_sets():
    w4 = inputs.adjoint_case()
    m4 = inputs.solid_mask(w4)
    p4 = inputs.probe_cells(w4, m4)
    assert len(p4) == 32 * 16 and (m4.reshape(-1)[p4] == 0).all()
    assert (p4 % w4.nx == 96).all()
    w5 = inputs.assimilation_case()
    m5 = inputs.solid_mask(w5)
    p5 = inputs.probe_cells(w5, m5)
    assert len(p5) == 64 and len(set(p5.tolist())) == 64
    assert (m5.reshape(-1)[p5] == 0).all()
    assert (p5 // (w5.nx * w5.ny) == 10).all()


def test_table1_lattice_velocity():
    """Table 1: Ma = 0.034641 with Ma = u / c_s and c_s^2 = 1/3 (Sec. 2.2) gives
    the lattice velocity 0.02, the magnitude of the workloads' inflow speeds."""
    from oracle import oracle as orc
    with open(os.path.join(GOLDEN, "paper_table1.json")) as fh:
        t = json.load(fh)
    c, w, _ = orc.lattice()
    cs = math.sqrt((w * c[:, 0] ** 2).sum())
    assert abs(t["Ma"] * cs - 0.02) < 1e-6
    assert t["collocation_points_per_dim"] ** 2 == t["collocation_points_total"]


def test_cylinder_mask_rules():
    w = inputs.cylinder_gpc()
    m = inputs.solid_mask(w)
    R = w.cylinder_radius
    assert m.shape == (40, 544, 544) and w.nx == w.ny == 2 * int(R) + 4
    mant = m[0] == 2
    # a ring of mantle cells surrounds the disk: the box border is mantle
    assert mant[0].all() and mant[-1].all() and mant[:, 0].all() and mant[:, -1].all()
    # the disk holds about pi R^2 columns (Gauss circle problem: error O(R))
    assert abs((~mant).sum() - math.pi * R * R) < 4 * R
    # the mantle region is the same in every layer and symmetric under a half
    # turn and a quarter turn about the axis
    assert ((m == 2) == mant[None]).all()
    assert (mant == mant[::-1, ::-1]).all() and (mant == mant.T[:, ::-1]).all()
    # two blocks on the ground, inside the central square of side R
    from scipy.ndimage import label
    lab, n = label(m[0] == 1)
    assert n == 2
    ys, xs = np.nonzero(m[0] == 1)
    c = w.nx // 2
    assert xs.min() >= c - R // 2 and xs.max() < c + R // 2
    assert (m[-1] != 1).all()
