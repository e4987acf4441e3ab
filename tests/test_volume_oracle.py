"""Pins of the oracle's volume-level driver (Sec. 4.1): the split into
curtained sub-volumes and the linear-interpolation merge, against facts that
do not come from the oracle's own code."""
import numpy as np
import pytest

import oracle


def P(sigma=1.0):
    return oracle.params_array(sigma, 1.0, 1.0, 0.001, 1.0, 0.1, 1.0, 1e-10)


@pytest.mark.parametrize("shape,block,curtain", [((30, 41, 52), 14, 3), ((17, 60, 9), 20, 4),
                                                 ((64, 64, 64), 21, 5), ((12, 12, 12), 100, 3)])
def test_weights_partition_unity_and_cover(shape, block, curtain):
    boxes = oracle.volume_boxes(shape, block, curtain)
    total = np.zeros(shape)
    for sl, w in boxes:
        assert w.shape == tuple(s.stop - s.start for s in sl)
        assert np.all(w >= 0) and np.all(w <= 1)
        total[sl] += w
    assert np.max(np.abs(total - 1.0)) < 1e-14


def test_cores_are_near_equal_and_at_most_block():
    for n in (7, 50, 100, 101, 512, 1000):
        for block in (7, 20, 64, 500):
            cuts = oracle.volume_cores(n, block)
            sizes = np.diff(cuts)
            assert cuts[0] == 0 and cuts[-1] == n
            assert sizes.max() <= block and sizes.max() - sizes.min() <= 1


def test_merge_is_linear_across_the_curtain():
    """Two parts along x holding constants a and b: the merged profile is a,
    then a straight line from a to b across the 2C overlap, then b."""
    shape, block, C = (4, 5, 40), 20, 4
    boxes = oracle.volume_boxes(shape, block, C)
    assert len(boxes) == 2
    a, b = 2.0, -1.0
    fields = [np.full([s.stop - s.start for s in sl], v) for (sl, _), v in zip(boxes, (a, b))]
    row = oracle.merge_boxes(shape, boxes, fields)[2, 3]
    assert np.allclose(row[:20 - C], a) and np.allclose(row[20 + C:], b)
    ramp = row[20 - C:20 + C]
    assert np.allclose(np.diff(ramp), (b - a) / (2 * C))
    assert abs(ramp.mean() - 0.5 * (a + b)) < 1e-14      # symmetric about the core face


def test_zero_iterations_reproduce_phi0():
    r = np.random.default_rng(3)
    I = r.uniform(0, 1, size=(20, 24, 28))
    phi0 = r.normal(size=I.shape)
    got = oracle.evolve_volume(I, phi0, P(), 0, 10, 2)
    assert np.max(np.abs(got - phi0)) < 1e-14


def test_single_subvolume_is_plain_evolution():
    r = np.random.default_rng(4)
    I = r.uniform(0, 1, size=(14, 15, 16))
    phi0 = np.where(r.uniform(size=I.shape) > 0.5, 2.0, -2.0)
    a = oracle.evolve_volume(I, phi0, P(), 3, 64, 3)
    b, _ = oracle.evolve(I, phi0, P(), 3)
    assert np.array_equal(a, b)


def test_outside_overlaps_the_merge_is_the_whole_volume_result():
    """One iteration with sigma = 1 reaches R + 2 = 5 voxels (Gaussian
    radius 3, then the 2-voxel update stencil).  A voxel outside every
    overlap has weight one in a single sub-volume and lies at least 2C from
    that sub-volume's cut faces, so with 2C >= 5 its merged value is the
    whole-volume value (volume faces are treated alike in both).  Inside the
    overlaps the blend only reduces the seam: sub-volume values near their
    cut faces keep a small weight, as the paper's curtains minimise rather
    than remove template artefacts."""
    r = np.random.default_rng(5)
    I = r.uniform(0, 1, size=(24, 26, 40))
    phi0 = r.normal(size=I.shape)
    whole, _ = oracle.evolve(I, phi0, P(), 1)
    C = 3
    split = oracle.evolve_volume(I, phi0, P(), 1, 12, C)
    single = np.zeros(I.shape, dtype=bool)
    for sl, w in oracle.volume_boxes(I.shape, 12, C):
        single[sl] |= w == 1.0
    assert single.mean() > 0.05
    assert np.max(np.abs(whole - split)[single]) < 1e-12
    assert np.max(np.abs(whole - split)[~single]) > 1e-6      # the seam is reduced, not removed
