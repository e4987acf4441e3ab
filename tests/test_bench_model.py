"""The measurement model of bench.py (host only): the algorithmic bytes per
voxel of each pass, the volume driver's curtained extents against the
oracle's own sub-volume boxes, and the counter calibration."""
import numpy as np
import pytest

import bench
import oracle


def test_path_bytes_per_voxel_iteration():
    # RSF force: 72 B in FP32, 42 B with FP16 storage and a uint16 image
    assert sum(bench.pass_bytes(4, 4).values()) == 72
    assert sum(bench.pass_bytes(2, 2).values()) == 42
    # Sec. 4.2 force, sigma2 = 0: 48 B; fused update with the next stage-1
    # pass: 44 B (FP32), 30 B (FP16 storage, uint16 image)
    assert sum(bench.pass_bytes(4, 4, paper=True).values()) == 48
    assert sum(bench.pass_bytes(4, 4, paper=True, fused=True).values()) == 44
    assert sum(bench.pass_bytes(2, 2, paper=True, fused=True).values()) == 30
    assert "z_heaviside" not in bench.pass_bytes(4, 4, paper=True, fused=True)


@pytest.mark.parametrize("shape,block,curtain", [((100, 50, 70), 30, 4), ((64, 64, 64), 32, 9),
                                                 ((37, 90, 41), 20, 3), ((30, 30, 30), 100, 5)])
def test_curtained_extents_match_the_oracle_boxes(shape, block, curtain):
    boxes = oracle.volume_boxes(shape, block, curtain)
    want = sum(int(np.prod([s.stop - s.start for s in sl])) for sl, _ in boxes)
    got = 1
    for n in shape:
        got *= sum(bench.curtained_extents(n, block, curtain))
    assert got == want


def test_roofline_prices_the_dominant_pass():
    prof = {"z_heaviside": (10, 4.0), "xy_fits": (10, 5.0), "z_update": (10, 7.0),
            "reduce": (10, 0.05)}
    r = bench.roofline(prof, bench.pass_bytes(4, 4), 1_000_000, "no-such-workload")
    assert r["kernel"] == "z_update"
    assert r["avg_launch_ms"] == pytest.approx(0.7)
    assert r["achieved"] == pytest.approx(20 * 1_000_000 / 0.7e-3 / 1e9, rel=1e-3)
    assert r["traffic"] is None
