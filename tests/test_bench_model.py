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


def _counter_csv(path, counter, rows):
    import csv
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, kib) in enumerate(rows):
            w.writerow([i + 1, name, counter, kib])


def test_counter_calibration_takes_the_reference_copy(tmp_path, monkeypatch):
    """The counters are scaled by what they read for the 1 GiB reference copy,
    which the run repeats; a larger clone of phi (2 GiB here) in the same run
    must not be taken for it."""
    gib = 1 << 30
    copy = "__amd_rocclr_copyBuffer"
    update = "void rsf::(anonymous namespace)::z_update_kernel<9, false, float, float, false, true>"
    fetch_dir, write_dir = tmp_path / "f", tmp_path / "w"
    fetch_dir.mkdir()
    write_dir.mkdir()
    # FETCH_SIZE reads half the bytes a copy moves, WRITE_SIZE all of them
    clone = [(copy, 2 * gib / 1024 * 0.5)]
    ref = [(copy, gib / 1024 * 0.5)] * 5
    _counter_csv(fetch_dir / "p_counter_collection.csv", "FETCH_SIZE",
                 clone + ref + [(copy, 2.0), (update, 3000.0 * 0.5), (update, 3000.0 * 0.5)])
    clone_w = [(copy, 2 * gib / 1024)]
    ref_w = [(copy, gib / 1024)] * 5
    _counter_csv(write_dir / "p_counter_collection.csv", "WRITE_SIZE",
                 clone_w + ref_w + [(copy, 0.03125), (update, 1000.0), (update, 1000.0)])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "synthetic")
    data = bench.ingest_counters(str(fetch_dir), str(write_dir), "synthetic", gib)
    entry = data["z_update@synthetic"]
    assert entry["fetch_factor"] == pytest.approx(0.5)
    assert entry["write_factor"] == pytest.approx(1.0)
    assert entry["bytes_per_launch"] == pytest.approx((3000.0 + 1000.0) * 1024, rel=1e-6)
    assert (tmp_path / "profiles" / "traffic.json").exists()
