"""Host-side rules of bench.py (no GPU): which counter-measured traffic a
bench line may carry, and the cell count the bulk kernel skips on open faces."""
import json
import os

import numpy as np

import bench
from paper_2506_21804_amd import inputs as I


def _write(tmp_path, name, **kw):
    t = {"kernel_hash": bench.kernel_source_hash(), "collision": "bgk", "fd_weight": 0.0, "bytes_per_launch": 123}
    t.update(kw)
    (tmp_path / f"k_bulk_{name}_traffic.json").write_text(json.dumps(t))


def test_traffic_only_for_the_kernel_it_was_measured_on(tmp_path):
    _write(tmp_path, "w")
    assert bench.measured_traffic("w", "bgk", 0.0, str(tmp_path)) == 123
    assert bench.measured_traffic("w", "rr3", 0.0, str(tmp_path)) is None
    assert bench.measured_traffic("w", "rr3", 0.3, str(tmp_path)) is None
    assert bench.measured_traffic("other", "bgk", 0.0, str(tmp_path)) is None
    _write(tmp_path, "stale", kernel_hash="0000")
    assert bench.measured_traffic("stale", "bgk", 0.0, str(tmp_path)) is None
    _write(tmp_path, "old")  # files written before the collision was recorded
    t = json.loads((tmp_path / "k_bulk_old_traffic.json").read_text())
    del t["collision"]
    (tmp_path / "k_bulk_old_traffic.json").write_text(json.dumps(t))
    assert bench.measured_traffic("old", "bgk", 0.0, str(tmp_path)) is None


def test_committed_traffic_files_name_their_collision():
    prof = os.path.join(bench.ROOT, "profiles")
    for f in os.listdir(prof):
        if f.endswith("_traffic.json"):
            t = json.load(open(os.path.join(prof, f)))
            assert t["collision"] in ("bgk", "rr3") and "fd_weight" in t and "kernel_hash" in t, f


def test_open_face_cells():
    c = I.urban(64, 32, 16, q=27, with_wall_dist=False, open_x=True, fringe_len=8, x_lo=8, x_hi=40, h_mean=6.0,
                h_max=12, fp_lo=4, fp_hi=8)
    m = np.asarray(c.mask).reshape(16, 32, 64)[:-1] != 0  # the lid plane stays a lid
    assert bench.open_face_cells(c) == int(m[:, :, 0].sum() + m[:, :, -1].sum())
    assert bench.open_face_cells(I.channel(16, 8, 10, q=19)) == 0
