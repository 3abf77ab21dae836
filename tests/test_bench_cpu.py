"""CPU checks of the bench's host logic: the one-GPU guard, the algorithmic
byte count of the dominant kernel, the counter-traffic record and the
autotuner database handling."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_schwarz_bytes_formula():
    # 8 bytes per stored inverse entry, (index + value) per gathered residual
    # entry, (index, read, write) per owned correction
    info = {"sum_om": 10, "sum_m": 3, "n_owned": 2}
    assert bench.ras_bytes(info, 8, 8) == 8 * 10 + 12 * 3 + 20 * 2
    assert bench.ras_bytes(info, 2, 4) == 2 * 10 + 8 * 3 + 12 * 2


def test_traffic_record_matches_the_kernel_source():
    """The committed counter traffic is reported only for the kernel code it
    was measured on; the current source must still be that code."""
    t = bench.measured_traffic()
    assert t is not None and 1.0 < t / 224534136 < 1.1


def test_tuning_database(tmp_path, monkeypatch):
    monkeypatch.delenv("FSI_TUNING_DB", raising=False)
    bench._TUNING_DB = None
    fresh = bench.tuning_db()
    assert os.path.exists(fresh) and os.path.getsize(fresh) == 0
    assert bench.tuning_db() == fresh                     # one file per run
    db = tmp_path / "t.db"
    db.write_text("spmv:J:f64:10:10:30 8\ngj3:372:336:1 3\ngjg:372:336:1:3 168\n")
    monkeypatch.setenv("FSI_TUNING_DB", str(db))
    assert bench.tuning_db() == str(db)
    ch = bench.tuning_choices(str(db))
    assert ch["gj_variant"] == {"gj3:372:336:1": "NB32 x 512, LDS panel, FP64"}
    assert ch["gj_grid"] == {"gjg:372:336:1:3": 168}
    assert bench.tuning_choices(str(tmp_path / "missing.db")) == {}


def test_inversion_traffic_record_matches_the_kernel_source():
    """The batched inversion's counter traffic is reported only for the code
    and the variant it was measured on; against the streamed-update model
    16 sum m^3 / (columns per streamed panel) of the 2D system
    (sum m^3 = 15,524,440,128) it is above 1 and below 1.5."""
    import re
    txt = open(bench.GJ_TRAFFIC_PROFILE).read()
    vid = int(re.search(r"^variant:\s*(\d+)", txt, re.M).group(1))
    t = bench.measured_traffic(bench.GJ_TRAFFIC_PROFILE, bench.gj_kernel_digest, vid)
    assert t is not None and 1.0 < t / (16 * 15524440128 / bench.GJ_VARIANTS[vid][1]) < 1.5
    assert bench.measured_traffic(bench.GJ_TRAFFIC_PROFILE, bench.gj_kernel_digest, vid + 1) is None
