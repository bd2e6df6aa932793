"""Host logic of bench.py (no GPU): the one-GPU contract and the traffic
records taken from rocprofv3 counter databases, one per step-kernel
workgroup shape."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def counter_db(path, counter, step_kib, shape, warmup, steps, copy_kib):
    """A database shaped like rocprofv3's: warm-up and timed launches of the
    step kernel between other kernels, then the calibration copy."""
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, "
                "counter_name text, value real)")
    d = 0
    rows = []
    for k in range(warmup + steps):
        d += 1
        kib = step_kib[k - warmup] if k >= warmup else 1.0  # warm-up launches read differently
        # a dispatch's counter arrives in several instances, summed per dispatch
        rows += [(d, f"void ppf::k_step_spot<13, {shape}>(ppf::Model, ppf::Buffers, float const*)",
                  counter, kib / 2), (d, f"void ppf::k_step_spot<13, {shape}>(ppf::Model, "
                                         "ppf::Buffers, float const*)", counter, kib / 2)]
        d += 1
        rows.append((d, "void ppf::k_anc(ppf::Model, ppf::Buffers, ppf::WeightSrc)", counter, 5.0))
    d += 1
    rows.append((d, "__amd_rocclr_copyBuffer", counter, copy_kib))
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()


@pytest.fixture
def records(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "traffic_path",
                        lambda kernel, workload, shape:
                        str(tmp_path / f"traffic_{kernel}_shape{shape}_{workload}.json"))
    return tmp_path


def test_traffic_record_from_counter_databases(tmp_path, records):
    steps, warmup = 4, 3
    f = str(tmp_path / "fetch.db")
    w = str(tmp_path / "write.db")
    # FETCH_SIZE reads half of the copy's bytes (scale 2), WRITE_SIZE all (scale 1)
    counter_db(f, "FETCH_SIZE", [100.0, 110.0, 90.0, 100.0], 1, warmup, steps, 512.0 * 1024)
    counter_db(w, "WRITE_SIZE", [200.0, 200.0, 200.0, 200.0], 1, warmup, steps, 1024.0 * 1024)
    rec = bench.traffic_from(f, w, "wl", 1024, warmup, steps, 1)
    assert rec["shape"] == 1
    assert rec["counters"]["FETCH_SIZE"]["kernel_kib_avg"] == 100.0  # the timed launches only
    assert rec["counters"]["FETCH_SIZE"]["scale"] == 2.0
    assert rec["counters"]["WRITE_SIZE"]["scale"] == 1.0
    assert rec["traffic_bytes_per_launch"] == (100.0 * 2.0 + 200.0) * 1024
    assert "--shape 1" in rec["command"][0]
    # reported only for its own shape and while the kernel sources are unchanged
    assert bench.load_traffic("k_step", "wl", 1) == rec["traffic_bytes_per_launch"]
    assert bench.load_traffic("k_step", "wl", 0) is None
    path = bench.traffic_path("k_step", "wl", 1)
    stale = json.load(open(path))
    stale["source_sha256"] = "0" * 64
    json.dump(stale, open(path, "w"))
    assert bench.load_traffic("k_step", "wl", 1) is None


def test_traffic_record_refuses_another_shape(tmp_path, records):
    f = str(tmp_path / "fetch.db")
    w = str(tmp_path / "write.db")
    counter_db(f, "FETCH_SIZE", [1.0] * 4, 0, 3, 4, 512.0)
    counter_db(w, "WRITE_SIZE", [1.0] * 4, 0, 3, 4, 1024.0)
    with pytest.raises(SystemExit, match="shape 1"):
        bench.traffic_from(f, w, "wl", 1, 3, 4, 1)
    # too few launches for the warm-up and timed steps
    with pytest.raises(SystemExit, match="expected at least"):
        bench.traffic_from(f, w, "wl", 1, 10, 4, 0)
