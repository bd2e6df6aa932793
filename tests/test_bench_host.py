"""Host logic of bench.py (no GPU): the one-GPU contract, the traffic
records taken from rocprofv3 counter databases (one per step-kernel
workgroup shape, one for the resampling pair), and the correctness gate,
exercised on a stand-in filter that runs the oracle's Algorithm 1 on the
host, with mistakes planted in it."""
import json
import math
import os
import sqlite3
import subprocess
import sys

import numpy as np
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
        rows.append((d, "void ppf::k_fill(ppf::Model, ppf::Buffers)", counter, 1.5))
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


def test_resampling_pair_traffic_record(tmp_path, records):
    f = str(tmp_path / "fetch.db")
    w = str(tmp_path / "write.db")
    counter_db(f, "FETCH_SIZE", [1.0] * 4, 0, 3, 4, 512.0 * 1024)
    counter_db(w, "WRITE_SIZE", [1.0] * 4, 0, 3, 4, 1024.0 * 1024)
    rec = bench.traffic_from(f, w, "wl", 1024, 3, 4, 0, kernel="k_resample")
    assert rec["shape"] is None
    # k_anc 5.0 + k_fill 1.5 KiB per step, scaled 2 (fetch) and 1 (write)
    assert rec["traffic_bytes_per_launch"] == (6.5 * 2.0 + 6.5) * 1024
    assert bench.load_traffic("k_resample", "wl", 1) == rec["traffic_bytes_per_launch"]


def test_batched_step_traffic_record(tmp_path, records):
    """The batch's record sums its fused and wide-patch step launches per step."""
    f = str(tmp_path / "fetch.db")
    w = str(tmp_path / "write.db")
    for path, counter, copy_kib in ((f, "FETCH_SIZE", 512.0 * 1024), (w, "WRITE_SIZE", 1024.0 * 1024)):
        con = sqlite3.connect(path)
        con.execute("create table counters_collection (dispatch_id integer, kernel_name text, "
                    "counter_name text, value real)")
        rows, d = [], 0
        for k in range(3 + 4):
            for name, kib in (("void ppf::k_step_batch_fused<1>(ppf::Model const*)", 30.0),
                              ("void ppf::k_step_batch_wide<15>(ppf::Model const*)", 4.0),
                              ("void ppf::k_anc_batch(ppf::Model const*)", 2.0)):
                d += 1
                rows.append((d, name, counter, kib if k >= 3 else 1.0))
        rows.append((d + 1, "__amd_rocclr_copyBuffer", counter, copy_kib))
        con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
        con.commit()
        con.close()
    rec = bench.traffic_from(f, w, "mt", 1024, 3, 4, 1, kernel="k_step_batch")
    assert rec["shape"] is None
    assert rec["traffic_bytes_per_launch"] == (34.0 * 2.0 + 34.0) * 1024
    assert bench.load_traffic("k_step_batch", "mt", None) == rec["traffic_bytes_per_launch"]


# ------------------------------------------------------- correctness gate
class OracleFilter:
    """Stand-in for the library's Filter, stepped by the oracle on the host
    with the library's storage: fp32 states, fp64 normalised log weights,
    the ancestors of the last resampling. `plant` plants one mistake."""

    def __init__(self, m, plant=None):
        import oracle
        self.o, self.m, self.n, self.plant = oracle, m, m.n, plant
        x, lw = oracle.init(m)
        self.x, self.lw = x.astype(np.float32), lw
        self.anc = np.arange(m.n, dtype=np.int32)
        self.resampled, self.k = False, 0
        self.st = dict(k=0, resampled=False, ess=float(m.n), max_logw=0.0, delta=0.0,
                       mean=np.zeros(5))

    def step(self, frame):
        o, m, n = self.o, self.m, self.n
        k = self.k + 1
        xp = o.propagate(m, k, self.x.astype(np.float64), self.anc if self.resampled else None)
        if self.plant == "propagate":
            xp[0] += 0.01
        x = xp.astype(np.float32)
        lw_in = np.full(n, -math.log(n)) if (k == 1 or self.resampled) else self.lw
        l = lw_in + o.loglik(m, frame, x.astype(np.float64))
        w, s = o.normalize(l)
        self.x, self.k = x, k
        self.lw = l - s["delta"]
        if self.plant == "weights":
            self.lw[::7] += 1e-3
        self.resampled = bool(s["ess"] < m.ess_threshold)
        self.anc = (o.resample_systematic(w, o.resample_uniform(m, k)) if self.resampled
                    else np.arange(n, dtype=np.int32))
        if self.plant == "ancestors" and self.resampled:
            self.anc = self.anc[::-1].copy()
        self.st = dict(k=k, resampled=self.resampled, ess=s["ess"], max_logw=s["m"],
                       delta=s["delta"], mean=o.estimate(w, x.astype(np.float64)))
        if self.plant == "ess":
            self.st["ess"] *= 1.01

    def stats(self):
        return dict(self.st)

    def particles(self):
        return self.x.copy(), self.lw.copy(), self.anc.copy()


@pytest.fixture(scope="module")
def small():
    from paper_1310_5045_amd import synth
    # the 128 x 128 workload with 2^16 particles over the central half of the
    # frame (4096 spread over the whole frame can lock onto the border, where
    # pixels read as noise-free background)
    w = dict(bench.WORKLOADS["sir_128x128_n4096_p9"], n=1 << 16, box=(32, 96, 32, 96))
    mv = synth.render_movie(w["W"], w["H"], w["T"], intensity=30.0, sigma=w["s"], background=10.0,
                            noise_sd=3.0, seed=1)
    return w, mv


def run_stand_in(w, mv, plant=None, steps=5):
    f = OracleFilter(bench.oracle_model(w, w["n"], 2), plant)
    for k in range(steps):
        f.step(mv.frames[k])
    return f


def test_gate_passes_a_correct_filter(small):
    w, mv = small
    f = run_stand_in(w, mv)
    err, st = bench.check_state(None, f, w, mv, 4, 0)
    assert err < 1.0 and st["k"] == 5
    bench.oracle_check_step(f, w, mv.frames, mv.frames, w["T"], 2)


@pytest.mark.parametrize("plant", ["ess", "ancestors", "weights"])
def test_gate_catches_a_wrong_state(small, plant):
    w, mv = small
    f = run_stand_in(w, mv, plant)
    with pytest.raises(bench.GateError):
        bench.check_state(None, f, w, mv, 4, 0)


@pytest.mark.parametrize("plant", ["propagate", "weights"])
def test_oracle_check_catches_a_wrong_step(small, plant):
    w, mv = small
    f = run_stand_in(w, mv)
    f.plant = plant  # the checked step goes wrong
    with pytest.raises(bench.GateError):
        bench.oracle_check_step(f, w, mv.frames, mv.frames, w["T"], 2)


def test_gate_catches_a_lost_track(small):
    w, mv = small
    f = run_stand_in(w, mv)
    far = mv.truth.copy()
    far[4, 0] += 5.0  # the truth is elsewhere: tracking error above 1 px
    with pytest.raises(bench.GateError, match="tracking"):
        bench.check_state(None, f, w, type(mv)(**{**mv.__dict__, "truth": far}), 4, 0)
