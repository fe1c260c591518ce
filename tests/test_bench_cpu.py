"""The benchmark's command-line contract, checked without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, env=env)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "single GPU" in r.stderr
    assert r.stdout == ""


def test_a_distributed_launch_is_refused_too():
    env = dict(os.environ, WORLD_SIZE="4")
    r = _bench(env=env)
    assert r.returncode == 2
    assert "single GPU" in r.stderr


def test_help_lists_the_modes():
    r = _bench("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--batched-only", "--serving-only", "--streaming-only",
                 "--copy-probe", "--placement-probe", "--sweep-only", "--launch"):
        assert flag in r.stdout


def test_trace_summary_of_a_synthetic_kernel_trace(tmp_path):
    # A rocprofv3-shaped `kernels` table: two overlapping batches on two
    # queues, a gap, a third batch; a run break; a kernel on another queue.
    import json
    import sqlite3
    db = tmp_path / "t_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start int, end int, duration int, queue_id int)")
    rows = [("batch_kernel", 0, 100_000, 3), ("batch_kernel", 50_000, 150_000, 4),
            ("batch_kernel", 160_000, 200_000, 3), ("gen_kernel", 0, 10, 2),
            ("batch_kernel", 20_000_000, 20_100_000, 3), ("batch_kernel", 20_100_000, 20_200_000, 4),
            ("batch_kernel", 30_000_000, 30_050_000, 2)]
    for name, a, b, q in rows:
        con.execute("insert into kernels values (?,?,?,?,?)", (name, a, b, b - a, q))
    con.commit()
    con.close()
    r = _bench("--trace-summary", str(db), "--trace-kernels", "batch", "--trace-queues", "3,4")
    assert r.returncode == 0, r.stderr
    runs = [json.loads(l) for l in r.stdout.splitlines()]
    assert len(runs) == 2
    a, b = runs
    assert a["kernels"] == 3 and a["queues"] == [3, 4]
    assert a["span_ms"] == 0.2 and a["busy_ms"] == 0.19 and a["gaps"] == 1
    assert a["gap_max_us"] == 10.0 and a["kernel_sum_ms"] == 0.24
    assert a["mean_in_flight"] == round(0.24 / 0.19, 3)
    assert b["kernels"] == 2 and b["busy_frac"] == 1.0 and b["gaps"] == 0
    # Without the queue filter the queue-2 batch forms a third run.
    r = _bench("--trace-summary", str(db))
    assert [json.loads(l)["kernels"] for l in r.stdout.splitlines()] == [3, 2, 1]


def test_trace_overlap_of_a_synthetic_kernel_trace(tmp_path):
    import json
    import sqlite3
    db = tmp_path / "o_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start int, end int, duration int, queue_id int)")
    us = 1000
    rows = [("gen_kernel", 0, 10 * us, 1), ("d2h_kernel", 5 * us, 20 * us, 2),
            ("gen_kernel", 20 * us, 30 * us, 1), ("d2h_kernel", 25 * us, 40 * us, 2),
            ("d2h_kernel", 39 * us, 45 * us, 3), ("gen_kernel", 42 * us, 50 * us, 1),
            ("gen_kernel", 100 * us, 110 * us, 1)]
    for name, a, b, q in rows:
        con.execute("insert into kernels values (?,?,?,?,?)", (name, a, b, b - a, q))
    con.commit()
    con.close()
    r = _bench("--trace-overlap", str(db), "gen_kernel", "d2h_kernel")
    assert r.returncode == 0, r.stderr
    d = json.loads(r.stdout)
    assert d["a_kernels"] == 4 and d["a_queues"] == {"1": 4}
    assert d["b_kernels"] == 3 and d["b_queues"] == {"2": 2, "3": 1}
    assert d["a_total_ms"] == 0.038 and d["b_total_ms"] == 0.036
    # 5 + 5 + 3 us: the last two copies overlap each other and count once.
    assert d["overlap_ms"] == 0.013


def test_trace_stats_of_a_synthetic_kernel_trace(tmp_path):
    import json
    import sqlite3
    db = tmp_path / "s_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start int, end int, duration int, queue_id int)")
    name = "void rngx::(anonymous namespace)::batch_kernel<256, 16, false>(rngx::BatchDesc const*)"
    for i, d in enumerate([1000, 2000, 3000, 4000]):
        con.execute("insert into kernels values (?,?,?,?,?)", (name, 10**6 * i, 10**6 * i + d, d, 3))
    con.execute("insert into kernels values (?,?,?,?,?)", ("init_kernel(unsigned long*)", 0, 500, 500, 1))
    con.commit()
    con.close()
    r = _bench("--trace-stats", str(db))
    assert r.returncode == 0, r.stderr
    rows = [json.loads(l) for l in r.stdout.splitlines()]
    assert rows[0] == {"kernel": "void rngx::batch_kernel<256, 16, false>", "queue": 3, "calls": 4,
                       "total_us": 10.0, "mean_us": 2.5, "p50_us": 3.0, "p99_us": 4.0,
                       "max_us": 4.0}
    assert rows[1]["kernel"] == "init_kernel" and rows[1]["calls"] == 1


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counter_traffic_matches_the_kernel_code_of_the_launch():
    # Each committed headline counter line applies to launches that run the
    # same kernel code (chunks, non-temporal stores, scheduled or not),
    # whatever the block size or the schedule's rate, and to nothing else.
    b = _bench_module()
    lines = [l for l in open(os.path.join(ROOT, "profiles", "gen_kernel_u64_2p26x256.md"))
             if l.startswith("machine:")]
    assert lines
    alg = 8 * (1 << 26) * 256 + 16 * (1 << 26)
    keys = set()
    for line in lines:
        kv = dict(tok.split("=", 1) for tok in line.split()[1:])
        blk, ch, nt, pace = (int(x) for x in kv["launch"].split(","))
        same = {"block": blk, "chunks": ch, "nontemporal": bool(nt), "pace_gbs": pace}
        keys.add(b.launch_key(same))
        t = b.counter_traffic(same)
        assert t == int(kv["traffic_bytes_per_launch"]) and abs(t / alg - 1) < 1e-3
        assert b.counter_traffic(dict(same, block=1024 if blk != 1024 else 256)) == t
        if pace:
            assert b.counter_traffic(dict(same, pace_gbs=pace + 250)) == t
    for ch in (1, 2, 4):
        for nt in (False, True):
            for pace in (0, 7000):
                cfg = {"block": 512, "chunks": ch, "nontemporal": nt, "pace_gbs": pace}
                if b.launch_key(cfg) not in keys:
                    assert b.counter_traffic(cfg) is None
