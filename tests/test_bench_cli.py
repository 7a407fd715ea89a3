"""bench.py's command-line contract on the host: more than one GPU is refused with exit
status 2 and a message, before anything touches a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_refuses_a_distributed_launch():
    env = dict(os.environ, WORLD_SIZE="2")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], capture_output=True, text=True,
                       timeout=120, cwd=ROOT, env=env)
    assert r.returncode == 2
    assert "--gpus 1" in r.stderr


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_budget_counts_from_process_start_and_skips():
    b = _bench_module()
    bud = b.Budget(5.0)
    assert bud.left() <= 5.0
    assert not bud.fits(10.0)
    rec = b.skipped(10.0, bud)
    assert rec["skipped"] == "budget" and rec["estimate_s"] == 10.0
    assert b.Budget(0).fits(1e9)  # 0 = no budget


def test_guarded_arm_turns_errors_into_records():
    b = _bench_module()
    assert b.guarded(lambda: {"ok": 1}) == {"ok": 1}
    rec = b.guarded(lambda: 1 / 0)
    assert "ZeroDivisionError" in rec["error"]


def test_profiles_of_several_timed_solves_add_up():
    b = _bench_module()
    p = {"fp_stage": {"launches": 2, "total_ms": 1.5, "alg_bytes": 10.0}}
    q = {"fp_stage": {"launches": 3, "total_ms": 2.0, "alg_bytes": 5.0}}
    assert b.add_prof(None, p) == p
    assert b.add_prof(p, q) == {"fp_stage": {"launches": 5, "total_ms": 3.5, "alg_bytes": 15.0}}


def test_traffic_ratio_only_for_its_shape_kernel_and_source(tmp_path, monkeypatch):
    # the counter ratio of a committed summary is used only for the launch shape, the kernel
    # and the stencil source it was taken on
    import json
    b = _bench_module()
    shape = [3, 8, 2, 64, 2, 4]
    assert b.traffic_kernel(shape, triple=True) == "ztrip_kernel"
    assert b.traffic_kernel(shape, triple=False) == "zpair_tall_kernel<0>"
    assert b.traffic_kernel([2, 8, 3, 64, 1, 4]) == "zpair_dma_kernel<0, 4>"
    assert "three middle factors" in b.middle_kernel_name(shape, triple=True)
    monkeypatch.setattr(b, "PROFILES", str(tmp_path))
    rec = {"kernel": "ztrip_kernel", "source_hash": b.source_hash(), "shape": shape,
           "bytes_per_launch": 3.0e9, "alg_bytes_per_launch": 2.5e9}
    with open(b.traffic_file(shape), "w") as fh:
        json.dump(rec, fh)
    assert abs(b.measured_traffic(shape, "ztrip_kernel") - 1.2) < 1e-12
    assert b.measured_traffic(shape, "zpair_tall_kernel<0>") is None
    assert b.measured_traffic([3, 8, 2, 64, 2, 1], "ztrip_kernel") is None
    rec["source_hash"] = "0" * 16
    with open(b.traffic_file(shape), "w") as fh:
        json.dump(rec, fh)
    assert b.measured_traffic(shape, "ztrip_kernel") is None
