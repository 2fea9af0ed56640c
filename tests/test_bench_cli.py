"""Host logic of bench.py that runs without a GPU: it measures one GPU only, so a request for
several GPUs (or a multi-rank launch) ends with a message and exit status 2 before anything
touches the device; and the HBM traffic it reports is read from the committed counter summary
only when that summary belongs to the same apply kernels and workload."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, env=e, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "8"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout


def test_multi_rank_launch_is_refused():
    r = _run([], env={"WORLD_SIZE": "2"})
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_taken_only_from_a_matching_profile(tmp_path, monkeypatch):
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench
    prof = json.load(open(os.path.join(ROOT, "profiles", "apply_counters.json")))
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2009_10173_amd", "csrc", "apply.hip"),
                              "rb").read()).hexdigest()
    got = bench.profiled_traffic(prof["workload"], "fp32", "adjoint")
    if prof["apply_hip_sha256"] == sha:
        assert got == prof["kernels"]["apply fp32 adjoint"]["bytes"]
    else:
        assert got is None
    assert bench.profiled_traffic("another_workload", "fp32", "adjoint") is None
    # a summary taken with other apply kernels is ignored
    fake = tmp_path / "profiles"
    fake.mkdir()
    (fake / "apply_counters.json").write_text(json.dumps(dict(prof, apply_hip_sha256="0" * 64)))
    src = tmp_path / "paper_2009_10173_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "apply.hip").write_bytes(b"// other kernels\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic(prof["workload"], "fp32", "adjoint") is None
