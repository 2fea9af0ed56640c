"""Host logic of bench.py that runs without a GPU: it measures one GPU only, so a request for
several GPUs (or a multi-rank launch) ends with a message and exit status 2 before anything
touches the device; and the HBM traffic it reports is read from the committed counter summary
only when that summary belongs to the same apply kernels and workload."""
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
    got = bench.profiled_traffic(prof["workload"], "fp32", "adjoint")
    if prof["kernel_code_digest"] == bench.kernel_code_digest():
        assert got == prof["kernels"]["apply fp32 adjoint"]["bytes"]
    else:
        assert got is None
    assert bench.profiled_traffic("another_workload", "fp32", "adjoint") is None
    # the digest ignores comments and layout but not code
    src = tmp_path / "paper_2009_10173_amd" / "csrc"
    src.mkdir(parents=True)
    for name in bench.KERNEL_SOURCES:
        path = os.path.join(ROOT, "paper_2009_10173_amd", "csrc", name)
        (src / name).write_text(open(path).read())
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "apply_counters.json").write_text(json.dumps(prof))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_code_digest()
    apply_src = src / "apply.hip"
    text = apply_src.read_text()
    apply_src.write_text("// a new comment line\n" + text.replace("\n", "\n\n", 3))
    assert bench.kernel_code_digest() == base
    apply_src.write_text(text + "\nstatic int one_more_symbol = 1;\n")
    assert bench.kernel_code_digest() != base
    assert bench.profiled_traffic(prof["workload"], "fp32", "adjoint") is None
