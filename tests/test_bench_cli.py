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


def test_cpu_detail_scales_its_sample_to_the_whole_workload():
    """The oracle timing leg on the 16x16 case: the band entries it counts on the full table
    equal the count it is given, and every figure is scaled from a sample that is a fraction
    of the workload (so the scaled time is at least the sample's)."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import numpy as np

    import bench
    import workloads as W
    from oracle import model as omodel
    cfg = W.config("tiny")
    g = cfg["grid"]
    H = omodel.build_table(cfg["sensor"], g)
    nzr = H != 0
    present = nzr.any(axis=-1)
    first = np.argmax(nzr, axis=-1)
    last = g["nt"] - 1 - np.argmax(nzr[..., ::-1], axis=-1)
    length = np.where(present, last - first + 1, 0)
    K = g["k_half"]
    d = np.abs(np.arange(-K, K + 1))
    pairs = (g["ny"] - d)[:, None] * (g["nx"] - d)[None, :]
    nnz, mac = int(length.sum()), int(np.sum(pairs[:, :, None] * length))
    out = bench.cpu_detail(cfg, nnz, mac, iters=3)
    assert out["table_band_entries"] == {"oracle": nnz, "model": nnz}
    assert out["1"]["blas_threads"] == 1 and out["1"]["workers"] == 1
    for label in ("1", "all"):
        r = out[label]
        smp = r["sample_s"]
        assert r["pair_s"] >= smp["forward"] + smp["adjoint"] > 0
        assert r["recon_s"] > 0
    assert out["1"]["table_build_s"] >= out["1"]["sample_s"]["table"]
    assert "depth slabs" in out["sample"]


def test_cpu_baseline_reports_the_oracle_rate_on_its_sample():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench
    import workloads as W
    from oracle import model as omodel
    cfg = W.config("tiny")
    g = cfg["grid"]
    _, mac = bench._sample_work(omodel.build_table(cfg["sensor"], g), g)
    out = bench.cpu_baseline(cfg, mac)
    assert out["kind"] == "oracle" and out["unit"] == "A+A^T pairs/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "depth slabs" in out["sample"]
