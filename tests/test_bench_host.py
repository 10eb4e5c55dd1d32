"""Host logic of the benchmark (no device): committed counter summaries are
used only when they were taken on the current traversal sources and on
dispatches of the benchmark's grid size (one summary per walk split), and the benchmark refuses more than
one GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_profiles_are_matched_by_source_digest_and_grid(tmp_path, monkeypatch):
    """A summary in the committed format is used only with the current
    traversal digest and the same grid (whether the committed summaries are
    current is not a property of the code: the bench line shows it)."""
    import bench
    from paper_2405_16634_amd.profiling import traversal_digest
    name = "traffic_traverse_A_torusknot500k_split512"
    d = json.load(open(os.path.join(ROOT, "profiles", name + ".json")))
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    cur = dict(d, source_sha=traversal_digest())
    (tmp_path / "profiles" / (name + ".json")).write_text(json.dumps(cur))
    assert bench.load_profile(name, d["grid_threads"])["bytes_per_launch"] == d["bytes_per_launch"]
    assert bench.load_profile(name, d["grid_threads"] + 64) is None
    # a summary taken on other sources is not used
    stale = dict(d, source_sha="0" * 16)
    (tmp_path / "profiles" / (name + ".json")).write_text(json.dumps(stale))
    assert bench.load_profile(name, d["grid_threads"]) is None
    assert bench.load_profile("missing_profile") is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stdout + p.stderr
