"""Host-side pieces of bench.py (no GPU): the counter-summary lookup, the
multi-GPU refusal and the CPU model of the baseline."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _fake_tree(tmp_path, kernel_src, sha, lines):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_1902_00088_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "paper_1902_00088_amd" / "csrc" / "kernels.hip").write_bytes(kernel_src)
    text = "# counters\n\ntraffic_sha256: " + sha + "\n" + "\n".join(lines) + "\n"
    (tmp_path / "profiles" / "stage_traffic_counters.md").write_text(text)


def test_counter_traffic_reads_the_line_of_the_tiling_while_the_source_matches(tmp_path, monkeypatch):
    src = b"// kernel source\n"
    sha = hashlib.sha256(src).hexdigest()
    _fake_tree(tmp_path, src, sha, ["traffic_bytes_per_launch c2 nsub 4: 2047807",
                                    "traffic_bytes_per_launch c2 nsub 1 t512: 2094173"])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("c2 nsub 4") == 2047807.0
    assert bench.counter_traffic("c2 nsub 1" + bench.tkey({"stage_threads": 512})) == 2094173.0
    assert bench.counter_traffic("c2 nsub 2") is None          # not measured
    assert bench.tkey({"stage_threads": 256}) == "" and bench.tkey({}) == ""


def test_traffic_key_names_the_kernel_the_run_used():
    stage = {"stage_tiles": 4, "stage_threads": 256}
    assert bench.traffic_key("c2", stage, "stage") == "c2 nsub 4"
    tile = {"rk4_tile": {"tiles": 2, "analysis_folded": [1, 1024], "refine_folded": [1, 1, 512],
                         "mothers_folded": [1, 256]}}
    assert bench.traffic_key("c2", tile, "rk4_tile") == "c2 rk4_tile nsub 1 t256 analysis refine mothers"
    tile["rk4_tile"]["mothers_folded"] = [0, 256]
    assert bench.traffic_key("c2", tile, "rk4_tile") == "c2 rk4_tile nsub 1 t512 analysis refine"
    tile["rk4_tile"]["refine_folded"] = [0, 1, 512]
    assert bench.traffic_key("c2", tile, "rk4_tile") == "c2 rk4_tile nsub 1 t1024 analysis"
    tile["rk4_tile"]["analysis_folded"] = [-1, 256]
    assert bench.traffic_key("c2", tile, "rk4_tile") == "c2 rk4_tile nsub 2"
    assert bench.traffic_key("c2", stage, "mr") is None and bench.counter_traffic(None) is None


def test_counter_traffic_is_void_once_the_kernel_source_changes(tmp_path, monkeypatch):
    src = b"// kernel source\n"
    _fake_tree(tmp_path, src, hashlib.sha256(b"// older source\n").hexdigest(),
               ["traffic_bytes_per_launch c2 nsub 4: 2047807"])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("c2 nsub 4") is None


def test_committed_counter_summary_parses():
    """The committed summary has a hash line and at least one figure per workload."""
    text = open(os.path.join(ROOT, "profiles", "stage_traffic_counters.md")).read()
    assert any(l.startswith("traffic_sha256: ") for l in text.splitlines())
    for w in ("c2", "c4"):
        vals = [float(l.split(":", 1)[1]) for l in text.splitlines()
                if l.startswith(f"traffic_bytes_per_launch {w} nsub ")]
        assert vals and all(v > 0 for v in vals)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_cpu_model_names_the_host_processor():
    name = bench.cpu_model()
    assert name is None or (isinstance(name, str) and name.strip())
    if name and os.path.exists("/proc/cpuinfo"):
        want = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")), None)
        if want:
            assert name.startswith(want)
