"""Host-side parts of the benchmark's contract (no GPU needed): the refusal
of more than one GPU, the algorithmic byte model of a cell-update, and the
rule that a measured L2 traffic is reported only for the solver sources it
was measured on."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_algorithmic_bytes_per_cell():
    b = _bench()
    # E_g, F_g (3 N_g), E_gas, v (3) read and written in FP64, rho and the
    # opacity scale read, three int32 counters written
    for ng in (1, 4, 16, 64, 256):
        assert b.bytes_per_cell(ng) == 2 * 8 * (ng + 3 * ng + 1 + 3) + 2 * 8 + 3 * 4
    assert b.bytes_per_cell(16) == 1116 and b.bytes_per_cell(64) == 4188


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    b = _bench()
    sha = b.kernel_source_sha()
    assert len(sha) == 16 and sha == b.kernel_source_sha()   # deterministic
    kernel = "k_source_update<2, 32, 1, 4, false, true>"
    os.makedirs(tmp_path / "profiles")
    rec = {"kernel": kernel, "source_sha": sha, "traffic_bytes": 123.0}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps({"config2": rec}))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    # kernel_source_sha reads the sources under ROOT: point it back at the tree
    monkeypatch.setattr(b, "kernel_source_sha", lambda: sha)
    assert b.measured_traffic("config2", kernel) == 123.0
    assert b.measured_traffic("config1", kernel) is None                 # no record
    assert b.measured_traffic("config2", kernel.replace("32", "16")) is None  # other kernel
    monkeypatch.setattr(b, "kernel_source_sha", lambda: "0" * 16)
    assert b.measured_traffic("config2", kernel) is None                 # sources changed
