"""Host-side logic of bench.py (no GPU): the one-GPU guard and the rule
that a recorded HBM-traffic figure is reported only while the kernel source
it was measured on is unchanged."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    for args, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})):
        e = dict(os.environ, **env)
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args,
                           capture_output=True, text=True, env=e, timeout=120)
        assert r.returncode == 2, (args, env, r.stderr)
        assert "one GPU" in r.stderr
        assert r.stdout == ""


def test_recorded_traffic_follows_the_source(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2006_15367_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = csrc / "m2l.hip"
    src.write_bytes(b"// kernel source\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "profiles" / "m2l_sphere262k_hbm_traffic.txt"
    prof.write_text("# header = ignored\ntraffic_bytes_per_launch = 1234\nnrhs = 1\n"
                    "source_sha256 = %s\n" % digest)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("m2l", "sphere262k", 1) == 1234.0
    assert bench.recorded_traffic("m2l", "sphere262k", 64) is None  # other RHS count
    assert bench.recorded_traffic("m2l", "spheroid1m", 1) is None  # no profile
    src.write_bytes(b"// kernel source, changed\n")
    assert bench.recorded_traffic("m2l", "sphere262k", 1) is None
