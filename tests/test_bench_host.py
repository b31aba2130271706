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
    # a summary that names its per-level forms applies only to those forms
    prof.write_text("traffic_bytes_per_launch = 1234\nnrhs = 1\nsource_sha256 = %s\n"
                    "forms = [-1, -1, 8, 7, 7, 8, 7]\n" % digest)
    assert bench.recorded_traffic("m2l", "sphere262k", 1, [-1, -1, 8, 7, 7, 8, 7]) == 1234.0
    assert bench.recorded_traffic("m2l", "sphere262k", 1, [-1, -1, 8, 7, 7, 5, 5]) is None
    src.write_bytes(b"// kernel source, changed\n")
    assert bench.recorded_traffic("m2l", "sphere262k", 1) is None


def _fake_levels():
    tinfo = {"n_points": 1000, "n_levels": 4, "n_p2p_pairs": 50000}
    levels = [{"level": 1, "nbox": 1}, {"level": 2, "nbox": 8},
              {"level": 3, "nbox": 20, "L": 13, "ntheta": 14, "nphi": 28, "K": 392,
               "n_far": 300, "n_types": 40},
              {"level": 4, "nbox": 100, "L": 8, "ntheta": 9, "nphi": 18, "K": 162,
               "n_far": 2000, "n_types": 100}]
    return tinfo, levels


def test_onepass_work_split_books_on_the_onepass_kernel():
    """A one-pass pair in any work split (variant 1 + k) books all of its
    work on "interp"/"anterp" and none on the staged kernels."""
    tinfo, levels = _fake_levels()
    staged = bench.algorithmic_work(tinfo, levels, 4, [-1, -1, 0, -1], [-1, -1, 0, -1])
    for v in (1, 2, 3):
        w = bench.algorithmic_work(tinfo, levels, 4, [-1, -1, v, -1], [-1, -1, v, -1])
        for k in ("interp_s1", "interp_s2", "interp_s3", "anterp_s1", "anterp_s2", "anterp_s3"):
            assert w[k]["flops"] == 0 and w[k]["bytes"] == 0, (v, k)
        up = sum(staged[k]["flops"] for k in ("interp_s1", "interp_s2", "interp_s3"))
        dn = sum(staged[k]["flops"] for k in ("anterp_s1", "anterp_s2", "anterp_s3"))
        assert w["interp"]["flops"] == up > 0
        assert w["anterp"]["flops"] == dn > 0


def test_phase_rooflines_sum_the_kernels_of_each_phase():
    """Each phase books the work and the time of its kernels; its floor is
    the larger of the HBM and compute times at peak, and the whole-matvec
    floor is the sum of the phase floors."""
    tinfo, levels = _fake_levels()
    work = bench.algorithmic_work(tinfo, levels, 1, [-1, -1, 0, -1], [-1, -1, 0, -1])
    ms = {"p2p": 0.5, "interp_s1": 0.1, "interp_s2": 0.2, "interp_s3": 0.3, "m2l": 1.0}
    ph, floor = bench.phase_rooflines(work, ms, False)
    m2m_flops = sum(work[k]["flops"] for k in ("interp_s1", "interp_s2", "interp_s3"))
    assert abs(ph["m2m"]["achieved"] - round(m2m_flops / 0.6e-3 / 1e12, 3)) < 1e-3
    assert ph["m2m"]["bound"] == "mfma" and ph["p2p"]["bound"] == "alu"
    assert "l2l" not in ph          # no time booked: not reported
    expect = 0.0
    for p, ks in bench.PHASES.items():
        fl = sum(work[k]["flops"] for k in ks)
        by = sum(work[k]["bytes"] for k in ks)
        expect += max(by / 8e12, fl / 157.3e12) * 1e3
    assert abs(floor - expect) < 1e-12
    ph3, _ = bench.phase_rooflines(work, ms, True)
    assert ph3["m2m"]["peak"] == bench.PEAK_BF16_TFLOPS


def test_fft_grid_sizes_are_7_smooth_and_minimal():
    import bench
    for L in range(0, 200):
        P = bench.smooth_phi_count(L)
        assert P % 2 == 0 and P >= 2 * L + 2
        m = P
        for r in (2, 3, 5, 7):
            while m % r == 0:
                m //= r
        assert m == 1
        for Q in range(2 * L + 2, P, 2):
            m = Q
            for r in (2, 3, 5, 7):
                while m % r == 0:
                    m //= r
            assert m != 1, (L, Q)
    assert [bench.smooth_phi_count(L) for L in (8, 13, 20, 33, 57)] == [18, 28, 42, 70, 120]
