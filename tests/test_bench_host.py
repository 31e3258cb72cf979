"""Host checks of the benchmark's measurement logic (no GPU): the one-GPU
contract, the algorithmic bytes and nominal flops that the roofline divides
by the measured launch time, the source-hash guard on the recorded HBM
traffic, and the roofline arithmetic against the published peaks."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402  (module level holds no torch or GPU work)


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""                      # no JSON line for a refused run


@pytest.mark.parametrize("N,T", [(1024, 4096), (512, 1000), (256, 7)])
def test_algorithmic_bytes_per_frame(N, T):
    """One read of every stored input and one write of every stored output,
    float32, P = 2N: the shift passes move N x N in and out, the first
    x-shear N x N in and N x P out, the y-shear N x P in and out, the last
    x-shear N x P in and N x N out; both medians of a step read the stack
    twice, write it once and write two images."""
    P = 2 * N
    b = lambda fam: bench.alg_bytes_per_frame(fam, N, P, T)
    assert b("shift_y") == b("shift_x") == 8 * N * N
    assert b("shear_x1") == b("shear_x2") == 4 * N * N + 4 * N * P
    assert b("shear_y") == 8 * N * P
    assert b("median") == pytest.approx(12 * N * N + 8 * N * N / T, rel=0, abs=1e-9)
    assert b("aux") is None
    # the shift + rotate headline: 56 N^2 bytes per frame at P = 2N
    assert sum(b(f) for f in ("shift_y", "shift_x", "shear_x1", "shear_y", "shear_x2")) == 56 * N * N


def test_nominal_flops_per_frame():
    """5 P log2 P per complex length-P transform, forward and back, one
    transform per pair of real lines: N / 2 pairs for the shift passes and
    x-shears, P / 2 for the y-shear (230.7 MFLOP per 1024^2 frame)."""
    N, P = 1024, 2048
    per_pair = 2 * 5 * P * 11
    for fam in ("shift_y", "shift_x", "shear_x1", "shear_x2"):
        assert bench.alg_flops_per_frame(fam, N, P) == (N // 2) * per_pair
    assert bench.alg_flops_per_frame("shear_y", N, P) == (P // 2) * per_pair
    assert round(bench.alg_flops_per_frame("shear_y", N, P) / 1e6, 1) == 230.7
    assert bench.alg_flops_per_frame("median", N, P) is None


def test_peaks():
    """The published MI355X peaks, and the derived non-packed FP32 rate."""
    assert bench.HBM_PEAK_GBS == 8000.0
    assert bench.FP32_PEAK_TFLOPS == 157.3
    # derived: FP32 vector without packed instructions, 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
    assert round(bench.FP32_NONPACKED_TFLOPS, 1) == 78.6


def test_roofline_is_hbm_over_algorithmic_bytes():
    """frac = algorithmic bytes per launch / mean launch time / 8 TB/s; the
    line passes' nominal FFT rate is reported beside it."""
    alg = 512 * 16 * 1024 * 1024          # shear_y of a 512-frame chunk at 1024^2 (16 N^2 per frame)
    ms = 3.926
    gbps = alg / (ms * 1e-3) / 1e9
    r = bench.roofline({"achieved_GBps": gbps, "achieved_TFLOPs": 29.84, "alg_bytes_per_launch": alg,
                        "avg_launch_ms": ms}, "shear_y", 12345)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["kernel"] == "shear_y"
    assert r["peak"] == 8000.0 and r["traffic"] == 12345
    assert abs(r["frac"] - 0.2735) < 1e-3
    assert abs(r["alu"]["frac_published"] - 29.84 / 157.3) < 1e-4
    assert abs(r["alu"]["frac_nonpacked"] - 29.84 / bench.FP32_NONPACKED_TFLOPS) < 1e-4
    m = bench.roofline({"achieved_GBps": 4761.0, "alg_bytes_per_launch": 1e9, "avg_launch_ms": 0.21}, "median",
                       None)
    assert m["bound"] == "hbm" and m["unit"] == "GB/s" and m["peak"] == 8000.0 and "alu" not in m
    assert abs(m["frac"] - 4761.0 / 8000.0) < 1e-4 and m["traffic"] is None


def test_traffic_is_used_only_for_the_sources_it_was_taken_from(tmp_path):
    good = tmp_path / "good.txt"
    good.write_text("traffic shear_y N=1024 P=2048 bytes_per_frame=18491485\n"
                    "source_sha256 %s\n" % bench.sources_sha256())
    assert bench.read_traffic(str(good), "shear_y", 1024, 2048) == 18491485.0
    assert bench.read_traffic(str(good), "shear_y", 512, 1024) is None       # another geometry
    assert bench.read_traffic(str(good), "median", 1024, 2048) is None       # another family
    stale = tmp_path / "stale.txt"
    stale.write_text("traffic shear_y N=1024 P=2048 bytes_per_frame=18491485\n"
                     "source_sha256 %s\n" % ("0" * 64))
    assert bench.read_traffic(str(stale), "shear_y", 1024, 2048) is None     # kernels changed since
    unsigned = tmp_path / "unsigned.txt"
    unsigned.write_text("traffic shear_y N=1024 P=2048 bytes_per_frame=18491485\n")
    assert bench.read_traffic(str(unsigned), "shear_y", 1024, 2048) is None
    assert bench.read_traffic(str(tmp_path / "missing.txt"), "shear_y", 1024, 2048) is None


def test_source_hash_covers_every_library_source(tmp_path, monkeypatch):
    """Changing any file of the library sources changes the hash."""
    import shutil
    src = os.path.join(ROOT, "paper_1510_04331_amd", "csrc")
    fake = tmp_path / "repo"
    shutil.copytree(src, fake / "paper_1510_04331_amd" / "csrc")
    monkeypatch.setattr(bench, "HERE", str(fake))
    h0 = bench.sources_sha256()
    assert h0 == bench.sources_sha256()
    for name in sorted(os.listdir(src)):
        p = fake / "paper_1510_04331_amd" / "csrc" / name
        if not p.is_file():
            continue
        orig = p.read_bytes()
        p.write_bytes(orig + b" ")
        assert bench.sources_sha256() != h0, name
        p.write_bytes(orig)
    assert bench.sources_sha256() == h0
