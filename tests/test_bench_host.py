"""Host-side parts of bench.py (no GPU): the one-GPU refusal, the board power / clock sampler
and the stage-kernel code hash of the built library."""
import os
import subprocess
import sys
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


class _FakeSolver:
    def __init__(self):
        self.steps = 0

    def run(self, st, nsteps):
        self.steps += nsteps
        time.sleep(0.001 * nsteps)


class _FakeTorch:
    class cuda:
        @staticmethod
        def synchronize():
            pass


def test_board_sampler_reads_power_and_clock(tmp_path, monkeypatch):
    pw, clk = tmp_path / "power1_input", tmp_path / "pp_dpm_sclk"
    pw.write_text("1385000000\n")  # microwatts
    clk.write_text("0: 500Mhz\n1: 2231Mhz *\n2: 2400Mhz\n")
    monkeypatch.setattr(bench, "_sysfs_board", lambda: (str(pw), str(clk)))
    s = _FakeSolver()
    out = bench.board_state(_FakeTorch, s, None, seconds=0.4)
    assert out["stage_board_w"] == pytest.approx(1385.0)
    assert out["idle_board_w"] == pytest.approx(1385.0)
    assert out["stage_shader_mhz"] == 2231
    assert out["stage_steps"] == s.steps and s.steps % 20 == 0 and s.steps > 0
    assert out["samples"] >= 8


def test_board_sampler_without_sysfs(monkeypatch):
    monkeypatch.setattr(bench, "_sysfs_board", lambda: (None, None))
    assert bench.board_state(_FakeTorch, _FakeSolver(), None, seconds=0.1) is None


def test_stage_code_hash_of_the_built_library():
    lib = os.path.join(ROOT, "paper_2208_01260_amd", "libswe_hweno.so")
    if not os.path.exists(lib):
        pytest.skip("library not built")
    h = bench.device_code_sha(lib)
    assert h is not None and len(h) == 16 and int(h, 16) >= 0
    assert bench.device_code_sha(lib) == h
    assert bench.device_code_sha(os.path.join(ROOT, "bench.py")) is None
