"""Host logic of bench.py, on the CPU with stand-ins for the library.

* time_plan reads the scheduler's status word only after an execution has
  written it (with --warmup 0 the workspace is still uninitialised after the
  warmup loop).
* measured_traffic reports the committed HBM traffic only while the kernel
  source hashes to the value recorded beside it.
* --gpus above 1 exits with a message, since the path is single-GPU.
* chase_bytes (the bulge chase's algorithmic bytes) equals 16 bytes per entry
  that a brute-force count finds changed in each step.
"""
import hashlib
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
import bench  # noqa: E402


class _FakeTorch:
    class cuda:
        @staticmethod
        def synchronize():
            pass

    @staticmethod
    def empty_like(x):
        return _FakeBuf()


class _FakeBuf:
    def copy_(self, other):
        pass


class _FakePlan:
    def __init__(self, log):
        self.log = log

    def alloc(self):
        return "vt", "ws"

    def execute(self, S, m, vt, ws):
        self.log.append("execute")

    def last_kernel_ms(self):
        return 1.0


class _FakeLib:
    def __init__(self, log):
        self.log = log

    def poll_error(self, ws):
        # the status word is undefined until an execution has written it
        assert "execute" in self.log, "status polled before any execution"
        self.log.append("poll")
        return 0


@pytest.mark.parametrize("warmup", [0, 1, 2])
def test_time_plan_polls_only_after_an_execution(warmup):
    log = []
    ms, kms, S, vt = bench.time_plan(_FakeLib(log), _FakeTorch, _FakePlan(log), _FakeBuf(), 8, 2, warmup)
    assert log.count("execute") == warmup + 2
    assert log[-1] == "poll"
    assert len(kms) == 2


def test_measured_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    name = "persistent_kernel_square_graded_64x64_nb32_bidiag_auto.md"
    (tmp_path / "profiles").mkdir()
    src_dir = tmp_path / "paper_1611_06892_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (src_dir / "kernels.hip").write_bytes(b"// kernel source\n")
    sha = hashlib.sha256(b"// kernel source\n").hexdigest()[:16]
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    summary = tmp_path / "profiles" / name
    summary.write_text("traffic_bytes: 12345\nkernel_source_sha256_prefix: %s\n" % sha)
    assert bench.measured_traffic("square_graded", 64, 64, 32, "bidiag", "auto", "f64") == 12345.0
    assert bench.measured_traffic("square_graded", 64, 64, 32, "bidiag", "auto", "f64_upd_f32") is None
    summary.write_text("traffic_bytes: 12345\nkernel_source_sha256_prefix: %s\n" % ("0" * 16))
    assert bench.measured_traffic("square_graded", 64, 64, 32, "bidiag", "auto", "f64") is None
    summary.unlink()
    assert bench.measured_traffic("square_graded", 64, 64, 32, "bidiag", "auto", "f64") is None


def test_committed_headline_traffic_matches_the_source():
    """The committed summary of the headline kernel names the current source."""
    v = bench.measured_traffic("square_graded", 16384, 16384, 256, "bidiag", "auto", "f64")
    assert v is not None and v > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _chase_changed_entries(n, nb):
    """Entries each step of the bulge chase changes, counted as sets from the
    step's definition: the right reflector of step t of sweep k (column
    c = k + 1 + t nb) acts on columns c .. c+L-1 of rows rr .. c+L-1 (the
    cleared row rr = k, or c - nb after the first step, and every row below
    it down to the diagonal block); the left one on rows c .. c+L-1 of
    columns c .. min(c + 2 nb, n) - 1.  L = min(nb, n - c)."""
    total = 0
    if nb <= 1:
        return 0
    for k in range(max(n - 2, 0)):
        c, t = k + 1, 0
        while c < n:
            L = min(nb, n - c)
            rr = k if t == 0 else c - nb
            cells = {(i, j) for i in range(rr, c + L) for j in range(c, c + L)}
            cells |= {(i, j) for i in range(c, c + L) for j in range(c, min(c + 2 * nb, n))}
            total += len(cells)
            c += nb
            t += 1
    return total


@pytest.mark.parametrize("n,nb", [(1, 4), (2, 1), (5, 2), (9, 3), (17, 4), (40, 7), (33, 16), (12, 20)])
def test_chase_bytes_counts_every_changed_entry_once_per_step(n, nb):
    """The chase's algorithmic bytes (16 per changed entry and step, read and
    written once) against a brute-force count of the changed entries."""
    assert bench.chase_bytes(n, nb) == 16 * _chase_changed_entries(n, nb)
