"""Host-side checks of the bench harness (no GPU): the one-GPU contract,
the algorithmic byte count behind the roofline, and script replay."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single MI355X" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_bytes_of_one_granule_call():
    # one active granule OR-ing 3 support-row segments (512 B each), its
    # currTable words read and written (2 x 512 B), one trailed granule
    # (64 words + 8 B header), two residue checks (2 words each), one
    # scanned granule (64 currTable + 64 support words), 5 domain words in
    # and out
    d = {"granule_rows": 3, "granules_in": 1, "trail_granules": 1, "residue_checks": 2, "scan_granules": 1}
    want = 3 * 512 + 2 * 512 + (512 + 8) + 2 * 16 + 2 * 512 + 5 * 16
    assert bench.algorithmic_bytes(d, 5, 1) == want == 4216


def test_replay_counts_propagations_and_keeps_order():
    seen = []

    class Fake:
        def push(self):
            seen.append("push")

        def pop(self):
            seen.append("pop")

        def propagate(self, d):
            seen.append(("prop", d))

    script = [("push", None), ("prop", 1), ("prop", 2), ("pop", None), ("push", None), ("prop", 3)]
    lat = []
    assert bench.replay(Fake(), script, lat) == 3
    assert len(lat) == 3 and all(x >= 0 for x in lat)
    assert seen == ["push", ("prop", 1), ("prop", 2), "pop", "push", ("prop", 3)]
