"""bench.py's contract, checked on the CPU: the committed counter summary
belongs to the current walk kernel (so the benchmark line can report HBM
traffic), the cycle model adds up, and more than one GPU is refused."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_committed_traffic_profile_matches_the_kernel():
    import bench
    t = bench.traffic_from_profile("annulus_fp32_8x8x129")
    # None means the kernel changed since the counters were taken: re-profile
    assert t is not None, "profiles/walk_annulus_fp32_8x8x129_traffic.txt is stale for the current kernel"
    # at least the algorithmic bytes: the node table and the node sums
    assert t >= bench.WALK_BYTES_PER_NODE * 3633


def test_source_hash_ignores_comments(tmp_path):
    import bench
    src = os.path.join(ROOT, "paper_1310_3435_amd", "csrc")
    for f in ("walk.hip", "walk.h", "walk_core.h", "common.h", "rng.h"):
        text = open(os.path.join(src, f)).read()
        (tmp_path / f).write_text("// a comment\n" + text.replace("\n", "\n  ") + "\n/* another */\n")
    assert bench.kernel_source_hash(str(tmp_path)) == bench.kernel_source_hash()
    (tmp_path / "rng.h").write_text(open(os.path.join(src, "rng.h")).read() + "\nint changed;\n")
    assert bench.kernel_source_hash(str(tmp_path)) != bench.kernel_source_hash()


def test_cycle_model_adds_up():
    import bench
    common = 160 / 3 + 20 + 36 + 16 + 8
    for kind, drift in {"ring": 56, "gauss": 42, "sech2": 46, "sin2": 46}.items():
        assert bench.CYCLES_PER_WAVE_STEP[kind] == pytest.approx(common + drift)
    assert bench.ISSUE_PEAK_G == pytest.approx(256 * 4 * 2.4)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
