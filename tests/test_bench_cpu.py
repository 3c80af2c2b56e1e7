"""Host-side checks of bench.py that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_flop_counts_of_the_roofline():
    sys.path.insert(0, ROOT)
    import bench
    # 3 PSF components, 6 + 8 galaxy prototypes: the figures the design notes quote
    assert bench.flop_full_per_px(3, 6, 8) == 4729
    assert bench.flop_value_per_px(3, 6, 8) == 3 * (13 + 8 * 14) + 30
