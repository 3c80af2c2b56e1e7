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


def test_oracle_pattern_counts():
    """The CPU baseline's pixel-evaluation counts: the stats of fits without trial derivatives are
    the oracle's own pattern; with them, trial-point passes count as the oracle's value evaluations
    and the pixels of accepted steps as its value+gradient+Hessian evaluations."""
    sys.path.insert(0, ROOT)
    import bench
    st = {"full_px": 500, "value_px": 300, "trial_full_px": 0, "taken_px": 0}
    assert bench.oracle_pattern_px(st) == (500, 300)
    # 100 px per source and 10 sources: start pass 1,000 px, 7 trial passes of 1,000 px, 5 accepted
    st = {"full_px": 1000 + 7000, "value_px": 2000, "trial_full_px": 7000, "taken_px": 5000}
    assert bench.oracle_pattern_px(st) == (1000 + 5000, 2000 + 7000)


def test_flop_counts_of_the_roofline():
    sys.path.insert(0, ROOT)
    import bench
    # 3 PSF components, 6 + 8 galaxy prototypes: the figures the design notes quote
    assert bench.flop_full_per_px(3, 6, 8) == 4311
    assert bench.flop_value_per_px(3, 6, 8) == 3 * (13 + 8 * 14) + 30
    # algorithmic figure of the roofline: 170 per galaxy component, 30 per star component, 400 per pixel
    assert bench.flop_full_per_px_algorithmic(3, 6, 8) == 170 * 42 + 90 + 400


def test_stratified_sample_takes_one_source_per_size_stratum():
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    npx = np.random.default_rng(0).integers(1000, 700000, size=2000)
    pick = bench.stratified_sample(npx, 40, 5)
    assert len(pick) == 40 and len(set(pick)) == 40
    rank = np.argsort(np.argsort(npx, kind="stable"), kind="stable")
    assert sorted(rank[pick] // 50) == list(range(40))


def test_host_pixels_drawn_in_chunks_equal_one_draw():
    """The host-generated workload (bench --host-generated, rebuilt by --oracle-fits-from) draws
    its sky counts in chunks of whole images; the chunk size changes no value."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import synth
    a = synth.make_config(1, n_sources=12, pixel_chunk=1)
    b = synth.make_config(1, n_sources=12, pixel_chunk=1 << 27)
    c = synth.make_config(1, n_sources=12, pixel_chunk=3000)
    assert a.pixels.dtype == np.float32 and np.array_equal(a.pixels, b.pixels) and np.array_equal(b.pixels, c.pixels)


def test_oracle_fits_from_refuses_device_generated_fits(tmp_path):
    import numpy as np
    p = tmp_path / "fits.npz"
    np.savez(p, n_sources=10, host_generated=False, plain_elbo=np.zeros(10), plain_status=np.zeros(10, np.int32),
             head_elbo=np.zeros(10), head_status=np.zeros(10, np.int32), head="plain")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--oracle-fits-from", str(p)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0 and "host-generated" in r.stderr
