"""Host-side checks of the benchmark's contract (no GPU needed).

- The algorithmic access counts per grid point follow the sweep structure of
  Algorithms 1-4: Van Cittert 4 per pass, CG 8 per pass (3 in the first,
  whose p0 = r0 is not re-read), BiCGSTAB 15 per pass (13 in the first,
  whose p0 = q0 = 0 are not read), steepest descent 5 per pass, plus the
  init sweep and the exit true residual (2).
- The committed HBM-traffic summaries belong to the current kernel sources,
  so that the bench's roofline.traffic is reported rather than null.
- More than one GPU is refused with a message and exit status 2.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_access_model():
    for n in (1, 2, 5, 18):
        assert bench.accesses("vc", n) == 3 + 4 * n + 2
        assert bench.accesses("sd", n) == 3 + 5 * n + 2
        assert bench.accesses("cg", n) == 3 + 7 + 8 * (n - 1) + 2
        assert bench.accesses("bicgstab", n) == 4 + 13 + 15 * (n - 1) + 2
    # the per-pass increments: 4, 8, 15 field accesses
    assert bench.accesses("vc", 6) - bench.accesses("vc", 5) == 4
    assert bench.accesses("cg", 6) - bench.accesses("cg", 5) == 8
    assert bench.accesses("bicgstab", 6) - bench.accesses("bicgstab", 5) == 15


def test_committed_traffic_matches_the_kernel_sources():
    for key in ("2048sq_x16", "256cube_x3", "uneven200"):
        t = bench.measured_traffic(key)
        assert t is not None, f"profiles/ traffic for {key} was taken on other solve-kernel sources"
        assert t > 0
    for key in ("closure_256cube", "closure_2048sq_x8"):
        t = bench.measured_traffic(key, bench.CLOSURE_TRAFFIC_FILE, bench.CLOSURE_SOURCES)
        assert t is not None, f"profiles/ traffic for {key} was taken on other closure-kernel sources"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env={**os.environ, "WORLD_SIZE": "1"})
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
