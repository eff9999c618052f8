"""Host-side checks of the benchmark's contract (no GPU needed).

- The algorithmic access counts per grid point: the method's count (every
  vector of Algorithms 1-4 read or written once per pass: 4, 5, 8 and 15
  per pass for Van Cittert, steepest descent, CG and BiCGSTAB, plus init and
  the exit true residual), and the count the fused kernels make, derived
  here from the sweep functors' operand lists in csrc/gd_ops.h (stencil
  inputs + centre inputs + stores of each sweep).
- The committed HBM-traffic summaries belong to the current kernel sources,
  so that the bench's roofline.traffic is reported rather than null.
- More than one GPU is refused with a message and exit status 2.
"""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def sweep_accesses(with_f0: bool) -> dict:
    """Full-field accesses of every sweep functor in gd_ops.h: its NI stencil
    inputs and NO centre inputs are read once, each store writes one field
    (the optional shadow residual f0 only where the solver keeps it)."""
    src = open(os.path.join(ROOT, "paper_1707_09177_amd", "csrc", "gd_ops.h")).read()
    out = {}
    for m in re.finditer(r"struct (Op\w+) \{(.*?)\n\};", src, re.S):
        name, body = m.group(1), m.group(2)
        ni, no = map(int, re.search(r"NI = (\d+), NO = (\d+)", body).groups())
        stores = len(re.findall(r"(?:store_c|vst)<", body))
        optional = len(re.findall(r"if \(f0\) (?:store_c|vst)<", body))
        out[name] = ni + no + stores - (0 if with_f0 else optional)
    return out


def test_algorithmic_access_model():
    # the method's count: per pass 4 / 5 / 8 / 15, plus init and exit
    for n in (1, 2, 5, 18):
        assert bench.accesses("vc", n) == 4 * n + 5
        assert bench.accesses("sd", n) == 5 * n + 5
        assert bench.accesses("cg", n) == 8 * n + 6
        assert bench.accesses("bicgstab", n) == 15 * n + 6
    # the kernels' count from their sweeps: init, the first pass, the later
    # passes, and the exit true residual
    a, af = sweep_accesses(False), sweep_accesses(True)
    seq = {
        "vc": (a["OpInitUbar"], a["OpVC"], a["OpVC"]),
        "sd": (a["OpInitUbar"], a["OpSD1"] + a["OpSD2"], a["OpSD1"] + a["OpSD2"]),
        "cg": (a["OpInitUbar"], a["OpCG1First"] + a["OpCG2"], a["OpCG1"] + a["OpCG2"]),
        "bicgstab": (af["OpInitUbar"], af["OpBiAFirst"] + af["OpBiB"] + af["OpBiC"],
                     af["OpBiA"] + af["OpBiB"] + af["OpBiC"]),
    }
    for solver, (init, first, later) in seq.items():
        for n in (1, 2, 5, 18):
            assert bench.kernel_accesses(solver, n) == init + first + later * (n - 1) + a["OpResNorm"], solver
    # later passes make exactly the method's per-pass count; the kernels save
    # only the unread zero vectors of the first pass (and CG's copy p0 = r0)
    for solver in seq:
        assert bench.kernel_accesses(solver, 6) - bench.kernel_accesses(solver, 5) == \
            bench.accesses(solver, 6) - bench.accesses(solver, 5)
        assert 0 <= bench.accesses(solver, 5) - bench.kernel_accesses(solver, 5) <= 2


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
