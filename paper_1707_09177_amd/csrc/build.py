"""Build libgdecon.so for gfx950 from the HIP sources in this directory.

Each translation unit is compiled in parallel into ../_build/*.o, then linked
into ../libgdecon.so (the package directory, so the shared library travels with
the source tree).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC",
    # no packed-FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", HERE,
    # the FFT twiddle table is evaluated at compile time
    "-fconstexpr-steps=50000000",
]


def _compile(src: str, obj: str) -> tuple[str, int, str]:
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (p.stdout + p.stderr).splitlines() if "packed-fp32" not in l and l.strip())
    return src, p.returncode, err


def build(out: str | None = None, jobs: int | None = None, verbose: bool = False) -> str:
    out = out or os.path.join(PKG, "libgdecon.so")
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(HERE, "*.hip")))
    objs = [os.path.join(bdir, os.path.basename(s)[:-4] + ".o") for s in srcs]
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda so: _compile(*so), zip(srcs, objs)))
    bad = [(s, e) for s, rc, e in results if rc != 0]
    for s, rc, e in results:
        if e and (verbose or rc != 0):
            print(f"--- {os.path.basename(s)}\n{e}", file=sys.stderr)
    if bad:
        raise RuntimeError("HIP compile failed: " + ", ".join(os.path.basename(s) for s, _ in bad))
    tmp = out + f".tmp{os.getpid()}"
    subprocess.check_call([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
