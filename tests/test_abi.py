"""The C ABI library loads on the CPU host and exports every declared symbol.

No compute call is made here (there is no GPU in the CPU test run).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]
LIB = os.path.join(ROOT, "paper_1707_09177_amd", "libgdecon.so")


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                             text, flags=re.M):
            name = m.group(1)
            if name not in ("if", "while", "for", "return", "sizeof"):
                names.append(name)
    return sorted(set(names))


def test_header_declares_the_path_entry_points():
    names = declared_functions()
    for required in ("filter_apply", "deconvolve_vancittert", "deconvolve_cg", "deconvolve_bicgstab",
                     "deconvolve_workspace_bytes", "gd_status_string"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdecon.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdecon.so not built")
def test_status_strings_and_host_side_validation():
    """Host-only paths: status names and argument checks that return before any launch."""
    from paper_1707_09177_amd import gdecon
    lib = gdecon.load()
    assert lib.gd_status_string(3).decode() == "GD_BREAKDOWN_OMEGA"
    assert lib.gd_status_string(-2).decode() == "GD_EWORKSPACE"
    g = gdecon.Grid()
    g.ndim = 4
    g.dtype = 1
    assert lib.deconvolve_workspace_bytes(ctypes.byref(g), 2) == 0
    assert lib.filter_apply(ctypes.byref(g), None, None, None) == -1
    assert "ndim" in lib.gd_last_error().decode()
    g.ndim = 2
    g.n[0], g.n[1], g.batch = 64, 64, 1
    assert lib.deconvolve_workspace_bytes(ctypes.byref(g), 2) > 7 * 64 * 64 * 4
    assert lib.deconvolve_workspace_bytes(ctypes.byref(g), 9) == 0
    o = gdecon.Opts()
    o.max_iter = 3
    info = ctypes.c_void_p(0x1000)
    # NULL workspace is rejected before anything touches the device
    rc = lib.deconvolve_bicgstab(ctypes.byref(g), ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000),
                                 ctypes.byref(o), None, 0, info, None)
    assert rc == -2
    # misaligned workspace
    rc = lib.deconvolve_cg(ctypes.byref(g), ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000),
                           ctypes.byref(o), ctypes.c_void_p(0x30010), 1 << 30, info, None)
    assert rc == -4
    # aliasing ubar / u
    rc = lib.deconvolve_cg(ctypes.byref(g), ctypes.c_void_p(0x10000), ctypes.c_void_p(0x10000),
                           ctypes.byref(o), ctypes.c_void_p(0x100000), 1 << 30, info, None)
    assert rc == -1
    o.init = 7
    rc = lib.deconvolve_vancittert(ctypes.byref(g), ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000),
                                   ctypes.byref(o), ctypes.c_void_p(0x100000), 1 << 30, info, None)
    assert rc == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdecon.so not built")
def test_batch_host_side_validation():
    """Uneven-batch workspace sizing and the argument checks made before any launch."""
    from paper_1707_09177_amd import gdecon
    lib = gdecon.load()
    n = 3
    lst = (gdecon.Instance * n)()
    sizes = [(2, (64, 48, 1)), (3, (16, 12, 10)), (2, (9, 7, 1))]
    for i, (nd, sz) in enumerate(sizes):
        lst[i].ndim = nd
        for d in range(3):
            lst[i].n[d] = sz[d]
    ws = lib.deconvolve_batch_workspace_bytes(2, 1, lst, n)
    pts = 64 * 48 + 16 * 12 * 10 + 9 * 7
    assert ws > 7 * pts * 4                      # BiCGSTAB keeps 7 work vectors per instance
    assert lib.deconvolve_batch_workspace_bytes(0, 1, lst, n) < ws   # Van Cittert keeps 2
    assert lib.deconvolve_batch_workspace_bytes(2, 1, lst, 0) == 0
    assert lib.deconvolve_batch_workspace_bytes(9, 1, lst, n) == 0
    o = gdecon._make_opts(5, 0.0, "ubar", "r0ubar", None, 0)
    # NULL field pointers
    assert lib.deconvolve_batch(2, 1, lst, n, ctypes.byref(o), 256, ws, 256, None) == -1
    # fake, non-dereferenced addresses: the second output overlaps the first input
    base = 1 << 40
    for i in range(n):
        lst[i].ubar = base + i * (1 << 24)
        lst[i].u = base + (1 << 30) + i * (1 << 24)
    lst[1].u = lst[0].ubar + 64
    work = base + (1 << 34)
    assert lib.deconvolve_batch(2, 1, lst, n, ctypes.byref(o), work, ws, work + ws, None) == -1
    assert "overlaps" in lib.gd_last_error().decode()
    # workspace too small / misaligned
    lst[1].u = base + (1 << 30) + (1 << 24)
    assert lib.deconvolve_batch(2, 1, lst, n, ctypes.byref(o), work, ws - 256, work + ws, None) == -2
    assert lib.deconvolve_batch(2, 1, lst, n, ctypes.byref(o), work + 8, ws, work + ws, None) == -4
    # bad instance
    lst[2].ndim = 1
    assert lib.deconvolve_batch(2, 1, lst, n, ctypes.byref(o), work, ws, work + ws, None) == -1
    assert "instance 2" in lib.gd_last_error().decode()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdecon.so not built")
def test_tune_set_validates_choices():
    from paper_1707_09177_amd import gdecon
    lib = gdecon.load()
    g = gdecon.Grid()
    g.ndim, g.dtype, g.batch = 2, 1, 1
    g.n[0], g.n[1], g.n[2] = 64, 32, 1
    bad = gdecon._choice(tiles_per_wave=0)
    assert lib.gd_tune_set(2, ctypes.byref(g), 256, 512, ctypes.byref(bad)) == -1
    bad = gdecon._choice(wave_claims=2)
    assert lib.gd_tune_set(2, ctypes.byref(g), 256, 512, ctypes.byref(bad)) == -1
    for bpc in (-1, 17):
        bad = gdecon._choice(blocks_per_cu=bpc)
        assert lib.gd_tune_set(2, ctypes.byref(g), 256, 512, ctypes.byref(bad)) == -1
    for segs in (-1, 65):
        bad = gdecon._choice(segments=segs)
        assert lib.gd_tune_set(2, ctypes.byref(g), 256, 512, ctypes.byref(bad)) == -1
    assert lib.gd_tune_set(2, ctypes.byref(g), 256, 512, ctypes.byref(gdecon._choice(segments=64))) == 0
    lib.gd_tune_reset()
    assert lib.gd_tune_set(7, ctypes.byref(g), 256, 512, ctypes.byref(gdecon._choice())) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdecon.so not built")
def test_closure_stress_host_side_validation():
    """closure_stress rejects bad grids, NULL pointers and an output that
    overlaps an input before any launch."""
    from paper_1707_09177_amd import gdecon
    lib = gdecon.load()
    g = gdecon.Grid()
    g.ndim, g.dtype, g.batch = 4, 1, 1
    g.n[0], g.n[1], g.n[2] = 8, 8, 8
    assert lib.closure_stress(ctypes.byref(g), 4096, 8192, 1 << 20, None) == -1
    assert "ndim" in lib.gd_last_error().decode()
    g.ndim = 3
    assert lib.closure_stress(ctypes.byref(g), None, 8192, 1 << 20, None) == -1
    assert "NULL" in lib.gd_last_error().decode()
    g.n[1] = 0
    assert lib.closure_stress(ctypes.byref(g), 4096, 8192, 1 << 20, None) == -1
    g.n[1] = 8
    # 3 components of 512 FP32 points = 6 KiB per input; 6 pairs = 12 KiB out
    ub, us = 1 << 20, 2 << 20
    assert lib.closure_stress(ctypes.byref(g), ub, us, us + 4096, None) == -1
    assert "overlaps" in lib.gd_last_error().decode()
    assert lib.closure_stress(ctypes.byref(g), ub, us, us - 12288 + 4, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdecon.so not built")
def test_germano_host_side_validation():
    """The differential-filter entry points accept power-of-two sizes only and
    check gamma, pointers and the workspace before any launch."""
    from paper_1707_09177_amd import gdecon
    lib = gdecon.load()
    g = gdecon.make_grid((2, 64, 32), 2, gdecon.torch.float32)
    assert lib.germano_workspace_bytes(ctypes.byref(g), -1) >= 2 * 64 * (32 + 4) * 4
    assert lib.germano_workspace_bytes(ctypes.byref(g), 2) > lib.deconvolve_workspace_bytes(ctypes.byref(g), 2)
    assert lib.germano_workspace_bytes(ctypes.byref(g), 9) == 0
    bad = gdecon.make_grid((2, 48, 32), 2, gdecon.torch.float32)
    assert lib.germano_workspace_bytes(ctypes.byref(bad), -1) == 0
    assert lib.germano_filter_apply(ctypes.byref(bad), 0.1, 0x10000, 0x20000, 0x100000, 1 << 30, None) == -1
    assert "power-of-two" in lib.gd_last_error().decode()
    big = gdecon.make_grid((8192, 2), 2, gdecon.torch.float32)
    assert lib.germano_workspace_bytes(ctypes.byref(big), -1) == 0
    f64 = gdecon.make_grid((4096, 2), 2, gdecon.torch.float64)
    assert lib.germano_workspace_bytes(ctypes.byref(f64), -1) == 0
    assert lib.germano_filter_apply(ctypes.byref(g), 0.0, 0x10000, 0x20000, 0x100000, 1 << 30, None) == -1
    assert "gamma" in lib.gd_last_error().decode()
    assert lib.germano_filter_apply(ctypes.byref(g), 0.1, 0x10000, 0x20000, None, 0, None) == -2
    assert lib.germano_filter_apply(ctypes.byref(g), 0.1, 0x10000, 0x20000, 0x100010, 1 << 30, None) == -4
    o = gdecon.Opts()
    o.max_iter = 3
    info = ctypes.c_void_p(0x1000)
    assert lib.deconvolve_germano(2, ctypes.byref(g), 0.1, 0x10000, 0x10000, ctypes.byref(o), 0x1000000, 1 << 30,
                                  info, None) == -1
    assert "overlap" in lib.gd_last_error().decode()
    assert lib.deconvolve_germano(7, ctypes.byref(g), 0.1, 0x10000, 0x20000, ctypes.byref(o), 0x1000000, 1 << 30,
                                  info, None) == -1
    assert lib.deconvolve_germano(2, ctypes.byref(g), 0.1, 0x10000, 0x40000, ctypes.byref(o), 0x1000000, 16,
                                  info, None) == -2
    t = gdecon.TuneInfo()
    assert lib.deconvolve_germano_autotune(2, ctypes.byref(g), 0.1, 0x1000100, 0x40000, 0x1000000, 1 << 30, info,
                                           None, ctypes.byref(t)) == -1
    assert "overlaps the workspace" in lib.gd_last_error().decode()
    assert lib.deconvolve_germano_autotune(2, ctypes.byref(g), 0.1, 0x10000, 0x40000, 0x1000000, 16, info,
                                           None, ctypes.byref(t)) == -2


def test_binding_output_check_on_host():
    """The binding's output check (shape, dtype, device must match exactly)."""
    from paper_1707_09177_amd import gdecon
    torch = gdecon.torch
    x = torch.zeros(2, 3, dtype=torch.float32)
    assert gdecon._out(None, (2, 3), x).shape == (2, 3)
    y = torch.zeros(2, 3)
    assert gdecon._out(y, (2, 3), x) is y
    for bad in (torch.zeros(2, 2), torch.zeros(3, 2), torch.zeros(2, 3, dtype=torch.float64)):
        with pytest.raises(ValueError):
            gdecon._out(bad, (2, 3), x)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdecon.so not built")
def test_sizes_that_would_overflow_are_rejected():
    """Extents whose product passes 2^63, and batches whose byte counts would
    pass it, are refused on the host: no size computation wraps round."""
    from paper_1707_09177_amd import gdecon
    lib = gdecon.load()

    def grid(n, batch=1, ndim=3):
        g = gdecon.Grid()
        g.ndim, g.dtype, g.batch = ndim, 1, batch
        for d in range(3):
            g.n[d] = n[d]
        return g

    for n, b in [((2, 1 << 62, 2), 1), ((1 << 20, 1 << 40, 1 << 20), 1), ((1024, 1024, 1), 1 << 30)]:
        g = grid(n, b)
        assert lib.deconvolve_workspace_bytes(ctypes.byref(g), 2) == 0
        assert lib.filter_apply(ctypes.byref(g), 4096, 8192, None) == -1
        assert "too large" in lib.gd_last_error().decode()
    g = grid((1 << 29, 1 << 29, 1 << 29))
    assert lib.closure_stress(ctypes.byref(g), 1 << 20, 2 << 20, 3 << 20, None) == -1
    assert "too large" in lib.gd_last_error().decode()
    net = gdecon.Cnn()
    net.ndim, net.channels, net.layers, net.params = 2, 32, 6, 4096
    assert lib.warmstart_workspace_bytes(ctypes.byref(net), ctypes.byref(grid((1 << 40, 1 << 40, 1), ndim=2)), 0) == 0
    assert lib.warmstart_workspace_bytes(ctypes.byref(net), ctypes.byref(grid((64, 64, 1), 1 << 40, 2)), 0) == 0
    assert lib.warmstart_workspace_bytes(ctypes.byref(net), ctypes.byref(grid((64, 64, 1), 4, 2)), 0) > 0

    def instances(k):
        lst = (gdecon.Instance * k)()
        for i in range(k):
            lst[i].ndim = 2
            lst[i].n[0], lst[i].n[1], lst[i].n[2] = 1 << 20, 1 << 20, 1
        return lst
    assert lib.deconvolve_batch_workspace_bytes(2, 1, instances(64), 64) > 0   # 2^46 points in all
    assert lib.deconvolve_batch_workspace_bytes(2, 1, instances(65), 65) == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdecon.so not built")
def test_blocked_vancittert_limits_max_iter():
    """The blocked Van Cittert issues its sweeps from the host, so max_iter is
    bounded (2^20); the check comes before any launch."""
    from paper_1707_09177_amd import gdecon
    lib = gdecon.load()
    g = gdecon.make_grid((64, 32), 2, gdecon.torch.float32)
    ws = lib.vancittert_blocked_workspace_bytes(ctypes.byref(g))
    o = gdecon._make_opts((1 << 20) + 1, 0.0, "ubar", "r0ubar", None, 0)
    assert lib.deconvolve_vancittert_blocked(ctypes.byref(g), 1 << 20, 2 << 20, ctypes.byref(o), 4 << 20, ws,
                                             8 << 20, None) == -1
    assert "max_iter" in lib.gd_last_error().decode()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgdecon.so not built")
def test_empty_inputs_are_rejected():
    """An empty batch or a zero extent is an argument error (GD_EINVAL) for
    every entry point, reported before any launch; workspace queries give 0."""
    from paper_1707_09177_amd import gdecon
    lib = gdecon.load()
    o = gdecon._make_opts(3, 0.0, "ubar", "r0ubar", None, 0)
    info = ctypes.c_void_p(0x1000)
    for shape, batch in [((0, 64), 1), ((64, 0), 1), ((64, 64), 0), ((0, 8, 8), 1), ((8, 8, 0), 1)]:
        g = gdecon.Grid()
        g.ndim, g.dtype, g.batch = len(shape), 1, batch
        for d in range(3):
            g.n[d] = shape[::-1][d] if d < len(shape) else 1
        gr = ctypes.byref(g)
        assert lib.deconvolve_workspace_bytes(gr, 2) == 0
        assert lib.germano_workspace_bytes(gr, 2) == 0
        assert lib.spectrum_workspace_bytes(gr) == 0
        assert lib.vancittert_blocked_workspace_bytes(gr) == 0
        for rc in (lib.filter_apply(gr, 1 << 20, 2 << 20, None),
                   lib.deconvolve_bicgstab(gr, 1 << 20, 2 << 20, ctypes.byref(o), 4 << 20, 1 << 30, info, None),
                   lib.deconvolve_vancittert_blocked(gr, 1 << 20, 2 << 20, ctypes.byref(o), 4 << 20, 1 << 30, info,
                                                     None),
                   lib.deconvolve_germano(2, gr, 0.1, 1 << 20, 2 << 20, ctypes.byref(o), 4 << 20, 1 << 30, info, None),
                   lib.germano_filter_apply(gr, 0.1, 1 << 20, 2 << 20, 4 << 20, 1 << 30, None),
                   lib.energy_spectrum(gr, 0.0, 1 << 20, 2 << 20, 4 << 20, 1 << 30, None),
                   lib.pdf_counts(gr, -1.0, 1.0, 10, 1 << 20, 2 << 20, None)):
            assert rc == -1, (shape, batch, lib.gd_last_error().decode())
        assert ">= 1" in lib.gd_last_error().decode()
