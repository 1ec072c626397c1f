"""CPU-side checks of the C ABI: the HIP library loads, exports every symbol
the public header declares, and rejects invalid configurations before any
device call."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_2106_10278_amd import binding


@pytest.fixture(scope="module")
def lib():
    return binding.load_library()


def test_exports_every_header_symbol(lib):
    syms = binding.header_symbols()
    assert len(syms) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [s for s in syms if s not in exported]
    assert not missing, missing
    for s in syms:
        assert hasattr(lib, s)


def test_library_is_gfx950_code_object():
    out = subprocess.run(["strings", binding.LIB_PATH], capture_output=True, text=True).stdout
    assert "gfx950" in out


def test_strerror_and_version(lib):
    for st in range(6):
        assert binding.strerror(st)
    assert "unknown" in binding.strerror(99)
    assert "gfx950" in binding.version()


def _plan(lib, **kw):
    edges = np.asarray(kw.pop("edges", [1.0, 2.0, 3.0]), dtype=np.float64)
    cfg = binding._Config()
    cfg.D = kw.get("D", 3)
    cfg.N = kw.get("N", 3)
    cfg.lmax = kw.get("lmax", 2)
    cfg.nbins = kw.get("nbins", len(edges) - 1)
    cfg.edges = edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if kw.get("edges_ok", True) else None
    box = kw.get("box", [10.0, 10.0, 10.0, 10.0])
    for k in range(4):
        cfg.box[k] = box[k]
    cfg.periodic = kw.get("periodic", 1)
    cfg.btuple_mode = kw.get("btuple_mode", 0)
    cfg.precision = kw.get("precision", 0)
    cfg.norm = kw.get("norm", 0)
    cfg.geometry = kw.get("geometry", 0)
    h = ctypes.c_void_p()
    st = lib.npcf_plan(ctypes.byref(cfg), None, kw.get("max_points", 100), ctypes.byref(h))
    if st == 0:
        lib.npcf_destroy(h)
    return st


@pytest.mark.parametrize("kw,expect", [
    (dict(D=5), binding.NPCF_E_UNSUPPORTED),
    (dict(D=1), binding.NPCF_E_UNSUPPORTED),
    (dict(N=6), binding.NPCF_E_UNSUPPORTED),
    (dict(D=2, N=5), binding.NPCF_E_UNSUPPORTED),        # N = 5 needs D = 3
    (dict(N=5, lmax=6), binding.NPCF_E_UNSUPPORTED),     # lmax above 5 for N = 5
    (dict(D=4, N=4), binding.NPCF_E_UNSUPPORTED),
    (dict(lmax=-1), binding.NPCF_E_INVALID),
    (dict(D=3, lmax=11), binding.NPCF_E_UNSUPPORTED),
    (dict(edges=[0.0, 1.0, 2.0]), binding.NPCF_E_INVALID),
    (dict(edges=[1.0, 1.0, 2.0]), binding.NPCF_E_INVALID),
    (dict(edges=[1.0, np.nan, 2.0]), binding.NPCF_E_INVALID),
    (dict(edges=[1.0, 2.0, 6.0]), binding.NPCF_E_INVALID),      # 2 r_max >= box
    (dict(box=[10.0, -1.0, 10.0, 1.0]), binding.NPCF_E_INVALID),
    (dict(nbins=0, edges=[1.0]), binding.NPCF_E_INVALID),
    (dict(btuple_mode=2), binding.NPCF_E_INVALID),
    (dict(precision=7), binding.NPCF_E_INVALID),
    (dict(precision=4), binding.NPCF_E_INVALID),
    (dict(norm=3), binding.NPCF_E_INVALID),
    (dict(max_points=0), binding.NPCF_E_INVALID),
    (dict(edges_ok=False), binding.NPCF_E_INVALID),
    # no radial tuple b1 < ... < b_{N-1}: fewer than N - 1 bins in the default mode
    (dict(N=5, lmax=2, edges=[1.0, 1.5, 2.0, 3.0]), binding.NPCF_E_INVALID),
    (dict(N=4, edges=[1.0, 2.0, 3.0]), binding.NPCF_E_INVALID),
    (dict(N=3, edges=[1.0, 2.0]), binding.NPCF_E_INVALID),
    # the unit D-sphere: D = 2 or 3, edges in (0, pi], cos(edges[0]) below 1
    (dict(geometry=1, D=4), binding.NPCF_E_UNSUPPORTED),
    (dict(geometry=1, D=3, lmax=6), binding.NPCF_E_UNSUPPORTED),
    (dict(geometry=1, D=3, edges=[1.0, 2.0, 3.5]), binding.NPCF_E_INVALID),
    (dict(geometry=1, D=3, edges=[1e-9, 1.0, 2.0]), binding.NPCF_E_INVALID),
    (dict(geometry=1, D=2, edges=[1e-9, 1.0, 2.0]), binding.NPCF_E_INVALID),
    # hyperbolic space: D = 2 or 3, cosh(edges[0]) >= 1 + 1e-9, edges up to 20, V = box[0] > 0
    (dict(geometry=2, D=4), binding.NPCF_E_UNSUPPORTED),
    (dict(geometry=2, D=3, lmax=6), binding.NPCF_E_UNSUPPORTED),
    (dict(geometry=2, D=3, edges=[1e-6, 1.0, 2.0]), binding.NPCF_E_INVALID),
    (dict(geometry=2, D=3, edges=[1.0, 2.0, 25.0]), binding.NPCF_E_INVALID),
    (dict(geometry=2, D=3, box=[0.0, 1.0, 1.0, 1.0]), binding.NPCF_E_INVALID),
    (dict(geometry=3), binding.NPCF_E_INVALID),
])
def test_plan_validation(lib, kw, expect):
    assert _plan(lib, **kw) == expect


def test_null_handles(lib):
    assert lib.npcf_plan(None, None, 10, None) == binding.NPCF_E_INVALID
    assert lib.npcf_accumulate(None, None, None, 1, 0, 1, 0) == binding.NPCF_E_INVALID
    assert lib.npcf_finalize(None, None, 0) == binding.NPCF_E_INVALID
    assert lib.npcf_reset(None) == binding.NPCF_E_INVALID
    assert lib.npcf_destroy(None) == binding.NPCF_OK
    assert lib.npcf_describe(None, None, None, None, None, None) == binding.NPCF_E_INVALID


def test_valid_plan_needs_a_device(lib):
    """Without a GPU a valid configuration fails with NPCF_E_DEVICE (no CPU fallback)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _plan(lib) == binding.NPCF_E_DEVICE
    assert _plan(lib, geometry=1, D=3, lmax=5, edges=[0.5, 1.0, 1.5]) == binding.NPCF_E_DEVICE
    assert _plan(lib, geometry=2, D=3, lmax=5, edges=[0.5, 1.0, 1.5]) == binding.NPCF_E_DEVICE


def test_single_hip_runtime_per_process():
    """Loading the library first (before any torch import) must not bring a
    second HIP runtime next to the one PyTorch ships: one libamdhip64 and one
    libhsa-runtime64 mapped, in a fresh interpreter."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2106_10278_amd import binding\n"
        "binding.load_library()\n"
        "import torch\n"
        "maps = open('/proc/self/maps').read().splitlines()\n"
        "libs = {l.split()[-1] for l in maps if 'libamdhip64' in l or 'libhsa-runtime64' in l}\n"
        "print(len([l for l in libs if 'amdhip64' in l]), len([l for l in libs if 'hsa-runtime64' in l]))\n"
    ) % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split()[-2:] == ["1", "1"]
