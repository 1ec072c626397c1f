"""ctypes binding of the C ABI in include/npcf.h.

Argument marshalling only: every step of the estimator runs in the HIP
library ``_build/libnpcf.so``.  There is no CPU fallback; a missing library
raises :class:`NPCFLibraryMissing`.  Device tensors come from PyTorch (it
provides device memory and the stream); the library never sees torch types.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("NPCF_LIBRARY", os.path.join(HERE, "_build", "libnpcf.so"))
HEADER = os.path.join(HERE, "..", "include", "npcf.h")

NPCF_OK, NPCF_E_INVALID, NPCF_E_UNSUPPORTED, NPCF_E_NOMEM, NPCF_E_DEVICE, NPCF_E_STATE = range(6)
PRECISION = {"plain": 0, "mixed_bf16": 1, "mixed_fp16": 2, "mixed_bf16x6": 3}
NORM = {"raw": 0, "by_randoms": 1}
ROLE = {"data": 0, "randoms": 1}


class NPCFLibraryMissing(RuntimeError):
    pass


class NPCFError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        detail = ""
        if status in (NPCF_E_DEVICE, NPCF_E_NOMEM, NPCF_E_UNSUPPORTED):
            detail = load_library().npcf_last_error_detail().decode()
        super().__init__(f"{what}: {strerror(status)} (status {status})" + (f" [{detail}]" if detail else ""))


class _Config(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int), ("N", ctypes.c_int), ("lmax", ctypes.c_int), ("nbins", ctypes.c_int),
        ("edges", ctypes.POINTER(ctypes.c_double)),
        ("box", ctypes.c_double * 4),
        ("periodic", ctypes.c_int), ("btuple_mode", ctypes.c_int),
        ("precision", ctypes.c_int), ("norm", ctypes.c_int),
        ("basis", ctypes.c_int), ("Lmax", ctypes.c_int),
        ("geometry", ctypes.c_int),
    ]


class _Tuning(ctypes.Structure):
    _fields_ = [("cell_subdiv", ctypes.c_int), ("couple_block", ctypes.c_int), ("chunk_rows", ctypes.c_int64),
                ("harmonic_blocks_per_cu", ctypes.c_int), ("curved_bins_per_pass", ctypes.c_int)]


_lib = None


def load_library():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NPCFLibraryMissing(
            f"{LIB_PATH} not found: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 (same
    # soname), which must be loaded first so that the library binds to it;
    # loaded the other way round, torch would bring a second runtime and the
    # two would contend for the device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64
    ip = ctypes.POINTER(ctypes.c_int)
    lib.npcf_plan.argtypes = [ctypes.POINTER(_Config), vp, i64, ctypes.POINTER(vp)]
    lib.npcf_accumulate.argtypes = [vp, vp, vp, i64, i64, i64, ctypes.c_int]
    lib.npcf_accumulate_static.argtypes = [vp, vp, vp, i64, i64, i64, ctypes.c_int]
    lib.npcf_finalize.argtypes = [vp, dp, ctypes.c_size_t]
    lib.npcf_describe.argtypes = [vp, ip, ip, ip, ip, ctypes.POINTER(ctypes.c_size_t)]
    lib.npcf_accumulate_grid.argtypes = [vp, vp, ip, i64, i64, ctypes.c_int]
    lib.npcf_alm_grid.argtypes = [vp, vp, ip, i64, i64, dp, ctypes.c_size_t]
    lib.npcf_pair_count.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.npcf_alm.argtypes = [vp, vp, vp, i64, i64, i64, dp, ctypes.c_size_t]
    lib.npcf_accumulate_batch.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i64)]
    lib.npcf_finalize_batch.argtypes = [vp, ctypes.c_int, dp, ctypes.c_size_t, dp, ctypes.POINTER(i64)]
    lib.npcf_reset.argtypes = [vp]
    lib.npcf_destroy.argtypes = [vp]
    lib.npcf_set_tuning.argtypes = [vp, ctypes.c_int, ctypes.c_int, i64]
    lib.npcf_stage_ms.argtypes = [vp, dp]
    lib.npcf_autotune.argtypes = [vp, vp, vp, i64, i64, ip, ip, dp]
    lib.npcf_get_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
    lib.npcf_apply_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
    lib.npcf_strerror.argtypes = [ctypes.c_int]
    lib.npcf_strerror.restype = ctypes.c_char_p
    lib.npcf_version.restype = ctypes.c_char_p
    lib.npcf_last_error_detail.restype = ctypes.c_char_p
    for name in ("npcf_plan", "npcf_accumulate", "npcf_accumulate_static", "npcf_finalize", "npcf_describe", "npcf_pair_count", "npcf_alm",
                 "npcf_accumulate_batch", "npcf_finalize_batch", "npcf_reset", "npcf_destroy", "npcf_set_tuning",
                 "npcf_stage_ms", "npcf_autotune", "npcf_accumulate_grid", "npcf_alm_grid", "npcf_get_tuning",
                 "npcf_apply_tuning"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def header_symbols() -> list:
    """Every function the public header declares."""
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(npcf_[a-z_0-9]+)\s*\(", src, re.M)))


def strerror(status: int) -> str:
    return load_library().npcf_strerror(int(status)).decode()


def version() -> str:
    return load_library().npcf_version().decode()


def _check(st: int, what: str):
    if st != NPCF_OK:
        raise NPCFError(st, what)


def _dptr(t):
    """Device pointer of a contiguous float64 torch tensor (or an int)."""
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor on the GPU")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


class NPCF:
    """One estimator plan (npcf_plan ... npcf_destroy)."""

    def __init__(self, D: int, N: int, lmax: int, edges, box, periodic: bool = True, btuple_mode: int = 0,
                 precision: str = "plain", norm: str = "raw", max_points: int = 1 << 20, stream=None,
                 Lmax=None, sphere: bool = False, hyperbolic: bool = False):
        lib = load_library()
        self.D, self.N, self.lmax = int(D), int(N), int(lmax)
        self.edges = np.ascontiguousarray(edges, dtype=np.float64)
        cfg = _Config()
        cfg.D, cfg.N, cfg.lmax, cfg.nbins = self.D, self.N, self.lmax, len(self.edges) - 1
        cfg.edges = self.edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        b = [float(x) for x in box] + [1.0] * (4 - len(box))
        for k in range(4):
            cfg.box[k] = b[k]
        cfg.periodic = 1 if periodic else 0
        cfg.btuple_mode = int(btuple_mode)
        cfg.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
        cfg.norm = NORM[norm] if isinstance(norm, str) else int(norm)
        # Lmax given: the line-of-sight basis P^{0L}_{l1 l2} (D = 3, N = 3)
        cfg.basis = 0 if Lmax is None else 1
        cfg.Lmax = 0 if Lmax is None else int(Lmax)
        # points on the unit D-sphere (D = 2 or 3): pos [D + 1][n] unit vectors, edges in radians;
        # hyperbolic: points of H^D on the hyperboloid (pos [D + 1][n]), box[0] = the region's volume
        cfg.geometry = 2 if hyperbolic else (1 if sphere else 0)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        h = ctypes.c_void_p()
        _check(lib.npcf_plan(ctypes.byref(cfg), ctypes.c_void_p(stream), int(max_points), ctypes.byref(h)), "npcf_plan")
        self._h = h
        nl, nb_ = ctypes.c_int(), ctypes.c_int()
        olen = ctypes.c_size_t()
        _check(lib.npcf_describe(h, ctypes.byref(nl), None, ctypes.byref(nb_), None, ctypes.byref(olen)), "npcf_describe")
        # N = 5: labels (l1, l2, l12, l3, l4) and radial tuples of 4; else 3 each
        lab = np.zeros((nl.value, 5 if self.N == 5 else 3), dtype=np.int32)
        bt = np.zeros((nb_.value, 4 if self.N == 5 else 3), dtype=np.int32)
        _check(lib.npcf_describe(h, None, lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), None,
                                 bt.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), None), "npcf_describe")
        self.lambda_labels = lab
        self.btuples = bt[:, : self.N - 1].copy()
        self.out_len = olen.value

    # ---------------------------------------------------------------------
    def accumulate(self, pos, w, prim_begin: int = 0, prim_end: int | None = None, role: str = "data"):
        n = int(w.shape[0])
        if prim_end is None:
            prim_end = n
        _check(load_library().npcf_accumulate(self._h, _dptr(pos), _dptr(w), n, int(prim_begin), int(prim_end),
                                              ROLE[role]), "npcf_accumulate")

    def accumulate_static(self, pos, w, prim_begin: int = 0, prim_end: int | None = None, role: str = "data"):
        """npcf_accumulate with every per-call device buffer in the library's
        static workspace (no device allocation; calls overlapping on one device race)."""
        n = int(w.shape[0])
        if prim_end is None:
            prim_end = n
        _check(load_library().npcf_accumulate_static(self._h, _dptr(pos), _dptr(w), n, int(prim_begin),
                                                     int(prim_end), ROLE[role]), "npcf_accumulate_static")

    def accumulate_grid(self, field, prim_begin: int = 0, prim_end: int | None = None, role: str = "data"):
        """Gridded data: `field` is a contiguous float64 CUDA tensor of shape
        (dims[0], ..., dims[D-1]) on the periodic box; its nodes [prim_begin,
        prim_end) (row-major) are the primaries."""
        dims = np.ascontiguousarray(list(field.shape), dtype=np.int32)
        if len(dims) != self.D:
            raise ValueError(f"field must have {self.D} dimensions")
        ng = int(np.prod(dims))
        if prim_end is None:
            prim_end = ng
        _check(load_library().npcf_accumulate_grid(self._h, _dptr(field), dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                                   int(prim_begin), int(prim_end), ROLE[role]), "npcf_accumulate_grid")

    def alm_grid(self, field, prim_begin: int = 0, prim_end: int | None = None) -> np.ndarray:
        """a^b_[l] of the grid nodes [prim_begin, prim_end) from the FFT path."""
        dims = np.ascontiguousarray(list(field.shape), dtype=np.int32)
        ng = int(np.prod(dims))
        if prim_end is None:
            prim_end = ng
        nb = len(self.edges) - 1
        nst = stored_states(self.D, self.lmax)
        out = np.zeros((prim_end - prim_begin, nb, nst, 2))
        _check(load_library().npcf_alm_grid(self._h, _dptr(field), dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                            int(prim_begin), int(prim_end),
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size),
               "npcf_alm_grid")
        return out[..., 0] + 1j * out[..., 1]

    def finalize(self) -> np.ndarray:
        out = np.zeros(self.out_len)
        _check(load_library().npcf_finalize(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.out_len),
               "npcf_finalize")
        return self._shape(out)

    def _shape(self, out):
        nl, nbt = len(self.lambda_labels), len(self.btuples)
        if self.D == 2:
            z = out.reshape(nl, nbt, 2)
            return z[..., 0] + 1j * z[..., 1]
        return out.reshape(nl, nbt)

    def pair_count(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(load_library().npcf_pair_count(self._h, ctypes.byref(a), ctypes.byref(b)), "npcf_pair_count")
        return a.value, b.value

    def alm(self, pos, w, prim_begin: int = 0, prim_end: int | None = None) -> np.ndarray:
        n = int(w.shape[0])
        if prim_end is None:
            prim_end = n
        nb = len(self.edges) - 1
        nst = stored_states(self.D, self.lmax)
        out = np.zeros((prim_end - prim_begin, nb, nst, 2))
        _check(load_library().npcf_alm(self._h, _dptr(pos), _dptr(w), n, int(prim_begin), int(prim_end),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size), "npcf_alm")
        return out[..., 0] + 1j * out[..., 1]

    def accumulate_batch(self, pos_list, w_list):
        ncat = len(pos_list)
        P = (ctypes.c_void_p * ncat)(*[_dptr(p).value for p in pos_list])
        W = (ctypes.c_void_p * ncat)(*[_dptr(w).value for w in w_list])
        Ns = (ctypes.c_int64 * ncat)(*[int(w.shape[0]) for w in w_list])
        _check(load_library().npcf_accumulate_batch(self._h, ncat, P, W, Ns), "npcf_accumulate_batch")

    def finalize_batch(self, cat: int):
        """(zeta of catalogue `cat`, its completion time in ms after the batch
        start, its in-range pair count)."""
        out = np.zeros(self.out_len)
        done = ctypes.c_double()
        pairs = ctypes.c_int64()
        _check(load_library().npcf_finalize_batch(self._h, int(cat), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                  self.out_len, ctypes.byref(done), ctypes.byref(pairs)),
               "npcf_finalize_batch")
        return self._shape(out), done.value, pairs.value

    def stage_ms(self):
        ms = (ctypes.c_double * 3)()
        _check(load_library().npcf_stage_ms(self._h, ms), "npcf_stage_ms")
        return {"harmonic": ms[0], "coupling": ms[1], "cells": ms[2]}

    def set_tuning(self, cell_subdiv: int = 0, couple_block: int = 0, chunk_rows: int = 0):
        _check(load_library().npcf_set_tuning(self._h, int(cell_subdiv), int(couple_block), int(chunk_rows)),
               "npcf_set_tuning")

    def autotune(self, pos, w, sample: int = 8192):
        """Tune the cell subdivision and the harmonic grid (flat geometry) or
        the bins per pass (curved geometries), the coupling block size and the
        chunk rows on this catalogue (npcf_autotune; resets the accumulators).
        Returns every knob of the resulting tuning and the timed ms."""
        cs, cb, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(load_library().npcf_autotune(self._h, _dptr(pos), _dptr(w), int(w.shape[0]), int(sample),
                                            ctypes.byref(cs), ctypes.byref(cb), ctypes.byref(ms)), "npcf_autotune")
        return self.tuning() | {"sample_ms": ms.value}

    def tuning(self):
        t = _Tuning()
        _check(load_library().npcf_get_tuning(self._h, ctypes.byref(t)), "npcf_get_tuning")
        return {"cell_subdiv": t.cell_subdiv, "couple_block": t.couple_block, "chunk_rows": t.chunk_rows,
                "harmonic_blocks_per_cu": t.harmonic_blocks_per_cu, "curved_bins_per_pass": t.curved_bins_per_pass}

    def apply_tuning(self, cell_subdiv=0, couple_block=0, chunk_rows=0, harmonic_blocks_per_cu=0,
                     curved_bins_per_pass=0):
        t = _Tuning(int(cell_subdiv), int(couple_block), int(chunk_rows), int(harmonic_blocks_per_cu),
                    int(curved_bins_per_pass))
        _check(load_library().npcf_apply_tuning(self._h, ctypes.byref(t)), "npcf_apply_tuning")

    def reset(self):
        _check(load_library().npcf_reset(self._h), "npcf_reset")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().npcf_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stored_states(D: int, L: int) -> int:
    if D == 2:
        return L + 1
    if D == 3:
        return (L + 1) * (L + 2) // 2
    return (L + 1) * (L + 2) * (L + 3) // 6


def stored_state_labels(D: int, L: int) -> np.ndarray:
    """(l1, l2, l3) of every stored state (l1 >= 0 half), in the library's order."""
    out = []
    if D == 2:
        out = [(l, 0, 0) for l in range(L + 1)]
    elif D == 3:
        out = [(m, l, 0) for l in range(L + 1) for m in range(l + 1)]
    else:
        out = [(l1, l2, l3) for l3 in range(L + 1) for l2 in range(l3 + 1) for l1 in range(l2 + 1)]
    return np.array(out, dtype=np.int32)
