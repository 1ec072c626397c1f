"""FP64 CPU oracle for the separable NPCF estimator (Philcox & Slepian,
arXiv:2106.10278, section "Application to Discrete Data").

TEST INFRASTRUCTURE ONLY: imported by tests/, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of bench.py.  The GPU library never imports it.

The C source ``npcf_oracle.c`` is compiled with gcc into ``_build/liboracle.so``
by :func:`build`.  This module is a thin ctypes wrapper plus the output
conventions of the paper:

* eq. basis-parity-conj / the parity remark after eq. zeta-basis-decomp: with
  a real field and vec L = 0, even sum of l_{D-1} gives a purely real
  coefficient, odd gives a purely imaginary one, so for D >= 3 the reported
  value is Re (even) or Im (odd); D = 2 coefficients are reported complex.
* N = 5 (D = 3, section "Hydrodynamic Turbulence"): labels are
  (l1, l2, l12, l3, l4) and radial tuples (b1, b2, b3, b4); the parity sum is
  l1 + l2 + l3 + l4.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "npcf_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int), ("N", ctypes.c_int), ("lmax", ctypes.c_int), ("nbins", ctypes.c_int),
        ("edges", ctypes.POINTER(ctypes.c_double)),
        ("box", ctypes.c_double * 4),
        ("periodic", ctypes.c_int), ("btuple_mode", ctypes.c_int),
        ("basis", ctypes.c_int), ("Lmax", ctypes.c_int),
        ("geometry", ctypes.c_int),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lp = ctypes.POINTER(ctypes.c_long)
    lib.oracle_num_states.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.oracle_state_labels.argtypes = [ctypes.c_int, ctypes.c_int, ip]
    lib.oracle_harmonics.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
    lib.oracle_ferrers_neg.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double]
    lib.oracle_ferrers_neg.restype = ctypes.c_double
    lib.oracle_wigner3j.argtypes = [ctypes.c_int] * 6
    lib.oracle_wigner3j.restype = ctypes.c_double
    lib.oracle_cg3.argtypes = [ctypes.c_int] * 6
    lib.oracle_cg3.restype = ctypes.c_double
    lib.oracle_dim_states.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.oracle_dim_states.restype = ctypes.c_double
    lib.oracle_num_lambda.argtypes = [ctypes.c_int] * 3
    lib.oracle_lambda_labels.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip]
    lib.oracle_num_btuples.argtypes = [ctypes.c_int] * 3
    lib.oracle_btuple_labels.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip]
    lib.oracle_bin_volume.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
    lib.oracle_bin_volume.restype = ctypes.c_double
    lib.oracle_coupling_terms.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip, dp]
    lib.oracle_num_lambda_los.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.oracle_lambda_labels_los.argtypes = [ctypes.c_int, ctypes.c_int, ip]
    lib.oracle_coupling_terms_los.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip, dp]
    lib.oracle_alm.argtypes = [ctypes.POINTER(_Cfg), dp, dp, ctypes.c_long, lp, ctypes.c_long, dp, lp]
    lib.oracle_npcf.argtypes = [ctypes.POINTER(_Cfg), dp, dp, ctypes.c_long, lp, ctypes.c_long, dp, lp]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _lp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


def state_labels(D: int, lmax: int) -> np.ndarray:
    """All [l] sets (l1 first) with |l1| <= l2 <= ... <= l_{D-1} <= lmax."""
    lib = _load()
    n = lib.oracle_num_states(D, lmax)
    lab = np.zeros((n, D - 1), dtype=np.int32)
    lib.oracle_state_labels(D, lmax, _ip(lab))
    return lab


def harmonics(D: int, lmax: int, x) -> np.ndarray:
    """Y_[l](xhat) for every state of :func:`state_labels` (complex)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = lib.oracle_num_states(D, lmax)
    re = np.zeros(n)
    im = np.zeros(n)
    st = lib.oracle_harmonics(D, lmax, _dp(x), _dp(re), _dp(im))
    if st != 0:
        raise ValueError(f"oracle_harmonics status {st}")
    return re + 1j * im


def ferrers_neg(mu: float, n: int, x: float) -> float:
    """Ferrers P^{-mu}_{mu+n}(x) (first kind, DLMF 14.3)."""
    return _load().oracle_ferrers_neg(float(mu), int(n), float(x))


def wigner3j(j1, j2, j3, m1, m2, m3) -> float:
    return _load().oracle_wigner3j(j1, j2, j3, m1, m2, m3)


def cg3(j1, m1, j2, m2, J, M) -> float:
    """<m1 j1, m2 j2 | M J> for D = 3 as written in eq. CG-examples."""
    return _load().oracle_cg3(j1, m1, j2, m2, J, M)


def dim_states(D: int, l: int) -> float:
    return _load().oracle_dim_states(D, l)


def lambda_labels(D: int, N: int, lmax: int, Lmax=None) -> np.ndarray:
    """Lambda labels; with Lmax given (D = 3, N = 3), the line-of-sight basis
    labels (l1, l2, L) with L <= Lmax."""
    lib = _load()
    if Lmax is not None:
        if (D, N) != (3, 3):
            raise ValueError("the line-of-sight basis needs D = 3, N = 3")
        n = lib.oracle_num_lambda_los(lmax, Lmax)
        lab = np.zeros((n, 3), dtype=np.int32)
        lib.oracle_lambda_labels_los(lmax, Lmax, _ip(lab))
        return lab
    n = lib.oracle_num_lambda(D, N, lmax)
    if n < 0:
        raise ValueError("unsupported (D, N)")
    lab = np.zeros((n, 5 if N == 5 else 3), dtype=np.int32)
    lib.oracle_lambda_labels(D, N, lmax, _ip(lab))
    return lab


def btuple_labels(nbins: int, N: int, mode: int = 0) -> np.ndarray:
    lib = _load()
    n = lib.oracle_num_btuples(nbins, N, mode)
    bt = np.zeros((n, 4 if N == 5 else 3), dtype=np.int32)
    lib.oracle_btuple_labels(nbins, N, mode, _ip(bt))
    return bt[:, : N - 1].copy()


def bin_volume(D: int, e0: float, e1: float) -> float:
    return _load().oracle_bin_volume(D, e0, e1)


def coupling_terms(D: int, N: int, lmax: int, Lmax=None):
    """(lambda index, state-index tuple, C) for every non-zero coupling term
    (with Lmax: the line-of-sight basis, D = 3, N = 3)."""
    lib = _load()
    if Lmax is not None:
        cnt = lib.oracle_coupling_terms_los(lmax, Lmax, 0, None, None, None)
        lam = np.zeros(cnt, dtype=np.int32)
        s = np.zeros((cnt, 3), dtype=np.int32)
        c = np.zeros(cnt)
        lib.oracle_coupling_terms_los(lmax, Lmax, cnt, _ip(lam), _ip(s), _dp(c))
        return lam, s, c
    cnt = lib.oracle_coupling_terms(D, N, lmax, 0, None, None, None)
    if cnt < 0:
        raise ValueError("unsupported (D, N)")
    lam = np.zeros(cnt, dtype=np.int32)
    s = np.zeros((cnt, 4 if N == 5 else 3), dtype=np.int32)
    c = np.zeros(cnt)
    lib.oracle_coupling_terms(D, N, lmax, cnt, _ip(lam), _ip(s), _dp(c))
    return lam, s, c


def _cfg(D, N, lmax, edges, box, periodic=True, btuple_mode=0, Lmax=None, sphere=False, hyperbolic=False):
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    cfg = _Cfg()
    cfg.D, cfg.N, cfg.lmax, cfg.nbins = D, N, lmax, len(edges) - 1
    cfg.edges = _dp(edges)
    b = list(box) + [1.0] * (4 - len(box))
    for k in range(4):
        cfg.box[k] = float(b[k])
    cfg.periodic = 1 if periodic else 0
    cfg.btuple_mode = btuple_mode
    cfg.basis = 0 if Lmax is None else 1
    cfg.Lmax = 0 if Lmax is None else int(Lmax)
    # sphere: points on the unit D-sphere (D = 2: S^2 in R^3; D = 3: S^3 in R^4);
    # hyperbolic: points of H^D on the hyperboloid in R^{D,1}, box[0] = V
    cfg.geometry = 3 if hyperbolic else ((D - 1) if sphere else 0)
    return cfg, edges


def _prep(pos, w, prims):
    pos = np.ascontiguousarray(pos, dtype=np.float64)  # [D][n]
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = pos.shape[1]
    if prims is None:
        prims = np.arange(n, dtype=np.int64)
    prims = np.ascontiguousarray(prims, dtype=np.int64)
    return pos, w, n, prims


def alm(D, lmax, edges, box, pos, w, prims=None, periodic=True, sphere=False, hyperbolic=False):
    """a^b_[l](y_j) for the listed primaries: complex [nprim][nbins][nstates].
    sphere: points on the unit D-sphere (D = 2: pos [3][n], D = 3: pos [4][n]
    unit vectors; edges in radians of geodesic angle).  hyperbolic: points of
    H^D on the hyperboloid x0^2 - |x|^2 = 1 (pos [D+1][n]; edges in geodesic
    distance; box[0] = V)."""
    lib = _load()
    cfg, edges = _cfg(D, 3, lmax, edges, box, periodic, sphere=sphere, hyperbolic=hyperbolic)
    pos, w, n, prims = _prep(pos, w, prims)
    nst = lib.oracle_num_states(D, lmax)
    out = np.zeros((len(prims), len(edges) - 1, nst, 2))
    pairs = ctypes.c_long(0)
    st = lib.oracle_alm(ctypes.byref(cfg), _dp(pos), _dp(w), n, _lp(prims), len(prims), _dp(out), ctypes.byref(pairs))
    if st != 0:
        raise ValueError(f"oracle_alm status {st}")
    return out[..., 0] + 1j * out[..., 1], int(pairs.value)


def npcf(D, N, lmax, edges, box, pos, w, prims=None, periodic=True, btuple_mode=0, Lmax=None, sphere=False,
         hyperbolic=False):
    """Complex zeta^{Lambda,b} [nlambda][nbtuple] over the listed primaries
    (default: all) against all secondaries, plus the in-range pair count.
    With Lmax (D = 3, N = 3): the line-of-sight basis P^{0L}, L <= Lmax.
    sphere / hyperbolic: the curved geometries (see alm)."""
    lib = _load()
    cfg, edges = _cfg(D, N, lmax, edges, box, periodic, btuple_mode, Lmax, sphere, hyperbolic)
    pos, w, n, prims = _prep(pos, w, prims)
    nlam = len(lambda_labels(D, N, lmax, Lmax)) if Lmax is not None else lib.oracle_num_lambda(D, N, lmax)
    nbt = lib.oracle_num_btuples(len(edges) - 1, N, btuple_mode)
    if nlam < 0 or nbt < 0:
        raise ValueError("unsupported (D, N)")
    out = np.zeros((nlam, nbt, 2))
    pairs = ctypes.c_long(0)
    st = lib.oracle_npcf(ctypes.byref(cfg), _dp(pos), _dp(w), n, _lp(prims), len(prims), _dp(out), ctypes.byref(pairs))
    if st != 0:
        raise ValueError(f"oracle_npcf status {st}")
    return out[..., 0] + 1j * out[..., 1], int(pairs.value)


def reported_part(zeta: np.ndarray, labels: np.ndarray, D: int, N: int, los: bool = False) -> np.ndarray:
    """Apply the paper's parity rule: for D >= 3 report Re for even sum of the
    total angular momenta and Im for odd; D = 2 stays complex.  For the
    line-of-sight basis the sum is l1 + l2 + L (P^{0L}* = (-1)^{l1+l2+L} P^{0L})."""
    if D == 2:
        return zeta
    if N == 3 and not los:
        tot = 2 * labels[:, 0]
    elif N == 5:
        tot = labels[:, 0] + labels[:, 1] + labels[:, 3] + labels[:, 4]
    else:
        tot = labels[:, 0] + labels[:, 1] + labels[:, 2]
    odd = (tot % 2) == 1
    return np.where(odd[:, None], zeta.imag, zeta.real)
