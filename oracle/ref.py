"""ctypes wrapper of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import build as _build

PH_MAGNETIC = 1
PH_CHARGE = 2
PP_UPDOWN = 4
PH_LONG_UPUP = 8
PH_LONG_UPDOWN = 16
PH_TRANSVERSE = 32
PP_SINGLET = 64
PP_TRIPLET = 128


class _Shape(ctypes.Structure):
    _fields_ = [("lx", ctypes.c_int), ("ly", ctypes.c_int), ("nw", ctypes.c_int),
                ("nwex", ctypes.c_int), ("nq", ctypes.c_int),
                ("q_list", ctypes.POINTER(ctypes.c_int)),
                ("q_begin", ctypes.c_long), ("q_end", ctypes.c_long)]


_lib = None


def lib():
    """The compiled oracle.  G4_ORACLE_LIB may name another build of the same
    source (the mutation tests load copies with a planted mistake this way)."""
    global _lib
    if _lib is None:
        path = os.environ.get("G4_ORACLE_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_accumulate.argtypes = [ctypes.POINTER(_Shape), ctypes.c_int, dp, dp, dp,
                                        ctypes.c_int, dp, dp, ctypes.c_int]
        L.oracle_accumulate.restype = ctypes.c_int
        L.oracle_entries.argtypes = [ctypes.POINTER(_Shape), ctypes.c_int, dp, dp, dp,
                                     ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.c_long, dp]
        L.oracle_entries.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_gsigma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int), dp,
                                    ctypes.POINTER(ctypes.c_int64), ctypes.c_long, dp]
        L.oracle_gsigma.restype = ctypes.c_int
        L.oracle_accumulate_mo.argtypes = [ctypes.POINTER(_Shape), ctypes.c_int, ctypes.c_int, dp, dp, dp,
                                           ctypes.c_int, dp]
        L.oracle_accumulate_mo.restype = ctypes.c_int
        L.oracle_entries_mo.argtypes = [ctypes.POINTER(_Shape), ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.c_long, dp]
        L.oracle_entries_mo.restype = ctypes.c_int
        _lib = L
    return _lib


def _shape(w):
    q = np.ascontiguousarray(np.asarray(w.qs, dtype=np.int32))
    s = _Shape(w.lx, w.ly, w.nw, w.nwex, w.nq,
               q.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), w.q0, w.q1)
    return s, q


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c128(a, shape):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    assert a.shape == shape, (a.shape, shape)
    return a


def accumulate(w, channel: int, g_up: np.ndarray, g_dn: np.ndarray, sign: np.ndarray,
               g4: Optional[np.ndarray] = None, comp: Optional[np.ndarray] = None,
               nthreads: int = 0) -> np.ndarray:
    """G4 slice (complex128 [planes, N, N]) += sum_b s_b T_channel, in place if given."""
    sign = np.ascontiguousarray(sign, dtype=np.float64)
    batch = sign.shape[0]
    g_up = _c128(g_up, (batch, w.ng, w.ng))
    g_dn = _c128(g_dn, (batch, w.ng, w.ng))
    if g4 is None:
        g4 = np.zeros((w.planes, w.n, w.n), dtype=np.complex128)
    assert g4.dtype == np.complex128 and g4.flags.c_contiguous and g4.shape == (w.planes, w.n, w.n)
    if comp is not None:
        assert comp.dtype == np.complex128 and comp.shape == g4.shape and comp.flags.c_contiguous
    s, q = _shape(w)
    rc = lib().oracle_accumulate(ctypes.byref(s), channel, _dp(g_up), _dp(g_dn), _dp(sign), batch,
                                 _dp(g4), _dp(comp) if comp is not None else None, nthreads)
    if rc:
        raise ValueError("oracle_accumulate rejected the shape or arguments")
    return g4


def accumulate_mo(w, nb: int, channel: int, g_up: np.ndarray, g_dn: np.ndarray, sign: np.ndarray,
                  g4: Optional[np.ndarray] = None) -> np.ndarray:
    """Multi-orbital slice (complex128 [planes, N nb^2, N nb^2]; rows (K2, b3, b4),
    columns (K1, b1, b2)) += sum_b s_b T_channel; G: batch x (Ng nb)^2."""
    sign = np.ascontiguousarray(sign, dtype=np.float64)
    batch = sign.shape[0]
    ngb = w.ng * nb
    g_up = _c128(g_up, (batch, ngb, ngb))
    g_dn = _c128(g_dn, (batch, ngb, ngb))
    side = w.n * nb * nb
    if g4 is None:
        g4 = np.zeros((w.planes, side, side), dtype=np.complex128)
    assert g4.dtype == np.complex128 and g4.flags.c_contiguous and g4.shape == (w.planes, side, side)
    s, q = _shape(w)
    rc = lib().oracle_accumulate_mo(ctypes.byref(s), nb, channel, _dp(g_up), _dp(g_dn), _dp(sign), batch, _dp(g4))
    if rc:
        raise ValueError("oracle_accumulate_mo rejected the shape or arguments")
    return g4


def entries_mo(w, nb: int, channel: int, g_up: np.ndarray, g_dn: np.ndarray, sign: np.ndarray,
               idx: np.ndarray) -> np.ndarray:
    """sum_b s_b T_channel of the multi-orbital slice at flattened entries idx."""
    sign = np.ascontiguousarray(sign, dtype=np.float64)
    batch = sign.shape[0]
    ngb = w.ng * nb
    g_up = _c128(g_up, (batch, ngb, ngb))
    g_dn = _c128(g_dn, (batch, ngb, ngb))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(idx.shape[0], dtype=np.complex128)
    s, q = _shape(w)
    rc = lib().oracle_entries_mo(ctypes.byref(s), nb, channel, _dp(g_up), _dp(g_dn), _dp(sign), batch,
                                 idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), idx.shape[0], _dp(out))
    if rc:
        raise ValueError("oracle_entries_mo rejected the shape or arguments")
    return out


def entries(w, channel: int, g_up: np.ndarray, g_dn: np.ndarray, sign: np.ndarray,
            idx: np.ndarray) -> np.ndarray:
    """sum_b s_b T_channel at flattened slice entries idx (complex128 array)."""
    sign = np.ascontiguousarray(sign, dtype=np.float64)
    batch = sign.shape[0]
    g_up = _c128(g_up, (batch, w.ng, w.ng))
    g_dn = _c128(g_dn, (batch, w.ng, w.ng))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(idx.shape[0], dtype=np.complex128)
    s, q = _shape(w)
    rc = lib().oracle_entries(ctypes.byref(s), channel, _dp(g_up), _dp(g_dn), _dp(sign), batch,
                              idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), idx.shape[0],
                              _dp(out))
    if rc:
        raise ValueError("oracle_entries rejected the shape or arguments")
    return out


def max_threads() -> int:
    return lib().oracle_max_threads()


def gsigma(w, spin: int, tau, site, M, idx=None) -> np.ndarray:
    """G_sigma of one expansion configuration (n vertices: imaginary times tau,
    cluster sites site, n x n matrix M): the full Ng x Ng matrix, or the
    flattened entries idx (K1*Ng + K2)."""
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    site = np.ascontiguousarray(site, dtype=np.int32)
    n = tau.shape[0]
    M = np.ascontiguousarray(M, dtype=np.complex128).reshape(n, n)
    full = idx is None
    if full:
        idx = np.arange(w.ng * w.ng, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(idx.shape[0], dtype=np.complex128)
    rc = lib().oracle_gsigma(w.lx, w.ly, w.nw, w.nwex, w.beta, w.mu, w.h, w.t, spin, n, _dp(tau),
                             site.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(M),
                             idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), idx.shape[0], _dp(out))
    if rc:
        raise ValueError("oracle_gsigma rejected the arguments")
    return out.reshape(w.ng, w.ng) if full else out
