"""Python binding of the G4 slice library (include/g4.h), by ctypes.

Argument marshalling only: every step of the accumulation runs in the HIP
library libg4.so next to this file.  Functions keep the C names.  Device
buffers are passed as torch tensors (or raw integer device pointers); the
binding checks their dtype, device, contiguity and element count against the
slice's shape before handing the pointer over, because the library cannot
see the size of a device allocation.

Failures raise G4Error(code, message).  If the library has not been built the
import raises ImportError: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libg4.so")

G4_ABI_VERSION = 1
G4_OK, G4_E_ARG, G4_E_OOM, G4_E_HIP, G4_E_STATE, G4_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
G4_PH_MAGNETIC, G4_PH_CHARGE, G4_PP_UPDOWN = 1, 2, 4
G4_PH_LONG_UPUP, G4_PH_LONG_UPDOWN, G4_PH_TRANSVERSE = 8, 16, 32
G4_PP_SINGLET, G4_PP_TRIPLET = 64, 128
G4_IN_C128, G4_IN_C64 = 0, 1
G4_PROD_F64, G4_PROD_F32, G4_PROD_BF16X2, G4_PROD_F16X2 = 0, 1, 2, 3
G4_ACC_C128, G4_ACC_C64_KAHAN, G4_ACC_C64 = 0, 1, 2
G4_MODE_PLAIN, G4_MODE_BATCHED = 0, 1
G4_F_CHECK_FINITE, G4_F_KERNEL_TIMING, G4_F_GRAPH, G4_F_MFMA, G4_F_PACKED, G4_F_PACKED_DEEP, G4_F_PERSISTENT = \
    1, 2, 4, 8, 16, 32, 64
G4_VARIANT_VALU, G4_VARIANT_MFMA, G4_VARIANT_PACKED, G4_VARIANT_PACKED_DEEP, G4_VARIANT_PACKED_MFMA = 0, 1, 2, 3, 4

STATUS_NAMES = {0: "G4_OK", -1: "G4_E_ARG", -2: "G4_E_OOM", -3: "G4_E_HIP", -4: "G4_E_STATE",
                -5: "G4_E_UNSUPPORTED"}


class G4Error(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, code), message))
        self.code = code
        self.message = message


class g4_config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("lx", ctypes.c_int32), ("ly", ctypes.c_int32),
                ("nw", ctypes.c_int32), ("nwex", ctypes.c_int32), ("nq", ctypes.c_int32),
                ("q_list", ctypes.POINTER(ctypes.c_int32)),
                ("q_begin", ctypes.c_int64), ("q_end", ctypes.c_int64),
                ("channels", ctypes.c_uint32), ("g_in", ctypes.c_int32), ("prod", ctypes.c_int32),
                ("acc", ctypes.c_int32), ("mode", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p), ("flags", ctypes.c_uint32),
                ("tile", ctypes.c_int32), ("beta", ctypes.c_double)]


class g4_tune_result(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("tile", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("ms_per_measurement", ctypes.c_double),
                ("rel_err_fp64", ctypes.c_double)]


class g4_stats_t(ctypes.Structure):
    _fields_ = [("measurements", ctypes.c_uint64), ("sign_sum", ctypes.c_double),
                ("launches", ctypes.c_uint64), ("kernel_ms", ctypes.c_double),
                ("timed_launches", ctypes.c_uint64), ("entries", ctypes.c_uint64),
                ("channels", ctypes.c_uint32), ("batch", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("variant", ctypes.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError("libg4.so is not built (run __graft_entry__.build() or "
                      "python paper_2105_00027_amd/build.py)")
# torch ships its own HIP runtime.  Loading it first makes libg4.so bind to that
# same runtime (matched by soname), so device pointers and streams handed over
# by torch are valid in the library; loading libg4.so first would bring in a
# second HIP/HSA runtime that cannot open the device.
try:
    import torch  # noqa: F401
except ImportError:  # C callers and CPU-only use need no torch
    pass
_L = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_cfgp = ctypes.POINTER(g4_config)
_sig = {
    "g4_config_init": ([_cfgp], ctypes.c_int),
    "g4_slice_size": ([_cfgp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "g4_init_slice": ([_cfgp, ctypes.POINTER(_vp)], ctypes.c_int),
    "g4_accumulate": ([_vp, _vp, _vp, _dp, ctypes.c_int32], ctypes.c_int),
    "g4_sync": ([_vp], ctypes.c_int),
    "g4_readback": ([_vp, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, _dp], ctypes.c_int),
    "g4_load": ([_vp, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, _dp], ctypes.c_int),
    "g4_set_counts": ([_vp, ctypes.c_uint64, ctypes.c_double], ctypes.c_int),
    "g4_merge": ([_vp, _vp], ctypes.c_int),
    "g4_reset": ([_vp], ctypes.c_int),
    "g4_stats": ([_vp, ctypes.POINTER(g4_stats_t)], ctypes.c_int),
    "g4_set_plan": ([_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "g4_autotune": ([_vp, _vp, _vp, _dp, ctypes.c_int32, ctypes.c_double,
                     ctypes.POINTER(g4_tune_result)], ctypes.c_int),
    "g4_accumulate_into": ([_cfgp, _vp, _vp, _vp, _vp, _vp, _dp, ctypes.c_int32], ctypes.c_int),
    "g4_gsigma_workspace": ([ctypes.c_int32] * 7 + [ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "g4_gsigma": ([ctypes.c_int32] * 4 + [ctypes.c_double] * 4 + [ctypes.c_int32] * 3
                  + [_vp, _vp, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_uint64, _vp], ctypes.c_int),
    "g4_accumulate_mo": ([ctypes.c_int32] * 6 + [ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, ctypes.c_int64,
                          ctypes.c_uint32, ctypes.c_int32, _vp, _vp, _dp, ctypes.c_int32, _vp, _vp, _vp, _vp],
                         ctypes.c_int),
    "g4_destroy": ([_vp], None),
    "g4_last_error": ([], ctypes.c_char_p),
    "g4_synth_fill": ([_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                       ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                       ctypes.c_double, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32,
                       ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _vp], ctypes.c_int),
    "g4_index_maps": ([_cfgp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_L, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTS = tuple(_sig)


def g4_last_error() -> str:
    return (_L.g4_last_error() or b"").decode()


def _check(rc: int) -> None:
    if rc != G4_OK:
        raise G4Error(rc, g4_last_error())


class Config:
    """A g4_config plus the q_list storage it points to."""

    def __init__(self, **kw):
        self.c = g4_config()
        _check(_L.g4_config_init(ctypes.byref(self.c)))
        self._q = None
        q_list = kw.pop("q_list", None)
        for k, v in kw.items():
            if k == "stream":
                v = int(v) if v else None
            setattr(self.c, k, v)
        self.set_q_list(q_list)

    def set_q_list(self, q_list: Optional[Sequence[int]]):
        if q_list is None:
            self._q = None
            self.c.q_list = None
        else:
            self._q = (ctypes.c_int32 * len(q_list))(*[int(x) for x in q_list])
            self.c.q_list = ctypes.cast(self._q, ctypes.POINTER(ctypes.c_int32))

    # shapes
    @property
    def nc(self):
        return self.c.lx * self.c.ly

    @property
    def ng(self):
        return self.nc * (self.c.nw + self.c.nwex - 1)

    @property
    def n(self):
        return self.nc * self.c.nw

    @property
    def planes(self):
        return self.c.q_end - self.c.q_begin


def g4_config_init(**kw) -> Config:
    return Config(**kw)


def g4_slice_size(cfg: Config):
    e = ctypes.c_uint64()
    b = ctypes.c_uint64()
    _check(_L.g4_slice_size(ctypes.byref(cfg.c), ctypes.byref(e), ctypes.byref(b)))
    return int(e.value), int(b.value)


class Slice:
    """Handle returned by g4_init_slice; keeps the shape for argument checks."""

    def __init__(self, ptr, cfg: Config):
        self.ptr = ptr
        self.cfg = cfg
        self.ng = cfg.ng
        self.entries = cfg.planes * cfg.n * cfg.n


def g4_init_slice(cfg: Config) -> Slice:
    h = _vp()
    _check(_L.g4_init_slice(ctypes.byref(cfg.c), ctypes.byref(h)))
    return Slice(h, cfg)


def _device_ptr(x, nbytes_expected: int, elem_bytes: int) -> int:
    """Pointer of a device tensor holding at least nbytes_expected bytes."""
    if isinstance(x, int):
        return x
    import torch
    if not isinstance(x, torch.Tensor):
        raise G4Error(G4_E_ARG, "expected a torch tensor or an integer device pointer")
    if not x.is_cuda:
        raise G4Error(G4_E_ARG, "G buffer must live in device memory")
    if not x.is_contiguous():
        raise G4Error(G4_E_ARG, "G buffer must be contiguous")
    if x.element_size() != elem_bytes or not x.is_complex():
        raise G4Error(G4_E_ARG, "G buffer dtype %s does not match the slice's input type" % x.dtype)
    if x.numel() * x.element_size() < nbytes_expected:
        raise G4Error(G4_E_ARG, "G buffer holds %d bytes, %d needed"
                      % (x.numel() * x.element_size(), nbytes_expected))
    return x.data_ptr()


def g4_accumulate(h: Slice, G_up, G_dn, sign, batch: Optional[int] = None) -> None:
    s = np.ascontiguousarray(np.asarray(sign, dtype=np.float64).reshape(-1))
    if batch is None:
        batch = s.shape[0]
    if batch > s.shape[0]:
        raise G4Error(G4_E_ARG, "sign has %d entries, batch=%d" % (s.shape[0], batch))
    el = 16 if h.cfg.c.g_in == G4_IN_C128 else 8
    need = batch * h.ng * h.ng * el
    pu = _device_ptr(G_up, need, el)
    pd = _device_ptr(G_dn, need, el)
    _check(_L.g4_accumulate(h.ptr, _vp(pu), _vp(pd), s.ctypes.data_as(_dp), int(batch)))


def _acc_ptr(x, nbytes_expected: int) -> int:
    """Pointer of a caller-owned device accumulator (None for an absent channel)."""
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda or not x.is_contiguous():
        raise G4Error(G4_E_ARG, "accumulators must be contiguous device tensors")
    if x.numel() * x.element_size() < nbytes_expected:
        raise G4Error(G4_E_ARG, "accumulator holds %d bytes, %d needed"
                      % (x.numel() * x.element_size(), nbytes_expected))
    return x.data_ptr()


def g4_accumulate_into(cfg: Config, acc_mag, acc_chg, acc_pp, G_up, G_dn, sign,
                       batch: Optional[int] = None) -> None:
    """Allocation-free accumulation into caller-owned accumulators (device
    layout [plane][k2][k1][i2][i1]); see include/g4.h."""
    s = np.ascontiguousarray(np.asarray(sign, dtype=np.float64).reshape(-1))
    if batch is None:
        batch = s.shape[0]
    if batch > s.shape[0]:
        raise G4Error(G4_E_ARG, "sign has %d entries, batch=%d" % (s.shape[0], batch))
    el = 16 if cfg.c.g_in == G4_IN_C128 else 8
    need = batch * cfg.ng * cfg.ng * el
    pu = _device_ptr(G_up, need, el)
    pd = _device_ptr(G_dn, need, el)
    ab = cfg.planes * cfg.n * cfg.n * (8 if cfg.c.acc == G4_ACC_C64 else 16)
    accs = [_acc_ptr(a, ab) for a in (acc_mag, acc_chg, acc_pp)]
    _check(_L.g4_accumulate_into(ctypes.byref(cfg.c), *[_vp(a) if a else None for a in accs],
                                 _vp(pu), _vp(pd), s.ctypes.data_as(_dp), int(batch)))


def _dev_buf(x, nbytes: int, what: str, dtype=None) -> int:
    """Pointer of a contiguous device tensor of at least nbytes bytes (and of
    the given torch dtype, if one is named), or an integer device pointer."""
    if isinstance(x, int):
        return x
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda or not x.is_contiguous():
        raise G4Error(G4_E_ARG, "%s must be a contiguous device tensor" % what)
    if dtype is not None and x.dtype != dtype:
        raise G4Error(G4_E_ARG, "%s must be %s, got %s" % (what, dtype, x.dtype))
    if x.numel() * x.element_size() < nbytes:
        raise G4Error(G4_E_ARG, "%s holds %d bytes, %d needed" % (what, x.numel() * x.element_size(), nbytes))
    return x.data_ptr()


def g4_gsigma_workspace(lx: int, ly: int, nw: int, nwex: int, n: int, count: int, dtype: int) -> int:
    out = ctypes.c_uint64(0)
    _check(_L.g4_gsigma_workspace(lx, ly, nw, nwex, n, count, dtype, ctypes.byref(out)))
    return out.value


def g4_gsigma(lx: int, ly: int, nw: int, nwex: int, beta: float, mu: float, h: float, t: float, spin: int,
              tau, site, M, G, workspace, stream=None) -> None:
    """G_sigma of count configurations (tau: count x n float64, site: count x n
    int32, M: count x n x n complex) into G (count x Ng x Ng, M's dtype); see
    include/g4.h."""
    import torch
    if not isinstance(M, torch.Tensor) or M.dim() != 3 or M.shape[1] != M.shape[2]:
        raise G4Error(G4_E_ARG, "M must be a count x n x n device tensor")
    count, n = int(M.shape[0]), int(M.shape[1])
    dtype = {torch.complex128: G4_IN_C128, torch.complex64: G4_IN_C64}.get(M.dtype)
    if dtype is None:
        raise G4Error(G4_E_ARG, "M must be complex128 or complex64")
    el = 16 if dtype == G4_IN_C128 else 8
    ng = lx * ly * (nw + nwex - 1)
    pt = _dev_buf(tau, count * n * 8, "tau", torch.float64) if n else 0
    ps = _dev_buf(site, count * n * 4, "site", torch.int32) if n else 0
    pm = _dev_buf(M, count * n * n * el, "M")
    pg = _dev_buf(G, count * ng * ng * el, "G", M.dtype)
    need = g4_gsigma_workspace(lx, ly, nw, nwex, n, count, dtype)
    pw = _dev_buf(workspace, need, "workspace")
    wbytes = workspace.numel() * workspace.element_size() if not isinstance(workspace, int) else need
    _check(_L.g4_gsigma(lx, ly, nw, nwex, beta, mu, h, t, spin, n, count, _vp(pt), _vp(ps), _vp(pm), dtype,
                        _vp(pg), _vp(pw), wbytes, _vp(int(stream) if stream else 0)))


def g4_accumulate_mo(lx: int, ly: int, nw: int, nwex: int, nb: int, nq: int, q_list, q_begin: int, q_end: int,
                     channels: int, prod: int, G_up, G_dn, sign, acc_mag=None, acc_chg=None, acc_pp=None,
                     stream=None) -> None:
    """Multi-orbital accumulation into caller-owned complex128 accumulators
    (planes x (N nb^2)^2 each); see include/g4.h."""
    s = np.ascontiguousarray(np.asarray(sign, dtype=np.float64).reshape(-1))
    batch = s.shape[0]
    ngb = lx * ly * (nw + nwex - 1) * nb
    el = 16 if prod == G4_PROD_F64 else 8
    pu = _device_ptr(G_up, batch * ngb * ngb * el, el)
    pd = _device_ptr(G_dn, batch * ngb * ngb * el, el)
    side = lx * ly * nw * nb * nb
    ab = (q_end - q_begin) * side * side * 16
    accs = [_acc_ptr(a, ab) for a in (acc_mag, acc_chg, acc_pp)]
    ql = None
    if q_list is not None:
        qa = np.ascontiguousarray(np.asarray(q_list, dtype=np.int32))
        if qa.shape[0] != nq:
            raise G4Error(G4_E_ARG, "q_list has %d entries, nq=%d" % (qa.shape[0], nq))
        ql = qa.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    _check(_L.g4_accumulate_mo(lx, ly, nw, nwex, nb, nq, ql, q_begin, q_end, channels, prod, _vp(pu), _vp(pd),
                               s.ctypes.data_as(_dp), batch, *[_vp(a) if a else None for a in accs],
                               _vp(int(stream) if stream else 0)))


def g4_sync(h: Slice) -> None:
    _check(_L.g4_sync(h.ptr))


def g4_readback(h: Slice, channel: int, first: int = 0, count: Optional[int] = None) -> np.ndarray:
    if count is None:
        count = h.entries - first
    out = np.empty(count, dtype=np.complex128)
    _check(_L.g4_readback(h.ptr, channel, first, count, out.ctypes.data_as(_dp)))
    return out


def g4_load(h: Slice, channel: int, first: int, values) -> None:
    v = np.ascontiguousarray(np.asarray(values, dtype=np.complex128).reshape(-1))
    _check(_L.g4_load(h.ptr, channel, first, v.shape[0], v.ctypes.data_as(_dp)))


def g4_set_counts(h: Slice, measurements: int, sign_sum: float) -> None:
    _check(_L.g4_set_counts(h.ptr, measurements, sign_sum))


def g4_merge(dst: Slice, src: Slice) -> None:
    _check(_L.g4_merge(dst.ptr, src.ptr))


def g4_reset(h: Slice) -> None:
    _check(_L.g4_reset(h.ptr))


def g4_stats(h: Slice) -> dict:
    st = g4_stats_t()
    _check(_L.g4_stats(h.ptr, ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in g4_stats_t._fields_}


def g4_set_plan(h: Slice, tile: int = 0, batch: int = 0, variant: int = -1) -> None:
    _check(_L.g4_set_plan(h.ptr, tile, batch, variant))


def g4_autotune(h: Slice, G_up, G_dn, sign, batch: Optional[int] = None, tol: float = 1e-6) -> dict:
    s = np.ascontiguousarray(np.asarray(sign, dtype=np.float64).reshape(-1))
    if batch is None:
        batch = s.shape[0]
    if batch > s.shape[0]:
        raise G4Error(G4_E_ARG, "sign has %d entries, batch=%d" % (s.shape[0], batch))
    el = 16 if h.cfg.c.g_in == G4_IN_C128 else 8
    need = batch * h.ng * h.ng * el
    pu = _device_ptr(G_up, need, el)
    pd = _device_ptr(G_dn, need, el)
    r = g4_tune_result()
    _check(_L.g4_autotune(h.ptr, _vp(pu), _vp(pd), s.ctypes.data_as(_dp), int(batch), tol,
                          ctypes.byref(r)))
    return {f: getattr(r, f) for f, _ in g4_tune_result._fields_}


def g4_destroy(h: Slice) -> None:
    if h is not None and h.ptr:
        _L.g4_destroy(h.ptr)
        h.ptr = None


def g4_synth_fill(out, dtype: int, lx: int, ly: int, nw: int, nwex: int, beta: float, t: float,
                  mu: float, h: float, noise: float, seed: int, wid: int, b0: int, count: int,
                  spin: int, stream=None) -> None:
    ng = lx * ly * (nw + nwex - 1)
    el = 16 if dtype == G4_IN_C128 else 8
    p = _device_ptr(out, count * ng * ng * el, el)
    _check(_L.g4_synth_fill(_vp(p), dtype, lx, ly, nw, nwex, beta, t, mu, h, noise, seed, wid,
                            b0, count, spin, _vp(int(stream) if stream else 0)))


def g4_index_maps(cfg: Config):
    nc = cfg.nc
    ka = np.zeros(nc * nc, dtype=np.int32)
    ks = np.zeros(nc * nc, dtype=np.int32)
    pq = np.zeros(cfg.planes, dtype=np.int32)
    pm = np.zeros(cfg.planes, dtype=np.int32)
    ip = ctypes.POINTER(ctypes.c_int32)
    _check(_L.g4_index_maps(ctypes.byref(cfg.c), ka.ctypes.data_as(ip), ks.ctypes.data_as(ip),
                            pq.ctypes.data_as(ip), pm.ctypes.data_as(ip)))
    return ka, ks, pq, pm
