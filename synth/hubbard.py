"""Seeded synthetic single-particle Green's functions shaped like a 2D Hubbard
cluster measurement, and the workload shapes they are drawn for.

Recipe (stands in for the QMC walker output G_sigma that the paper's ring
circulates; the paper's own 6x6 Hubbard runs are not available):

    G_sigma,b(r, c) = delta_rc * g0_sigma(r) + noise * (x + i y),   x, y ~ N(0,1) iid
    g0_sigma(k, n)  = 1 / (i w_n + mu + sigma*h - eps_k),  w_n = (2n+1) pi / beta
    eps_k           = -2 t (cos kx + cos ky),  (kx, ky) = 2 pi (ix/Lx, iy/Ly),  k = ix + Lx*iy

over the G frequency window n in [-Nw/2, Nw/2 + Nwex - 2] (Nwg = Nw + Nwex - 1
values, local index n + Nw/2), combined row/column index r = k*Nwg + (n + Nw/2).
The two spins draw independent noise; the per-measurement sign is +1 with
probability 0.95, else -1.

Random numbers: Philox4x32-10 with key (seed, workload id) and counter
(element r*Ng + c, measurement b, stream, 0), stream 0 = spin up,
1 = spin down, 2 = sign.  Each call yields two 53-bit uniforms, turned into
one complex normal by Box-Muller.

This module holds input synthesis only: nothing of the G4 accumulation.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

from .philox import box_muller, philox4x32_10, u53

PH_MAGNETIC = 1
PH_CHARGE = 2
PP_UPDOWN = 4

STREAM_UP = 0
STREAM_DN = 1
STREAM_SIGN = 2


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shapes and input recipe of one workload.  Sizes follow the notation
    Nc = lx*ly, Nwg = nw + nwex - 1, Ng = Nc*Nwg, N = Nc*nw, NQ = nq*nwex."""
    name: str
    lx: int
    ly: int
    nw: int
    nwex: int
    nq: int
    q_list: Optional[Sequence[int]] = None  # None -> 0..nq-1
    q_begin: int = 0
    q_end: int = -1                         # -1 -> nq*nwex
    channels: int = PH_MAGNETIC
    beta: float = 10.0
    t: float = 1.0
    mu: float = 0.0
    h: float = 0.0                           # Zeeman shift (0 = paramagnetic)
    noise: float = 0.1
    seed: int = 1
    wid: int = 1                             # workload id, second Philox key word
    measurements: int = 64
    batch: int = 1
    p_plus: float = 0.95

    @property
    def nc(self) -> int:
        return self.lx * self.ly

    @property
    def nwg(self) -> int:
        return self.nw + self.nwex - 1

    @property
    def ng(self) -> int:
        return self.nc * self.nwg

    @property
    def n(self) -> int:
        return self.nc * self.nw

    @property
    def nQ(self) -> int:
        return self.nq * self.nwex

    @property
    def q0(self) -> int:
        return self.q_begin

    @property
    def q1(self) -> int:
        return self.nQ if self.q_end < 0 else self.q_end

    @property
    def planes(self) -> int:
        return self.q1 - self.q0

    @property
    def entries(self) -> int:
        """Entries of one channel of this GPU's slice."""
        return self.planes * self.n * self.n

    @property
    def qs(self) -> list:
        return list(range(self.nq)) if self.q_list is None else list(self.q_list)

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# The workloads of the build (sizes from the paper's 2D Hubbard setting).
C1_TINY = Workload("tiny 2x2 Nw16 Nq1 Nwex1 PH-magnetic, 64 measurements",
                   lx=2, ly=2, nw=16, nwex=1, nq=1, beta=5.0, seed=1, wid=1,
                   measurements=64, channels=PH_MAGNETIC)
C2_PLAIN = Workload("4x4 Nw64 Nq16 Nwex8 PH-magnetic c128 slice, 512 measurements one per launch",
                    lx=4, ly=4, nw=64, nwex=8, nq=16, beta=10.0, seed=2, wid=2,
                    measurements=512, channels=PH_MAGNETIC)
C3_BATCHED = Workload("4x4 Nw64 Nq16 Nwex8 PH-magnetic slice, 4096 measurements batched",
                      lx=4, ly=4, nw=64, nwex=8, nq=16, beta=10.0, seed=3, wid=3,
                      measurements=4096, batch=16, channels=PH_MAGNETIC)
C4_RING = Workload("6x6 Nw128 Nq36 Nwex16 1/8 slice, 8 walkers x 16 measurements",
                   lx=6, ly=6, nw=128, nwex=16, nq=36, beta=10.0, seed=4, wid=4,
                   q_begin=0, q_end=72, measurements=128, batch=16,
                   channels=PH_MAGNETIC)
C5_SPLIT = Workload("8x8 Nw64 Nq64 Nwex4 1/4 slice, 3 channels, 256 measurements",
                    lx=8, ly=8, nw=64, nwex=4, nq=64, beta=10.0, seed=5, wid=5,
                    q_begin=0, q_end=64, measurements=256, batch=32,
                    channels=PH_MAGNETIC | PH_CHARGE | PP_UPDOWN)

WORKLOADS = {"c1": C1_TINY, "c2": C2_PLAIN, "c3": C3_BATCHED, "c4": C4_RING, "c5": C5_SPLIT}


def g0_diag(w: Workload, spin: int) -> np.ndarray:
    """Diagonal g0_sigma over the G window, length Ng, spin 0 = up, 1 = down."""
    sig = 1.0 if spin == 0 else -1.0
    k = np.arange(w.nc)
    ix = k % w.lx
    iy = k // w.lx
    eps = -2.0 * w.t * (np.cos(2.0 * math.pi * ix / w.lx) + np.cos(2.0 * math.pi * iy / w.ly))
    n = np.arange(w.nwg) - w.nw // 2
    wn = (2.0 * n + 1.0) * math.pi / w.beta
    z = 1j * wn[None, :] + (w.mu + sig * w.h) - eps[:, None]
    return (1.0 / z).reshape(-1)


def noise_elements(w: Workload, b, stream: int, r, c) -> np.ndarray:
    """Noise term of G at (measurement b, stream, row r, col c); arrays broadcast."""
    b = np.asarray(b, dtype=np.int64)
    r = np.asarray(r, dtype=np.int64)
    c = np.asarray(c, dtype=np.int64)
    e = (r * w.ng + c).astype(np.uint64)
    b, e = np.broadcast_arrays(b, e)
    x0, x1, x2, x3 = philox4x32_10(e.astype(np.uint32), b.astype(np.uint32),
                                   np.uint32(stream), np.uint32(0),
                                   np.uint32(w.seed), np.uint32(w.wid))
    x, y = box_muller(u53(x0, x1), u53(x2, x3))
    return w.noise * (x + 1j * y)


def g_elements(w: Workload, b, spin: int, r, c) -> np.ndarray:
    """Elements G_spin,b(r, c) (complex128), regenerated from their counters."""
    r = np.asarray(r, dtype=np.int64)
    c = np.asarray(c, dtype=np.int64)
    val = noise_elements(w, b, STREAM_UP if spin == 0 else STREAM_DN, r, c)
    d = g0_diag(w, spin)
    diag = np.broadcast_to(r == c, val.shape)
    rr = np.broadcast_to(r, val.shape)
    val = val.copy()
    val[diag] += d[rr[diag]]
    return val


def g_matrices(w: Workload, b0: int, count: int, spin: int) -> np.ndarray:
    """Full G_spin for measurements b0..b0+count-1: complex128 [count, Ng, Ng]."""
    ng = w.ng
    out = np.empty((count, ng, ng), dtype=np.complex128)
    r = np.arange(ng)[:, None]
    c = np.arange(ng)[None, :]
    d = g0_diag(w, spin)
    for j in range(count):
        out[j] = noise_elements(w, b0 + j, STREAM_UP if spin == 0 else STREAM_DN, r, c)
        out[j][np.arange(ng), np.arange(ng)] += d
    return out


def signs(w: Workload, b0: int, count: int) -> np.ndarray:
    """Per-measurement weights: +1 with probability p_plus, else -1."""
    b = np.arange(b0, b0 + count, dtype=np.uint32)
    x0, x1, _, _ = philox4x32_10(np.uint32(0), b, np.uint32(STREAM_SIGN), np.uint32(0),
                                 np.uint32(w.seed), np.uint32(w.wid))
    return np.where(u53(x0, x1) < w.p_plus, 1.0, -1.0)


def expansion_configs(w: Workload, seed: int, count: int, n: int):
    """Seeded stand-ins for walker expansion configurations: for each of count
    measurements, n vertex times uniform in [0, beta), n cluster sites uniform
    over the Nc sites, and an n x n complex matrix with independent normal
    real and imaginary parts scaled by 1/sqrt(n) (so that M E^H stays O(1)
    per entry as n grows).  Returns (tau[count, n] float64, site[count, n]
    int32, M[count, n, n] complex128)."""
    rng = np.random.default_rng(seed)
    tau = rng.uniform(0.0, w.beta, size=(count, n))
    site = rng.integers(0, w.nc, size=(count, n)).astype(np.int32)
    sc = 1.0 / math.sqrt(max(n, 1))
    M = (rng.normal(size=(count, n, n)) + 1j * rng.normal(size=(count, n, n))) * sc
    return tau, site, M
