"""Per-entry FP64 oracle that regenerates the G elements it needs.

Test infrastructure only.  For slices too large to hold every measurement's G
on the host, each sampled entry (Q, K2, K1) is evaluated as the plain
definition

    sum_b s_b T_ch(K1, K2, Q)

(PH magnetic/charge: direct minus exchange Wick terms; the spin-resolved PH
channels: longitudinal up-up, longitudinal up-down, transverse; PP: the
paper's Eq. (1) with K3 -> Q, and its singlet and triplet projections), the G elements being regenerated one by one from their
Philox counters by the seeded input generator (a chunk of measurements at a
time).  Index arithmetic is done on cluster coordinates and integer Matsubara
labels, as in the C oracle: momenta add coordinate-wise modulo the cluster,
w_n + nu_m = w_{n+m}, nu_m - w_n = w_{m-n-1}.  Measurements are summed in
order.
"""
from __future__ import annotations

import numpy as np

from synth.hubbard import Workload, g_elements, signs

PH_MAGNETIC = 1
PH_CHARGE = 2
PP_UPDOWN = 4
PH_LONG_UPUP = 8
PH_LONG_UPDOWN = 16
PH_TRANSVERSE = 32
PP_SINGLET = 64
PP_TRIPLET = 128


def _mom_add(w: Workload, k, q):
    ix, iy = k % w.lx, k // w.lx
    jx, jy = q % w.lx, q // w.lx
    return (ix + jx) % w.lx + w.lx * ((iy + jy) % w.ly)


def _mom_sub(w: Workload, q, k):
    ix, iy = k % w.lx, k // w.lx
    jx, jy = q % w.lx, q // w.lx
    return (jx - ix) % w.lx + w.lx * ((jy - iy) % w.ly)


def _g_index(w: Workload, k, n):
    loc = n + w.nw // 2
    if np.any(loc < 0) or np.any(loc >= w.nwg):
        raise AssertionError("frequency outside the G window")
    return k * w.nwg + loc


def decode(w: Workload, idx):
    """Flattened slice entry -> (iQ, K2, K1)."""
    idx = np.asarray(idx, dtype=np.int64)
    n = w.n
    return w.q0 + idx // (n * n), (idx // n) % n, idx % n


def entries(w: Workload, channel: int, idx, b0: int = 0, count: int = None,
            sign=None) -> np.ndarray:
    """sum over measurements b0..b0+count-1 of s_b T_channel at entries idx."""
    if count is None:
        count = w.measurements
    if sign is None:
        sign = signs(w, b0, count)
    iQ, K2, K1 = decode(w, idx)
    qs = np.asarray(w.qs, dtype=np.int64)
    iq, m = iQ // w.nwex, iQ % w.nwex
    q = qs[iq]
    k1, n1 = K1 // w.nw, K1 % w.nw - w.nw // 2
    k2, n2 = K2 // w.nw, K2 % w.nw - w.nw // 2
    r_k1 = _g_index(w, k1, n1)
    r_k2 = _g_index(w, k2, n2)
    out = np.zeros(len(iQ), dtype=np.complex128)
    if channel in (PH_MAGNETIC, PH_CHARGE, PH_LONG_UPUP, PH_LONG_UPDOWN, PH_TRANSVERSE):
        r_k1q = _g_index(w, _mom_add(w, k1, q), n1 + m)
        r_k2q = _g_index(w, _mom_add(w, k2, q), n2 + m)
    elif channel in (PP_UPDOWN, PP_SINGLET, PP_TRIPLET):
        r_qk1 = _g_index(w, _mom_sub(w, q, k1), m - n1 - 1)
        r_qk2 = _g_index(w, _mom_sub(w, q, k2), m - n2 - 1)
    else:
        raise ValueError("unknown channel")

    def terms(b):
        """T_channel of measurements b (column) at every sampled entry (row
        vectors of indices): one row per measurement."""
        G = lambda spin, r, c: g_elements(w, b, spin, r[None, :], c[None, :])
        if channel in (PH_MAGNETIC, PH_CHARGE):
            pm = -1.0 if channel == PH_MAGNETIC else 1.0
            u1, d1 = G(0, r_k1q, r_k1), G(1, r_k1q, r_k1)
            u2, d2 = G(0, r_k2, r_k2q), G(1, r_k2, r_k2q)
            direct = (u1 + pm * d1) * (u2 + pm * d2)
            ex = G(0, r_k2, r_k1) * G(0, r_k1q, r_k2q) + G(1, r_k2, r_k1) * G(1, r_k1q, r_k2q)
            return direct - ex
        if channel == PH_LONG_UPUP:
            return G(0, r_k1q, r_k1) * G(0, r_k2, r_k2q) - G(0, r_k2, r_k1) * G(0, r_k1q, r_k2q)
        if channel == PH_LONG_UPDOWN:
            return G(0, r_k1q, r_k1) * G(1, r_k2, r_k2q)
        if channel == PH_TRANSVERSE:
            return -(G(1, r_k2, r_k1) * G(0, r_k1q, r_k2q) + G(0, r_k2, r_k1) * G(1, r_k1q, r_k2q))
        same = G(0, r_qk2, r_qk1) * G(1, r_k2, r_k1) + G(1, r_qk2, r_qk1) * G(0, r_k2, r_k1)
        if channel == PP_UPDOWN:
            return same
        pm = 1.0 if channel == PP_SINGLET else -1.0
        crossed = G(0, r_qk2, r_k1) * G(1, r_k2, r_qk1) + G(1, r_qk2, r_k1) * G(0, r_k2, r_qk1)
        return 0.5 * (same + pm * crossed)

    # measurements regenerated in chunks (vectorised), summed one by one in order
    chunk = max(1, min(count, (1 << 20) // max(1, len(iQ))))
    for j0 in range(0, count, chunk):
        nb = min(chunk, count - j0)
        t = terms(np.arange(b0 + j0, b0 + j0 + nb, dtype=np.int64)[:, None])
        for j in range(nb):
            out += sign[j0 + j] * t[j]
    return out


def sample_indices(w: Workload, count: int, seed: int = 12345) -> np.ndarray:
    """Seeded sample of flattened slice entries, always including the first and
    last entry of the slice and the edges of the first and last plane."""
    rng = np.random.default_rng(seed)
    e = w.entries
    fixed = np.array([0, w.n - 1, w.n * (w.n - 1), w.n * w.n - 1, e - 1, e - w.n, e - w.n * w.n],
                     dtype=np.int64)
    fixed = fixed[(fixed >= 0) & (fixed < e)]
    rnd = rng.integers(0, e, size=max(0, count - len(fixed)), dtype=np.int64)
    return np.unique(np.concatenate([fixed, rnd]))
