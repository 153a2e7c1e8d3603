"""Parity of the multi-orbital G4 path (g4_accumulate_mo through the C ABI)
with the FP64 oracle.

Bars: FP64 products 1e-12, FP32 products 1e-6 (relative Frobenius, Eq. (2)/(3)
on real and imaginary parts, and the small half of the entries), per channel.
Shapes: one to nine orbitals (four: rows of 384 columns, a full and a partial
block each; six: rows of 864 columns; nine: the one-thread-per-entry
kernel), a transfer list in a
different order, a slice cut through a transfer momentum, entry counts that
are not multiples of the 256-thread block; 70 measurements (three launches of
at most 32).  Argument
errors are rejected before any launch.
"""
import numpy as np
import pytest

from gpu_common import g4mod
from metrics import check_entries
from oracle import ref
from synth import Workload

pytestmark = pytest.mark.gpu

W2 = Workload("mo-3x1", lx=3, ly=1, nw=4, nwex=3, nq=3, q_list=(2, 0, 1), q_begin=1, q_end=8, beta=6.0)
W3 = Workload("mo-2x2", lx=2, ly=2, nw=6, nwex=2, nq=4, q_begin=0, q_end=5, beta=5.0)


def inputs(w, nb, count, seed):
    rng = np.random.default_rng(seed)
    ngb = w.ng * nb
    g = lambda: (rng.normal(size=(count, ngb, ngb)) + 1j * rng.normal(size=(count, ngb, ngb))) * 0.3
    s = np.where(rng.random(count) < 0.9, 1.0, -1.0)
    return g(), g(), s


def run(w, nb, channels, prod, gu, gd, s):
    import torch
    g4 = g4mod()
    dt = torch.complex128 if prod == 0 else torch.complex64
    du = torch.from_numpy(gu).to(device="cuda", dtype=dt)
    dd = torch.from_numpy(gd).to(device="cuda", dtype=dt)
    side = w.n * nb * nb
    accs = [torch.zeros((w.planes, side, side), dtype=torch.complex128, device="cuda") if channels & (1 << c)
            else None for c in range(3)]
    g4.g4_accumulate_mo(w.lx, w.ly, w.nw, w.nwex, nb, w.nq, w.q_list, w.q0, w.q1, channels, prod, du, dd, s, *accs)
    torch.cuda.synchronize()
    return {1 << c: a.cpu().numpy() for c, a in enumerate(accs) if a is not None}


@pytest.mark.parametrize("prod", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("w,nb,count", [(W2, 2, 5), (W3, 3, 3), (W2, 1, 70), (W3, 4, 3), (W2, 5, 2), (W3, 6, 2),
                                         (W2, 7, 2), (W2, 8, 2), (W2, 9, 1)],
                         ids=["3x1-nb2", "2x2-nb3", "3x1-nb1-70meas", "2x2-nb4", "3x1-nb5", "2x2-nb6",
                              "3x1-nb7", "3x1-nb8", "3x1-nb9-entry-kernel"])
def test_matches_oracle(w, nb, count, prod):
    print("\ncase %s nb=%d count=%d prod=%d" % (w.name, nb, count, prod), flush=True)
    gu, gd, s = inputs(w, nb, count, 10 * nb + count)
    if prod == 1:
        gu = gu.astype(np.complex64).astype(np.complex128)
        gd = gd.astype(np.complex64).astype(np.complex128)
    got = run(w, nb, 7, prod, gu, gd, s)
    tol = 1e-12 if prod == 0 else 1e-6
    for ch in (1, 2, 4):
        want = ref.accumulate_mo(w, nb, ch, gu, gd, s)
        check_entries(got[ch], want, tol, what="channel %d" % ch)


def test_channel_subset_and_accumulation():
    """One channel, two calls: the second adds to the first."""
    w, nb = W3, 2
    gu, gd, s = inputs(w, nb, 4, 3)
    import torch
    g4 = g4mod()
    du = torch.from_numpy(gu).cuda()
    dd = torch.from_numpy(gd).cuda()
    side = w.n * nb * nb
    acc = torch.zeros((w.planes, side, side), dtype=torch.complex128, device="cuda")
    g4.g4_accumulate_mo(w.lx, w.ly, w.nw, w.nwex, nb, w.nq, None, w.q0, w.q1, 4, 0, du[:2], dd[:2], s[:2],
                        None, None, acc)
    g4.g4_accumulate_mo(w.lx, w.ly, w.nw, w.nwex, nb, w.nq, None, w.q0, w.q1, 4, 0, du[2:], dd[2:], s[2:],
                        None, None, acc)
    torch.cuda.synchronize()
    check_entries(acc.cpu().numpy(), ref.accumulate_mo(w, nb, 4, gu, gd, s), 1e-12)


def test_argument_errors():
    import torch
    g4 = g4mod()
    w, nb = W2, 2
    gu, gd, s = inputs(w, nb, 1, 1)
    du = torch.from_numpy(gu).cuda()
    dd = torch.from_numpy(gd).cuda()
    side = w.n * nb * nb
    acc = torch.zeros((w.planes, side, side), dtype=torch.complex128, device="cuda")
    bad = [dict(channels=8), dict(channels=3), dict(prod=2), dict(nb=0), dict(q_end=100)]
    for kw in bad:
        a = dict(channels=1, prod=0, nb=nb, q_end=w.q1)
        a.update(kw)
        with pytest.raises(g4.G4Error) as e:
            g4.g4_accumulate_mo(w.lx, w.ly, w.nw, w.nwex, a["nb"], w.nq, w.q_list, w.q0, a["q_end"], a["channels"],
                                a["prod"], du, dd, s, acc if a["nb"] == nb else 0)
        assert e.value.code == g4.G4_E_ARG, kw
    torch.cuda.synchronize()
    assert float(acc.abs().max()) == 0.0
