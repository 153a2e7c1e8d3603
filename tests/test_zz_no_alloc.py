"""The allocation-free entry point g4_accumulate_into against g4_accumulate.

Both run the same kernels on the same inputs; g4_accumulate_into keeps its
workspace in the library's static device array and writes caller-owned
accumulators in the device layout [plane][k2][k1][i2][i1].  Two calls in a
row (the second on a smaller slice with fewer measurements, so that the
workspace holds the first call's leftovers) must each equal the slice
handle's result bit for bit, and the FP64 oracle within the path's bar."""
import numpy as np
import pytest

from gpu_common import config_for, g4mod, host_inputs, run_slice, to_dev
from metrics import check_entries
from oracle import ref
from synth import PH_CHARGE, PH_MAGNETIC, PP_UPDOWN, Workload

pytestmark = pytest.mark.gpu

ALL = PH_MAGNETIC | PH_CHARGE | PP_UPDOWN
BIG = Workload("noalloc-a", lx=3, ly=2, nw=24, nwex=5, nq=6, q_list=(4, 0, 5, 1, 3, 2),
               q_begin=3, q_end=27, beta=7.0, seed=41, wid=41, channels=ALL)
SMALL = BIG.with_(name="noalloc-b", q_begin=9, q_end=14, seed=42, wid=42)


def from_device_layout(buf, w, kind):
    """Caller accumulator (device layout) -> documented [plane][K2][K1] complex128."""
    a = buf.cpu().numpy()
    if kind == 0:
        v = a.view(np.complex128)
    elif kind == 1:
        f = a.view(np.float32).reshape(-1, 4).astype(np.float64)
        v = (f[:, 0] - f[:, 2]) + 1j * (f[:, 1] - f[:, 3])
    else:
        v = a.view(np.complex64).astype(np.complex128)
    v = v.reshape(w.planes, w.nc, w.nc, w.nw, w.nw)          # plane, k2, k1, i2, i1
    return v.transpose(0, 1, 3, 2, 4).reshape(w.planes, w.n, w.n)


def run_into(cfg, w, gu, gd, s, kind):
    import torch
    g4 = g4mod()
    eb = 8 if kind == 2 else 16
    accs = [torch.zeros(w.entries * eb, dtype=torch.uint8, device="cuda") if cfg.c.channels & ch else None
            for ch in (1, 2, 4)]
    g4.g4_accumulate_into(cfg, *accs, gu, gd, s)
    return {ch: from_device_layout(accs[i], w, kind) for i, ch in enumerate((1, 2, 4)) if accs[i] is not None}


@pytest.mark.parametrize("kw,bar", [(dict(mode=0), 1e-12),
                                    (dict(mode=1, prod=1, g_in=1, acc=1, batch=3), 1e-6),
                                    (dict(mode=1, prod=1, g_in=1, acc=0, batch=2), 1e-6),
                                    (dict(mode=1, prod=0, g_in=0, acc=0, batch=4), 1e-12)],
                         ids=["plain-fp64", "batched-fp32-kahan", "batched-fp32-c128", "batched-fp64"])
def test_accumulate_into_matches_slice_handle(kw, bar):
    for w, count in ((BIG, 5), (SMALL, 2)):
        g_in = kw.get("g_in", 0)
        gu, gd, s = host_inputs(w, count)
        du, dd = to_dev(gu, g_in), to_dev(gd, g_in)
        cfg = config_for(w, **kw)
        want, _ = run_slice(cfg, du, dd, s)
        got = run_into(cfg, w, du, dd, s, kw.get("acc", 0))
        for ch in want:
            assert np.array_equal(got[ch], want[ch]), (w.name, ch)
            exp = ref.accumulate(w, ch, gu, gd, s)
            check_entries(got[ch], exp, bar, what="%s channel %d" % (w.name, ch))


def test_accumulate_into_rejects_what_it_cannot_hold():
    import torch
    g4 = g4mod()
    # the 4x4 slice with 64 measurements per pass: 134 MB of direct vectors
    w = Workload("too-big", lx=4, ly=4, nw=64, nwex=8, nq=16, channels=PH_MAGNETIC)
    cfg = config_for(w, mode=1, prod=1, g_in=1, batch=64)
    g = torch.zeros((1, w.ng, w.ng), dtype=torch.complex64, device="cuda")
    acc = torch.zeros(w.entries * 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(g4.G4Error) as e:
        g4.g4_accumulate_into(cfg, acc, None, None, g, g, [1.0])
    assert e.value.code == g4.G4_E_UNSUPPORTED and "workspace" in str(e.value)
    del acc
    small = config_for(SMALL, mode=1, prod=1, g_in=1, batch=2, flags=g4.G4_F_PACKED)
    with pytest.raises(g4.G4Error) as e:
        g4.g4_accumulate_into(small, None, None, None, g, g, [1.0])
    assert e.value.code == g4.G4_E_UNSUPPORTED
