"""The C-ABI library on the CPU: it loads, exports every declared entry point,
validates configurations before any HIP call, and its integer index maps equal
the oracle's coordinate arithmetic bit for bit."""
import os
import re

import numpy as np
import pytest

from oracle import sampled
from synth import Workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
g4 = pytest.importorskip("paper_2105_00027_amd.g4", reason="libg4.so not built")


def declared_functions():
    with open(os.path.join(ROOT, "include", "g4.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(g4_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(g4._L, n), n
    assert set(names) == set(g4.EXPORTS)


def test_every_declaration_names_its_passage():
    """Each entry point's comment names the passage of the paper it implements
    (a section, an equation or an algorithm), or says that none exists; the
    allocation-free variant names the callers it is for instead."""
    with open(os.path.join(ROOT, "include", "g4.h")) as f:
        text = f.read()
    for name in declared_functions():
        m = re.search(r"/\*((?:(?!\*/).)*)\*/\s*(?:int|void|const char \*)\s*\*?\s*%s\s*\(" % name,
                      text, re.S)
        assert m, "%s has no comment block right before it" % name
        comment = m.group(1)
        if "callers that cannot allocate" in comment:
            continue                      # the allocation-free variant names its callers instead
        assert "Paper:" in comment, "%s: no 'Paper:' line" % name
        cite = comment[comment.index("Paper:"):]
        assert re.search(r"section|Eq\. \(\d\)|Algorithm \d|no passage", cite), (name, cite)


def base(**kw):
    d = dict(lx=4, ly=4, nw=64, nwex=8, nq=16, q_begin=0, q_end=128)
    d.update(kw)
    return g4.Config(**d)


BAD = [
    dict(abi_version=7), dict(lx=0), dict(nw=63), dict(nw=0), dict(nwex=0), dict(nq=17),
    dict(q_list=[0, 1, 1] + list(range(3, 16))), dict(q_list=[0] * 15 + [16]),
    dict(q_begin=5, q_end=5), dict(q_end=129), dict(q_begin=-1), dict(channels=0),
    dict(channels=256), dict(channels=9), dict(channels=7 | 56), dict(channels=4 | 64), dict(channels=32 | 128),
    dict(g_in=2), dict(prod=9), dict(acc=3), dict(mode=2), dict(flags=1 << 9), dict(flags=128),
    dict(device=-1), dict(mode=1, max_batch=0), dict(mode=1, max_batch=257),
    dict(mode=0, prod=1), dict(mode=0, acc=1), dict(mode=1, max_batch=8, prod=0, g_in=1),
    dict(tile=-1),
]


def test_mfma_plan_accepted_where_it_fits():
    c = base(mode=1, max_batch=16, prod=1, g_in=1, flags=8)
    assert g4.g4_slice_size(c)[0] == 128 * 1024 * 1024


@pytest.mark.parametrize("kw", BAD, ids=lambda k: ",".join("%s=%s" % i for i in k.items())[:40])
def test_invalid_configs_rejected_without_hip(kw):
    c = base(**kw)
    with pytest.raises(g4.G4Error) as e:
        g4.g4_slice_size(c)
    assert e.value.code == g4.G4_E_ARG
    with pytest.raises(g4.G4Error) as e:
        g4.g4_init_slice(c)
    assert e.value.code == g4.G4_E_ARG
    assert g4.g4_last_error()


def test_split_precision_plans_accepted():
    for prod in (2, 3):
        for flags in (0, g4.G4_F_PACKED):
            assert g4.g4_slice_size(base(mode=1, max_batch=8, prod=prod, g_in=1, flags=flags))[0] > 0
    with pytest.raises(g4.G4Error) as e:                       # plain mode is FP64 throughout
        g4.g4_slice_size(base(mode=0, prod=2))
    assert e.value.code == g4.G4_E_ARG


def test_packed_plan_accepted_and_sized():
    plain = base(mode=1, max_batch=16, prod=1, g_in=1)
    packed = base(mode=1, max_batch=16, prod=1, g_in=1, flags=g4.G4_F_PACKED)
    e0, b0 = g4.g4_slice_size(plain)
    e1, b1 = g4.g4_slice_size(packed)
    ng = 16 * (64 + 8 - 1)
    pcb = (64 + 8 - 1 + 7) // 8 * 8                     # momentum blocks of columns on 128 bytes
    ldp = (16 * pcb + 1 + 7) // 8 * 8
    per = ng * ldp * 16 + 2 * 128 * 1024 * 8          # G rows + direct vectors a, b
    assert e0 == e1 and b1 - b0 == 16 * ((per + 255) // 256 * 256)


def test_packed_rejections():
    P = g4.G4_F_PACKED
    for flags in (P | g4.G4_F_PACKED_DEEP, g4.G4_F_MFMA | g4.G4_F_PACKED_DEEP,
                  P | g4.G4_F_MFMA | g4.G4_F_PACKED_DEEP):      # exclusive variants
        with pytest.raises(g4.G4Error) as e:
            g4.g4_slice_size(base(mode=1, max_batch=8, prod=1, g_in=1, flags=flags))
        assert e.value.code == g4.G4_E_ARG
    D = g4.G4_F_PACKED_DEEP
    with pytest.raises(g4.G4Error) as e:                       # deep blocks: at most 2 rows/thread
        g4.g4_slice_size(base(mode=1, max_batch=8, prod=1, g_in=1, flags=D, tile=32))
    assert e.value.code == g4.G4_E_UNSUPPORTED
    assert g4.g4_slice_size(base(mode=1, max_batch=8, prod=1, g_in=1, flags=D, tile=16))[0] > 0
    for kw in (dict(mode=0, flags=P),                          # plain FP64
               dict(mode=1, max_batch=8, prod=0, g_in=0, flags=P),   # batched FP64
               dict(nw=130, mode=1, max_batch=8, prod=1, g_in=1, flags=P, tile=1)):   # odd tile
        with pytest.raises(g4.G4Error) as e:
            g4.g4_slice_size(base(**kw))
        assert e.value.code == g4.G4_E_UNSUPPORTED, kw


def test_channel_families_on_valu_plans_only():
    """The spin-resolved family sizes like the standard one (one accumulator
    per channel, direct vectors for up-up and up-down only), the PP singlet /
    triplet family like PP up-down; both run on the VALU kernels: packed,
    MFMA and split plans are G4_E_UNSUPPORTED."""
    for ch in (8, 16, 32, 24, 40, 48, 56):
        for kw in (dict(mode=0), dict(mode=1, max_batch=8, prod=0), dict(mode=1, max_batch=8, prod=1, g_in=1)):
            e, b = g4.g4_slice_size(base(channels=ch, **kw))
            std = {8: 1, 16: 2, 32: 4, 24: 3, 40: 5, 48: 6, 56: 7}[ch]
            e0, b0 = g4.g4_slice_size(base(channels=std, **kw))
            assert e == e0 and b == b0, (ch, kw)       # same accumulators, same direct-vector slots
    for ch in (8, 64):
        for kw in (dict(flags=g4.G4_F_PACKED), dict(flags=g4.G4_F_MFMA), dict(flags=g4.G4_F_PACKED_DEEP),
                   dict(flags=g4.G4_F_PACKED | g4.G4_F_MFMA), dict(prod=2), dict(prod=3)):
            with pytest.raises(g4.G4Error) as e:
                g4.g4_slice_size(base(channels=ch, mode=1, max_batch=8, **dict(dict(prod=1, g_in=1), **kw)))
            assert e.value.code == g4.G4_E_UNSUPPORTED, (ch, kw)
    # PP singlet / triplet: one accumulator each, no direct vectors (as PP up-down)
    for kw in (dict(mode=0), dict(mode=1, max_batch=8, prod=1, g_in=1)):
        e4, b4 = g4.g4_slice_size(base(channels=4, **kw))
        for ch in (64, 128):
            assert g4.g4_slice_size(base(channels=ch, **kw)) == (e4, b4)
        e, b = g4.g4_slice_size(base(channels=192, **kw))
        assert b - b4 == e4 * 16


def test_unsupported_is_distinguished():
    mfma = 8
    for kw in (dict(nw=512), dict(mode=1, max_batch=8, prod=2, g_in=1, flags=8), dict(tile=3),
               dict(flags=mfma),                                    # plain mode
               dict(mode=1, max_batch=8, prod=1, g_in=1, flags=mfma, nw=24),
               dict(mode=1, max_batch=8, prod=1, g_in=1, flags=mfma, channels=7),
               dict(mode=1, max_batch=8, prod=1, g_in=1, flags=mfma, tile=8)):
        with pytest.raises(g4.G4Error) as e:
            g4.g4_slice_size(base(**kw))
        assert e.value.code == g4.G4_E_UNSUPPORTED


def test_oom_cap_before_any_allocation(monkeypatch):
    c = base()
    entries, nbytes = g4.g4_slice_size(c)
    assert entries == 128 * 1024 * 1024
    assert nbytes >= entries * 16
    monkeypatch.setenv("G4_TEST_DEVICE_MEM_LIMIT", str(nbytes - 1))
    with pytest.raises(g4.G4Error) as e:
        g4.g4_init_slice(c)
    assert e.value.code == g4.G4_E_OOM


def test_slice_size_matches_paper_arithmetic():
    # 6x6 cluster, 64 fermionic frequencies, 40 planes -> 212,336,640 entries;
    # a sub-ring of three holds a third of them (Results: accuracy and memory analysis)
    c = base(lx=6, ly=6, nw=64, nwex=1, nq=36, q_begin=0, q_end=36)
    e, _ = g4.g4_slice_size(c)
    assert e == (36 * 64) ** 2 * 36
    e40 = (36 * 64) ** 2 * 40
    assert e40 == 212336640
    c3 = base(lx=6, ly=6, nw=64, nwex=1, nq=36, q_begin=0, q_end=12)
    assert g4.g4_slice_size(c3)[0] * 3 == e


def test_null_handle_calls():
    with pytest.raises(g4.G4Error) as e:
        g4._check(g4._L.g4_sync(None))
    assert e.value.code == g4.G4_E_ARG
    with pytest.raises(g4.G4Error) as e:
        g4._check(g4._L.g4_merge(None, None))
    assert e.value.code == g4.G4_E_ARG
    g4._L.g4_destroy(None)


SHAPES = [Workload("3x5", lx=3, ly=5, nw=4, nwex=3, nq=4, q_list=(14, 0, 7, 3), q_begin=2, q_end=11),
          Workload("6x6", lx=6, ly=6, nw=8, nwex=4, nq=36, q_begin=37, q_end=100),
          Workload("8x8", lx=8, ly=8, nw=4, nwex=2, nq=64)]


@pytest.mark.parametrize("w", SHAPES, ids=lambda w: w.name)
def test_index_maps_bit_exact(w):
    c = base(lx=w.lx, ly=w.ly, nw=w.nw, nwex=w.nwex, nq=w.nq, q_list=w.q_list,
             q_begin=w.q0, q_end=w.q1)
    ka, ks, pq, pm = g4.g4_index_maps(c)
    k = np.arange(w.nc)
    kk, qq = np.meshgrid(k, k, indexing="ij")
    assert np.array_equal(ka.reshape(w.nc, w.nc), sampled._mom_add(w, kk, qq))
    assert np.array_equal(ks.reshape(w.nc, w.nc), sampled._mom_sub(w, kk, qq))   # [q][k] = q - k
    iQ = np.arange(w.q0, w.q1)
    assert np.array_equal(pq, np.asarray(w.qs)[iQ // w.nwex])
    assert np.array_equal(pm, iQ % w.nwex)


def test_persistent_flag_accepted_everywhere():
    """G4_F_PERSISTENT changes only how the packed plans launch (a persistent
    grid instead of one block per tile): accepted with every plan, no device
    memory of its own."""
    for f in (g4.G4_F_PACKED, g4.G4_F_PACKED | g4.G4_F_MFMA, g4.G4_F_PACKED_DEEP, 0, g4.G4_F_MFMA):
        a = base(mode=1, max_batch=16, prod=1, g_in=1, flags=f)
        b = base(mode=1, max_batch=16, prod=1, g_in=1, flags=f | g4.G4_F_PERSISTENT)
        assert g4.g4_slice_size(b) == g4.g4_slice_size(a), f


def test_packed_mfma_plan_accepted_and_bounded():
    """G4_F_PACKED | G4_F_MFMA: packed operands with the direct term on MFMA;
    nw = 64, 8-row tiles, plane pairs (nwex >= 2), PH channels (one or both);
    the packed buffer is sized as for G4_F_PACKED."""
    PM = g4.G4_F_PACKED | g4.G4_F_MFMA
    ok = base(mode=1, max_batch=16, prod=1, g_in=1, flags=PM)
    packed = base(mode=1, max_batch=16, prod=1, g_in=1, flags=g4.G4_F_PACKED, tile=8)
    assert g4.g4_slice_size(ok) == g4.g4_slice_size(packed)      # same buffers at the same tile
    assert g4.g4_slice_size(base(mode=1, max_batch=16, prod=1, g_in=1, flags=PM, tile=8))[0] > 0
    assert g4.g4_slice_size(base(mode=1, max_batch=8, prod=1, g_in=1, flags=PM, nwex=4, q_end=64,
                                 channels=g4.G4_PH_MAGNETIC | g4.G4_PH_CHARGE))[0] > 0
    assert g4.g4_slice_size(base(mode=1, max_batch=8, prod=1, g_in=1, flags=PM,
                                 channels=g4.G4_PH_MAGNETIC | g4.G4_PH_CHARGE))[0] > 0
    for kw in (dict(nw=128),                                        # 64 columns per block
               dict(nw=32),
               dict(channels=g4.G4_PP_UPDOWN),                      # PH channels only
               dict(channels=g4.G4_PH_MAGNETIC | g4.G4_PP_UPDOWN),
               dict(tile=16),                                       # 8-row tiles
               dict(nwex=1, q_end=16),                              # plane pairs
               dict(prod=2)):                                       # split direct term runs apart
        with pytest.raises(g4.G4Error) as e:
            g4.g4_slice_size(base(**{**dict(mode=1, max_batch=8, prod=1, g_in=1, flags=PM), **kw}))
        assert e.value.code == g4.G4_E_UNSUPPORTED, kw
    with pytest.raises(g4.G4Error) as e:                            # batched FP32 only
        g4.g4_slice_size(base(mode=1, max_batch=8, prod=0, g_in=0, flags=PM))
    assert e.value.code == g4.G4_E_UNSUPPORTED
