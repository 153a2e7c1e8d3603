"""Parity of the HIP G_sigma path (g4_gsigma through the C ABI) with the
oracle's entry-by-entry double sum.

Bars, as relative Frobenius error of the correction G - diag(g0) (over every
entry, or over the sampled entries at full size):
- complex128 (FP64 phases and MFMA products): 1e-12;
- complex64 (FP32 products of n terms, twice, plus the FP32 rounding of E and
  M): (2n + 16) * 2^-24, a norm-wise bound for two chained n-term FP32
  inner products.
The G window of the small shapes spans several 64 x 64 output tiles with a
ragged tail, and n spans several 16-wide k chunks with a ragged last chunk;
n = 0 (G = g0 on the diagonal), count = 0 and argument errors are covered."""

import numpy as np
import pytest

from gpu_common import g4mod
from oracle import ref
from synth import Workload, expansion_configs, g0_diag

pytestmark = pytest.mark.gpu

SMALL = Workload("gsig-small", lx=3, ly=2, nw=6, nwex=3, nq=1, beta=4.0, mu=0.3, h=0.2, t=1.0)
TILES = Workload("gsig-tiles", lx=4, ly=4, nw=8, nwex=3, nq=1, beta=6.0, mu=-0.2, h=0.1, t=1.0)
FULL = Workload("gsig-4x4", lx=4, ly=4, nw=64, nwex=8, nq=1, beta=10.0, mu=0.0, h=0.0, t=1.0)


def tol_for(c128, n):
    return 1e-12 if c128 else (2 * n + 16) * 2.0 ** -24


def run(w, spin, tau, site, M, c128):
    import torch
    g4 = g4mod()
    count, n = M.shape[0], M.shape[1]
    dt = torch.complex128 if c128 else torch.complex64
    dev = dict(device="cuda")
    tau_d = torch.from_numpy(np.ascontiguousarray(tau)).to(**dev)
    site_d = torch.from_numpy(np.ascontiguousarray(site)).to(**dev)
    M_d = torch.from_numpy(np.ascontiguousarray(M)).to(dtype=dt, **dev)
    G = torch.full((count, w.ng, w.ng), complex(float("nan"), float("nan")), dtype=dt, **dev)
    ws = torch.empty(g4.g4_gsigma_workspace(w.lx, w.ly, w.nw, w.nwex, n, count,
                                            g4.G4_IN_C128 if c128 else g4.G4_IN_C64), dtype=torch.uint8, **dev)
    g4.g4_gsigma(w.lx, w.ly, w.nw, w.nwex, w.beta, w.mu, w.h, w.t, spin, tau_d, site_d, M_d, G, ws)
    torch.cuda.synchronize()
    return G.cpu().numpy().astype(np.complex128)


def oracle_inputs(M, c128):
    """The oracle sees M exactly as the kernel does (rounded to complex64 for
    the single-precision path)."""
    return M if c128 else M.astype(np.complex64).astype(np.complex128)


def corr_err(got, want, g0_rows, diag_mask):
    d = np.where(diag_mask, g0_rows, 0.0)
    c_want = want - d
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(c_want), 1e-300))


@pytest.mark.parametrize("c128", [True, False], ids=["c128", "c64"])
@pytest.mark.parametrize("w,n,spin", [(SMALL, 1, 0), (SMALL, 17, 1), (SMALL, 70, 0), (TILES, 33, 1),
                                      (TILES, 100, 0)], ids=lambda v: getattr(v, "name", str(v)))
def test_full_matrix_matches_oracle(w, n, spin, c128):
    print(f"\ncase {w.name} n={n} spin={spin} c128={c128}", flush=True)
    count = 3
    tau, site, M = expansion_configs(w, 100 + n + spin, count, n)
    got = run(w, spin, tau, site, M, c128)
    assert np.isfinite(got).all()
    Mo = oracle_inputs(M, c128)
    g0 = g0_diag(w, spin)
    eye = np.eye(w.ng, dtype=bool)
    for b in range(count):
        want = ref.gsigma(w, spin, tau[b], site[b], Mo[b])
        err = corr_err(got[b], want, g0[:, None], eye)
        assert err <= tol_for(c128, n), (b, err)


@pytest.mark.parametrize("c128", [True, False], ids=["c128", "c64"])
def test_no_vertices_gives_g0(c128):
    print(f"\ncase n=0 c128={c128}", flush=True)
    w = TILES
    tau, site, M = expansion_configs(w, 7, 2, 0)
    got = run(w, 0, tau, site, M, c128)
    want = np.diag(g0_diag(w, 0))
    rel = 1e-15 if c128 else 2.0 ** -23
    for b in range(2):
        assert np.max(np.abs(got[b] - want)) <= rel * np.max(np.abs(want))


def test_count_zero_launches_nothing():
    import torch
    g4 = g4mod()
    M = torch.zeros((0, 5, 5), dtype=torch.complex128, device="cuda")
    G = torch.zeros((0, SMALL.ng, SMALL.ng), dtype=torch.complex128, device="cuda")
    tau = torch.zeros((0, 5), dtype=torch.float64, device="cuda")
    site = torch.zeros((0, 5), dtype=torch.int32, device="cuda")
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    g4.g4_gsigma(SMALL.lx, SMALL.ly, SMALL.nw, SMALL.nwex, SMALL.beta, SMALL.mu, SMALL.h, SMALL.t, 0,
                 tau, site, M, G, ws)


def test_argument_errors():
    import torch
    g4 = g4mod()
    w = SMALL
    n, count = 4, 1
    tau, site, M = expansion_configs(w, 3, count, n)
    tau_d = torch.from_numpy(tau).cuda()
    site_d = torch.from_numpy(site).cuda()
    M_d = torch.from_numpy(M).cuda()
    G = torch.zeros((count, w.ng, w.ng), dtype=torch.complex128, device="cuda")
    need = g4.g4_gsigma_workspace(w.lx, w.ly, w.nw, w.nwex, n, count, g4.G4_IN_C128)
    short = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(g4.G4Error) as e:
        g4.g4_gsigma(w.lx, w.ly, w.nw, w.nwex, w.beta, w.mu, w.h, w.t, 0, tau_d, site_d, M_d, G, short)
    assert e.value.code == g4.G4_E_ARG
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    with pytest.raises(g4.G4Error) as e:
        g4.g4_gsigma(w.lx, w.ly, w.nw, w.nwex, w.beta, w.mu, w.h, w.t, 2, tau_d, site_d, M_d, G, ws)
    assert e.value.code == g4.G4_E_ARG
    with pytest.raises(g4.G4Error) as e:
        g4.g4_gsigma(w.lx, w.ly, 5, w.nwex, w.beta, w.mu, w.h, w.t, 0, tau_d, site_d, M_d, G, ws)
    assert e.value.code == g4.G4_E_ARG
    # nothing was written by the rejected calls
    assert float(G.abs().max()) == 0.0


@pytest.mark.parametrize("c128", [True, False], ids=["c128", "c64"])
def test_full_size_sampled_entries(c128):
    """The 4x4 cluster window (Ng = 1136) at expansion order 512, eight
    measurements in one call: 512 sampled entries per measurement (diagonal
    ones included) against the oracle, and Hermitian symmetry of the
    correction for a Hermitian M."""
    w, n, count = FULL, 512, 8
    print(f"\ncase {w.name} n={n} count={count} c128={c128}", flush=True)
    tau, site, M = expansion_configs(w, 555, count, n)
    M[1] = M[1] + M[1].conj().T
    got = run(w, 1, tau, site, M, c128)
    assert np.isfinite(got).all()
    Mo = oracle_inputs(M, c128)
    g0 = g0_diag(w, 1)
    rng = np.random.default_rng(9)
    for b in range(count):
        idx = rng.integers(0, w.ng * w.ng, size=512)
        idx[:16] = rng.integers(0, w.ng, size=16) * (w.ng + 1)   # diagonal entries
        want = ref.gsigma(w, 1, tau[b], site[b], Mo[b], idx)
        r, c = idx // w.ng, idx % w.ng
        diag = r == c
        err = corr_err(got[b].reshape(-1)[idx], want, g0[r], diag)
        assert err <= tol_for(c128, n), (b, err)
    c1 = (got[1] - np.diag(g0)) / (g0[:, None] * g0[None, :])
    herm = np.linalg.norm(c1 - c1.conj().T) / np.linalg.norm(c1)
    assert herm <= 2 * tol_for(c128, n), herm
