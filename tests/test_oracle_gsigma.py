"""Pins of the oracle's G_sigma from an expansion configuration.

The walker's G_sigma (Background section, the solver workflow: a
nonuniform Fourier transform implemented by matrix-matrix multiplication) is
written out in the oracle entry by entry as a double sum over vertex pairs.
Pinned here, independently of that code, by:
- no vertices: the noninteracting diagonal g0 (the input generator's own g0);
- the same transform as three library matrix products, E M E^H, with E built
  by numpy's exponential;
- translation of every vertex by a lattice vector and of every time by a
  constant: phases e^{i(k1-k2).a} and e^{i(w1-w2)c} on the correction only;
- a Hermitian M gives a Hermitian correction E M E^H;
- one vertex: the correction has modulus |g0(K1) g0(K2) m| / (beta Nc) at
  every entry, whatever its time and site.
"""
import numpy as np
import pytest

from oracle import ref
from synth import Workload, g0_diag

W = Workload("gsig", lx=3, ly=2, nw=6, nwex=3, nq=1, beta=4.0, mu=0.3, h=0.2, t=1.0)


def config(seed, n, w=W):
    rng = np.random.default_rng(seed)
    tau = rng.uniform(0.0, w.beta, size=n)
    site = rng.integers(0, w.nc, size=n).astype(np.int32)
    M = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return tau, site, M


def kw(w):
    """(k index, fermionic label n) of every G-window index K, and the
    momentum coordinates."""
    K = np.arange(w.ng)
    k, nn = K // w.nwg, K % w.nwg - w.nw // 2
    return k, nn, k % w.lx, k // w.lx


def library_form(w, spin, tau, site, M):
    k, nn, kx, ky = kw(w)
    wn = (2 * nn + 1) * np.pi / w.beta
    rx, ry = site % w.lx, site // w.lx
    th = wn[:, None] * tau[None, :] + 2 * np.pi * (np.outer(kx, rx) / w.lx + np.outer(ky, ry) / w.ly)
    E = np.exp(1j * th)
    corr = E @ M @ E.conj().T / (w.beta * w.nc)
    g0 = g0_diag(w, spin)
    return np.diag(g0) - g0[:, None] * corr * g0[None, :]


@pytest.mark.parametrize("spin", [0, 1])
def test_no_vertices_gives_g0(spin):
    G = ref.gsigma(W, spin, np.zeros(0), np.zeros(0, dtype=np.int32), np.zeros((0, 0)))
    want = np.diag(g0_diag(W, spin))
    assert np.max(np.abs(G - want)) <= 1e-15 * np.max(np.abs(want))


@pytest.mark.parametrize("spin", [0, 1])
@pytest.mark.parametrize("n", [1, 5, 17])
def test_matches_library_matrix_products(spin, n):
    tau, site, M = config(n + 10 * spin, n)
    G = ref.gsigma(W, spin, tau, site, M)
    want = library_form(W, spin, tau, site, M)
    assert np.linalg.norm(G - want) <= 1e-13 * np.linalg.norm(want)


def test_sampled_entries_equal_full_matrix():
    tau, site, M = config(3, 7)
    G = ref.gsigma(W, 0, tau, site, M)
    idx = np.array([0, 5, W.ng + 3, W.ng * W.ng - 1, 77], dtype=np.int64)
    assert np.array_equal(ref.gsigma(W, 0, tau, site, M, idx), G.reshape(-1)[idx])


def test_translation_in_space_and_time():
    tau, site, M = config(4, 6)
    g0 = g0_diag(W, 1)
    base = ref.gsigma(W, 1, tau, site, M) - np.diag(g0)
    k, nn, kx, ky = kw(W)
    ax, ay, c = 2, 1, 0.7
    moved = (site % W.lx + ax) % W.lx + W.lx * ((site // W.lx + ay) % W.ly)
    shifted = ref.gsigma(W, 1, tau + c, moved.astype(np.int32), M) - np.diag(g0)
    ph_k = np.exp(2j * np.pi * (kx * ax / W.lx + ky * ay / W.ly))
    ph_w = np.exp(1j * (2 * nn + 1) * np.pi / W.beta * c)
    ph = ph_k * ph_w
    want = base * ph[:, None] * ph.conj()[None, :]
    assert np.linalg.norm(shifted - want) <= 1e-13 * np.linalg.norm(base)


def test_hermitian_matrix_gives_hermitian_correction():
    tau, site, M = config(5, 9)
    M = M + M.conj().T
    g0 = g0_diag(W, 0)
    corr = (np.diag(g0) - ref.gsigma(W, 0, tau, site, M)) / (g0[:, None] * g0[None, :])
    assert np.linalg.norm(corr - corr.conj().T) <= 1e-13 * np.linalg.norm(corr)


def test_one_vertex_has_constant_modulus():
    m = 0.8 - 0.6j
    for seed in range(3):
        tau, site, _ = config(20 + seed, 1)
        g0 = g0_diag(W, 0)
        corr = np.diag(g0) - ref.gsigma(W, 0, tau, site, np.array([[m]]))
        want = np.abs(g0[:, None] * g0[None, :] * m) / (W.beta * W.nc)
        assert np.max(np.abs(np.abs(corr) - want)) <= 1e-14 * want.max()
