"""The seeded input generator: Philox4x32-10 against its published known-answer
vectors, and the Hubbard-shaped G recipe's basic properties."""
import os

import numpy as np

from synth import C1_TINY, C2_PLAIN, g0_diag, g_elements, g_matrices, signs
from synth.philox import box_muller, philox4x32_10, u53

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = philox4x32_10(*[np.uint32(x) for x in r[:6]])
        assert [int(x) for x in out] == r[6:]


def test_uniform_and_normal_moments():
    n = 1 << 18
    c = np.arange(n, dtype=np.uint32)
    x0, x1, x2, x3 = philox4x32_10(c, np.uint32(0), np.uint32(0), np.uint32(0),
                                   np.uint32(7), np.uint32(9))
    u1, u2 = u53(x0, x1), u53(x2, x3)
    assert u1.min() >= 0.0 and u1.max() < 1.0
    assert abs(u1.mean() - 0.5) < 5e-3
    x, y = box_muller(u1, u2)
    for v in (x, y):
        assert abs(v.mean()) < 1e-2
        assert abs(v.var() - 1.0) < 1e-2
    assert abs(np.mean(x * y)) < 1e-2


def test_g_recipe_diagonal_and_noise():
    w = C1_TINY
    g = g_matrices(w, 0, 3, 0)
    d = g0_diag(w, 0)
    # g0 = 1/(i w_n + mu - eps_k): k=0 has eps=-4t, n=-Nw/2 gives w=-(Nw-1) pi/beta
    wn = -(w.nw - 1) * np.pi / w.beta
    assert np.isclose(d[0], 1.0 / (1j * wn + w.mu + 4.0 * w.t))
    off = g[:, ~np.eye(w.ng, dtype=bool)]
    assert abs(off.real.std() - w.noise) < 0.01 and abs(off.imag.std() - w.noise) < 0.01
    # elements regenerate identically from their counters
    r = np.array([0, 5, 17, 63])
    c = np.array([0, 9, 17, 2])
    for b in range(3):
        assert np.array_equal(g_elements(w, b, 0, r, c), g[b, r, c])
    # spins draw independent noise
    gd = g_matrices(w, 0, 1, 1)
    assert not np.allclose(gd[0], g[0])


def test_signs_fraction():
    s = signs(C2_PLAIN, 0, 20000)
    assert set(np.unique(s)) == {-1.0, 1.0}
    assert abs((s > 0).mean() - 0.95) < 0.01
    assert np.array_equal(s[100:200], signs(C2_PLAIN, 100, 100))
