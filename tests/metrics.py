"""Error measures used by the tests.

rel_fro:   ||A - B||_F / ||B||_F over complex entries.
l1_error, l2_error:  the paper's normalized entrywise errors, Eq. (2) and
Eq. (3) (Results section, "Accuracy Analysis"), applied to the real and the
imaginary parts separately as its Table 1 reports them.
check_entries:  the parity gate of the GPU tests: the relative Frobenius
error, the four Eq. (2)/(3) numbers, and the relative Frobenius error over
the smaller half of the entries by magnitude, each against its bar.
"""
import numpy as np


def rel_fro(a, ref):
    a = np.asarray(a).ravel()
    ref = np.asarray(ref).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(a - ref) / (den if den > 0 else 1.0))


def l1_error(a, ref):
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.abs(a - ref).sum() / np.abs(ref).sum())


def l2_error(a, ref):
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def paper_errors(a, ref):
    """Eq. (2)/(3) on real and imaginary parts: dict of four numbers."""
    a = np.asarray(a)
    ref = np.asarray(ref)
    return {"l1_re": l1_error(a.real, ref.real), "l1_im": l1_error(a.imag, ref.imag),
            "l2_re": l2_error(a.real, ref.real), "l2_im": l2_error(a.imag, ref.imag)}


def check_entries(got, want, tol, what=""):
    """Assert parity of got with want (the oracle) at relative bar tol:
    - relative Frobenius error <= tol;
    - Eq. (2) and Eq. (3) on real and imaginary parts, each <= 4 tol;
    - relative Frobenius error over the entries whose |want| is at most the
      median (the half that the large entries would hide in a whole-slice
      norm) <= 16 tol.  Rounding of FP32 products scales with the sizes of the
      terms, not of their sum, so small entries carry a larger relative error:
      the looser bar covers that and still catches a defect confined to them.
    Returns the numbers."""
    got = np.asarray(got).ravel()
    want = np.asarray(want).ravel()
    assert got.shape == want.shape, (got.shape, want.shape)
    out = {"rel_fro": rel_fro(got, want)}
    out.update(paper_errors(got, want))
    mag = np.abs(want)
    med = np.median(mag)
    small = mag <= med
    out["rel_fro_small_half"] = rel_fro(got[small], want[small]) if med > 0 else 0.0
    assert out["rel_fro"] <= tol, (what, out)
    for k in ("l1_re", "l1_im", "l2_re", "l2_im"):
        assert out[k] <= 4 * tol, (what, k, out)
    assert out["rel_fro_small_half"] <= 16 * tol, (what, out)
    return out
