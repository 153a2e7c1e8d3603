"""Error measures used by the tests.

rel_fro:   ||A - B||_F / ||B||_F over complex entries.
l1_error, l2_error:  the paper's normalized entrywise errors, Eq. (2) and
Eq. (3) (Results section, "Accuracy Analysis"), applied to the real and the
imaginary parts separately as its Table 1 reports them.
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
