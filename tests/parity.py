"""Comparison of a GPU result with the FP64 oracle's, shared by the GPU tests.

One global relative Frobenius error can hide a single wrong frontal slice or a
few wrong entries, so every comparison also bounds
  * the largest per-slice error, ||got_p - ref_p|| / max(||ref_p||, ||ref|| / sqrt(P))
    over the frontal slices p (the floor keeps slices of a nearly zero
    reference from dividing by ~0), and
  * the largest entry error, max |got - ref| / max |ref|.
"""
import numpy as np


def errors(got, ref):
    """(global relative error, worst per-slice error, worst entry error)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    d = got - ref
    nref = float(np.linalg.norm(ref))
    glob = float(np.linalg.norm(d)) / max(nref, 1e-300)
    I1, I2 = ref.shape[0], (ref.shape[1] if ref.ndim > 1 else 1)
    P = ref.size // max(I1 * I2, 1)
    dr = d.reshape((I1 * I2, P), order="F")
    rr = ref.reshape((I1 * I2, P), order="F")
    floor = max(nref / np.sqrt(max(P, 1)), 1e-300)
    per = np.linalg.norm(dr, axis=0) / np.maximum(np.linalg.norm(rr, axis=0), floor)
    worst = float(per.max()) if per.size else 0.0
    amax = float(np.abs(ref).max()) if ref.size else 0.0
    elem = float(np.abs(d).max()) / max(amax, 1e-300) if d.size else 0.0
    return glob, worst, elem


def check(got, ref, tol, slice_factor=10.0, elem_factor=10.0, label=""):
    """Assert the global error <= tol, the worst per-slice error <=
    slice_factor * tol and the worst entry error <= elem_factor * tol; return
    the three errors."""
    glob, worst, elem = errors(got, ref)
    print("  %s parity: global %.3e, worst slice %.3e, worst entry %.3e (tol %.1e)"
          % (label, glob, worst, elem, tol), flush=True)
    assert glob <= tol, ("global", glob, tol)
    assert worst <= slice_factor * tol, ("slice", worst, slice_factor * tol)
    assert elem <= elem_factor * tol, ("entry", elem, elem_factor * tol)
    return glob, worst, elem
