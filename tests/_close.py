"""Comparison of a GPU result with its oracle value, normwise and entry by entry.

A result passes when both its normwise relative error ||got - ref|| / ||ref|| and
its largest entry error relative to the largest reference entry,
max |got - ref| / max |ref|, are within the tolerance. The second bound catches a
single wrong entry that a normwise ratio over many entries would hide.
"""
import numpy as np


def errors(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    diff = got - ref
    norm = float(np.linalg.norm(diff) / np.linalg.norm(ref))
    entry = float(np.max(np.abs(diff)) / np.max(np.abs(ref)))
    return norm, entry


def assert_close(got, ref, tol, what=""):
    norm, entry = errors(got, ref)
    assert np.all(np.isfinite(got)), f"{what}: non-finite entries"
    assert norm <= tol and entry <= tol, f"{what}: normwise {norm:.3e}, entrywise {entry:.3e} > {tol:g}"
    return norm, entry


def assert_close_per_matrix(got, ref, tol, what=""):
    """assert_close for each matrix along the first axis (S_l, l = 1..d); returns the worst pair."""
    worst = (0.0, 0.0)
    for l in range(ref.shape[0]):
        norm, entry = assert_close(got[l], ref[l], tol, f"{what} matrix {l}")
        worst = (max(worst[0], norm), max(worst[1], entry))
    return worst
