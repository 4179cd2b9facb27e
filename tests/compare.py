"""Error measures of the GPU parity tests.

Every comparison with the oracle (or between two GPU paths) is held to its
bar in two norms at once: the norm-wise relative error ||a - b||_2 / ||b||_2
and the element-wise one max_j |a_j - b_j| / max_j |b_j| (for far-field maps:
over the directions).  On the contour the iterates and the far field vary by
orders of magnitude over the grid and over the angles, so a wrong border
row, ragged tile or single direction can hide under the norm of the rest;
the element-wise measure catches it.
"""
import numpy as np


def normwise(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def elementwise(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)) if b.size else 0.0


def rel(a, b):
    """The larger of the norm-wise and the element-wise relative errors."""
    return max(normwise(a, b), elementwise(a, b))
