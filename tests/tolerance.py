"""Error measure of the GPU parity tests.

``rel(a, b)`` is the larger of the relative l2 error ||a - b||_2 / ||b||_2 and the
max-norm error max|a - b| / max|b|, so that every tolerance bounds both the overall
error and the error of the worst single entry (an entry that is far off cannot hide
in the l2 norm of a long vector)."""
import numpy as np


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rel_max(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def rel(a, b):
    return max(rel_l2(a, b), rel_max(a, b))
