"""Lloyd's k-means in FP64, used only to check the device build (Sec. 3).

Test infrastructure only (see the package docstring).

The paper builds its partitions with k-means but does not fix the
initialisation, the iteration count or the empty-cluster policy; the
centroids the device build returns are therefore *parity unpinned*.  What is
pinned: every vector sits in its nearest centroid's partition (checked by
``ivf.assignment_violations``), and Lloyd's objective never rises from one
iteration to the next (textbook property, checked here on tiny inputs).
"""

from __future__ import annotations

import numpy as np

from .knn import distances


def objective(X: np.ndarray, assign: np.ndarray, C: np.ndarray) -> float:
    """Sum of squared distances from each row to its assigned centroid."""
    X64 = np.asarray(X, dtype=np.float64)
    C64 = np.asarray(C, dtype=np.float64)
    diff = X64 - C64[np.asarray(assign, dtype=np.int64)]
    return float(np.einsum("ij,ij->", diff, diff))


def assign_nearest(X: np.ndarray, C: np.ndarray) -> np.ndarray:
    D = distances(X, C, "l2")
    return np.argmin(D, axis=1)


def lloyd(X: np.ndarray, C0: np.ndarray, iters: int):
    """Plain Lloyd iterations; an empty cluster keeps its previous centroid."""
    X64 = np.asarray(X, dtype=np.float64)
    C = np.array(C0, dtype=np.float64)
    hist = []
    for _ in range(iters):
        a = assign_nearest(X64, C)
        hist.append(objective(X64, a, C))
        for j in range(C.shape[0]):
            sel = a == j
            if sel.any():
                C[j] = X64[sel].mean(0)
    a = assign_nearest(X64, C)
    hist.append(objective(X64, a, C))
    return C, a, hist
