"""Jacobi iteration for the Laplace equation on a 2-D grid, written out plainly.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper's method also sped up a sample program that solves the Laplace
equation with Jacobi's method (Sec. 4, the implementation paragraph before
Sec. 5); it gives no code, so the iteration here is the textbook one:
the grid ``u`` ([n][m], FP64) keeps its boundary rows and columns fixed
(Dirichlet values) and every interior point becomes the average of its four
neighbours from the previous iterate,

    u'[i][j] = 0.25 * (u[i-1][j] + u[i+1][j] + u[i][j-1] + u[i][j+1]),

summed left to right in that order.  ``max_change`` of an iteration is the
largest ``|u'[i][j] - u[i][j]|`` over the interior.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def step(u: np.ndarray) -> Tuple[np.ndarray, float]:
    """One Jacobi iteration; returns (new grid, max change over the interior)."""
    u = np.asarray(u, dtype=np.float64)
    v = u.copy()
    if u.shape[0] > 2 and u.shape[1] > 2:
        s = u[:-2, 1:-1] + u[2:, 1:-1]
        s = s + u[1:-1, :-2]
        s = s + u[1:-1, 2:]
        v[1:-1, 1:-1] = 0.25 * s
        change = float(np.max(np.abs(v[1:-1, 1:-1] - u[1:-1, 1:-1])))
    else:
        change = 0.0
    return v, change


def solve(u: np.ndarray, iters: int) -> Tuple[np.ndarray, float]:
    """``iters`` iterations; returns the final grid and the last iteration's max change."""
    change = 0.0
    for _ in range(iters):
        u, change = step(u)
    return u, change
