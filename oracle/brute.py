"""Exhaustive geometry for tiny systems (n <= 3) -- TEST INFRASTRUCTURE ONLY.

Independent of the oracle's C code: used to pin it.

* ``vertices`` -- vertex enumeration of M = {p : A p <= b} (every n-subset of
  rows with a non-singular matrix; keep the feasible intersection points).
* ``project`` -- the Euclidean projection of x onto M (section 2's distance
  d(x, M)), by enumeration of active sets: for every set S of at most n
  linearly independent rows, the minimiser of ||p - x|| on {A_S p = b_S} is a
  candidate; the projection is the feasible candidate nearest to x (it is one
  of them, by the KKT conditions with a linearly independent active subset).
* ``exact_sweep`` -- one sweep in exact rational arithmetic (fractions), for
  integer or dyadic inputs: residuals, h and y exactly; the distances squared
  exactly (the distances themselves need a square root).
* ``exact_scale`` -- the rounding-error scale of each residual,
  t_i = sum_j |a_ij x_j| + |b_i| (the quantity a forward error bound of the
  dot product <a_i, x> - b_i is proportional to; Higham, Accuracy and
  Stability of Numerical Algorithms, sect. 3.1), in exact rationals.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def vertices(A, b, tol=1e-9):
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    out = []
    for S in itertools.combinations(range(m), n):
        As = A[list(S)]
        if abs(np.linalg.det(As)) < 1e-12:
            continue
        p = np.linalg.solve(As, b[list(S)])
        if np.all(A @ p <= b + tol * (1 + np.abs(b))):
            if not any(np.allclose(p, q, atol=1e-9) for q in out):
                out.append(p)
    return np.array(out).reshape(-1, n)


def project(A, b, x, tol=1e-9):
    """Projection of x onto M and the distance d(x, M) (exact up to FP64 rounding)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    m, n = A.shape
    best, best_d = None, np.inf
    for k in range(0, n + 1):
        for S in itertools.combinations(range(m), k):
            if k == 0:
                p = x.copy()
            else:
                As = A[list(S)]
                G = As @ As.T
                if abs(np.linalg.det(G)) < 1e-12:
                    continue
                mu = np.linalg.solve(G, As @ x - b[list(S)])
                p = x - As.T @ mu
            if np.all(A @ p <= b + tol * (1 + np.abs(b))):
                d = float(np.linalg.norm(p - x))
                if d < best_d:
                    best, best_d = p, d
    return best, best_d


def exact_sweep(A, b, x):
    """Exact sweep in rationals: (r list, h, y list, d2 list of r_i^2/||a_i||^2 for violated rows)."""
    A = [[Fraction(v) for v in row] for row in np.asarray(A, dtype=np.float64).tolist()]
    b = [Fraction(v) for v in np.asarray(b, dtype=np.float64).tolist()]
    x = [Fraction(v) for v in np.asarray(x, dtype=np.float64).tolist()]
    m, n = len(A), len(x)
    r = []
    y = [Fraction(0)] * n
    h = 0
    d2 = []
    for i in range(m):
        ri = sum(A[i][j] * x[j] for j in range(n)) - b[i]
        r.append(ri)
        if ri > 0:
            nu = sum(a * a for a in A[i])
            w = ri / nu
            y = [y[j] + w * A[i][j] for j in range(n)]
            h += 1
            d2.append(ri * ri / nu)
    return r, h, y, d2


def exact_scale(A, b, x):
    """Exact t_i = sum_j |a_ij x_j| + |b_i| for every row (list of Fractions)."""
    A = [[Fraction(v) for v in row] for row in np.asarray(A, dtype=np.float64).tolist()]
    b = [Fraction(v) for v in np.asarray(b, dtype=np.float64).tolist()]
    x = [Fraction(v) for v in np.asarray(x, dtype=np.float64).tolist()]
    return [sum(abs(A[i][j] * x[j]) for j in range(len(x))) + abs(b[i]) for i in range(len(A))]
