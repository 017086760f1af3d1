"""Brute-force Lasso solution by enumeration of sign patterns (tiny K only).

TEST INFRASTRUCTURE ONLY.

The Lasso optimality conditions (equation (primaldual)) say that x solves the
problem iff D^T (y - D x) = lambda * s with s_i = sign(x_i) where x_i != 0 and
|s_i| <= 1 elsewhere.  For a guessed support A and signs s_A the active part
solves the normal equations D_A^T D_A x_A = D_A^T y - lambda s_A; the guess is
right iff the signs agree and the inactive correlations are at most lambda.
Enumerating every (A, s_A) therefore finds the solution exactly, independently
of any iterative method.  Cost 3^K small solves: keep K <= 12.
"""
from __future__ import annotations

import itertools

import numpy as np


def brute_force_lasso(D: np.ndarray, y: np.ndarray, lam: float, tol: float = 1e-11):
    D = np.asarray(D, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    N, K = D.shape
    assert K <= 12, "brute force is exponential in K"
    corr_y = D.T @ y
    if np.max(np.abs(corr_y)) <= lam:
        return np.zeros(K)
    found = []
    for size in range(1, min(N, K) + 1):
        for A in itertools.combinations(range(K), size):
            A = list(A)
            DA = D[:, A]
            G = DA.T @ DA
            if np.linalg.matrix_rank(G) < size:
                continue
            Ginv = np.linalg.inv(G)
            inactive = [i for i in range(K) if i not in A]
            for signs in itertools.product((-1.0, 1.0), repeat=size):
                s = np.array(signs)
                xA = Ginv @ (corr_y[A] - lam * s)
                if np.any(np.sign(xA) != s) or np.any(np.abs(xA) <= tol):
                    continue
                res = y - DA @ xA
                if inactive and np.max(np.abs(D[:, inactive].T @ res)) > lam * (1.0 + tol):
                    continue
                x = np.zeros(K)
                x[A] = xA
                found.append(x)
    assert len(found) >= 1, "no KKT point found (degenerate instance)"
    # the solution is unique for dictionaries in general position; report the first
    return found[0]
