"""Right-preconditioned flexible GMRES (oracle).

Sec. 4.1 of the paper: the outer solver is FGMRES (Saad 1993) with restart 10,
preconditioned on the right by one multigrid V-cycle; right preconditioning
keeps the residual that is tested the true residual of the high-order system.
Modified Gram-Schmidt Arnoldi, Givens rotations on the Hessenberg matrix,
x0 = 0 unless given.  Stopping rule (a reading): the Givens estimate of
||b - A x|| / ||b|| reaching rtol ends a cycle; the solve stops only when the
true relative residual, recomputed at the start of the next cycle, is <= rtol.

Parity: the solution is pinned against the sparse direct solve of the same
system (tests/test_oracle_mg.py).
"""
from __future__ import annotations

import math
from typing import Callable, List, Tuple

import numpy as np


def fgmres(A: Callable, M: Callable, b: np.ndarray, x0=None, rtol: float = 1e-10,
           restart: int = 10, max_iters: int = 500):
    """Returns (x, history, iterations, converged).  history holds one entry
    per inner iteration: the Givens estimate of the relative residual."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, [], 0, True
    hist: List[float] = []
    true_hist: List[float] = []
    its = 0
    while True:
        r = b - A(x)
        beta = np.linalg.norm(r)
        true_hist.append(beta / bnorm)
        if beta / bnorm <= rtol:
            return x, hist, its, True
        if its >= max_iters:
            return x, hist, its, False
        m = restart
        V = np.zeros((m + 1, b.size))
        Z = np.zeros((m, b.size))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = M(V[j])
            w = A(Z[j])
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= rtol or its >= max_iters:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
