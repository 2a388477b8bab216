"""Central second-derivative stencils and their von Neumann symbol (oracle).

Sec. 2.1: the interior Laplacian is a dimension-split sum of the standard
central second-derivative stencil of order n along each axis.
Sec. 2.5: for a stencil {a_j}, j = -w..w, the symbol is
    sigma(k) = 2 * sum_{j=1..w} a_j (1 - cos(j k)),
and the periodic eigenvalues are lambda(k) = -sum_i sigma(k_i h) / h^2.
Table 1 gives sigma_max = 4, 16/3, 272/45 for orders 2, 4, 6.

Parity: pinned by Table 1 (tests/golden/sigma_max.txt) and by the closed-form
periodic spectrum against a dense eigen-solve (tests/test_oracle_fd.py).  The
first-derivative stencils are pinned by their Taylor conditions, solved afresh
in exact arithmetic in the test.
"""
from fractions import Fraction

import numpy as np

# one side of the symmetric stencil: a_0, a_1, ..., a_w (exact rationals)
_STENCILS = {
    2: [Fraction(-2), Fraction(1)],
    4: [Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12)],
    6: [Fraction(-49, 18), Fraction(3, 2), Fraction(-3, 20), Fraction(1, 90)],
}


# one side of the antisymmetric central first-derivative stencil of order n:
# g_1, ..., g_w with  du/dx ~ sum_j g_j (u_{+j} - u_{-j}) / h  (the gradient
# post-processing of Sec. 2.3 uses the same half-width w as the Laplacian)
_FIRST = {
    2: [Fraction(1, 2)],
    4: [Fraction(2, 3), Fraction(-1, 12)],
    6: [Fraction(3, 4), Fraction(-3, 20), Fraction(1, 60)],
}


def first_stencil(order: int):
    """Coefficients [g_1, ..., g_w] of the order-n central first derivative."""
    return [float(v) for v in _FIRST[order]]


def first_stencil_exact(order: int):
    return list(_FIRST[order])


def stencil(order: int):
    """Coefficients [a_0, a_1, ..., a_w] of the order-n central second derivative."""
    return [float(v) for v in _STENCILS[order]]


def stencil_exact(order: int):
    return list(_STENCILS[order])


def half_width(order: int) -> int:
    return order // 2


def sigma(k, order: int):
    a = stencil(order)
    k = np.asarray(k, dtype=np.float64)
    return 2.0 * sum(a[j] * (1.0 - np.cos(j * k)) for j in range(1, len(a)))


def sigma_max_exact(order: int) -> Fraction:
    """sigma(pi) in exact arithmetic: 2 * sum_j a_j (1 - (-1)^j)."""
    a = _STENCILS[order]
    return 2 * sum(a[j] * (1 - (-1) ** j) for j in range(1, len(a)))


def periodic_matrix_1d(m: int, order: int, h: float = 1.0) -> np.ndarray:
    """Dense periodic 1D second-derivative matrix on m points."""
    a = stencil(order)
    A = np.zeros((m, m))
    for i in range(m):
        A[i, i] += a[0] / h ** 2
        for j in range(1, len(a)):
            A[i, (i + j) % m] += a[j] / h ** 2
            A[i, (i - j) % m] += a[j] / h ** 2
    return A
