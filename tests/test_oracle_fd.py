"""Pins for the interior stencils (Sec. 2.5, Table 1)."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import fd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sigma_max.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        o, num, den = (int(v) for v in line.split())
        out[o] = Fraction(num, den)
    return out


@pytest.mark.parametrize("order", [2, 4, 6])
def test_sigma_max_matches_table(order):
    g = _golden()[order]
    assert fd.sigma_max_exact(order) == g
    # sigma_max is the maximum of sigma over [0, pi] (not just its value at pi)
    k = np.linspace(0.0, np.pi, 200001)
    assert abs(fd.sigma(k, order).max() - float(g)) < 1e-12


@pytest.mark.parametrize("order", [2, 4, 6])
def test_stencil_consistency(order):
    """Second-derivative stencils: exact on x^q for q <= order+1 (symmetric)."""
    a = fd.stencil_exact(order)
    w = len(a) - 1
    for q in range(order + 2):
        val = a[0] * (0 if q else 1) + sum(a[j] * (Fraction(j) ** q + Fraction(-j) ** q) for j in range(1, w + 1))
        want = 2 if q == 2 else 0
        assert val == want


@pytest.mark.parametrize("order", [2, 4, 6])
def test_periodic_spectrum_closed_form(order):
    """With no immersed boundary the periodic eigenvalues are -sigma(k h)/h^2."""
    m, h = 24, 0.1
    A = fd.periodic_matrix_1d(m, order, h)
    ev = np.sort(np.linalg.eigvalsh(A))
    k = 2 * np.pi * np.arange(m) / m
    closed = np.sort(-fd.sigma(k, order) / h ** 2)
    assert np.allclose(ev, closed, atol=1e-9 * abs(closed).max())
    # 2D tensor product: -(sigma(k1 h) + sigma(k2 h)) / h^2, bounded by 2 sigma_max
    A2 = np.kron(A, np.eye(m)) + np.kron(np.eye(m), A)
    ev2 = np.linalg.eigvalsh(A2) * h ** 2
    assert ev2.max() <= 1e-9 and ev2.min() >= -2 * float(fd.sigma_max_exact(order)) - 1e-9


@pytest.mark.parametrize("order", [2, 4, 6])
def test_first_derivative_stencil_taylor(order):
    """First-derivative stencils: exact on x^q for q <= order (antisymmetric),
    and the order-n stencil is the unique one of half-width n/2 that is:
    solving the moment conditions in exact arithmetic reproduces it."""
    g = fd.first_stencil_exact(order)
    w = len(g)
    assert w == fd.half_width(order)
    for q in range(order + 1):
        val = sum(g[j - 1] * (Fraction(j) ** q - Fraction(-j) ** q) for j in range(1, w + 1))
        assert val == (1 if q == 1 else 0), (order, q)
    # the next odd moment is not matched: the stencil is of order n exactly
    q = order + 1
    assert sum(g[j - 1] * (Fraction(j) ** q - Fraction(-j) ** q) for j in range(1, w + 1)) != 0
    # moment system 2 sum_j g_j j^(2m+1) = [m == 0], m = 0..w-1, by Gaussian elimination
    A = [[2 * Fraction(j) ** (2 * m + 1) for j in range(1, w + 1)] + [Fraction(1 if m == 0 else 0)]
         for m in range(w)]
    for c in range(w):
        piv = A[c][c]
        A[c] = [v / piv for v in A[c]]
        for r in range(w):
            if r != c:
                f = A[r][c]
                A[r] = [a - f * b for a, b in zip(A[r], A[c])]
    assert [A[r][w] for r in range(w)] == g
