"""Pins for the oracle's GLL nodes, weights and derivative matrix.

Closed forms come from tests/golden/gll_closed_forms.json (textbook values,
cited there); the other checks are properties any GLL rule must have:
exactness of the quadrature to degree 2N-3 but not 2N-2, and exact
differentiation of polynomials of degree <= N-1."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def _num(s):
    s = s.strip()
    neg = s.startswith("-")
    if neg:
        s = s[1:]
    if s.startswith("sqrt(") and s.endswith(")"):
        v = math.sqrt(float(Fraction(s[5:-1])))
    else:
        v = float(Fraction(s))
    return -v if neg else v


def test_closed_forms(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "gll_closed_forms.json")))
    for N, rule in g["rules"].items():
        xi, w = O.gll(int(N))
        np.testing.assert_allclose(xi, [_num(s) for s in rule["nodes"]], rtol=0, atol=1e-15)
        np.testing.assert_allclose(w, [_num(s) for s in rule["weights"]], rtol=0, atol=1e-15)
    D3 = O.deriv(3)
    np.testing.assert_allclose(D3, [[_num(s) for s in row] for row in g["derivative_matrix_3"]],
                               rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", list(range(2, 17)))
def test_quadrature_exact_to_2N_minus_3(N):
    xi, w = O.gll(N)
    assert abs(w.sum() - 2.0) < 1e-14
    assert np.all(np.diff(xi) > 0) and xi[0] == -1.0 and xi[-1] == 1.0
    for m in range(0, 2 * N - 2):
        exact = 2.0 / (m + 1) if m % 2 == 0 else 0.0
        assert abs(np.dot(w, xi ** m) - exact) < 2e-14, (N, m)
    # not exact one degree higher (distinguishes Lobatto from Gauss rules)
    m = 2 * N - 2
    assert abs(np.dot(w, xi ** m) - 2.0 / (m + 1)) > 1e-11


@pytest.mark.parametrize("N", list(range(2, 17)))
def test_derivative_exact_on_polynomials(N):
    xi, _ = O.gll(N)
    D = O.deriv(N, xi)
    assert np.abs(D @ np.ones(N)).max() < 1e-12 * N * N
    for m in range(1, N):
        got = D @ xi ** m
        want = m * xi ** (m - 1)
        assert np.abs(got - want).max() < 1e-11 * N ** 2, (N, m)
    # end-point closed form of the diagonal
    p = N - 1
    assert D[0, 0] == pytest.approx(-p * (p + 1) / 4.0, rel=1e-15)
    assert D[-1, -1] == pytest.approx(p * (p + 1) / 4.0, rel=1e-15)


def test_symmetry_of_nodes():
    for N in range(2, 17):
        xi, w = O.gll(N)
        np.testing.assert_allclose(xi, -xi[::-1], atol=1e-15)
        np.testing.assert_allclose(w, w[::-1], atol=1e-15)
