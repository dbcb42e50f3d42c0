"""Pins for the oracle's AX operator (Section II-B).

(a) against the dense Kronecker element matrix built by brute force;
(b) invariants: AX(const) = 0, symmetry, positive semi-definiteness;
(c) exact integration of polynomial gradients on affine (also sheared)
    elements;
plus the paper's printed flop counts (tests/golden/paper_flop_counts.json).
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import synthetic as S
from brute import dense_element_matrix, grad_inner_exact


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_ax_matches_dense_element_matrix(N):
    E = 3
    D = O.deriv(N)
    G = S.random_factors(E, N, seed=N)
    u = S.uniform_field(E, N, seed=N + 100)
    w = O.ax(u, G, D)
    for e in range(E):
        A = dense_element_matrix(G[e], D)
        ref = A @ u[e]
        assert np.abs(w[e] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_ax_matches_dense_element_matrix_N10():
    N, E = 10, 1
    D = O.deriv(N)
    G = S.random_factors(E, N, seed=7)
    u = S.uniform_field(E, N, seed=8)
    w = O.ax(u, G, D)
    A = dense_element_matrix(G[0], D)
    ref = A @ u[0]
    assert np.abs(w[0] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_dense_matrix_detects_transposed_operand():
    """A plausible slip (applying D^T where D belongs) must be caught by the
    dense comparison: the element matrix built from D^T differs."""
    N = 4
    D = O.deriv(N)
    G = S.random_factors(1, N, seed=3)
    u = S.uniform_field(1, N, seed=4)
    w = O.ax(u, G, D)[0]
    wrong = dense_element_matrix(G[0], D.T) @ u[0]
    assert np.abs(w - wrong).max() > 1e-3 * np.abs(w).max()


@pytest.mark.parametrize("N", [4, 7, 10])
def test_invariants_on_deformed_mesh(N):
    b = S.scaled_c2_brick(3, N)
    xi, wq = O.gll(N)
    D = O.deriv(N, xi)
    x, y, z = O.brick_coords(b, xi)
    G, bm, jmin = O.geom(N, D, wq, x, y, z)
    assert jmin > 0
    E = b.E
    one = np.ones((E, N ** 3))
    w1 = O.ax(one, G, D)
    assert np.abs(w1).max() < 1e-12 * np.abs(G).max() * N ** 2
    u = S.uniform_field(E, N, seed=1)
    v = S.uniform_field(E, N, seed=2)
    Au = O.ax(u, G, D); Av = O.ax(v, G, D)
    lhs = float(np.sum(v * Au)); rhs = float(np.sum(Av * u))
    assert abs(lhs - rhs) <= 1e-13 * np.sqrt(np.sum(u * Au) * np.sum(v * Av))
    # element matrices are PSD: u^T A_e u >= 0 for each element
    per_elem = np.sum(u * Au, axis=1)
    assert np.all(per_elem >= -1e-13 * np.abs(per_elem).max())


@pytest.mark.parametrize("N,dims", [(3, (1, 1, 1)), (4, (2, 3, 1)), (6, (2, 2, 2)), (8, (1, 2, 3))])
def test_exact_integration_affine(N, dims):
    """v^T A u = int grad u . grad v for monomials of degree <= N-2 per
    direction (GLL quadrature is exact to degree 2N-3)."""
    b = S.Brick(*dims, N)
    xi, wq = O.gll(N)
    D = O.deriv(N, xi)
    x, y, z = O.brick_coords(b, xi)
    G, _, _ = O.geom(N, D, wq, x, y, z)
    q = N - 2
    rng = np.random.default_rng(N)
    for _ in range(6):
        pu = tuple(int(t) for t in rng.integers(0, q + 1, size=3))
        pv = tuple(int(t) for t in rng.integers(0, q + 1, size=3))
        u = x ** pu[0] * y ** pu[1] * z ** pu[2]
        v = x ** pv[0] * y ** pv[1] * z ** pv[2]
        got = float(np.dot(v, O.ax(u, G, D).reshape(-1)))
        want = grad_inner_exact(pu, pv)
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (pu, pv, got, want)


@pytest.mark.parametrize("N", [3, 5, 7])
def test_exact_integration_sheared(N):
    """Physical coordinates x = M X for a general matrix M (off-diagonal
    terms exercise g2, g3, g5):  int_{M Omega} grad u . grad v dx =
    det(M) int_Omega grad_X u^T (M^-1 M^-T) grad_X v dX  for u, v monomials
    in the reference coordinates X."""
    M = np.array([[1.0, 0.3, -0.2], [0.1, 0.8, 0.25], [-0.15, 0.2, 1.2]])
    K = np.linalg.inv(M) @ np.linalg.inv(M).T
    b = S.Brick(2, 1, 2, N)
    xi, wq = O.gll(N)
    D = O.deriv(N, xi)
    X, Y, Z = O.brick_coords(b, xi)
    P = M @ np.stack([X, Y, Z])
    G, bm, _ = O.geom(N, D, wq, P[0].copy(), P[1].copy(), P[2].copy())
    assert abs(np.abs(G[:, 1]).max()) > 1e-3          # cross factors present
    assert abs(bm.sum() - np.linalg.det(M)) < 1e-13
    q = N - 2
    rng = np.random.default_rng(10 + N)
    for _ in range(6):
        pu = tuple(int(t) for t in rng.integers(0, q + 1, size=3))
        pv = tuple(int(t) for t in rng.integers(0, q + 1, size=3))
        u = X ** pu[0] * Y ** pu[1] * Z ** pu[2]
        v = X ** pv[0] * Y ** pv[1] * Z ** pv[2]
        got = float(np.dot(v, O.ax(u, G, D).reshape(-1)))
        want = np.linalg.det(M) * grad_inner_exact(pu, pv, K)
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (pu, pv, got, want)


def test_flop_model_matches_paper(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "paper_flop_counts.json")))
    n = g["nodes_per_direction"]
    assert n ** 3 == g["grid_points_per_element"]
    assert O.ax_flops(n, 1) == g["flops_per_element"]
    assert O.ax_flops(n, 1) // n ** 3 == g["flops_per_grid_point"]
