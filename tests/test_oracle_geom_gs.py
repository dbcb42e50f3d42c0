"""Pins for the oracle's mesh set-up, geometric factors, gather-scatter
(dssum), Dirichlet mask and Jacobi diagonal."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import synthetic as S
from brute import dense_element_matrix, scatter_matrix


def test_affine_factors_closed_form():
    """Cube elements of side h: J = (h/2) I, so G_aa = W (h/2)^3 (2/h)^2 =
    W h / 2 and the cross factors vanish (for h = 1/4: W/8)."""
    b = S.c1_brick()
    N = b.N
    xi, wq = O.gll(N)
    D = O.deriv(N, xi)
    G, bm, jmin = O.geom(N, D, wq, *O.brick_coords(b, xi))
    W = np.einsum("k,j,i->kji", wq, wq, wq).reshape(-1)
    for f, want in zip(range(6), [W / 8, 0, 0, W / 8, 0, W / 8]):
        np.testing.assert_allclose(G[:, f, :], np.broadcast_to(want, G[:, f, :].shape),
                                   rtol=0, atol=1e-16)
    assert jmin == pytest.approx((0.25 / 2) ** 3, rel=1e-13)


def test_factors_against_numpy_inverse():
    """A general affine map: G = W det(J) J^-1 J^-T with J = M (h/2) from
    numpy's inverse (independent of the oracle's adjugate formula)."""
    N = 4
    M = np.array([[0.9, 0.2, 0.1], [-0.3, 1.1, 0.05], [0.2, -0.1, 0.7]])
    b = S.Brick(1, 1, 1, N)
    xi, wq = O.gll(N)
    D = O.deriv(N, xi)
    X = np.stack(O.brick_coords(b, xi))
    P = M @ X
    G, bm, _ = O.geom(N, D, wq, *[p.copy() for p in P])
    J = M * 0.5
    Ji = np.linalg.inv(J)
    K = np.linalg.det(J) * (Ji @ Ji.T)
    W = np.einsum("k,j,i->kji", wq, wq, wq).reshape(-1)
    for f, (a, c) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        np.testing.assert_allclose(G[0, f], W * K[a, c], rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("N", [6, 10])
def test_deformed_geometry_properties(N):
    """C2's mapping: factors form SPD matrices, the discrete volume is 1
    (the map fixes the cube), and for any linear field u = a.x the discrete
    energy u^T A u equals |a|^2 times the discrete volume exactly (the
    isoparametric gradient of a linear field is exact)."""
    b = S.scaled_c2_brick(4, N)
    xi, wq = O.gll(N)
    D = O.deriv(N, xi)
    x, y, z = O.brick_coords(b, xi)
    G, bm, jmin = O.geom(N, D, wq, x, y, z)
    assert jmin > 0
    g1, g2, g3, g4, g5, g6 = [G[:, f, :] for f in range(6)]
    m1 = g1
    m2 = g1 * g4 - g2 * g2
    m3 = g1 * (g4 * g6 - g5 * g5) - g2 * (g2 * g6 - g5 * g3) + g3 * (g2 * g5 - g4 * g3)
    assert np.all(m1 > 0) and np.all(m2 > 0) and np.all(m3 > 0)
    vol = bm.sum()
    assert abs(vol - 1.0) < 1e-6
    a = np.array([0.7, -1.3, 0.4])
    u = a[0] * x + a[1] * y + a[2] * z
    energy = float(np.dot(u, O.ax(u, G, D).reshape(-1)))
    assert abs(energy - np.dot(a, a) * vol) < 1e-12 * np.dot(a, a)


@pytest.mark.parametrize("dims,N", [((2, 2, 2), 3), ((3, 2, 1), 4), ((2, 3, 2), 5)])
def test_dssum_equals_scatter_matrix(dims, N):
    b = S.Brick(*dims, N, ((0.05, 2, 2, 2),) * 3)
    xi, _ = O.gll(N)
    x, y, z = O.brick_coords(b, xi)
    Q = scatter_matrix(x, y, z)
    gid, bnd = O.brick_ids(b)
    gs = O.GS(gid)
    v = S.uniform_field(b.E, N, seed=5).reshape(-1)
    got = gs.dssum(v)
    want = Q @ (Q.T @ v)
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=1e-15)
    # every copy of a global node holds the same bits
    for col in range(Q.shape[1]):
        rows = Q[:, col].nonzero()[0]
        assert np.all(got[rows] == got[rows[0]])
    # ids agree with coordinate identity
    assert len(np.unique(gid)) == Q.shape[1]


def test_multiplicity_and_mask_counts():
    b = S.Brick(3, 4, 5, 4)
    N = b.N
    gid, bnd = O.brick_ids(b)
    gs = O.GS(gid)
    m = gs.multiplicity()
    assert set(np.unique(m)) <= {1.0, 2.0, 4.0, 8.0}
    np.testing.assert_array_equal(gs.dssum(np.ones(b.n_local)), m)
    c = 1.0 / m
    np.testing.assert_allclose(gs.dssum(c), np.ones(b.n_local), rtol=0, atol=1e-15)
    # global nodes: sum of c over local nodes counts each once
    Gx, Gy, Gz = [d * (N - 1) + 1 for d in (b.ex, b.ey, b.ez)]
    assert round(c.sum()) == Gx * Gy * Gz
    # vertices of the element grid shared by 8 elements
    assert np.sum(m == 8) == 8 * (b.ex - 1) * (b.ey - 1) * (b.ez - 1)
    nb_global = Gx * Gy * Gz - (Gx - 2) * (Gy - 2) * (Gz - 2)
    assert round(np.sum(c * bnd)) == nb_global
    v = S.uniform_field(b.E, N, 3).reshape(-1)
    mv = O.mask(bnd, v)
    np.testing.assert_array_equal(O.mask(bnd, mv), mv)
    assert np.all(mv[bnd == 1] == 0) and np.all(mv[bnd == 0] == v[bnd == 0])


@pytest.mark.parametrize("N", [3, 5])
def test_jacobi_diag_brute_force(N):
    b = S.Brick(2, 2, 2, N, ((0.08, 1, 2, 1), (0.05, 2, 1, 1), (0.03, 1, 1, 2)))
    xi, wq = O.gll(N)
    D = O.deriv(N, xi)
    G, _, _ = O.geom(N, D, wq, *O.brick_coords(b, xi))
    d = O.jacobi_diag(G, D).reshape(b.E, -1)
    for e in range(b.E):
        A = dense_element_matrix(G[e], D)
        np.testing.assert_allclose(d[e], np.diag(A), rtol=1e-13, atol=1e-16)


def test_wdot_counts_each_global_node_once():
    b = S.Brick(2, 2, 2, 4)
    xi, _ = O.gll(4)
    x, y, z = O.brick_coords(b, xi)
    Q = scatter_matrix(x, y, z)
    gid, _ = O.brick_ids(b)
    gs = O.GS(gid)
    c = 1.0 / gs.multiplicity()
    rng = np.random.default_rng(0)
    ug = rng.standard_normal(Q.shape[1]); vg = rng.standard_normal(Q.shape[1])
    ul = Q @ ug; vl = Q @ vg
    assert O.wdot(c, ul, vl) == pytest.approx(float(ug @ vg), rel=1e-14)
