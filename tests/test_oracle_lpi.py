"""Pins for the learned element-interior preconditioner's FP64 reference
(oracle/lpi.py): index set by brute force, exactness against the brute-force
dense element matrix, symmetry and positivity of the operator, linearity and
geometric scale, the hand-written gradient against central differences, and
the closed form of the untrained map."""
import numpy as np
import pytest

import oracle as O
from oracle import lpi, mlp as M
import synthetic as S
from brute import dense_element_matrix


def test_interior_index_by_brute_force():
    for N in (2, 3, 4, 7):
        want = [i + N * (j + N * k) for k in range(N) for j in range(N) for i in range(N)
                if 0 < i < N - 1 and 0 < j < N - 1 and 0 < k < N - 1]
        assert list(lpi.interior_index(N)) == want
    assert list(lpi.interior_index(3)) == [13]


def _interior_block(G_e, D, N):
    idx = lpi.interior_index(N)
    return dense_element_matrix(G_e, D)[np.ix_(idx, idx)]


def _affine(N, n=3):
    P = O.setup(S.Brick(n, n, n, N, S.NO_DEFORM, "random", 5),
                rhs_values=S.rhs_values(S.Brick(n, n, n, N, S.NO_DEFORM, "random", 5)))
    return P


@pytest.mark.parametrize("N", [4, 5, 6])
def test_exact_parameters_invert_the_interior_block(N):
    """On a uniform affine brick every element has the same interior block
    A_SS (from the brute-force dense element matrix); parameters built from
    the eigenpairs of gd A_SS^-1 make the learned part of M its exact
    inverse: A_SS z_S = r_S on every element, Jacobi everywhere else."""
    P = _affine(N)
    shape = lpi.Shape(N, n_hid=16)
    F, gd = lpi.geom_features(P.G, N)
    A = _interior_block(P.G[0], P.D, N)
    prm = lpi.exact_params(shape, A, gd[0])
    r = S.uniform_field(P.E, N, seed=3).reshape(-1) * (1 - P.bnd)
    z = lpi.apply(P, shape, prm, r).reshape(P.E, N ** 3)
    idx = lpi.interior_index(N)
    R = r.reshape(P.E, N ** 3)
    for e in range(P.E):
        np.testing.assert_allclose(A @ z[e, idx], R[e, idx], rtol=0, atol=1e-11 * np.abs(R).max())
    rest = np.setdiff1d(np.arange(N ** 3), idx)
    np.testing.assert_array_equal(z[:, rest], (P.dinv * r).reshape(P.E, N ** 3)[:, rest])
    # an orientation slip (L for L^T) is not an inverse
    L, *rest_p = shape.unpack(prm)
    bad = shape.pack([L.T, *rest_p])
    zb = lpi.apply(P, shape, bad, r).reshape(P.E, N ** 3)
    assert np.abs(A @ zb[0, idx] - R[0, idx]).max() > 1e-3 * np.abs(R).max()


def test_training_rows_are_fitted_exactly_by_the_inverse():
    """Rows built from solver vectors satisfy T = gd A_SS^-1 X: the exact
    parameters give a loss at rounding level, the untrained ones do not."""
    N = 5
    P = _affine(N)
    shape = lpi.Shape(N, n_hid=16)
    F, gd = lpi.geom_features(P.G, N)
    A = _interior_block(P.G[0], P.D, N)
    prm = lpi.exact_params(shape, A, gd[0])
    st = O.pcg_iterate(P, O.pcg_start(P), 7)
    xs = O.pcg(P, max_iter=2000, rtol=1e-13).x
    for v in (xs - st[0], st[1]):
        X, T, Fr, ok = lpi.sample_rows(P, v)
        assert X.shape[0] == ok.size > 0
        np.testing.assert_allclose(np.linalg.norm(T, axis=1), 1.0, rtol=1e-14)
        loss, _ = lpi.loss_and_grad(shape, prm, X, T, Fr)
        assert loss <= 1e-24, loss
        loss0, _ = lpi.loss_and_grad(shape, lpi.init_params(shape, 0.01), X, T, Fr)
        assert loss0 > 1e-6


def _random_params(shape, seed=7):
    rng = np.random.default_rng(seed)
    L, W1, b1, W2, b2, W3, b3 = shape.unpack(lpi.init_params(shape, 0.02, seed=seed))
    L = L + 0.3 * rng.standard_normal(L.shape)
    W3 = 0.2 * rng.standard_normal(W3.shape)
    b1 = 0.1 * rng.standard_normal(b1.shape)
    b2 = 0.1 * rng.standard_normal(b2.shape)
    return shape.pack([L, W1, b1, W2, b2, W3, b3])


def test_operator_is_symmetric_positive_linear_and_scales_with_the_geometry():
    b = S.Brick(3, 2, 2, 6, ((0.08, 2, 1, 3), (0.05, 1, 2, 2), (0.06, 3, 3, 1)))
    P = O.setup(b)
    shape = lpi.Shape(6, n_hid=32)
    prm = _random_params(shape)
    rng = np.random.default_rng(1)

    def consistent(seed):
        v = rng.standard_normal(P.n)
        return O.mask(P.bnd, P.gs.dssum(P.c * v))

    r, v = consistent(1), consistent(2)
    Mr, Mv = lpi.apply(P, shape, prm, r), lpi.apply(P, shape, prm, v)
    a, bb = O.wdot(P.c, v, Mr), O.wdot(P.c, Mv, r)
    assert abs(a - bb) <= 1e-12 * (abs(a) + abs(bb))
    for q in range(5):
        x = consistent(10 + q)
        assert O.wdot(P.c, x, lpi.apply(P, shape, prm, x)) > 0
    np.testing.assert_allclose(lpi.apply(P, shape, prm, 3.7 * r), 3.7 * Mr,
                               rtol=1e-13, atol=1e-13 * np.abs(Mr).max())
    # G -> lam G: the features are unchanged, gd -> lam gd, dinv -> dinv / lam
    lam = 8.0

    class Scaled:
        pass
    Q = Scaled()
    for k, val in vars(P).items():
        setattr(Q, k, val)
    Q.G, Q.dinv = P.G * lam, P.dinv / lam
    np.testing.assert_allclose(lpi.apply(Q, shape, prm, r), Mr / lam,
                               rtol=1e-13, atol=1e-13 * np.abs(Mr).max())


def test_untrained_map_closed_form():
    """L = identity and a perceptron that outputs zero: gamma = log 2, so the
    learned nodes get (log 2 / gd_e) r and the others Jacobi."""
    b = S.Brick(2, 2, 2, 5, ((0.05, 2, 2, 2),) * 3)
    P = O.setup(b)
    shape = lpi.Shape(5, n_hid=16)
    h, K, n = shape.n_hid, shape.K, shape.nI
    prm = shape.pack([np.eye(K, n), np.zeros((h, 6)), np.zeros(h), np.zeros((h, h)),
                      np.zeros(h), np.zeros((K, h)), np.zeros(K)])
    r = S.uniform_field(b.E, 5, seed=4).reshape(-1) * (1 - P.bnd)
    z = lpi.apply(P, shape, prm, r).reshape(b.E, 125)
    F, gd = lpi.geom_features(P.G, 5)
    idx = lpi.interior_index(5)
    np.testing.assert_allclose(z[:, idx], np.log(2.0) * r.reshape(b.E, 125)[:, idx] / gd[:, None],
                               rtol=1e-15)


def test_gradient_matches_central_differences():
    N = 4
    P = O.setup(S.Brick(2, 2, 1, N, ((0.07, 2, 1, 1), (0.04, 1, 1, 2), (0.05, 1, 2, 1))))
    shape = lpi.Shape(N, n_hid=16)
    prm = _random_params(shape, seed=3)
    v = S.uniform_field(P.E, N, seed=9).reshape(-1)
    X, T, F, _ = lpi.sample_rows(P, v)
    rng = np.random.default_rng(8)
    T = T + 0.1 * rng.standard_normal(T.shape)
    loss, g = lpi.loss_and_grad(shape, prm, X, T, F)
    idx = np.concatenate([rng.choice(shape.n_params, 60, replace=False),
                          np.arange(shape.sizes[0])[:5]])
    h = 1e-6
    for q in idx:
        pp = prm.copy(); pp[q] += h
        pm = prm.copy(); pm[q] -= h
        fd = (lpi.loss_and_grad(shape, pp, X, T, F)[0] -
              lpi.loss_and_grad(shape, pm, X, T, F)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(abs(fd), 1e-3 * abs(loss)) + 1e-12, (q, fd, g[q])


def test_bf16_operands_perturb_at_bfloat16_level():
    N = 5
    P = O.setup(S.Brick(2, 2, 2, N, ((0.05, 2, 2, 2),) * 3))
    shape = lpi.Shape(N, n_hid=32)
    prm = _random_params(shape, seed=5)
    r = S.uniform_field(P.E, N, seed=6).reshape(-1) * (1 - P.bnd)
    z = lpi.apply(P, shape, prm, r)
    zb = lpi.apply(P, shape, prm, r, bf16=True)
    err = np.abs(zb - z).max() / np.abs(z).max()
    assert 1e-5 < err < 2 ** -5


def test_flexible_cg_with_exact_interior_inverse_beats_jacobi():
    """The learned part at its exact optimum on an affine brick: the flexible
    CG converges to the assembled solution in fewer iterations than
    Jacobi-PCG."""
    N = 6
    b = S.Brick(4, 4, 3, N, S.NO_DEFORM, "random", 2)
    P = O.setup(b, rhs_values=S.rhs_values(b))
    shape = lpi.Shape(N, n_hid=16)
    F, gd = lpi.geom_features(P.G, N)
    prm = lpi.exact_params(shape, _interior_block(P.G[0], P.D, N), gd[0])
    ref = O.pcg(P, max_iter=3000, rtol=1e-10)
    x, it, hist = M.fpcg(P.apply_A, lambda r: lpi.apply(P, shape, prm, r), P.b, P.c,
                         max_iter=3000, rtol=1e-10)
    assert hist[-1] <= 1e-10
    assert it <= 0.8 * ref.iters, (it, ref.iters)
    assert np.abs(x - ref.x).max() <= 1e-8 * np.abs(ref.x).max()


def test_geometry_features_closed_form():
    """Affine brick with element sides hx, hy, hz: G_rr = W hy hz / (2 hx)
    and cyclically, cross factors 0, and the element mean of W = w_i w_j w_k
    is (2/N)^3 (the GLL weights sum to 2)."""
    N, (ex, ey, ez) = 5, (2, 3, 4)
    P = O.setup(S.Brick(ex, ey, ez, N))
    F, gd = lpi.geom_features(P.G, N)
    hx, hy, hz = 1 / ex, 1 / ey, 1 / ez
    mw = (2.0 / N) ** 3
    diag = np.array([hy * hz / (2 * hx), hx * hz / (2 * hy), hx * hy / (2 * hz)]) * mw
    np.testing.assert_allclose(gd, diag.mean(), rtol=1e-13)
    np.testing.assert_allclose(F[:, [0, 3, 5]], np.broadcast_to(diag / diag.mean(), (P.E, 3)),
                               rtol=1e-13)
    np.testing.assert_allclose(F[:, [1, 2, 4]], 0.0, atol=1e-14)


def test_shared_interior_node_keeps_jacobi_and_symmetry():
    """A plan that identifies an interior node of element 1 with the same
    node of element 0 (a valid SPD assembly): that node has two copies, so
    it is not learned in either element, and the operator stays symmetric
    in the 1/multiplicity-weighted dot product."""
    import dataclasses
    N = 5
    b = S.Brick(2, 1, 1, N, ((0.05, 2, 2, 2),) * 3)
    P0 = O.setup(b)
    q = 2 + N * (2 + N * 2)                      # node (2, 2, 2)
    gid = P0.gid.copy()
    gid[N ** 3 + q] = gid[q]
    gs = O.GS(gid)
    mult = gs.multiplicity()
    d = gs.dssum(O.jacobi_diag(P0.G, P0.D))
    P = dataclasses.replace(P0, gid=gid, gs=gs, mult=mult, c=1.0 / mult,
                            dinv=np.where(P0.bnd.astype(bool), 0.0, 1.0 / d))
    S_ = lpi.learned_mask(P)
    k = int(np.nonzero(lpi.interior_index(N) == q)[0][0])
    assert not S_[0, k] and not S_[1, k] and S_.sum() == 2 * (N - 2) ** 3 - 2
    shape = lpi.Shape(N, n_hid=16)
    prm = _random_params(shape, seed=11)
    rng = np.random.default_rng(3)
    r = O.mask(P.bnd, gs.dssum(P.c * rng.standard_normal(P.n)))
    v = O.mask(P.bnd, gs.dssum(P.c * rng.standard_normal(P.n)))
    z = lpi.apply(P, shape, prm, r)
    assert z[q] == z[N ** 3 + q] == P.dinv[q] * r[q]
    a, bb = O.wdot(P.c, v, z), O.wdot(P.c, lpi.apply(P, shape, prm, v), r)
    assert abs(a - bb) <= 1e-12 * (abs(a) + abs(bb))


def test_bf16_gradient_stays_within_the_bfloat16_bound_of_the_exact_one():
    """The rounding-emulating gradient (the library's operand roundings) is
    the exact chain rule when the rounding is switched off, and differs
    from it by the bfloat16 round-off, not more, when it is on."""
    N = 5
    P = O.setup(S.Brick(2, 2, 2, N, ((0.05, 2, 2, 2),) * 3))
    shape = lpi.Shape(N, n_hid=32)
    prm = _random_params(shape, seed=13)
    X, T, F, _ = lpi.sample_rows(P, S.uniform_field(P.E, N, seed=3).reshape(-1))
    l0, g0 = lpi.loss_and_grad(shape, prm, X, T, F)
    lx, gx = lpi.loss_and_grad_bf16(shape, prm, X, T, F, rnd=lambda a: a)
    assert abs(lx - l0) <= 1e-14 * l0
    np.testing.assert_allclose(gx, g0, rtol=1e-12, atol=1e-15)
    l1, g1 = lpi.loss_and_grad_bf16(shape, prm, X, T, F)
    assert abs(l1 - l0) <= 2 ** -6 * l0
    for a, b in zip(shape.unpack(g1), shape.unpack(g0)):
        assert np.abs(a - b).max() <= 2 ** -4 * np.abs(b).max()
