"""Pins for the FP64 reference network, Adam, bfloat16 rounding and
flexible PCG (oracle/mlp.py)."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
import synthetic as S


def _small():
    shape = M.Shape(20, 64, 10)
    init = S.mlp_init(20, 64, 10, seed=3)
    params = shape.from_init(init)
    # biases nonzero so that their gradients are exercised too
    rng = np.random.default_rng(4)
    W1, b1, W2, b2, W3, b3 = shape.unpack(params)
    params = shape.pack([W1, rng.normal(0, 0.1, b1.shape), W2, rng.normal(0, 0.1, b2.shape),
                         W3, rng.normal(0, 0.1, b3.shape)])
    X, T = S.mlp_batch(8, 20, 10, seed=5)
    Xp = np.zeros((8, shape.in_pad)); Xp[:, :20] = X
    Tp = np.zeros((8, shape.out_pad)); Tp[:, :10] = T
    return shape, params, Xp, Tp


def test_gradient_matches_central_differences():
    shape, params, X, T = _small()
    loss, g = M.loss_and_grad(shape, params, X, T)
    rng = np.random.default_rng(6)
    # parameters that influence the loss (padded columns/rows do not)
    live = np.ones(shape.n_params, bool)
    W1m = np.zeros((shape.n_hid, shape.in_pad), bool); W1m[:, :shape.n_in] = True
    W3m = np.zeros((shape.out_pad, shape.n_hid), bool); W3m[:shape.n_out] = True
    b3m = np.zeros(shape.out_pad, bool); b3m[:shape.n_out] = True
    live = shape.pack([W1m, np.ones(shape.n_hid), np.ones((shape.n_hid, shape.n_hid)),
                       np.ones(shape.n_hid), W3m, b3m]).astype(bool)
    idx = rng.choice(np.where(live)[0], size=80, replace=False)
    h = 1e-6
    for q in idx:
        pp = params.copy(); pp[q] += h
        pm = params.copy(); pm[q] -= h
        fd = (M.loss_and_grad(shape, pp, X, T)[0] - M.loss_and_grad(shape, pm, X, T)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (q, fd, g[q])
    # padded entries have exactly zero gradient
    assert np.all(g[~live] == 0.0)


def test_adam_first_step_moves_every_parameter_by_lr():
    shape, params, X, T = _small()
    _, g = M.loss_and_grad(shape, params, X, T)
    m = np.zeros_like(params); v = np.zeros_like(params)
    new, m, v = M.adam_step(params, g, m, v, 1, lr=1e-3)
    big = np.abs(g) > 1e-4
    np.testing.assert_allclose(np.abs(new - params)[big], 1e-3, rtol=1e-3)
    assert np.all(np.sign(params - new)[big] == np.sign(g[big]))


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.0e-3, 65504.0])
    r = M.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                     # tie -> even
    assert r[2] == 1.0 + 2 ** -6           # 1.0117 -> 1.015625 (tie -> even)
    assert r[3] == -2.5
    assert abs(r[4] - 3.0e-3) <= 3.0e-3 * 2 ** -8
    bits = M.bf16_bits(np.array([1.0, -2.0]))
    assert list(bits) == [0x3F80, 0xC000]


def test_fpcg_with_jacobi_equals_pcg():
    P = O.setup(S.scaled_c2_brick(3, 6))
    ref = O.pcg(P, max_iter=2000, rtol=1e-10)
    x, it, hist = M.fpcg(P.apply_A, lambda r: P.dinv * r, P.b, P.c, max_iter=2000, rtol=1e-10)
    assert abs(it - ref.iters) <= 1
    assert np.abs(x - ref.x).max() <= 1e-9 * np.abs(ref.x).max()


def test_fpcg_keeps_directions_conjugate_under_a_varying_preconditioner():
    """Notay's flexible CG with one stored direction A-orthogonalises each new
    preconditioned residual against the previous direction, so consecutive
    directions stay A-conjugate even when M changes every step.  A diagonal
    preconditioner dinv (1 + 0.8 u_k), u_k ~ U[-1, 1] drawn afresh per step
    (averaged over shared copies, so z stays consistent), is SPD at every
    step but different each time: PCG's beta <r', z'>/<r, z> loses conjugacy
    (and does not converge in 5000 steps on this mesh), as does the variant
    <r', z' - z>/<r, z>; both fail this test."""
    P = O.setup(S.scaled_c2_brick(3, 6))
    rng = np.random.default_rng(11)
    draws = []

    def varying(r):
        u = rng.uniform(-1.0, 1.0, size=P.n)
        draws.append(1)
        return O.mask(P.bnd, P.gs.dssum(P.c * P.dinv * (1.0 + 0.8 * u) * r))

    steps = []
    x, it, hist = M.fpcg(P.apply_A, varying, P.b, P.c, max_iter=2000, rtol=1e-10,
                         on_step=lambda k, p, w: steps.append((p.copy(), w.copy())))
    assert hist[-1] <= 1e-10 and it < 2000
    # the solution is the assembled system's (checked by the oracle's PCG)
    ref = O.pcg(P, max_iter=2000, rtol=1e-12)
    assert np.abs(x - ref.x).max() <= 1e-8 * np.abs(ref.x).max()
    for (p0, w0), (p1, w1) in zip(steps[:40], steps[1:41]):
        a01 = O.wdot(P.c, p1, w0)
        n0 = np.sqrt(O.wdot(P.c, p0, w0))
        n1 = np.sqrt(O.wdot(P.c, p1, w1))
        assert abs(a01) <= 1e-8 * n0 * n1, abs(a01) / (n0 * n1)


def test_fpcg_detects_breakdown():
    # M = -Jacobi is negative definite: <r, M r> < 0 at once
    P = O.setup(S.scaled_c2_brick(2, 4))
    with pytest.raises(M.FpcgBreakdown) as ei:
        M.fpcg(P.apply_A, lambda r: -P.dinv * r, P.b, P.c, max_iter=50)
    assert ei.value.iteration == 0
    # a preconditioner that turns indefinite after the first step
    calls = []

    def flip(r):
        calls.append(1)
        return P.dinv * r if len(calls) == 1 else -P.dinv * r
    with pytest.raises(M.FpcgBreakdown) as ei:
        M.fpcg(P.apply_A, flip, P.b, P.c, max_iter=50)
    assert ei.value.iteration == 1


def test_rounding_emulation_without_rounding_is_the_chain_rule():
    """The rounding-emulating gradient with the rounding switched off is
    the exact chain rule (every term and transpose in it is the same); with
    bfloat16 rounding the forward pass stays within the bfloat16 bound."""
    shape, params, X, T = _small()
    l0, g0 = M.loss_and_grad(shape, params, X, T)
    l1, g1, Y1 = M.loss_and_grad_bf16(shape, params, X, T, rnd=lambda a: a)
    _, _, Y0 = M.forward(shape, params, X)
    np.testing.assert_allclose(Y1, Y0, rtol=1e-14, atol=1e-14)
    assert abs(l1 - l0) <= 1e-14 * l0
    np.testing.assert_allclose(g1, g0, rtol=1e-12, atol=1e-15)
    _, _, Yb = M.loss_and_grad_bf16(shape, params, X, T)
    assert np.abs(Yb - Y0).max() <= 2 ** -5 * np.abs(Y0).max()
