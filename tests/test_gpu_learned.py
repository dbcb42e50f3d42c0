"""The learned element-local preconditioner and flexible PCG (nbx_lp_*,
nbx_pcg_learned) against the FP64 reference (oracle/mlp.py, oracle PCG).

Tolerances: the network runs with BF16 operands and BF16 hidden
activations on the GPU; the reference rounds inputs and weights the same
way but keeps FP64 activations, so the learned correction agrees to
~2e-2 normwise (as the network test); everything outside the network
(features, scales, the Jacobi part, dssum, mask) is FP64 or FP32 and agrees
to rounding.  Solves are compared through what is unique: the solution of
A x = b."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from oracle import mlp as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_04981_amd as nbx  # noqa: E402
from paper_2011_04981_amd import learned as LL  # noqa: E402

HID = 64


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _pair(brick, seed=0, out_scale=1.0, bias=0.05):
    """GPU set-up + oracle set-up of one brick, and a network with seeded
    weights (FP32 on the GPU) and the same weights as the reference sees
    them (BF16 W, FP32 b)."""
    N3 = brick.N ** 3
    shape = M.Shape(N3 + 6, HID, N3)
    W1, b1, W2, b2, W3, b3 = shape.unpack(shape.from_init(S.mlp_init(N3 + 6, HID, N3, seed)))
    rng = np.random.default_rng(seed + 7)
    params = shape.pack([W1, rng.normal(0, bias, b1.shape), W2, rng.normal(0, bias, b2.shape),
                         out_scale * W3, out_scale * np.concatenate(
                             [rng.normal(0, bias, N3), np.zeros(shape.out_pad - N3)])])
    net = nbx.Mlp(N3 + 6, HID, N3, max_batch=128)
    net.set_params(cuda(params, torch.float32))
    f32 = [a.astype(np.float32).astype(np.float64) for a in shape.unpack(params)]
    pr = shape.pack([M.bf16_round(f32[0]), f32[1], M.bf16_round(f32[2]), f32[3],
                     M.bf16_round(f32[4]), f32[5]])
    st = nbx.setup_brick(brick.ex, brick.ey, brick.ez, brick.N, brick.deform_array())
    P = O.setup(brick)
    return st, P, net, shape, params, pr


def test_geometric_features_match_reference():
    b = S.scaled_c2_brick(3, 6)
    st, P, net, *_ = _pair(b)
    lp = nbx.LearnedPrecond(st.problem, net)
    g = host(lp.geom_features())
    gf, gd = M.element_features(P.G, b.N)
    np.testing.assert_allclose(g[:, :6], gf, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(g[:, 6], gd, rtol=1e-6)
    assert np.all(g[:, 7] == 0)


@pytest.mark.parametrize("dims,N", [((3, 3, 3), 6), ((4, 3, 2), 5), ((5, 4, 4), 4)])
def test_apply_matches_reference(dims, N):
    b = S.Brick(*dims, N, ((0.05, 2, 2, 2),) * 3)
    print(f"lp apply {dims} N={N}", flush=True)
    st, P, net, shape, params, pr = _pair(b, seed=N)
    lp = nbx.LearnedPrecond(st.problem, net)
    r = S.uniform_field(b.E, N, seed=31 + N)
    r[0] = 0.0                                   # an element with r_e = 0
    z = host(lp.apply(cuda(r)))
    gf, gd = M.element_features(P.G, N)
    want = M.apply_learned(P, shape, pr, r.reshape(-1), gf, gd, round_inputs=True)
    jac = P.dinv * r.reshape(-1)
    err = rel(z.reshape(-1) - jac, want - jac)
    print(f"learned correction normwise error {err:.2e}")
    assert err <= 2e-2
    # Dirichlet nodes stay zero; the correction agrees between the copies
    # of a shared node
    assert np.all(z.reshape(-1)[P.bnd.astype(bool)] == 0)
    zc = z.reshape(-1) - jac
    np.testing.assert_allclose(P.gs.dssum(zc * P.c), zc, rtol=1e-12,
                               atol=1e-14 * np.abs(zc).max())


def test_zero_network_is_jacobi():
    b = S.scaled_c2_brick(3, 8)
    st, P, _, shape, *_ = _pair(b)
    net = nbx.Mlp(b.N ** 3 + 6, HID, b.N ** 3, max_batch=64)      # parameters start at 0
    lp = nbx.LearnedPrecond(st.problem, net)
    r = S.uniform_field(b.E, b.N, seed=3)
    z = host(lp.apply(cuda(r)))
    assert np.array_equal(z, host(st.problem.dinv()) * r)     # exactly the Jacobi step
    x, res = lp.pcg(st.b, rtol=1e-10, max_iter=5000, check_every=5)
    ora = O.pcg(P, max_iter=5000, rtol=1e-10)
    print(f"zero-network FPCG {res.iters} it, Jacobi oracle {ora.iters} it")
    assert res.status == 0 and res.fell_back == 0
    assert abs(res.iters - ora.iters) <= 2
    assert rel(host(x), ora.x) <= 1e-8


def test_samples_match_reference():
    b = S.scaled_c2_brick(3, 6)
    st, P, net, shape, *_ = _pair(b)
    lp = nbx.LearnedPrecond(st.problem, net)
    r = S.uniform_field(b.E, b.N, seed=41)
    xs = S.uniform_field(b.E, b.N, seed=42)
    x = S.uniform_field(b.E, b.N, seed=43)
    r[5] = 0.0
    elems = np.array([0, 5, 26, 3, 3, -1, 27, 11], dtype=np.int32)
    X, T = lp.samples(cuda(r), cuda(xs), cuda(x), cuda(elems, torch.int32))
    X = host(X.float())
    T = host(T)
    gf, gd = M.element_features(P.G, b.N)
    F, s = M.features(r.reshape(-1), gf, gd, b.N, shape.in_pad)
    N3 = b.N ** 3
    for q, e in enumerate(elems):
        if e < 0 or e >= b.E:
            assert np.all(X[q] == 0) and np.all(T[q] == 0)
            continue
        # features: BF16 of the FP64 values (one BF16 ulp for double rounding)
        np.testing.assert_allclose(X[q], M.bf16_round(F[e]), rtol=2 ** -7, atol=1e-30)
        dl = P.dinv.reshape(-1, N3)[e]
        want = (xs[e] - x[e]) - dl * r[e]
        want = want / s[e] if s[e] > 0 else np.zeros(N3)
        np.testing.assert_allclose(T[q, :N3], want, rtol=1e-6, atol=1e-6 * np.abs(want).max())
        assert np.all(T[q, N3:] == 0)


def test_residual_after_fixed_iterations_matches_oracle():
    b = S.scaled_c2_brick(3, 6)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    P = O.setup(b)
    net = nbx.Mlp(b.N ** 3 + 6, HID, b.N ** 3, max_batch=64)
    lp = nbx.LearnedPrecond(st.problem, net)
    st.problem.pcg(st.b, max_iter=12, fixed_iters=1, check_every=4)
    r = host(lp.residual())
    _, r12, *_ = O.pcg_iterate(P, O.pcg_start(P), 12)
    assert rel(r, r12) <= 1e-10


@pytest.mark.parametrize("graph", [1, 0])
def test_learned_fpcg_matches_reference_fpcg(graph):
    b = S.scaled_c2_brick(3, 6)
    # a small random correction keeps <r, M r> > 0 (larger untrained
    # outputs make M indefinite and flexible CG breaks down)
    st, P, net, shape, params, pr = _pair(b, seed=2, out_scale=0.003)
    lp = nbx.LearnedPrecond(st.problem, net)
    gf, gd = M.element_features(P.G, b.N)
    ora_x, ora_it, _ = M.fpcg(P.apply_A,
                              lambda v: M.apply_learned(P, shape, pr, v, gf, gd, True),
                              P.b, P.c, max_iter=3000, rtol=1e-10)
    x, res = lp.pcg(st.b, rtol=1e-10, max_iter=3000, check_every=6, use_graph=graph)
    print(f"learned FPCG: gpu {res.iters} it, reference {ora_it} it, fell back {res.fell_back}")
    assert res.status == 0 and res.fell_back == 0 and res.true_relres <= 1e-9
    assert abs(res.iters - ora_it) <= max(3, ora_it // 10)
    jac = O.pcg(P, max_iter=3000, rtol=1e-10)
    assert rel(host(x), jac.x) <= 1e-8


def test_fallback_reaches_tolerance():
    b = S.scaled_c2_brick(3, 6)
    st, P, net, shape, _, pr = _pair(b, seed=4, out_scale=30.0, bias=1.0)
    lp = nbx.LearnedPrecond(st.problem, net)
    x, res = lp.pcg(st.b, rtol=1e-10, max_iter=5, check_every=5)
    print(f"fallback: {res.iters} it, flag {res.flag}, relres {res.true_relres:.2e}")
    # the reference's flexible CG with this network cannot proceed either
    gf, gd = M.element_features(P.G, b.N)
    with pytest.raises(M.FpcgBreakdown):
        M.fpcg(P.apply_A, lambda v: M.apply_learned(P, shape, pr, v, gf, gd, True), P.b, P.c,
               max_iter=200)
    assert res.fell_back == 1 and res.status == 0 and res.true_relres <= 1e-9
    jac = O.pcg(P, max_iter=3000, rtol=1e-10)
    assert rel(host(x), jac.x) <= 1e-8


def test_training_pipeline_reduces_loss_and_solves():
    bricks = [S.Brick(4, 4, 4, 6, S.deformation_family(s), "random", s, f"t{s}")
              for s in range(3)]
    fac = LL.MeshFactory()
    net = LL.new_network(6, max_batch=256, hidden=HID, seed=1)
    data = LL.collect_samples(fac, bricks, net, n_iterates=4, elems_per_iterate=64, seed=0)
    assert data.rows > 0 and data.rows % 64 == 0
    assert np.all(np.isfinite(host(data.T)))
    losses = LL.train(net, data, epochs=40, batch=64, lr=2e-3)
    print(f"training loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < losses[0]
    ev = LL.evaluate(fac, S.Brick(4, 4, 4, 6, S.deformation_family(99), "sine", 0, "ev"), net,
                     reps=1)
    print(ev)
    assert ev.learned_relres <= 1e-9
    assert ev.learned_iters <= ev.jacobi_iters or ev.fell_back == 1
