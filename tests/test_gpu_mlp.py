"""The BF16 matrix-core kernels of the learned preconditioner's network
against the FP64 reference (oracle/mlp.py).

Operands are rounded to bfloat16 on both sides, so products are exact and
only FP32 accumulation (GEMM: ~K * 2^-24) and the bfloat16 rounding of the
hidden activations (network: ~2^-8 per layer) separate the results."""
import numpy as np
import pytest

import synthetic as S
from oracle import mlp as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_04981_amd as nbx  # noqa: E402


def bf16_tensor(a):
    bits = M.bf16_bits(a).astype(np.int16)
    return torch.from_numpy(bits).view(torch.bfloat16).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_gemm_all_transposes(ta, tb):
    Mm, N, K = 128, 192, 96
    rng = np.random.default_rng(10 + 2 * ta + tb)
    A = rng.standard_normal((K, Mm) if ta else (Mm, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    Ar, Br = M.bf16_round(A), M.bf16_round(B)
    want = (Ar.T if ta else Ar) @ (Br.T if tb else Br)
    got = host(nbx.gemm_bf16(bf16_tensor(A), bf16_tensor(B), bool(ta), bool(tb)))
    assert rel(got, want) <= 2e-6


def test_gemm_rejects_bad_shapes():
    A = bf16_tensor(np.ones((100, 64)))
    B = bf16_tensor(np.ones((64, 64)))
    with pytest.raises(nbx.NbxError):
        nbx.gemm_bf16(A, B)


def _net(B=128, seed=0):
    n_in, n_hid, n_out = 1006, 128, 1000
    shape = M.Shape(n_in, n_hid, n_out)
    params = shape.from_init(S.mlp_init(n_in, n_hid, n_out, seed=seed))
    W1, b1, W2, b2, W3, b3 = shape.unpack(params)
    rng = np.random.default_rng(seed + 1)
    params = shape.pack([W1, rng.normal(0, 0.05, b1.shape), W2, rng.normal(0, 0.05, b2.shape),
                         W3, np.concatenate([rng.normal(0, 0.05, n_out), np.zeros(24)])])
    X, T = S.mlp_batch(B, n_in, n_out, seed=seed + 2)
    Xp = np.zeros((B, shape.in_pad)); Xp[:, :n_in] = X
    Tp = np.zeros((B, shape.out_pad)); Tp[:, :n_out] = T
    net = nbx.Mlp(n_in, n_hid, n_out, max_batch=256)
    assert (net.in_pad, net.out_pad, net.n_params) == (shape.in_pad, shape.out_pad, shape.n_params)
    net.set_params(torch.as_tensor(params, dtype=torch.float32).cuda())
    # the reference sees the GPU's operands: BF16 weights (rounded from the
    # FP32 master copy), FP32 biases, BF16 inputs
    f32 = [a.astype(np.float32).astype(np.float64) for a in shape.unpack(params)]
    pr = shape.pack([M.bf16_round(f32[0]), f32[1], M.bf16_round(f32[2]), f32[3],
                     M.bf16_round(f32[4]), f32[5]])
    return shape, net, params, pr, Xp, Tp


def test_forward_matches_reference():
    shape, net, params, pr, X, T = _net()
    Y = host(net.forward(bf16_tensor(X)))
    _, _, want = M.forward(shape, pr, M.bf16_round(X))
    err = rel(Y[:, :shape.n_out], want[:, :shape.n_out])
    print(f"forward normwise error {err:.2e}")
    assert err <= 2e-2


def test_gradients_match_reference():
    shape, net, params, pr, X, T = _net(seed=5)
    Xt = bf16_tensor(X)
    Tt = torch.as_tensor(T, dtype=torch.float32).cuda()
    loss = host(net.grad(Xt, Tt))[0]
    g = host(net.get_params(grads=True))
    want_loss, want = M.loss_and_grad(shape, pr, M.bf16_round(X), T)
    assert abs(loss - want_loss) <= 1e-2 * want_loss
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], shape.unpack(g),
                          shape.unpack(want)):
        err = rel(a, b)
        print(f"grad {name}: normwise error {err:.2e}")
        assert err <= 5e-2, name


def _close_but_for_flips(got, want, name):
    """got agrees with the rounding-emulating reference but for bfloat16
    rounding flips (an intermediate that lands within the FP32-vs-FP64
    accumulation difference of a rounding boundary rounds the other way on
    one side): the typical entry to 1e-6 of the block's scale, the block as
    a whole to 2^-10 (a quarter of one bfloat16 rounding step) in the
    Frobenius norm, every entry within 2e-3 (a flip moves one operand by
    2^-8 of itself; a weight gradient entry sums many rows, so one flip
    reaches a whole row of it, and the first layer's gradient, fed by the
    flips of both hidden layers, measured 2.9e-4).  A reference without the
    rounding points differs by percents."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    scale = max(np.abs(want).max(), 1e-300)
    d = np.abs(got - want) / scale
    fro = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)
    print(f"{name}: Frobenius {fro:.2e}, max {d.max():.2e}, median {np.median(d):.2e}")
    assert np.median(d) <= 1e-6, name
    assert fro <= 2.0 ** -10, name
    assert d.max() <= 2e-3, name


def test_forward_and_gradients_match_the_rounding_emulating_reference():
    """The same network against a reference that rounds the library's
    bfloat16 operands, hidden activations and back-propagated gradients:
    forward and every gradient block agree but for rare rounding flips."""
    shape, net, params, pr, X, T = _net(seed=7)
    f32 = shape.pack([a.astype(np.float32).astype(np.float64) for a in shape.unpack(params)])
    Xt = bf16_tensor(X)
    Tt = torch.as_tensor(T, dtype=torch.float32).cuda()
    Y = host(net.forward(Xt))
    loss = host(net.grad(Xt, Tt))[0]
    g = host(net.get_params(grads=True))
    want_loss, want, want_Y = M.loss_and_grad_bf16(shape, f32, X, T)
    _close_but_for_flips(Y[:, :shape.n_out], want_Y[:, :shape.n_out], "forward")
    assert abs(loss - want_loss) <= 1e-5 * want_loss
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], shape.unpack(g),
                          shape.unpack(want)):
        _close_but_for_flips(a, b, f"grad {name}")


def test_adam_first_step_and_training_reduces_loss():
    shape, net, params, pr, X, T = _net(seed=9)
    Xt = bf16_tensor(X)
    Tt = torch.as_tensor(T, dtype=torch.float32).cuda()
    p0 = host(net.get_params())
    l0 = host(net.train_step(Xt, Tt, 1e-3))[0]
    g = host(net.get_params(grads=True))
    p1 = host(net.get_params())
    big = np.abs(g) > 1e-3
    np.testing.assert_allclose(np.abs(p1 - p0)[big], 1e-3, rtol=1e-2)
    for _ in range(150):
        l = host(net.train_step(Xt, Tt, 1e-3))[0]
    print(f"loss {l0:.4f} -> {l:.4f}")
    assert l < 0.5 * l0
