"""FP64 reference for the 3-layer perceptron of the learned preconditioner
(oracle/lpi.py builds the preconditioner on it) and for flexible PCG.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The network is not in
the paper; this follows the textbook definitions: a 3-layer perceptron
y = W3 relu(W2 relu(W1 x + b1) + b2) + b3, the chain rule for its gradients
(hand-written, pinned by central finite differences), Adam (Kingma & Ba
2015, pinned by its first-step property), and flexible PCG (Notay 2000,
truncated to one previous direction: the new preconditioned residual is
made A-orthogonal to the last direction, beta = -<z_new, A p> / <p, A p>,
which equals PCG's beta for a fixed SPD preconditioner).

Parameters use one flat arena: W1[hid][in_pad], b1[hid], W2[hid][hid],
b2[hid], W3[out_pad][hid], b3[out_pad] (row-major W[out][in]).
"""
from __future__ import annotations

import numpy as np


def pad64(n: int) -> int:
    return (n + 63) // 64 * 64


class Shape:
    def __init__(self, n_in: int, n_hid: int, n_out: int):
        self.n_in, self.n_hid, self.n_out = n_in, n_hid, n_out
        self.in_pad, self.out_pad = pad64(n_in), pad64(n_out)
        h, i, o = n_hid, self.in_pad, self.out_pad
        self.sizes = [h * i, h, h * h, h, o * h, o]
        self.n_params = sum(self.sizes)

    def unpack(self, p):
        h, i, o = self.n_hid, self.in_pad, self.out_pad
        out, k = [], 0
        for sz, shp in zip(self.sizes, [(h, i), (h,), (h, h), (h,), (o, h), (o,)]):
            out.append(np.asarray(p[k:k + sz], dtype=np.float64).reshape(shp))
            k += sz
        return out

    def pack(self, parts):
        return np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for a in parts])

    def from_init(self, init: dict):
        """Arena from synthetic.mlp_init weights (unpadded), zero-padded."""
        h, i, o = self.n_hid, self.in_pad, self.out_pad
        W1 = np.zeros((h, i)); W1[:, :self.n_in] = init["W1"]
        W3 = np.zeros((o, h)); W3[:self.n_out] = init["W3"]
        b3 = np.zeros(o); b3[:self.n_out] = init["b3"]
        return self.pack([W1, init["b1"], init["W2"], init["b2"], W3, b3])


def relu(a):
    return np.maximum(a, 0.0)


def forward(shape: Shape, params, X):
    """(H1, H2, Y) for X[B][in_pad]."""
    W1, b1, W2, b2, W3, b3 = shape.unpack(params)
    X = np.asarray(X, dtype=np.float64)
    H1 = relu(X @ W1.T + b1)
    H2 = relu(H1 @ W2.T + b2)
    Y = H2 @ W3.T + b3
    return H1, H2, Y


def loss_and_grad(shape: Shape, params, X, T):
    """Mean squared error over the first n_out outputs and its gradient
    with respect to every parameter (chain rule, relu'(0) = 0)."""
    W1, b1, W2, b2, W3, b3 = shape.unpack(params)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    B = X.shape[0]
    H1, H2, Y = forward(shape, params, X)
    D = np.zeros_like(Y)
    D[:, :shape.n_out] = Y[:, :shape.n_out] - T[:, :shape.n_out]
    loss = float(np.sum(D ** 2) / (B * shape.n_out))
    dY = 2.0 * D / (B * shape.n_out)
    dW3 = dY.T @ H2
    db3 = dY.sum(axis=0)
    dH2 = (dY @ W3) * (H2 > 0)
    dW2 = dH2.T @ H1
    db2 = dH2.sum(axis=0)
    dH1 = (dH2 @ W2) * (H1 > 0)
    dW1 = dH1.T @ X
    db1 = dH1.sum(axis=0)
    return loss, shape.pack([dW1, db1, dW2, db2, dW3, db3])


def adam_step(params, grads, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update; returns (params, m, v)."""
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads ** 2
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(a):
    """bfloat16 bit patterns (uint16) of a, ties to even."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


# ------------------------------------------------------------ flexible PCG

class FpcgBreakdown(ArithmeticError):
    """<r, M(r)> or <p, A p> was not positive: the CG step is undefined
    (a preconditioner that is not positive on r)."""

    def __init__(self, iteration: int):
        super().__init__(f"flexible PCG breakdown at iteration {iteration}")
        self.iteration = iteration


def fpcg(apply_A, precond, b, c, x0=None, max_iter=1000, rtol=1e-10, on_step=None):
    """Flexible preconditioned CG with c-weighted dots (Notay 2000 with one
    stored direction): r = b - A x, z = M(r), p = z; per iteration
    w = A p, alpha = <r,z>/<p,w>, x += alpha p, r -= alpha w, z' = M(r),
    beta = -<z', w> / <p, w>, p = z' + beta p, so that every new direction
    is A-orthogonal to the previous one whatever M does.  (For a fixed
    symmetric M this is PCG's <r', z'> / <r, z>.)  ``on_step(k, p, w)`` sees
    each direction and its image.  Returns (x, iterations, relative residual
    history); raises FpcgBreakdown when <r, z> or <p, w> is not positive."""
    def dot(a, b_):
        return float(np.sum(c * a * b_))
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    z = precond(r)
    p = z.copy()
    rho = dot(r, z)
    bb = dot(b, b)
    hist = []
    if not rho > 0:
        raise FpcgBreakdown(0)
    for k in range(max_iter):
        w = apply_A(p)
        if on_step is not None:
            on_step(k, p, w)
        pw = dot(p, w)
        if not pw > 0:
            raise FpcgBreakdown(k)
        alpha = rho / pw
        x += alpha * p
        r -= alpha * w
        rel = np.sqrt(dot(r, r) / bb)
        hist.append(rel)
        if rel <= rtol:
            return x, k + 1, np.array(hist)
        z = precond(r)
        rho = dot(r, z)
        if not rho > 0:
            raise FpcgBreakdown(k + 1)
        beta = -dot(z, w) / pw
        p = z + beta * p
    return x, max_iter, np.array(hist)


def loss_and_grad_bf16(shape: Shape, params, X, T, rnd=None):
    """loss_and_grad (and the output) with the library's bfloat16 rounding
    points: the products take X, the weights, the hidden activations, the
    output gradient and the back-propagated hidden gradients rounded to
    bfloat16 (FP64 accumulation here, FP32 in the library); bias gradients
    sum the unrounded output gradient and the rounded hidden ones, as the
    library's column sums do.  Returns (loss, gradient arena, Y).  rnd
    replaces the rounding (the identity gives loss_and_grad back)."""
    r = bf16_round if rnd is None else rnd
    W1, b1, W2, b2, W3, b3 = shape.unpack(params)
    Xr = r(X)
    W1r, W2r, W3r = r(W1), r(W2), r(W3)
    T = np.asarray(T, dtype=np.float64)
    B = Xr.shape[0]
    H1 = r(relu(Xr @ W1r.T + b1))
    H2 = r(relu(H1 @ W2r.T + b2))
    Y = H2 @ W3r.T + b3
    D = np.zeros_like(Y)
    D[:, :shape.n_out] = Y[:, :shape.n_out] - T[:, :shape.n_out]
    loss = float(np.sum(D ** 2) / (B * shape.n_out))
    dY = 2.0 * D / (B * shape.n_out)
    dYr = r(dY)
    dW3 = dYr.T @ H2
    db3 = dY.sum(axis=0)
    dH2 = r((dYr @ W3r) * (H2 > 0))
    dW2 = dH2.T @ H1
    db2 = dH2.sum(axis=0)
    dH1 = r((dH2 @ W2r) * (H1 > 0))
    dW1 = dH1.T @ Xr
    db1 = dH1.sum(axis=0)
    return loss, shape.pack([dW1, db1, dW2, db2, dW3, db3]), Y
