"""FP64 reference for the learned element-interior preconditioner.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The learned part is not
in the paper; this module writes out the definitions the library's kernels
follow, in plain numpy.

Preconditioner (a fixed, symmetric positive definite operator):
  * every local node that is not a "learned" node keeps Jacobi,
    z_l = dinv_l r_l;
  * the learned nodes of element e are its interior nodes (1 <= i,j,k <= N-2)
    that have one copy and are not on the Dirichlet boundary; on them
        z_S = (1/gd_e) L^T diag(gamma_e) L r_S,
    with L a K x nI matrix shared by all elements (nI = (N-2)^3 interior
    nodes, row-major over the interior's own (i,j,k), i fastest) and
    gamma_e = softplus(f(g_e)) > 0 from a 3-layer perceptron
    f(g) = W3 relu(W2 relu(W1 g + b1) + b2) + b3 on the six element-mean
    geometric factors divided by gd_e, the element mean of the diagonal
    factors (g1 + g4 + g6) / 3.  Inputs outside S are taken as zero and the
    outputs outside S discarded, so z_S depends on r_S only.
  L^T diag(gamma) L is symmetric and positive semidefinite for any L and
  positive gamma (definite when L has full column rank), and the learned
  nodes of different elements are disjoint, so the whole operator is
  symmetric in the 1/multiplicity-weighted dot product; a zero perceptron
  output and L = identity give gamma = log 2 on S.

Training rows: for a vector v that the FP64 solver produced (an error
x* - x_k or a residual r_k), per element with v_S != 0:
    X = A_SS v_S / (||v_S|| gd_e),  T = v_S / ||v_S||,  F = g_e / gd_e,
where A_SS is the element matrix restricted to S (AX of v with every node
outside S set to zero, read on S).  A model with
L^T diag(gamma) L = gd_e A_SS^{-1} fits these rows exactly.  Loss: mean
squared error over the rows and the nI outputs.
"""
from __future__ import annotations

import numpy as np

from . import ax
from .mlp import bf16_round


def interior_index(N: int) -> np.ndarray:
    """Local node numbers (i + N(j + N k)) of the interior nodes, in the
    interior's own row-major order (i fastest)."""
    if N < 3:
        return np.zeros(0, dtype=np.int64)
    r = np.arange(1, N - 1)
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    return (i + N * (j + N * k)).reshape(-1).astype(np.int64)


def learned_mask(P) -> np.ndarray:
    """[E][nI] booleans: interior nodes with a single copy, off the
    Dirichlet set."""
    N = P.N
    idx = interior_index(N)
    mult = P.mult.reshape(P.E, N ** 3)[:, idx]
    bnd = P.bnd.reshape(P.E, N ** 3)[:, idx]
    return (mult == 1) & (bnd == 0)


def geom_features(G, N: int):
    """(F [E][6], gd [E]): element means of the six factors over gd, and gd
    (the element mean of the three diagonal factors)."""
    G = np.asarray(G, dtype=np.float64).reshape(-1, 6, N ** 3)
    m = G.mean(axis=2)
    gd = (m[:, 0] + m[:, 3] + m[:, 5]) / 3.0
    return m / gd[:, None], gd


class Shape:
    """Parameter layout: L [K][nI], W1 [hid][6], b1 [hid], W2 [hid][hid],
    b2 [hid], W3 [K][hid], b3 [K] (row-major W[out][in])."""

    def __init__(self, N: int, n_hid: int = 128, K: int | None = None):
        self.N = N
        self.nI = max(N - 2, 0) ** 3
        self.K = self.nI if K is None else K
        self.n_hid = n_hid
        h, K, n = n_hid, self.K, self.nI
        self.shapes = [(K, n), (h, 6), (h,), (h, h), (h,), (K, h), (K,)]
        self.sizes = [int(np.prod(s)) for s in self.shapes]
        self.n_params = sum(self.sizes)

    def unpack(self, p):
        out, q = [], 0
        for sz, shp in zip(self.sizes, self.shapes):
            out.append(np.asarray(p[q:q + sz], dtype=np.float64).reshape(shp))
            q += sz
        return out

    def pack(self, parts):
        return np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for a in parts])


def softplus(a):
    """log(1 + e^a), evaluated without overflow."""
    a = np.asarray(a, dtype=np.float64)
    return np.log1p(np.exp(-np.abs(a))) + np.maximum(a, 0.0)


def softplus_inv(y):
    """The a with softplus(a) = y > 0."""
    y = np.asarray(y, dtype=np.float64)
    return y + np.log(-np.expm1(-y))


def sigmoid(a):
    return 1.0 / (1.0 + np.exp(-np.asarray(a, dtype=np.float64)))


def _relu(a):
    return np.maximum(a, 0.0)


def gains(shape: Shape, params, F, bf16=False):
    """gamma [B][K] = softplus(f(F)) and the perceptron's intermediates
    (H1, H2, A).  With bf16 the perceptron's operands (F, weights, hidden
    activations) are rounded to bfloat16 as the library's matrix-core
    products take them."""
    L, W1, b1, W2, b2, W3, b3 = shape.unpack(params)
    F = np.asarray(F, dtype=np.float64)
    r = bf16_round if bf16 else (lambda a: a)
    H1 = r(_relu(r(F) @ r(W1).T + b1))
    H2 = r(_relu(H1 @ r(W2).T + b2))
    A = H2 @ r(W3).T + b3
    return softplus(A), (H1, H2, A)


def apply_rows(shape: Shape, params, X, gamma, bf16=False):
    """Z = ((X L^T) * gamma) L for rows X [B][nI]: the map before the 1/gd
    scale.  With bf16, X, L and the scaled hidden rows are rounded to
    bfloat16 (the library's operands)."""
    L = shape.unpack(params)[0]
    r = bf16_round if bf16 else (lambda a: a)
    Lr = r(L)
    Q = r((r(X) @ Lr.T) * gamma)
    return Q @ Lr


def apply(P, shape: Shape, params, r, bf16=False):
    """z = M r for a local vector r (FP64; see the module docstring)."""
    N = P.N
    idx = interior_index(N)
    S = learned_mask(P)
    F, gd = geom_features(P.G, N)
    gamma, _ = gains(shape, params, F, bf16=bf16)
    R = np.asarray(r, dtype=np.float64).reshape(P.E, N ** 3)
    Z = (P.dinv * np.asarray(r, dtype=np.float64).reshape(-1)).reshape(P.E, N ** 3)
    XS = np.where(S, R[:, idx], 0.0)
    ZS = apply_rows(shape, params, XS, gamma, bf16=bf16) / gd[:, None]
    Zi = Z[:, idx]
    Zi[S] = ZS[S]
    Z[:, idx] = Zi
    return Z.reshape(-1)


def loss_and_grad(shape: Shape, params, X, T, F):
    """Mean squared error of apply_rows(X) against T over B rows and nI
    outputs, and its gradient with respect to every parameter (chain rule;
    relu'(0) = 0, softplus' = sigmoid)."""
    L, W1, b1, W2, b2, W3, b3 = shape.unpack(params)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    B, n = X.shape[0], shape.nI
    gamma, (H1, H2, A) = gains(shape, params, F)
    Hx = X @ L.T                     # [B][K]
    Q = Hx * gamma
    Z = Q @ L                        # [B][nI]
    Dl = Z - T
    loss = float(np.sum(Dl ** 2) / (B * n))
    dZ = 2.0 * Dl / (B * n)
    Pm = dZ @ L.T                    # gradient with respect to Q
    dL = Q.T @ dZ + (gamma * Pm).T @ X
    dA = Hx * Pm * sigmoid(A)
    dW3 = dA.T @ H2
    db3 = dA.sum(axis=0)
    dH2 = (dA @ W3) * (H2 > 0)
    dW2 = dH2.T @ H1
    db2 = dH2.sum(axis=0)
    dH1 = (dH2 @ W2) * (H1 > 0)
    dW1 = dH1.T @ np.asarray(F, dtype=np.float64)
    db1 = dH1.sum(axis=0)
    return loss, shape.pack([dL, dW1, db1, dW2, db2, dW3, db3])


def sample_rows(P, v):
    """Training rows (X, T, F) from one solver vector v (local, [E N^3]) for
    every element whose learned part of v is not zero (see the module
    docstring)."""
    N = P.N
    idx = interior_index(N)
    S = learned_mask(P)
    F, gd = geom_features(P.G, N)
    V = np.asarray(v, dtype=np.float64).reshape(P.E, N ** 3)
    VS = np.where(S, V[:, idx], 0.0)
    Vl = np.zeros_like(V)
    Vl[:, idx] = VS
    Y = ax(Vl, P.G, P.D)[:, idx]
    Y = np.where(S, Y, 0.0)
    nrm = np.sqrt(np.sum(VS ** 2, axis=1))
    ok = nrm > 0
    X = Y[ok] / (nrm[ok] * gd[ok])[:, None]
    T = VS[ok] / nrm[ok][:, None]
    return X, T, F[ok], np.nonzero(ok)[0]


def init_params(shape: Shape, s0: float, seed: int = 0):
    """L = identity (K = nI), perceptron weights He-uniform with W3 = 0,
    b1 = b2 = 0, b3 = softplus^-1(s0): gamma = s0 everywhere."""
    rng = np.random.default_rng(seed)
    h, K, n = shape.n_hid, shape.K, shape.nI
    L = np.eye(K, n)
    W1 = rng.uniform(-np.sqrt(6.0 / 6), np.sqrt(6.0 / 6), size=(h, 6))
    W2 = rng.uniform(-np.sqrt(6.0 / h), np.sqrt(6.0 / h), size=(h, h))
    return shape.pack([L, W1, np.zeros(h), W2, np.zeros(h), np.zeros((K, h)),
                       np.full(K, float(softplus_inv(s0)))])


def exact_params(shape: Shape, A_ref: np.ndarray, gd_ref: float):
    """Parameters for which L^T diag(gamma) L = gd_ref A_ref^{-1} on every
    element (W3 = 0, so gamma does not depend on the geometry): L the
    eigenvectors of the scaled inverse as rows, gamma its eigenvalues."""
    Minv = np.linalg.inv(np.asarray(A_ref, dtype=np.float64) / gd_ref)
    Minv = 0.5 * (Minv + Minv.T)
    lam, V = np.linalg.eigh(Minv)
    h = shape.n_hid
    return shape.pack([V.T, np.zeros((h, 6)), np.zeros(h), np.zeros((h, h)), np.zeros(h),
                       np.zeros((shape.K, h)), softplus_inv(lam)])


def loss_and_grad_bf16(shape: Shape, params, X, T, F, rnd=None):
    """loss_and_grad with the library's bfloat16 operand roundings: the
    products take X, F, L, the perceptron's weights and hidden activations,
    Q = Hx * gamma, the output gradient dZ, gamma * Pm and the perceptron's
    back-propagated gradients rounded to bfloat16 (FP64 accumulation here,
    FP32 in the library); bias gradients sum the unrounded dA and the
    rounded hidden gradients, as the library's column sums do.  rnd
    replaces the rounding (the identity gives loss_and_grad back)."""
    r = bf16_round if rnd is None else rnd
    L, W1, b1, W2, b2, W3, b3 = shape.unpack(params)
    Xr, Fr, Lr = r(X), r(F), r(L)
    W1r, W2r, W3r = r(W1), r(W2), r(W3)
    T = np.asarray(T, dtype=np.float64)
    B, n = Xr.shape[0], shape.nI
    H1 = r(_relu(Fr @ W1r.T + b1))
    H2 = r(_relu(H1 @ W2r.T + b2))
    A = H2 @ W3r.T + b3
    gamma = softplus(A)
    Hx = Xr @ Lr.T
    Q = r(Hx * gamma)
    Z = Q @ Lr
    Dl = Z - T
    loss = float(np.sum(Dl ** 2) / (B * n))
    dZ = r(2.0 * Dl / (B * n))
    Pm = dZ @ Lr.T
    dL = Q.T @ dZ + r(gamma * Pm).T @ Xr
    dA = Hx * Pm * sigmoid(A)
    dAr = r(dA)
    dW3 = dAr.T @ H2
    db3 = dA.sum(axis=0)
    dH2 = r((dAr @ W3r) * (H2 > 0))
    dW2 = dH2.T @ H1
    db2 = dH2.sum(axis=0)
    dH1 = r((dH2 @ W2r) * (H1 > 0))
    dW1 = dH1.T @ Fr
    db1 = dH1.sum(axis=0)
    return loss, shape.pack([dL, dW1, db1, dW2, db2, dW3, db3])
