"""Brute-force references used to pin the oracle (tests only).

They are independent formulations, not retypings of the oracle's loops:
  * the dense element matrix A_e = sum_{a,b} D_a^T diag(G_ab) D_b assembled
    from Kronecker products (O(N^6) storage) instead of sum factorisation;
  * the scatter matrix Q built by matching node coordinates instead of the
    global-id formula;
  * exact integrals of polynomial gradients from 1D monomial integrals in
    rational arithmetic.
"""
from fractions import Fraction

import numpy as np
import scipy.sparse as sp


def kron_ops(D):
    """D_r, D_s, D_t for the i-fastest node order idx = i + N(j + N k)."""
    N = D.shape[0]
    I = np.eye(N)
    Dr = np.kron(I, np.kron(I, D))
    Ds = np.kron(I, np.kron(D, I))
    Dt = np.kron(D, np.kron(I, I))
    return Dr, Ds, Dt


def dense_element_matrix(G_e, D):
    """A_e = sum_ab D_a^T diag(G_ab) D_b with G_e[6][N^3] in the order
    rr, rs, rt, ss, st, tt."""
    ops = kron_ops(D)
    pair = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}
    n = D.shape[0] ** 3
    A = np.zeros((n, n))
    for a in range(3):
        for b in range(3):
            f = pair[(min(a, b), max(a, b))]
            A += ops[a].T @ (G_e[f][:, None] * ops[b])
    return A


def scatter_matrix(x, y, z):
    """Q (n_local x n_global): Q[l, g] = 1 when local node l sits at global
    point g; points are identified by exact coordinate equality."""
    pts = np.stack([x, y, z], axis=1)
    _, inv = np.unique(pts, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    n = inv.size
    return sp.csr_matrix((np.ones(n), (np.arange(n), inv)), shape=(n, inv.max() + 1))


def mono_int(m, lo=Fraction(0), hi=Fraction(1)):
    """Exact integral of t^m over [lo, hi]."""
    return (Fraction(hi) ** (m + 1) - Fraction(lo) ** (m + 1)) / (m + 1)


def grad_inner_exact(pu, pv, K=None):
    """Exact  int_[0,1]^3 (grad u)^T K (grad v) dX  for monomials
    u = X^pu[0] Y^pu[1] Z^pu[2], v likewise (K = identity by default)."""
    if K is None:
        K = np.eye(3)
    total = 0.0
    for a in range(3):
        for b in range(3):
            if K[a][b] == 0:
                continue
            cu = pu[a]
            cv = pv[b]
            if cu == 0 or cv == 0:
                continue
            eu = list(pu); eu[a] -= 1
            ev = list(pv); ev[b] -= 1
            val = Fraction(cu * cv)
            for d in range(3):
                val *= mono_int(eu[d] + ev[d])
            total += float(K[a][b]) * float(val)
    return total
