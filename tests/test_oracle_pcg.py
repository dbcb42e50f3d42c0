"""Pins for the oracle's Jacobi-PCG: agreement with a direct sparse solve of
the assembled system on tiny meshes, finite termination, A-conjugacy of the
search directions, and spectral convergence to the manufactured solution."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
import synthetic as S
from brute import dense_element_matrix, scatter_matrix


def _assembled(P):
    Q = scatter_matrix(P.x, P.y, P.z)
    blocks = [sp.csr_matrix(dense_element_matrix(P.G[e], P.D)) for e in range(P.E)]
    A = sp.block_diag(blocks, format="csr")
    K = (Q.T @ A @ Q).tocsr()
    return Q, K


@pytest.mark.parametrize("dims,N,deform", [
    ((2, 2, 2), 3, S.NO_DEFORM),
    ((2, 2, 2), 5, ((0.05, 2, 2, 2),) * 3),
    ((3, 2, 2), 4, ((0.08, 1, 2, 3), (0.02, 2, 2, 1), (0.06, 3, 1, 1))),
])
def test_pcg_matches_direct_solve(dims, N, deform):
    b = S.Brick(*dims, N, deform)
    P = O.setup(b)
    Q, K = _assembled(P)
    # boundary flags and right-hand side on the global numbering
    bnd_g = (Q.T @ P.bnd.astype(float)) > 0
    rhs_g = Q.T @ (P.bm.reshape(-1) * O.sine_source(P.x, P.y, P.z))
    I = np.where(~bnd_g)[0]
    xg = np.zeros(Q.shape[1])
    xg[I] = spla.spsolve(K[I][:, I].tocsc(), rhs_g[I])
    res = O.pcg(P, max_iter=2000, rtol=1e-14)
    assert res.state == 1
    want = Q @ xg
    assert np.abs(res.x - want).max() <= 1e-11 * np.abs(want).max()
    # b as the oracle assembles it equals the global load vector
    np.testing.assert_allclose(P.b, Q @ np.where(bnd_g, 0.0, rhs_g), rtol=1e-13, atol=1e-15)


def test_finite_termination():
    """One element, N = 4: 2^3 = 8 unknowns, so CG must converge in about
    8 steps (exact arithmetic: at most 8)."""
    P = O.setup(S.Brick(1, 1, 1, 4, ((0.05, 1, 1, 1),) * 3))
    res = O.pcg(P, max_iter=50, rtol=1e-12)
    assert res.state == 1 and res.iters <= 10


def test_search_directions_are_conjugate():
    P = O.setup(S.Brick(2, 2, 2, 5, ((0.05, 2, 2, 2),) * 3))
    st = O.pcg_start(P)
    ps = []
    for _ in range(6):
        ps.append(st[3].copy())
        x, r, z, p, rho, it, flag, _ = O.pcg_iterate(P, st, 1)
        st = (x, r, z, p, rho)
    Ap = [P.apply_A(p) for p in ps]
    for i in range(len(ps)):
        for j in range(i):
            num = abs(O.wdot(P.c, ps[i], Ap[j]))
            den = np.sqrt(O.wdot(P.c, ps[i], Ap[i]) * O.wdot(P.c, ps[j], Ap[j]))
            assert num <= 1e-9 * den, (i, j)


def test_iterate_in_pieces_equals_one_run():
    P = O.setup(S.scaled_c2_brick(2, 6))
    st = O.pcg_start(P)
    a = O.pcg_iterate(P, st, 10)
    s = st
    for _ in range(10):
        x, r, z, p, rho, it, flag, _ = O.pcg_iterate(P, s, 1)
        s = (x, r, z, p, rho)
    for u, v in zip(a[:4], s[:4]):
        np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("deform", [S.NO_DEFORM, ((0.05, 2, 2, 2),) * 3])
def test_spectral_convergence(deform):
    """Manufactured u* = sin(pi x) sin(pi y) sin(pi z) on a 4^3 brick: the
    nodal max error falls monotonically and roughly exponentially in N."""
    errs = []
    for N in range(4, 12):
        P = O.setup(S.Brick(4, 4, 4, N, deform))
        res = O.pcg(P, max_iter=3000, rtol=1e-13)
        assert res.state == 1
        errs.append(np.abs(res.x - O.exact_solution(P.x, P.y, P.z)).max())
    errs = np.array(errs)
    assert np.all(np.diff(errs[:6]) < 0), errs
    # N = 10: the affine mesh resolves u* to ~1e-12; the curved map costs
    # accuracy but the error is still far below the N = 4 error
    assert errs[6] < (1e-9 if deform == S.NO_DEFORM else 1e-7), errs
    # roughly exponential: more than a decade per two added nodes early on
    assert errs[0] / errs[2] > 10 and errs[2] / errs[4] > 10
