"""Property-based pins of the oracle (Hypothesis draws the element order, the
mesh, the deformation and the seeds): AX against the brute-force dense
element matrix, the operator's invariants, dssum against the scatter matrix
built from coordinates, and Jacobi-PCG against a sparse direct solve."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

hyp = pytest.importorskip("hypothesis")
from hypothesis import assume, given, settings, HealthCheck  # noqa: E402
from hypothesis import strategies as st  # noqa: E402

import oracle as O  # noqa: E402
import synthetic as S  # noqa: E402
from brute import dense_element_matrix, scatter_matrix  # noqa: E402

SETTINGS = dict(max_examples=25, deadline=None,
                suppress_health_check=[HealthCheck.too_slow])

amplitude = st.floats(min_value=0.0, max_value=0.1)
wave = st.integers(min_value=1, max_value=3)
deform = st.tuples(*([st.tuples(amplitude, wave, wave, wave)] * 3))


@settings(**SETTINGS)
@given(N=st.integers(2, 7), E=st.integers(1, 4), seed=st.integers(0, 2 ** 31))
def test_ax_equals_dense_element_matrix(N, E, seed):
    D = O.deriv(N)
    G = S.random_factors(E, N, seed=seed)
    u = S.uniform_field(E, N, seed=seed + 1)
    w = O.ax(u, G, D)
    for e in range(E):
        ref = dense_element_matrix(G[e], D) @ u[e]
        assert np.abs(w[e] - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300)


@settings(**SETTINGS)
@given(N=st.integers(2, 12), dims=st.tuples(*([st.integers(1, 3)] * 3)), d=deform,
       seed=st.integers(0, 2 ** 31))
def test_operator_invariants_on_deformed_bricks(N, dims, d, seed):
    b = S.Brick(*dims, N, d)
    if b.E > 27:
        return
    xi, wq = O.gll(N)
    D = O.deriv(N, xi)
    G, _, jmin = O.geom(N, D, wq, *O.brick_coords(b, xi))
    assume(jmin > 0)            # a valid (non-inverted) isoparametric map
    u = S.uniform_field(b.E, N, seed=seed)
    v = S.uniform_field(b.E, N, seed=seed + 1)
    Au, Av = O.ax(u, G, D), O.ax(v, G, D)
    scale = np.abs(Au).max()
    # constants are in the kernel; symmetric; positive semi-definite
    assert np.abs(O.ax(np.ones_like(u), G, D)).max() <= 1e-12 * max(scale, 1.0)
    assert abs(np.sum(v * Au) - np.sum(u * Av)) <= 1e-11 * (np.abs(v).sum() * scale + 1e-300)
    assert np.sum(u * Au) >= -1e-12 * np.abs(u).sum() * scale


@settings(**SETTINGS)
@given(N=st.integers(2, 6), dims=st.tuples(*([st.integers(1, 3)] * 3)), d=deform,
       seed=st.integers(0, 2 ** 31))
def test_dssum_equals_scatter_matrix(N, dims, d, seed):
    b = S.Brick(*dims, N, d)
    xi, _ = O.gll(N)
    x, y, z = O.brick_coords(b, xi)
    gid, _ = O.brick_ids(b)
    Q = scatter_matrix(x, y, z)
    v = S.uniform_field(b.E, N, seed=seed).reshape(-1)
    want = Q @ (Q.T @ v)
    got = O.GS(gid).dssum(v)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


@settings(max_examples=10, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(N=st.integers(3, 6), dims=st.tuples(*([st.integers(1, 3)] * 3)), d=deform)
def test_pcg_reaches_the_direct_solution(N, dims, d):
    b = S.Brick(*dims, N, d)
    P = O.setup(b)
    # an under-resolved deformation can invert the degree N-1 map (then the
    # operator is indefinite and PCG rightly reports breakdown)
    assume(P.jmin > 0)
    res = O.pcg(P, max_iter=4000, rtol=1e-12)
    assert res.state == 1
    # the assembled system on the free global nodes, solved directly
    xi, _ = O.gll(N)
    Q = scatter_matrix(P.x, P.y, P.z)
    free = np.flatnonzero(np.asarray(Q.T @ (1.0 - P.bnd.astype(float))) > 0.5)
    blocks = [dense_element_matrix(P.G[e], P.D) for e in range(P.E)]
    import scipy.sparse as sp
    A = Q.T @ sp.block_diag(blocks) @ Q
    rhs = Q.T @ (P.b * P.c)
    xs = np.zeros(Q.shape[1])
    if free.size:
        xs[free] = spla.spsolve(A[free][:, free].tocsc(), rhs[free])
    want = Q @ xs
    assert np.abs(res.x - want).max() <= 1e-8 * max(np.abs(want).max(), 1e-300)
