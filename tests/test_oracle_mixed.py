"""Pins for the oracle's single-precision operator and its iterative
refinement: FP32 AX within single-precision accuracy of the FP64 AX,
refinement reaching an FP64 true residual of 1e-10 (recomputed with the
FP64 operator) and the FP64 solution."""
import numpy as np
import pytest

import oracle as O
import synthetic as S


@pytest.mark.parametrize("N", [3, 6, 10])
def test_ax_f32_within_single_precision(N):
    E = 20
    u = S.uniform_field(E, N, seed=N)
    G = S.random_factors(E, N, seed=N + 50)
    D = O.deriv(N)
    w64 = O.ax(u, G, D)
    # the FP64 AX of the float-rounded inputs isolates the arithmetic error
    w64r = O.ax(u.astype(np.float32).astype(np.float64),
                G.astype(np.float32).astype(np.float64),
                D.astype(np.float32).astype(np.float64))
    w32 = O.ax_f32(u, G, D).astype(np.float64)
    scale = np.abs(w64).max()
    assert np.abs(w32 - w64r).max() <= 64 * N * np.finfo(np.float32).eps * scale
    assert np.abs(w32 - w64).max() <= 1e-4 * scale
    # and it is genuinely single precision (not secretly double)
    assert np.abs(w32 - w64).max() > 1e-12 * scale


def test_dssum_f32_is_the_float_sum():
    b = S.Brick(3, 2, 2, 5)
    gid, _ = O.brick_ids(b)
    gs = O.GS(gid)
    v = S.uniform_field(b.E, 5, seed=3).reshape(-1).astype(np.float32)
    got = O.dssum_f32(gs, v)
    ref = gs.dssum(v.astype(np.float64))
    # at most 8 terms: within a few float ulps of the exact (double) sum
    assert np.abs(got - ref).max() <= 8 * np.finfo(np.float32).eps * np.abs(ref).max()
    mult = gs.multiplicity()
    np.testing.assert_array_equal(got[mult == 1], v[mult == 1])


@pytest.mark.parametrize("brick", [S.Brick(2, 2, 2, 5, ((0.05, 2, 2, 2),) * 3),
                                   S.c1_brick()])
def test_refinement_reaches_fp64_accuracy(brick):
    P = O.setup(brick)
    ref = O.pcg(P, max_iter=5000, rtol=1e-13)
    ir = O.ir_solve(P, rtol=1e-10, inner_rtol=1e-5)
    true = P.b - P.apply_A(ir.x)
    relres = np.sqrt(O.wdot(P.c, true, true) / O.wdot(P.c, P.b, P.b))
    assert relres <= 1e-10
    assert 2 <= ir.outer <= 5
    assert np.abs(ir.x - ref.x).max() <= 1e-8 * np.abs(ref.x).max()
