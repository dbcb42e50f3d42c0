"""Batched solves and the tile autotuner on the GPU.

Batched results must be bit-identical to solving each problem alone (same
kernel bodies, block counts and reduction order), and agree with the
oracle like any standalone solve."""
import numpy as np
import pytest

import oracle as O
import synthetic as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_04981_amd as nbx  # noqa: E402
from paper_2011_04981_amd import autotune  # noqa: E402


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _problems():
    """Uneven sizes and orders; random and sine right-hand sides."""
    specs = [S.Brick(2, 2, 2, 6, ((0.03, 2, 2, 2),) * 3, "random", 11),
             S.Brick(3, 2, 2, 8, ((0.05, 2, 2, 2),) * 3, "random", 12),
             S.Brick(4, 4, 4, 10, ((0.05, 2, 2, 2),) * 3, "sine", 0),
             S.Brick(2, 2, 1, 12, ((0.02, 2, 2, 2),) * 3, "random", 13),
             S.Brick(5, 3, 2, 6, S.NO_DEFORM, "sine", 0),
             S.Brick(3, 3, 3, 8, ((0.08, 2, 2, 2),) * 3, "random", 14)]
    out = []
    for b in specs:
        f = None
        if b.rhs == "random":
            f = torch.as_tensor(S.rhs_values(b)).cuda()
        out.append((b, nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array(), f=f)))
    return out


def test_batched_bit_identical_to_standalone_at_n16():
    """The largest order, one element per workgroup in both the standalone
    fused stage and the batched one: the solves agree bit for bit."""
    b = S.Brick(3, 2, 2, 16, ((0.05, 2, 1, 1), (0.04, 1, 2, 1), (0.03, 1, 1, 2)), "random", 3)
    f = torch.as_tensor(S.rhs_values(b)).cuda()
    st = nbx.setup_brick(b.ex, b.ey, b.ez, 16, b.deform_array(), f=f)
    x, r = st.problem.pcg(st.b, rtol=1e-10, max_iter=3000, check_every=10)
    xs, res, _ = nbx.pcg_batched([st.problem], [st.b], rtol=1e-10, max_iter=3000,
                                 check_every=10)
    print(f"N = 16: standalone {r.iters} it, batched {res[0].iters} it")
    assert r.status == 0 and res[0].status == 0 and res[0].iters == r.iters
    assert np.array_equal(host(xs[0]), host(x))


def test_batched_bit_identical_to_standalone():
    probs = _problems()
    refs = []
    for b, st in probs:
        x, r = st.problem.pcg(st.b, rtol=1e-10, max_iter=3000, check_every=10)
        assert r.status == 0
        refs.append((host(x), r.iters))
    xs, res, lat = nbx.pcg_batched([st.problem for _, st in probs], [st.b for _, st in probs],
                                   rtol=1e-10, max_iter=3000, check_every=10)
    for (b, st), (xr, it), x, r in zip(probs, refs, xs, res):
        print(f"{b.name or b}: standalone {it} it, batched {r.iters} it")
        assert r.status == 0 and r.flag == 1
        assert r.iters == it
        assert np.array_equal(host(x), xr)
        assert r.true_relres <= 1e-9
    # latencies: positive, within the batch wall time, slowest problem last
    wall = res[0].seconds
    assert all(0 < t <= wall * 1.05 for t in lat)
    # every graph iteration advances each unconverged problem by one
    # iteration, so the problem needing the most iterations finishes last
    iters = [r.iters for r in res]
    assert lat[int(np.argmax(iters))] >= 0.99 * max(lat)


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("graph", [1, 0])
def test_mixed_batched_bit_identical_to_standalone(prec, graph):
    """Mixed-precision batches (reliable updates): the FP32 iterations of all
    problems run together and each problem's FP64 residual replacement
    follows the standalone steps, so every problem's iterations, updates and
    solution agree bit for bit with its standalone mixed solve."""
    p = {"f32": nbx.F32, "f16": nbx.F16, "bf16": nbx.BF16}[prec]
    probs = _problems()
    kw = dict(rtol=1e-10, max_iter=6000, check_every=10, prec=p, use_graph=graph)
    refs = []
    for b, st in probs:
        x, r = st.problem.pcg(st.b, **kw)
        assert r.status == 0
        refs.append((host(x), r.iters, r.outer_iters, r.fell_back))
    xs, res, lat = nbx.pcg_batched([st.problem for _, st in probs], [st.b for _, st in probs],
                                   **kw)
    for (b, st), (xr, it, outer, fb), x, r in zip(probs, refs, xs, res):
        print(f"{prec} {b.name or b}: standalone {it} it / {outer} updates, "
              f"batched {r.iters} / {r.outer_iters}")
        assert r.status == 0 and r.flag == 1
        assert (r.iters, r.outer_iters, r.fell_back) == (it, outer, fb)
        assert np.array_equal(host(x), xr)
        assert r.true_relres <= 2e-10
    wall = res[0].seconds
    assert all(0 < t <= wall * 1.05 for t in lat)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_batched_large_orders_bit_identical(prec):
    """Large elements take the uniform entries of D slab by slab (FP64 from
    N = 11, FP32 arithmetic from N = 13), which the batched stages then read
    from constant memory instead of global: batched solves of orders 11-16
    must still equal the standalone ones bit for bit."""
    p = {"f64": nbx.F64, "f32": nbx.F32, "f16": nbx.F16}[prec]
    specs = [S.Brick(2, 2, 1, 11, ((0.04, 2, 2, 2),) * 3, "random", 31),
             S.Brick(2, 1, 1, 13, ((0.03, 2, 2, 2),) * 3, "random", 32),
             S.Brick(1, 2, 1, 14, S.NO_DEFORM, "sine", 0),
             S.Brick(1, 1, 2, 16, ((0.02, 2, 2, 2),) * 3, "random", 33),
             S.Brick(2, 2, 2, 12, ((0.05, 2, 2, 2),) * 3, "random", 34)]
    sets = []
    for b in specs:
        f = torch.as_tensor(S.rhs_values(b)).cuda() if b.rhs == "random" else None
        sets.append(nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array(), f=f))
    kw = dict(rtol=1e-10, max_iter=8000, check_every=10, prec=p)
    refs = []
    for st in sets:
        x, r = st.problem.pcg(st.b, **kw)
        assert r.status == 0
        refs.append((host(x), r.iters, r.outer_iters))
    xs, res, lat = nbx.pcg_batched([st.problem for st in sets], [st.b for st in sets], **kw)
    for b, (xr, it, outer), x, r in zip(specs, refs, xs, res):
        print(f"{prec} N={b.N}: standalone {it} it, batched {r.iters}")
        assert r.flag == 1 and (r.iters, r.outer_iters) == (it, outer)
        assert np.array_equal(host(x), xr)


def test_mixed_batched_breakdown_and_limit_are_per_problem():
    """A batch holding an indefinite problem (negated factors: <p, Ap> < 0 at
    once) next to ordinary ones: the indefinite one ends in breakdown after
    its FP64 fallback broke down too, the others converge as they would
    alone; a tiny iteration limit leaves every problem unconverged with the
    FP64 true residual and solution of its standalone solve."""
    probs = _problems()[:3]
    b0, st0 = probs[0]
    kw = dict(rtol=1e-10, max_iter=6000, check_every=10, prec=nbx.F16)
    refs = []
    for _, st in probs:
        x, r = st.problem.pcg(st.b, **kw)
        refs.append((host(x), r.iters, r.outer_iters))
    bad = nbx.Problem(-st0.G, st0.D, b0.N, st0.gs)
    plist = [st.problem for _, st in probs] + [bad]
    blist = [st.b for _, st in probs] + [st0.b]
    xs, res, lat = nbx.pcg_batched(plist, blist, **kw)
    print(f"indefinite member: flag {res[3].flag}, {res[3].iters} it, "
          f"fell back {res[3].fell_back}")
    for (xr, it, outer), x, r in zip(refs, xs, res):
        assert r.status == -5 and r.flag == 1 and r.true_relres <= 2e-10
        assert (r.iters, r.outer_iters) == (it, outer)
        assert np.array_equal(host(x), xr)
    assert res[3].flag == 2 and res[3].fell_back == 1 and res[3].iters <= 5
    assert np.all(np.isfinite(host(xs[3])))
    # the iteration limit: CG residuals are not monotone, so the reported
    # true residual is checked against the standalone solve, not against 1
    kw = dict(rtol=1e-10, max_iter=12, check_every=5, prec=nbx.F32)
    xs, res, lat = nbx.pcg_batched([st.problem for _, st in probs], [st.b for _, st in probs],
                                   **kw)
    for (_, st), x, r in zip(probs, xs, res):
        xr, rr = st.problem.pcg(st.b, **kw)
        print(f"limit: {r.iters} it, flag {r.flag}, true relres {r.true_relres:.2e}")
        assert r.status == 1 and r.flag == 0 and r.iters == rr.iters == 12
        assert r.true_relres == rr.true_relres and np.isfinite(r.true_relres)
        assert np.array_equal(host(x), host(xr))


@pytest.mark.parametrize("case", ["max_outer", "stall"])
def test_mixed_batched_host_ended_problems_stop_on_the_device(case):
    """A mixed solve can end on the host while its device flag still reads
    'continue': after max_outer residual replacements, or when two updates
    in a row fail to cut the true residual fourfold (forced here with an
    inner tolerance of 0.9, which then hands the solve to the FP64
    fallback).  In a batch every later replay would keep iterating such a
    problem; its iterations, updates, fallback and solution must still be
    exactly those of its standalone solve."""
    probs = _problems()[:4]
    kw = dict(rtol=1e-10, max_iter=6000, check_every=10, prec=nbx.F32)
    kw.update(max_outer=2) if case == "max_outer" else kw.update(inner_rtol=0.9)
    refs = []
    for _, st in probs:
        x, r = st.problem.pcg(st.b, **kw)
        refs.append((host(x), r.iters, r.outer_iters, r.fell_back, r.flag))
    xs, res, _ = nbx.pcg_batched([st.problem for _, st in probs], [st.b for _, st in probs],
                                 **kw)
    for (xr, it, outer, fb, fl), x, r in zip(refs, xs, res):
        print(f"{case}: standalone {it} it / {outer} updates / fell back {fb} / flag {fl}; "
              f"batched {r.iters} / {r.outer_iters} / {r.fell_back} / {r.flag}")
        assert (r.iters, r.outer_iters, r.fell_back, r.flag) == (it, outer, fb, fl)
        assert np.array_equal(host(x), xr)
    if case == "stall":
        assert any(r.fell_back == 1 for r in res) and all(r.flag == 1 for r in res)
    else:
        assert all(r.outer_iters == 2 and r.flag == 0 for r in res)


def test_mixed_batched_refuses_restarted_refinement():
    probs = _problems()[:2]
    with pytest.raises(nbx.NbxError):
        nbx.pcg_batched([st.problem for _, st in probs], [st.b for _, st in probs],
                        prec=nbx.F32, mixed_mode=1)


def test_batched_matches_oracle():
    b = S.Brick(3, 2, 2, 8, ((0.05, 2, 2, 2),) * 3, "random", 21)
    f = S.rhs_values(b)
    P = O.setup(b, rhs_values=f)
    ref = O.pcg(P, max_iter=3000, rtol=1e-10)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array(), f=torch.as_tensor(f).cuda())
    st2 = nbx.setup_brick(3, 3, 3, 6)
    xs, res, lat = nbx.pcg_batched([st.problem, st2.problem], [st.b, st2.b], rtol=1e-10,
                                   max_iter=3000)
    assert abs(res[0].iters - ref.iters) <= 1
    x = host(xs[0]).reshape(-1)
    assert np.abs(x - ref.x).max() <= 1e-8 * np.abs(ref.x).max()


def test_batched_fixed_iterations_and_limits():
    probs = _problems()[:3]
    xs, res, lat = nbx.pcg_batched([st.problem for _, st in probs], [st.b for _, st in probs],
                                   max_iter=25, fixed_iters=1, check_every=10)
    assert all(r.iters == 25 and r.flag == 0 for r in res)


def test_autotuner_picks_a_valid_tile_and_is_result_neutral():
    old = nbx.get_tile(nbx.F64, 8)
    try:
        table = autotune.tune(Ns=(8,), precs=(nbx.F64,), nodes=400_000, reps=3)
        row = table["f64"]["8"]
        assert row["epb"] in (1, 2, 4, 8) and nbx.get_tile(nbx.F64, 8) == row["epb"]
        assert set(row["us"]) <= {"1", "2", "4", "8"} and all(v > 0 for v in row["us"].values())
    finally:
        nbx.set_tile(nbx.F64, 8, old)


def test_breakdown_at_n16_standalone_and_batched():
    """At N = 16 the fused first stage (matrix cores) supplies <p, Ap> to
    the breakdown test: with negated factors the standalone and the batched
    FP64 solves both stop at once with the breakdown flag, at the same
    iteration and with the same x."""
    b = S.scaled_c2_brick(2, 16)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, 16, b.deform_array())
    bad = nbx.Problem(-st.G, st.D, 16, st.gs)
    x, r = bad.pcg(st.b, rtol=1e-10, max_iter=500, check_every=5)
    print(f"N = 16 indefinite: status {r.status}, flag {r.flag}, {r.iters} it")
    assert r.status == -5 and r.flag == 2 and r.iters <= 5
    xs, res, _ = nbx.pcg_batched([bad], [st.b], rtol=1e-10, max_iter=500, check_every=5)
    assert res[0].flag == 2 and res[0].iters == r.iters
    assert np.array_equal(host(xs[0]), host(x))
