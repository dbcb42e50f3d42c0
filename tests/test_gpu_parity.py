"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerance for FP64 results: normwise relative 1e-12,
max|gpu - oracle| <= 1e-12 * max|oracle| (pointwise relative error is
meaningless where AX cancels, e.g. AX(const) = 0).  dssum sums in the same
ascending order as the oracle, so it must agree bit for bit.  Each side
builds its own GLL rule, D and geometric factors from the same workload
description; the shared inputs are the seeded random fields only.
"""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from layout import pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_04981_amd as nbx  # noqa: E402

DEV = "cuda"
TOL = 1e-12


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


def assert_rel(a, b, tol):
    e = rel(a, b)
    assert e <= tol, f"normwise relative error {e:.3e} > {tol:.1e}"


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# --------------------------------------------------------------------- AX

@pytest.mark.parametrize("N,E", [(2, 1), (3, 5), (4, 37), (5, 3), (6, 64), (7, 9), (8, 33),
                                 (9, 2), (10, 1), (10, 129), (11, 4), (12, 17), (13, 2),
                                 (14, 3), (15, 2), (16, 5)])
def test_ax_random_factors(N, E):
    print(f"ax parity N={N} E={E}", flush=True)
    u = S.uniform_field(E, N, seed=N)
    G = S.random_factors(E, N, seed=N + 1)
    want = O.ax(u, G, O.deriv(N))
    D = nbx.deriv_device(N)
    got = host(nbx.ax(cuda(u), cuda(G), D))            # [E, 6, N^3], the contract
    assert_rel(got, want, TOL)
    # the factor-pair fast path computes the same bits
    assert np.array_equal(host(nbx.ax_paired(cuda(u), cuda(pairs(G)), D)), got)


def test_ax_zero_elements_is_noop():
    w = torch.full((0, 1000), 7.0, dtype=torch.float64, device=DEV)
    u = torch.zeros((0, 1000), dtype=torch.float64, device=DEV)
    G = torch.zeros((0, 6, 1000), dtype=torch.float64, device=DEV)
    D = nbx.deriv_device(10)
    assert nbx.lib().nbx_ax(0, nbx._dptr(torch.zeros(1, dtype=torch.float64, device=DEV)),
                            nbx._dptr(torch.zeros(1, dtype=torch.float64, device=DEV)),
                            nbx._dptr(D), 10, 0,
                            nbx._dptr(torch.zeros(2, dtype=torch.float64, device=DEV)),
                            None) == 0
    del w, u, G


@pytest.mark.parametrize("dims,N", [((3, 3, 3), 10), ((2, 3, 4), 6), ((4, 2, 2), 12)])
def test_geometry_and_ax_on_deformed_mesh(dims, N):
    """Each side builds G from the C2 mapping; factors, mass and AX agree."""
    print(f"deformed geometry dims={dims} N={N}", flush=True)
    b = S.Brick(*dims, N, ((0.05, 2, 2, 2),) * 3)
    P = O.setup(b)
    G, bm, xyz = nbx.geom_brick(*dims, N, b.deform_array(), with_xyz=True)
    assert tuple(G.shape) == (b.E, 6, N ** 3)
    assert_rel(host(G), P.G, TOL)
    assert_rel(host(bm), P.bm, TOL)
    assert_rel(host(xyz)[0], P.x, 1e-15)
    u = S.uniform_field(b.E, N, seed=3)
    got = host(nbx.ax(cuda(u), G, nbx.deriv_device(N)))
    assert_rel(got, O.ax(u, P.G, P.D), TOL)


def test_ax_full_size_seeded_factors():
    """Benchmark size and launch (E = 32768, N = 10, the library's default
    tile) on identical seeded inputs, checked on every element."""
    N, E = 10, 32768
    print("ax parity at E=32768 N=10 (seeded factors)", flush=True)
    u = S.uniform_field(E, N, seed=0)
    G = S.random_factors(E, N, seed=1)
    D = nbx.deriv_device(N)
    w = host(nbx.ax(cuda(u), cuda(G), D))
    assert_rel(w, O.ax(u, G, O.deriv(N)), TOL)
    assert np.array_equal(host(nbx.ax_paired(cuda(u), cuda(pairs(G)), D)), w)


def test_ax_full_size_deformed_c2():
    """The benchmark workload itself, each side with its own geometry.
    The factors agree to 1e-12; AX of the two factor sets is compared at
    1e-11 because the sides' sin() differ by an ulp in the coordinates and
    the derivative stencil amplifies that by ~10^2 in G, and AX by another
    order in w."""
    b = S.c2_brick()
    N = b.N
    print("ax at E=32768 N=10 with each side's own geometry", flush=True)
    G, bm, _ = nbx.geom_brick(b.ex, b.ey, b.ez, N, b.deform_array())
    xi, wq = O.gll(N)
    D = O.deriv(N, xi)
    x, y, z = O.brick_coords(b, xi)
    Go, bmo, _ = O.geom(N, D, wq, x, y, z)
    del x, y, z
    assert_rel(host(G), Go, TOL)
    assert_rel(host(bm), bmo, TOL)
    u = S.uniform_field(b.E, N, seed=0)
    w = nbx.ax(cuda(u), G, nbx.deriv_device(N))
    assert_rel(host(w), O.ax(u, Go, D), 1e-11)


def test_ax_is_deterministic():
    N, E = 10, 300
    u = cuda(S.uniform_field(E, N, 5)); G = cuda(S.random_factors(E, N, 6))
    D = nbx.deriv_device(N)
    a = host(nbx.ax(u, G, D)); b = host(nbx.ax(u, G, D))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("N", [4, 8, 10, 12])
def test_ax_fp32_error_vs_oracle(N):
    """FP32 storage and arithmetic: error reported against the FP64 oracle,
    gated at a bound of a few hundred FP32 ulps of the result scale."""
    E = 40
    u = S.uniform_field(E, N, seed=11)
    G = S.random_factors(E, N, seed=12)
    want = O.ax(u, G, O.deriv(N))
    got = host(nbx.ax(cuda(u, torch.float32), cuda(G, torch.float32), nbx.deriv_device(N)))
    err = rel(got, want)
    print(f"fp32 AX N={N}: normwise error {err:.3e}")
    assert err <= 300 * np.finfo(np.float32).eps


# ---------------------------------------------------- dssum / mask / Jacobi

@pytest.mark.parametrize("dims,N", [((3, 4, 5), 5), ((4, 4, 4), 10), ((2, 2, 1), 2)])
def test_dssum_bit_exact(dims, N):
    b = S.Brick(*dims, N)
    gid, bnd = nbx.brick_ids(*dims, N)
    gs = nbx.GS(gid, bnd)
    ogs = O.GS(O.brick_ids(b)[0])
    v = S.uniform_field(b.E, N, seed=21).reshape(-1)
    for mask in (False, True):
        t = cuda(v)
        gs.dssum(t, mask=mask)
        want = ogs.dssum(v)
        if mask:
            want = O.mask(bnd, want)
        assert np.array_equal(host(t), want), mask
    np.testing.assert_array_equal(host(gs.multiplicity()), ogs.multiplicity())


def test_dssum_fp32_matches_fp32_sum():
    b = S.Brick(3, 2, 2, 6)
    gid, bnd = nbx.brick_ids(3, 2, 2, 6)
    gs = nbx.GS(gid, bnd)
    v = S.uniform_field(b.E, 6, seed=2).reshape(-1).astype(np.float32)
    t = cuda(v, torch.float32)
    gs.dssum(t, mask=True)
    want = O.mask(bnd, O.GS(gid).dssum(v.astype(np.float64)))
    assert_rel(host(t), want, 4 * np.finfo(np.float32).eps)


@pytest.mark.parametrize("dims,N", [((3, 3, 3), 10), ((2, 3, 2), 7)])
def test_jacobi_and_rhs(dims, N):
    b = S.Brick(*dims, N, ((0.05, 2, 2, 2),) * 3)
    P = O.setup(b)
    st = nbx.setup_brick(*dims, N, b.deform_array())
    assert_rel(host(st.problem.dinv()), P.dinv, TOL)
    assert_rel(host(st.b), P.b, TOL)


# -------------------------------------------------------------------- PCG

def _gpu_state(st, x, r, p, rho):
    """Device state for one nbx_pcg_iterate step that starts from the
    oracle's (x, r, p, rho): z := p and beta = 0 make the kernel's
    p = z + beta p reproduce the oracle's search direction exactly."""
    n = st.E * st.N ** 3
    xs, rs = cuda(x).reshape(st.E, -1), cuda(r).reshape(st.E, -1)
    zs = cuda(p).reshape(st.E, -1)
    ps = torch.zeros_like(zs)
    scal = torch.zeros(nbx.SCAL_LEN, dtype=torch.float64, device=DEV)
    scal[nbx.S_RHO] = rho
    scal[nbx.S_STOP] = -1.0
    scal[nbx.S_MAXIT] = 1e9
    return xs, rs, zs, ps, scal


@pytest.mark.parametrize("case", ["c1", "deformed8", "deformed16"])
def test_pcg_one_step_parity(case):
    """One fused iteration from the oracle's state at k = 0 ... 99; at
    N = 16 the fused first stage is the matrix-core body, run on the
    oracle's own factors (the two sides' factors agree to 1e-12, and at
    N = 16 the derivative stencil lifts their last-bit differences to
    ~1e-12 in AX: test_ax16_on_deformed_geometry)."""
    b = {"c1": S.c1_brick, "deformed8": lambda: S.scaled_c2_brick(3, 8),
         "deformed16": lambda: S.scaled_c2_brick(2, 16)}[case]()
    P = O.setup(b)
    if case == "deformed16":
        gid, bnd = nbx.brick_ids(b.ex, b.ey, b.ez, b.N)
        prob = nbx.Problem(cuda(P.G), nbx.deriv_device(b.N), b.N, nbx.GS(gid, bnd))
    else:
        prob = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array()).problem
    state = O.pcg_start(P)
    done = 0
    for k in (0, 1, 10, 50, 99):
        if k > done:
            x, r, z, p, rho, *_ = O.pcg_iterate(P, state, k - done)
            state = (x, r, z, p, rho)
            done = k
        print(f"one-step parity {case} k={k}", flush=True)
        xs, rs, zs, ps, scal = _gpu_state(prob, state[0], state[1], state[3], state[4])
        prob.pcg_iterate(xs, rs, zs, ps, scal, 1)
        x1, r1, z1, p1, rho1, it, flag, _ = O.pcg_iterate(P, state, 1)
        sc = host(scal)
        assert sc[nbx.S_FLAG] == 0 and sc[nbx.S_ITER] == 1
        assert_rel(host(xs), x1, TOL)
        assert_rel(host(rs), r1, TOL)
        assert_rel(host(zs), z1, TOL)
        assert abs(sc[nbx.S_RHO] - rho1) <= TOL * abs(rho1)
        pnext = host(zs + sc[nbx.S_BETA] * ps)
        assert_rel(pnext, p1, TOL)


def test_pcg_100_iterations_c1():
    b = S.c1_brick()
    P = O.setup(b)
    ora = O.pcg(P, max_iter=100, rtol=0.0)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N)
    x, res = st.problem.pcg(st.b, max_iter=100, fixed_iters=1, check_every=10)
    assert res.iters == 100 and ora.iters == 100
    err = rel(host(x), ora.x)
    print(f"C1 100-iteration x difference {err:.3e}")
    assert err <= 1e-10


@pytest.mark.parametrize("graph", [1, 0])
def test_pcg_solve_to_1e10(graph):
    b = S.scaled_c2_brick(4, 8)
    P = O.setup(b)
    ora = O.pcg(P, max_iter=2000, rtol=1e-10)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    x, res = st.problem.pcg(st.b, rtol=1e-10, max_iter=2000, use_graph=graph, check_every=7)
    print(f"solve: gpu {res.iters} it, oracle {ora.iters} it, true relres {res.true_relres:.2e}")
    assert res.status == 0 and res.flag == 1
    assert abs(res.iters - ora.iters) <= 1
    assert res.relres <= 1e-10 and res.true_relres <= 1e-9
    assert_rel(host(x), ora.x, 1e-8)


def test_pcg_deterministic_and_reusable():
    b = S.scaled_c2_brick(3, 6)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    x1, r1 = st.problem.pcg(st.b, rtol=1e-10, check_every=5)
    x2, r2 = st.problem.pcg(st.b, rtol=1e-10, check_every=5)
    assert r1.iters == r2.iters
    assert np.array_equal(host(x1), host(x2))


def test_pcg_max_iter_limit_reports_not_converged():
    b = S.scaled_c2_brick(3, 6)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    x, res = st.problem.pcg(st.b, rtol=1e-14, max_iter=7, check_every=3)
    assert res.status == 1 and res.iters == 7 and res.flag == 0


def test_pcg_zero_rhs_returns_zero():
    b = S.Brick(2, 2, 2, 5)
    st = nbx.setup_brick(2, 2, 2, 5)
    zero = torch.zeros_like(st.b)
    x, res = st.problem.pcg(zero, rtol=1e-10)
    assert res.status == 0 and res.iters == 0
    assert float(host(x).__abs__().max()) == 0.0


def test_pcg_one_step_full_size_c2():
    """One fused iteration on the full benchmark mesh from the oracle's
    state after k = 0 and k = 10 iterations, on identical inputs: the GPU
    problem is built from the oracle's factors (its own geometry agrees to
    1e-12, which AX turns into 1e-11, see the deformed-mesh AX test)."""
    b = S.c2_brick()
    P = O.setup(b)
    ref = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    assert_rel(host(ref.b), P.b, TOL)
    del ref

    class St:
        pass
    st = St()
    st.E, st.N = b.E, b.N
    gid, bnd = nbx.brick_ids(b.ex, b.ey, b.ez, b.N)
    gs = nbx.GS(gid, bnd)
    st.problem = nbx.Problem(cuda(P.G), nbx.deriv_device(b.N), b.N, gs)
    state = O.pcg_start(P)
    for k in (0, 10):
        print(f"one-step parity at E=32768, k={k}", flush=True)
        if k:
            state = O.pcg_iterate(P, state, k)[:5]
        xs, rs, zs, ps, scal = _gpu_state(st, state[0], state[1], state[3], state[4])
        st.problem.pcg_iterate(xs, rs, zs, ps, scal, 1)
        x1, r1, z1, p1, rho1, *_ = O.pcg_iterate(P, state, 1)
        assert_rel(host(xs), x1, TOL)
        assert_rel(host(rs), r1, TOL)
        assert_rel(host(zs), z1, TOL)
        assert abs(host(scal)[nbx.S_RHO] - rho1) <= TOL * abs(rho1)


@pytest.mark.parametrize("N,E", [(4, 37), (8, 9), (10, 131), (12, 5), (16, 3)])
def test_every_tile_is_bit_identical(N, E):
    """The autotuner's search space: every elements-per-workgroup choice
    that fits computes the same bits (including the ragged last block)."""
    G6 = S.random_factors(E, N, seed=32)
    u = cuda(S.uniform_field(E, N, seed=31)); G = cuda(G6); Gp = cuda(pairs(G6))
    D = nbx.deriv_device(N)
    ref = None
    for epb in (1, 2, 4, 8):
        try:
            w = host(nbx.ax(u, G, D, epb=epb))
        except nbx.NbxError as e:
            assert e.status == -2   # tile does not fit in LDS
            continue
        if ref is None:
            ref = w
            assert_rel(w, O.ax(host(u), G6, O.deriv(N)), TOL)
        else:
            assert np.array_equal(w, ref), epb
        assert np.array_equal(host(nbx.ax_paired(u, Gp, D, epb=epb)), ref), epb


def test_tile_table_roundtrip():
    old = nbx.get_tile(nbx.F64, 10)
    nbx.set_tile(nbx.F64, 10, 4)
    assert nbx.get_tile(nbx.F64, 10) == 4
    nbx.set_tile(nbx.F64, 10, old)
    with pytest.raises(nbx.NbxError):
        nbx.set_tile(nbx.F64, 10, 3)


# ---------------------------------------------------------- mixed precision

@pytest.mark.parametrize("N", [6, 10])
def test_ax_fp32_matches_oracle_fp32(N):
    E = 33
    u = S.uniform_field(E, N, seed=41).astype(np.float32)
    G = S.random_factors(E, N, seed=42).astype(np.float32)
    want = O.ax_f32(u, G, O.deriv(N))
    got = host(nbx.ax(cuda(u, torch.float32), cuda(G, torch.float32), nbx.deriv_device(N)))
    assert_rel(got, want, 16 * N * np.finfo(np.float32).eps)


@pytest.mark.parametrize("case,mode", [("deformed8", 0), ("c1", 0), ("deformed8", 1), ("c1", 1)])
def test_mixed_precision_solve(case, mode):
    """mode 0: one FP32 Krylov sequence with FP64 reliable updates every
    tenfold residual drop; mode 1: restarted refinement, inner solves to
    1e-5.  Either way the FP64 true residual must reach 1e-10."""
    b = S.scaled_c2_brick(4, 8) if case == "deformed8" else S.c1_brick()
    P = O.setup(b)
    ref = O.pcg(P, max_iter=5000, rtol=1e-13)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    x, res = st.problem.pcg(st.b, rtol=1e-10, max_iter=5000, prec=nbx.F32,
                            inner_rtol=0.1 if mode == 0 else 1e-5, mixed_mode=mode)
    print(f"mixed {case} mode {mode}: {res.iters} it, {res.outer_iters} outer, "
          f"relres {res.relres:.2e} (fp64 oracle {ref.iters} it)")
    assert res.status == 0 and res.flag == 1 and res.fell_back == 0
    if mode == 1:
        assert 2 <= res.outer_iters <= 5
    else:
        assert 5 <= res.outer_iters <= 30
    xh = host(x).reshape(-1)
    true = P.b - P.apply_A(xh)          # the oracle's own FP64 operator
    assert np.sqrt(O.wdot(P.c, true, true) / O.wdot(P.c, P.b, P.b)) <= 2e-10
    assert_rel(xh, ref.x, 1e-8)


def test_mixed_precision_falls_back_when_refinement_stalls():
    """An inner tolerance of 0.5 cannot give the tenfold reduction per outer
    step the refinement loop demands, so it must finish with FP64 PCG."""
    b = S.scaled_c2_brick(3, 6)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    x, res = st.problem.pcg(st.b, rtol=1e-10, max_iter=5000, prec=nbx.F32, inner_rtol=0.5,
                            mixed_mode=1)
    assert res.fell_back == 1 and res.status == 0 and res.relres <= 1e-10
    # reliable updates every 1% of reduction cannot show the fourfold drop
    # per update the stall detector demands
    x, res = st.problem.pcg(st.b, rtol=1e-10, max_iter=5000, prec=nbx.F32, inner_rtol=0.99,
                            mixed_mode=0)
    assert res.fell_back == 1 and res.status == 0 and res.relres <= 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fused_stage_tile_change_reaches_captured_solves(prec):
    """The solvers replay captured graphs; after nbx_pcg_set_tile a solve on
    the same problem must run the new tile, i.e. agree bit for bit with a
    solve on a fresh problem (the tile decides how <p,w> partials group)."""
    b = S.scaled_c2_brick(4, 8)
    p = nbx.F64 if prec == "f64" else nbx.F32
    old = nbx.get_pcg_tile(p, b.N)
    kw = dict(rtol=1e-10, max_iter=3000, check_every=10, prec=p)
    try:
        st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
        results = {}
        for epb in (1, 4):
            nbx.set_pcg_tile(p, b.N, epb)
            x, r = st.problem.pcg(st.b, **kw)
            fresh = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
            xf, rf = fresh.problem.pcg(fresh.b, **kw)
            assert r.iters == rf.iters and np.array_equal(host(x), host(xf)), epb
            results[epb] = host(x)
        assert rel(results[1], results[4]) <= 1e-8      # both are solutions
    finally:
        nbx.set_pcg_tile(p, b.N, old)


def test_binding_refuses_mis_sized_tensors():
    """The C ABI takes raw pointers; the binding checks sizes before any
    launch could run past a buffer."""
    b = S.scaled_c2_brick(2, 4)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    n = st.E * st.N ** 3
    short = torch.zeros(n - 1, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        st.problem.pcg(short)
    with pytest.raises(ValueError):
        st.gs.dssum(short)
    with pytest.raises(ValueError):
        nbx.ax(torch.zeros((st.E, st.N ** 3), dtype=torch.float64, device=DEV), st.G, st.D,
               out=short)
    with pytest.raises(ValueError):
        nbx.ax(torch.zeros((st.E, st.N ** 3), dtype=torch.float64, device=DEV), st.G[:1], st.D)
    # the contract's [E, 6, N^3] factors and the pair layout are not
    # interchangeable: each entry point refuses the other's shape
    u0 = torch.zeros((st.E, st.N ** 3), dtype=torch.float64, device=DEV)
    Gp = nbx.pair_factors(st.G, st.N)
    with pytest.raises(ValueError):
        nbx.ax(u0, Gp, st.D)
    with pytest.raises(ValueError):
        nbx.ax_paired(u0, st.G, st.D)
    # a contiguous view that does not start on a 16-byte boundary
    buf = torch.zeros(n + 1, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        st.problem.pcg(st.b, x=buf[1:])
    with pytest.raises(ValueError):
        nbx.ax(buf[1:].view(st.E, -1), st.G, st.D)
    net = nbx.Mlp(st.N ** 3 + 6, 64, st.N ** 3, max_batch=64)
    with pytest.raises(ValueError):
        net.forward(torch.zeros((64, 8), dtype=torch.bfloat16, device=DEV))
    # the solve still works afterwards
    x, r = st.problem.pcg(st.b, rtol=1e-10)
    assert r.status == 0


def test_full_size_solves_checked_by_the_oracle_operator():
    """The benchmark's 32^3 deformed brick at N = 10 (32.8 M local nodes), in
    the configuration bench.py times: FP64 PCG and the FP32 / FP16-storage
    refinement solves to 1e-10; the oracle builds its own geometry and
    right-hand side and evaluates ||b - A x||_c / ||b||_c for each GPU
    solution with its own operator."""
    b = S.c2_brick()
    print("full-size set-up (oracle)", flush=True)
    P = O.setup(b)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    bb = O.wdot(P.c, P.b, P.b)
    for name, kw in (("fp64", dict(prec=nbx.F64)),
                     ("fp32", dict(prec=nbx.F32, inner_rtol=0.1)),
                     ("f16", dict(prec=nbx.F16, inner_rtol=0.1))):
        print(f"full-size solve {name}", flush=True)
        x, r = st.problem.pcg(st.b, rtol=1e-10, max_iter=10000, check_every=20, **kw)
        assert r.status == 0 and r.flag == 1, (name, r)
        xh = host(x).reshape(-1)
        res = P.b - P.apply_A(xh)
        rel_true = np.sqrt(O.wdot(P.c, res, res) / bb)
        print(f"{name}: {r.iters} it, oracle-operator relres {rel_true:.2e}")
        assert rel_true <= 2e-10, (name, rel_true)


def test_full_size_solves_at_n12_checked_by_the_oracle_operator():
    """The C2 mapping at N = 12 (32^3 elements, 56.6 M local nodes), one of
    the mixed-precision sweep's sizes: the FP64 solve and the FP16-stored
    mixed solve to 1e-10, each solution's residual evaluated by the oracle
    with its own geometry and operator."""
    b = S.c2_brick(12)
    print("full-size set-up at N=12 (oracle)", flush=True)
    P = O.setup(b)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    bb = O.wdot(P.c, P.b, P.b)
    for name, kw in (("fp64", dict(prec=nbx.F64)),
                     ("f16", dict(prec=nbx.F16, inner_rtol=0.1))):
        print(f"N=12 full-size solve {name}", flush=True)
        x, r = st.problem.pcg(st.b, rtol=1e-10, max_iter=20000, check_every=20, **kw)
        assert r.status == 0 and r.flag == 1, (name, r)
        xh = host(x).reshape(-1)
        res = P.b - P.apply_A(xh)
        rel_true = np.sqrt(O.wdot(P.c, res, res) / bb)
        print(f"{name}: {r.iters} it, oracle-operator relres {rel_true:.2e}")
        assert rel_true <= 2e-10, (name, rel_true)
        del x, xh, res


@pytest.mark.parametrize("N", [2, 3])
def test_pcg_tiny_elements(N):
    """Degenerate element orders: N = 2 (trilinear, no interior nodes) and
    N = 3; the solve must match the oracle's."""
    b = S.Brick(5, 4, 3, N, ((0.05, 2, 2, 2),) * 3)
    P = O.setup(b)
    ora = O.pcg(P, max_iter=3000, rtol=1e-10)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    x, r = st.problem.pcg(st.b, rtol=1e-10, max_iter=3000, check_every=3)
    assert r.status == 0 and abs(r.iters - ora.iters) <= 1
    assert rel(host(x), ora.x) <= 1e-8


def test_bandwidth_reference_streams():
    """nbx_copy_f64 / nbx_stream_f64: the copies are exact, the read-only
    stream stores nothing, odd lengths are refused."""
    src = torch.randn(1 << 20, dtype=torch.float64, device=DEV)
    dst = torch.zeros_like(src)
    nbx.copy_f64(src, dst)
    assert torch.equal(src, dst)
    dst.zero_()
    nbx.stream_f64(0, src, dst)
    assert torch.equal(src, dst)
    sink = torch.zeros(1, dtype=torch.float64, device=DEV)
    nbx.stream_f64(1, src, sink=sink)
    assert host(sink)[0] == 0.0
    with pytest.raises(nbx.NbxError):
        nbx.stream_f64(1, src[:-1], sink=sink)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_indefinite_operator_reports_breakdown(prec):
    """Negated factors make A negative definite: <p, Ap> < 0 at the first
    step.  Every solver must stop at once with the breakdown status (the
    mixed ones after their FP64 fallback has broken down too), not hang or
    return a bogus converged state."""
    b = S.scaled_c2_brick(2, 5)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    Gneg = -st.G
    P = nbx.Problem(Gneg, st.D, b.N, st.gs)
    p = {"f64": nbx.F64, "f32": nbx.F32, "f16": nbx.F16}[prec]
    x, r = P.pcg(st.b, rtol=1e-10, max_iter=500, prec=p, check_every=5)
    print(f"{prec}: status {r.status}, flag {r.flag}, iters {r.iters}, fell back {r.fell_back}")
    assert r.status == -5 and r.flag == 2
    assert r.iters <= 5
    assert np.all(np.isfinite(host(x)))


@pytest.mark.parametrize("N,E", [(2, 1), (3, 7), (10, 33), (16, 3)])
def test_factor_layout_conversions(N, E):
    """nbx_repack_g_aos_to_soa (from the layout of the operator's g
    argument, g(6, N^3, E) with the factor fastest) into one plane per
    factor, and nbx_pair_factors from planes into factor pairs, bit for bit
    (node counts below, at and off the kernels' 256-node blocks); AX agrees
    on the converted factors."""
    G6 = S.random_factors(E, N, seed=41)                 # [E, 6, N^3]
    want = cuda(G6)
    wantp = cuda(pairs(G6))                              # [E, 3, N^3, 2]
    aos = cuda(G6.transpose(0, 2, 1))                    # [E, N^3, 6]
    assert torch.equal(nbx.repack_g_aos_to_soa(aos, N), want)
    assert torch.equal(nbx.pair_factors(cuda(G6), N), wantp)
    out = torch.full_like(want, float("nan"))
    nbx.repack_g_aos_to_soa(aos, N, out=out)
    assert torch.equal(out, want)
    with pytest.raises(nbx.NbxError):                    # overlapping arrays
        nbx.repack_g_aos_to_soa(aos, N, out=aos)
    with pytest.raises(nbx.NbxError):
        nbx.pair_factors(wantp, N, out=wantp)
    empty = torch.empty((0, N ** 3, 6), dtype=torch.float64, device=DEV)
    assert nbx.repack_g_aos_to_soa(empty, N).shape == (0, 6, N ** 3)
    u = S.uniform_field(E, N, seed=42)
    D = nbx.deriv_device(N)
    w = host(nbx.ax(cuda(u), nbx.repack_g_aos_to_soa(aos, N), D))
    assert_rel(w, O.ax(u, G6, O.deriv(N)), TOL)
    assert np.array_equal(host(nbx.ax_paired(cuda(u), wantp, D)), w)


@pytest.mark.parametrize("N", [11, 13, 16])
def test_pcg_large_elements(N):
    """Element orders whose fused first stage loads part of the factor
    column inside the slab loop (FP64 from N = 11, FP32 from N = 13): FP64
    PCG and the FP32 / FP16-G mixed solves against the oracle's solution."""
    b = S.Brick(2, 2, 1, N, ((0.05, 2, 2, 2),) * 3)
    print(f"large-element solves N={N}", flush=True)
    P = O.setup(b)
    ora = O.pcg(P, max_iter=5000, rtol=1e-10)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    x, r = st.problem.pcg(st.b, rtol=1e-10, max_iter=5000, check_every=7)
    assert r.status == 0 and abs(r.iters - ora.iters) <= 1
    assert rel(host(x), ora.x) <= 1e-8
    for prec in (nbx.F32, nbx.F16):
        xm, rm = st.problem.pcg(st.b, rtol=1e-10, max_iter=8000, check_every=7, prec=prec)
        print(f"  prec {prec}: {rm.iters} it, {rm.outer_iters} updates, "
              f"true relres {rm.true_relres:.2e}")
        assert rm.status == 0 and rm.true_relres <= 2e-10
        assert rel(host(xm), ora.x) <= 1e-7


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_mixed_solve_with_interior_shared_node(prec):
    """Mixed solves on a plan that identifies two element-interior nodes
    (an unusual but valid SPD assembly: the exchange then also joins
    interior copies) agree with the FP64 solve."""
    ex, N = 2, 5
    gid, bnd = nbx.brick_ids(ex, 1, 1, N)
    N3 = N ** 3
    interior = (2 * N + 2) * N + 2                 # node (2, 2, 2) of each element
    gid = gid.copy()
    gid[N3 + interior] = gid[interior]
    gs = nbx.GS(gid, bnd)
    D = nbx.deriv_device(N)
    G, _, _ = nbx.geom_brick(ex, 1, 1, N)
    P = nbx.Problem(G, D, N, gs)
    b = torch.ones((ex, N3), dtype=torch.float64, device=DEV)
    gs.dssum(b)
    x64, r64 = P.pcg(b, rtol=1e-10, max_iter=500)
    x, r = P.pcg(b, rtol=1e-10, max_iter=2000, prec={"f32": nbx.F32, "f16": nbx.F16}[prec])
    print(f"{prec}: {r.iters} it, true relres {r.true_relres:.2e} (FP64 {r64.iters} it)")
    assert r64.status == 0 and r.status == 0 and r.true_relres <= 2e-10
    assert rel(host(x), host(x64)) <= 1e-8


@pytest.mark.parametrize("dims,N", [((1, 3, 2), 4), ((5, 2, 3), 2), ((4, 3, 3), 7),
                                    ((3, 2, 2), 16), ((7, 1, 1), 10), ((2, 5, 4), 5),
                                    ((1, 1, 1), 6)])
def test_x_face_pairs_summed_in_the_update_are_bit_identical(dims, N):
    """The solvers' iterations sum the two-copy x-face groups inside the
    update kernel instead of the exchange; nbx_pcg_iterate_noalloc runs the
    same iterations with the full exchange plan.  The two sums are formed in
    the same order, so every vector and scalar agrees bit for bit.  The pair
    offset is the brick's x element stride N^3 - N + 1 (no pairs with one
    element in x, and none at N = 2, where every face node is an element
    corner with four or more copies or lies on the Dirichlet boundary)."""
    print(f"x-pair update vs full exchange dims={dims} N={N}", flush=True)
    ex, ey, ez = dims
    b = S.Brick(*dims, N, ((0.05, 2, 2, 2),) * 3)
    st = nbx.setup_brick(*dims, N, b.deform_array())
    info = st.problem.exchange_info()
    want = (N ** 3 - N + 1 if ex > 1 and N > 2 else 0, 0, 0)
    print(f"  {info}", flush=True)
    assert info["pair_offsets"] == want
    assert (info["solver_groups"] < info["full_groups"]) == (want[0] != 0)
    bh = host(st.b).reshape(-1)
    dinv = st.problem.dinv()
    c = 1.0 / host(st.gs.multiplicity())
    z = host(dinv).reshape(-1) * bh
    scal = np.zeros(nbx.SCAL_LEN)
    scal[nbx.S_RHO] = float(np.sum(c * bh * z))
    scal[nbx.S_STOP] = -1.0
    scal[nbx.S_MAXIT] = 1e9
    s0 = [np.zeros_like(bh), bh, z, np.zeros_like(bh), scal]
    ref = [torch.as_tensor(a.copy()).cuda() for a in s0]
    new = [torch.as_tensor(a.copy()).cuda() for a in s0]
    w = torch.empty_like(ref[0])
    st.problem.pcg_iterate(*ref, n_iter=9)
    nbx.pcg_iterate_noalloc(nbx.pair_factors(st.G, N), st.D, N, st.gs, dinv, *new[:4], w,
                            new[4], n_iter=9)
    for name, a, c_ in zip(("x", "r", "z", "p", "scal"), ref, new):
        assert np.array_equal(host(a), host(c_)), name
    assert host(ref[4])[nbx.S_ITER] == 9
