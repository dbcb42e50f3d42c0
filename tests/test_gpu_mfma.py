"""The FP32 operator on matrix cores (nbx_ax_mfma, and the mixed solve's
inner operator with inner_mfma) against the oracle's single-precision AX.

Tolerance: FP32 products with FP32 accumulation in a different order from
the oracle's, 16 N single-precision unit round-offs normwise (as the
vector-unit FP32 kernel); against the FP64 oracle the FP32 storage error
is reported and gated at a few hundred unit round-offs.  Solves with the
matrix-core inner operator are checked like the other mixed solves: FP64
true residual by the oracle's own operator and the FP64 oracle solution."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from oracle import g16

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_04981_amd as nbx  # noqa: E402

EPS = np.finfo(np.float32).eps


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("N,E", [(2, 3), (3, 5), (4, 17), (5, 2), (6, 33), (7, 4), (8, 9),
                                 (9, 3), (10, 65), (11, 2), (12, 7), (13, 2), (16, 3)])
def test_ax_mfma_fp32_matches_oracle(N, E):
    print(f"mfma AX N={N} E={E}", flush=True)
    u = S.uniform_field(E, N, seed=N).astype(np.float32)
    G = S.random_factors(E, N, seed=N + 1).astype(np.float32)
    want = O.ax_f32(u, G, O.deriv(N))
    got = host(nbx.ax_mfma(cuda(u, torch.float32), cuda(G, torch.float32),
                           nbx.deriv_device(N)))
    assert rel(got, want) <= 16 * N * EPS
    w64 = O.ax(u.astype(np.float64), G.astype(np.float64), O.deriv(N))
    assert rel(got, w64) <= 300 * EPS


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("N,E", [(6, 9), (8, 20), (10, 33), (12, 5)])
def test_ax_mfma_16bit_factors_match_fp32_oracle(fmt, N, E):
    """16-bit factors with per-element scales: the dequantised factors in
    FP32 are the reference (elements over twelve decades of magnitude)."""
    gp = {"f16": nbx.F16, "bf16": nbx.BF16}[fmt]
    G = S.random_factors(E, N, seed=100 + N) * np.logspace(-10, 2, E)[:, None, None]
    u = S.uniform_field(E, N, seed=N).astype(np.float32)
    words, gs = g16.pack(G, N, fmt)
    Gd = g16.unpack(words, gs, N, fmt)
    want = O.ax_f32(u, Gd.astype(np.float32), O.deriv(N))
    G16, gsc = nbx.g16_pack(cuda(G), N, gp)
    got = host(nbx.ax_mfma(cuda(u, torch.float32), G16, nbx.deriv_device(N), gprec=gp,
                           gscale=gsc))
    for e in range(E):
        assert rel(got[e], want[e]) <= 16 * N * EPS, e


def test_ax_mfma_argument_errors():
    N, E = 4, 2
    u = torch.zeros((E, N ** 3), dtype=torch.float32, device="cuda")
    G = torch.zeros((E, 6, N ** 3), dtype=torch.float32, device="cuda")
    D = nbx.deriv_device(N)
    L = nbx.lib()
    with pytest.raises(ValueError):
        nbx.ax_mfma(u, G[:1], D)
    assert L.nbx_ax_mfma(nbx.F64, nbx._dptr(u), nbx._dptr(G), None, nbx._dptr(D), N, E,
                         nbx._dptr(torch.empty_like(u)), None) == -2
    assert L.nbx_ax_mfma(nbx.F32, nbx._dptr(u), nbx._dptr(G), None, nbx._dptr(D), N, E,
                         nbx._dptr(u), None) == -1               # u == w
    assert L.nbx_ax_mfma(nbx.F32, nbx._dptr(u), nbx._dptr(G), None, nbx._dptr(D), 17, E,
                         nbx._dptr(torch.empty_like(u)), None) == -1
    assert L.nbx_ax_mfma(nbx.F32, None, None, None, None, N, 0, None, None) == 0   # E = 0


@pytest.mark.parametrize("prec,N", [("f32", 8), ("f16", 10), ("bf16", 6), ("f16", 12)])
def test_mixed_solve_with_matrix_core_inner_operator(prec, N):
    b = S.scaled_c2_brick(3 if N >= 10 else 4, N)
    print(f"mixed solve {prec} N={N} on matrix cores", flush=True)
    P = O.setup(b)
    ref = O.pcg(P, max_iter=5000, rtol=1e-13)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, N, b.deform_array())
    p = {"f32": nbx.F32, "f16": nbx.F16, "bf16": nbx.BF16}[prec]
    x, r = st.problem.pcg(st.b, rtol=1e-10, max_iter=10000, prec=p, inner_rtol=0.1,
                          inner_mfma=1, check_every=7)
    _, rv = st.problem.pcg(st.b, rtol=1e-10, max_iter=10000, prec=p, inner_rtol=0.1,
                           check_every=7)
    print(f"  {r.iters} it / {r.outer_iters} updates (vector-unit kernel {rv.iters} it), "
          f"true relres {r.true_relres:.2e}")
    assert r.status == 0 and r.flag == 1 and r.fell_back == 0
    xh = host(x).reshape(-1)
    true = P.b - P.apply_A(xh)
    assert np.sqrt(O.wdot(P.c, true, true) / O.wdot(P.c, P.b, P.b)) <= 2e-10
    assert rel(xh, ref.x) <= 1e-8
    # the inner operator changed, not the method: a similar iteration count
    assert r.iters <= 1.2 * rv.iters + 10


def test_batched_refuses_matrix_core_inner_operator():
    b = S.scaled_c2_brick(2, 6)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, 6, b.deform_array())
    with pytest.raises(nbx.NbxError):
        nbx.pcg_batched([st.problem], [st.b], prec=nbx.F32, inner_mfma=1)
