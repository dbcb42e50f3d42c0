"""16-bit geometric factors (nbx_g16_pack, nbx_ax_g16) and the mixed-
precision solve that uses them as its inner operator, against the
reference (oracle/g16.py, the FP32 and FP64 oracle AX, the FP64 oracle
PCG).

Bars: the packed words are bit-identical (both sides round FP64 -> FP32 ->
16 bits to nearest-even); AX agrees with the FP32 oracle AX on the
dequantised factors to FP32 rounding (16 N eps, as the FP32 AX test: the
power-of-two scale commutes with rounding); solves reach a 1e-10 FP64 true
residual."""
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

FMT = {"f16": nbx.F16, "bf16": nbx.BF16}


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _factors(E, N, seed):
    # element magnitudes over twelve decades (as from element sizes 1..1e-4)
    G = S.random_factors(E, N, seed=seed)
    return G * np.logspace(-10, 2, E)[:, None, None]


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("N,E", [(2, 3), (5, 17), (10, 33), (16, 4)])
def test_pack_bit_exact(fmt, N, E):
    G = _factors(E, N, seed=N)
    G[1] = 0.0                                         # an all-zero element
    words, gs = g16.pack(G, N, fmt)                   # [E, 6, N^3]
    w_gpu, gs_gpu = nbx.g16_pack(cuda(G), N, FMT[fmt])
    assert np.array_equal(host(gs_gpu), gs)
    # the library stores factor pairs (g1,g2), (g3,g4), (g5,g6) per node
    want = words.reshape(E, 3, 2, N ** 3).transpose(0, 1, 3, 2)
    assert np.array_equal(host(w_gpu).view(np.uint16), want)


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("N,E", [(3, 7), (8, 20), (10, 65), (12, 9), (16, 3)])
def test_ax_g16_matches_fp32_oracle(fmt, N, E):
    print(f"ax_g16 {fmt} N={N} E={E}", flush=True)
    G = _factors(E, N, seed=100 + N)
    u = S.uniform_field(E, N, seed=N).astype(np.float32)
    words, gs = g16.pack(G, N, fmt)
    Gd = g16.unpack(words, gs, N, fmt)                 # exactly representable in FP32
    want = O.ax_f32(u, Gd.astype(np.float32), O.deriv(N))
    G16, gsc = nbx.g16_pack(cuda(G), N, FMT[fmt])
    got = host(nbx.ax_g16(cuda(u, torch.float32), G16, gsc, nbx.deriv_device(N), FMT[fmt]))
    for e in range(E):                                 # elements span twelve decades
        err = rel(got[e], want[e])
        assert err <= 16 * N * np.finfo(np.float32).eps, (e, err)
    # against FP64 AX with the exact factors: the storage error is reported
    w64 = O.ax(u.astype(np.float64), G, O.deriv(N))
    worst = max(rel(got[e], w64[e]) for e in range(E))
    print(f"{fmt} N={N}: worst element error vs FP64 AX with exact G {worst:.2e}")
    assert worst <= 64 * g16.unit_roundoff(fmt)


def test_g16_argument_errors():
    N, E = 4, 2
    G = cuda(_factors(E, N, 1))
    with pytest.raises(nbx.NbxError):
        nbx.g16_pack(G, N, nbx.F32)                    # not a 16-bit format
    G16, gs = nbx.g16_pack(G, N, nbx.F16)
    u = torch.zeros((E, N ** 3), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        nbx.ax_g16(u, G16, gs[:1], nbx.deriv_device(N), nbx.F16)
    # E = 0 is a no-op
    z = torch.zeros((0, N ** 3), dtype=torch.float32, device="cuda")
    nbx.ax_g16(z, torch.zeros((0, 6, N ** 3), dtype=torch.int16, device="cuda"),
               torch.zeros(0, dtype=torch.float32, device="cuda"), nbx.deriv_device(N), nbx.F16)


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
@pytest.mark.parametrize("mode", [0, 1])
def test_mixed_solve_with_16bit_operator(fmt, mode):
    b = S.scaled_c2_brick(4, 8)
    P = O.setup(b)
    ref = O.pcg(P, max_iter=5000, rtol=1e-13)
    st = nbx.setup_brick(b.ex, b.ey, b.ez, b.N, b.deform_array())
    x, res = st.problem.pcg(st.b, rtol=1e-10, max_iter=8000, prec=FMT[fmt],
                            inner_rtol=0.1 if mode == 0 else 1e-3, mixed_mode=mode)
    print(f"{fmt} mode {mode}: {res.iters} it, {res.outer_iters} outer, fell back "
          f"{res.fell_back}, relres {res.true_relres:.2e} (fp64 oracle {ref.iters} it)")
    assert res.status == 0 and res.flag == 1
    xh = host(x).reshape(-1)
    true = P.b - P.apply_A(xh)
    assert np.sqrt(O.wdot(P.c, true, true) / O.wdot(P.c, P.b, P.b)) <= 2e-10
    assert rel(xh, ref.x) <= 1e-8
    # the same problem again in FP32 then 16 bits: the formats switch cleanly
    x2, r2 = st.problem.pcg(st.b, rtol=1e-10, max_iter=8000, prec=nbx.F32)
    x3, r3 = st.problem.pcg(st.b, rtol=1e-10, max_iter=8000, prec=FMT[fmt],
                            inner_rtol=0.1 if mode == 0 else 1e-3, mixed_mode=mode)
    assert r2.flag == 1 and r3.flag == 1 and r3.iters == res.iters
    assert np.array_equal(host(x3), host(x))
