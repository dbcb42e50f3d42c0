"""The FP64 operator at N = 16 on the matrix cores: nbx_ax and nbx_ax_paired
run FP64 at N = 16 on ax16_mfma.hip's kernel; nbx_ax_tiled (an explicit
tile) keeps the vector-unit kernel.

Tolerance: normwise relative 1e-12 against the FP64 oracle, as for every
FP64 operator (max|gpu - oracle| <= 1e-12 max|oracle|, per element where
elements differ in scale).  At the paper's sizes (E = 800 and 8000, the
launches bench.py times) the oracle checks sampled elements, each computed
on its own, and the whole output is compared with the vector-unit kernel at
the same bound."""
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
N = 16


def cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("E", [1, 2, 7])
def test_ax16_matches_oracle_both_layouts(E):
    print(f"ax16 E={E}", flush=True)
    u = S.uniform_field(E, N, seed=160 + E)
    G = S.random_factors(E, N, seed=170 + E)
    D = nbx.deriv_device(N)
    w = host(nbx.ax(cuda(u), cuda(G), D))
    assert rel(w, O.ax(u, G, O.deriv(N))) <= TOL
    # the factor-pair layout runs the same kernel on the same values
    assert np.array_equal(host(nbx.ax_paired(cuda(u), cuda(pairs(G)), D)), w)


def test_ax16_on_deformed_geometry():
    """The deformed brick's factors: the operator on the oracle's factors at
    1e-12; each side's own factors agree at 1e-12, and AX on each side's
    own factors at 1e-11 (the derivative stencil, entries up to 60 at
    N = 16, amplifies the factors' last-bit differences, as on the full-size
    N = 10 brick)."""
    b = S.Brick(2, 2, 2, N, ((0.05, 2, 2, 2),) * 3)
    print("ax16 on the deformed 2x2x2 brick", flush=True)
    P = O.setup(b)
    G, _, _ = nbx.geom_brick(b.ex, b.ey, b.ez, N, b.deform_array(), with_xyz=True)
    assert rel(host(G), P.G) <= TOL
    u = S.uniform_field(b.E, N, seed=5)
    want = O.ax(u, P.G, P.D)
    D = nbx.deriv_device(N)
    assert rel(host(nbx.ax(cuda(u), cuda(P.G), D)), want) <= TOL
    assert rel(host(nbx.ax(cuda(u), G, D)), want) <= 1e-11


def test_ax16_element_scales_over_many_decades():
    """Factors scaled per element from 1e-150 to 1e150: every element is
    checked against the oracle on its own scale."""
    E = 9
    u = S.uniform_field(E, N, seed=7)
    G = S.random_factors(E, N, seed=8) * np.logspace(-150, 150, E)[:, None, None]
    w = host(nbx.ax(cuda(u), cuda(G), nbx.deriv_device(N)))
    want = O.ax(u, G, O.deriv(N))
    for e in range(E):
        assert rel(w[e], want[e]) <= TOL, e


@pytest.mark.parametrize("E", [800, 8000])
def test_ax16_paper_sizes(E):
    """The replay sizes (bench.py's seeded inputs and launch): sampled
    elements against the oracle, every element against the vector-unit
    kernel."""
    print(f"ax16 at the paper size E={E}", flush=True)
    u = S.uniform_field(E, N, seed=0)
    G = S.random_factors(E, N, seed=1)
    ud, Gd = cuda(u), cuda(G)
    D = nbx.deriv_device(N)
    w = host(nbx.ax(ud, Gd, D))
    assert np.isfinite(w).all()
    rng = np.random.default_rng(E)
    idx = np.unique(np.concatenate([[0, 1, E // 2, E - 1], rng.integers(0, E, 6)]))
    assert rel(w[idx], O.ax(u[idx], G[idx], O.deriv(N))) <= TOL
    wv = host(nbx.ax(ud, Gd, D, epb=1))                   # the vector-unit kernel
    assert rel(w, wv) <= TOL
