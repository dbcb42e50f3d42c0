"""The allocation-free entry point nbx_pcg_iterate_noalloc against
nbx_pcg_iterate on the same state: both run the same kernels in the same
order, so every vector and scalar must agree bit for bit.  Two calls in a
row, the second on a smaller problem, check that the shared device scratch
carries nothing from one call into the next; a problem whose partial sums
exceed the scratch is refused before anything runs."""
import numpy as np
import pytest

import synthetic as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2011_04981_amd as nbx  # noqa: E402


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _start(st):
    """x = 0, r = b, z = dinv r, p = 0 (the first step takes p = z), and the
    scalar block (rho = <r, z>_c, no stopping test)."""
    b = host(st.b).reshape(-1)
    dinv = host(st.problem.dinv()).reshape(-1)
    c = 1.0 / host(st.gs.multiplicity())
    z = dinv * b
    scal = np.zeros(nbx.SCAL_LEN)
    scal[nbx.S_RHO] = float(np.sum(c * b * z))
    scal[nbx.S_STOP] = -1.0
    scal[nbx.S_MAXIT] = 1e9
    return [np.zeros_like(b), b, z, np.zeros_like(b), scal]


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("order", [(6, 10), (8, 6), (16, 8)])
def test_noalloc_iterations_equal_the_allocating_entry_point(order):
    """Two calls in a row: a 6x5x4 brick, then a smaller problem (3x3x2,
    fewer local nodes in both orders)."""
    for dims, N in (((6, 5, 4), order[0]), ((3, 3, 2), order[1])):
        print(f"noalloc vs pcg_iterate dims={dims} N={N}", flush=True)
        b = S.Brick(*dims, N, ((0.05, 2, 2, 2),) * 3)
        st = nbx.setup_brick(*dims, N, b.deform_array())
        s0 = _start(st)
        ref = [_cuda(a) for a in s0]
        new = [_cuda(a) for a in s0]
        Gp = nbx.pair_factors(st.G, N)
        dinv = st.problem.dinv()
        w = torch.full_like(ref[0], float("nan"))
        st.problem.pcg_iterate(*ref, n_iter=7)
        nbx.pcg_iterate_noalloc(Gp, st.D, N, st.gs, dinv, *new[:4], w, new[4], n_iter=7)
        for name, a, c in zip(("x", "r", "z", "p", "scal"), ref, new):
            assert np.array_equal(host(a), host(c)), name
        assert np.all(np.isfinite(host(w)))
        assert host(new[4])[nbx.S_ITER] == 7


def test_noalloc_refuses_a_problem_beyond_its_scratch():
    """E elements of N = 2 with more fused-stage workgroups than the
    scratch holds partial sums for: refused with NBX_EUNSUPPORTED before
    any launch (the vectors are never touched)."""
    N = 2
    tile = nbx.get_pcg_tile(nbx.F64, N)
    E = nbx.NOALLOC_MAX_BLOCKS * tile + 1
    gs = nbx.GS(np.arange(E * N ** 3, dtype=np.int64))
    one = torch.zeros(16, dtype=torch.float64, device="cuda")
    L = nbx.lib()
    p = nbx._dptr(one)
    st = L.nbx_pcg_iterate_noalloc(p, p, N, E, gs.handle, p, p, p, p, p, p, p, 1, None)
    assert st == -2
