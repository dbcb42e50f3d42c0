"""FP64 CPU oracle for the spectral-element Poisson path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  It shares no code
with the HIP path (``paper_2011_04981_amd``) and never imports it.

The arithmetic lives in ``oracle.c`` (plain C, IEEE double, no fused
multiply-add); this module marshals numpy arrays into it and adds the few
steps that are plain elementwise numpy (the manufactured source term).
The MLP reference used by the learned preconditioner is in ``oracle.mlp``.

Parity status: every function here is pinned by tests under ``tests/``
against closed forms, brute-force dense matrices, exact integrals or
invariants (see each function's docstring for its pin).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_d = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def lib():
    """Loads liboracle.so, building it with gcc if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(HERE, "liboracle.so")
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    L = C.CDLL(path)
    L.ora_gll.argtypes = [C.c_int, _d, _d]
    L.ora_gll.restype = C.c_int
    L.ora_deriv.argtypes = [C.c_int, _d, _d]
    L.ora_brick_coords.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _d, _d, _d, _d, _d]
    L.ora_geom.argtypes = [C.c_int, C.c_int64, _d, _d, _d, _d, _d, _d, C.c_void_p]
    L.ora_geom.restype = C.c_double
    L.ora_brick_ids.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _i64, _u8]
    L.ora_ax.argtypes = [C.c_int, C.c_int64, _d, _d, _d, _d]
    L.ora_gs_create.argtypes = [_i64, C.c_int64]
    L.ora_gs_create.restype = C.c_void_p
    L.ora_gs_free.argtypes = [C.c_void_p]
    L.ora_dssum.argtypes = [C.c_void_p, _d]
    L.ora_mask.argtypes = [_u8, C.c_int64, _d]
    L.ora_multiplicity.argtypes = [C.c_void_p, _d]
    L.ora_jacobi_diag.argtypes = [C.c_int, C.c_int64, _d, _d, _d]
    L.ora_wdot.argtypes = [C.c_int64, _d, _d, _d]
    L.ora_wdot.restype = C.c_double
    L.ora_pcg_iterate.argtypes = [C.c_int, C.c_int64, _d, _d, C.c_void_p, _u8, _d, _d,
                                  _d, _d, _d, _d, _d, C.POINTER(C.c_double), C.c_int,
                                  C.c_double, C.c_void_p, C.POINTER(C.c_int)]
    L.ora_pcg_iterate.restype = C.c_int
    L.ora_pcg.argtypes = [C.c_int, C.c_int64, _d, _d, C.c_void_p, _u8, _d, _d, _d,
                          _d, _d, _d, _d, _d, C.c_int, C.c_double, C.c_void_p,
                          C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.ora_pcg.restype = C.c_int
    L.ora_num_threads.restype = C.c_int
    L.ora_set_num_threads.argtypes = [C.c_int]
    _f = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
    L.ora_ax_f32.argtypes = [C.c_int, C.c_int64, _f, _f, _d, _f]
    L.ora_dssum_f32.argtypes = [C.c_void_p, _f]
    _LIB = L
    return L


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------- basics

def gll(N: int):
    """GLL nodes and weights (pinned by closed forms for N=2,3,4, sum of
    weights, and exact quadrature to degree 2N-3)."""
    xi = np.zeros(N); w = np.zeros(N)
    if lib().ora_gll(N, xi, w) != 0:
        raise ValueError(f"GLL failed for N={N}")
    return xi, w


def deriv(N: int, xi: Optional[np.ndarray] = None) -> np.ndarray:
    """Row-major derivative matrix D[a, b] = l_b'(xi_a) (pinned by exact
    differentiation of polynomials of degree <= N-1 and the N=3 closed form)."""
    if xi is None:
        xi = gll(N)[0]
    D = np.zeros((N, N))
    lib().ora_deriv(N, _c(xi), D)
    return D


def brick_coords(brick, xi):
    N = brick.N
    n = brick.E * N ** 3
    x = np.zeros(n); y = np.zeros(n); z = np.zeros(n)
    lib().ora_brick_coords(brick.ex, brick.ey, brick.ez, N, _c(xi),
                           _c(brick.deform_array().ravel()), x, y, z)
    return x, y, z


def geom(N, D, w, x, y, z):
    """Geometric factors G[E][6][N^3] and mass bm[E][N^3]; returns
    (G, bm, min det J)."""
    N3 = N ** 3
    E = x.size // N3
    G = np.zeros(E * 6 * N3); bm = np.zeros(E * N3)
    jmin = lib().ora_geom(N, E, _c(D), _c(w), _c(x), _c(y), _c(z), G,
                          bm.ctypes.data_as(C.c_void_p))
    return G.reshape(E, 6, N3), bm.reshape(E, N3), jmin


def brick_ids(brick):
    n = brick.E * brick.N ** 3
    gid = np.zeros(n, dtype=np.int64); bnd = np.zeros(n, dtype=np.uint8)
    lib().ora_brick_ids(brick.ex, brick.ey, brick.ez, brick.N, gid, bnd)
    return gid, bnd


def ax(u, G, D, N: Optional[int] = None):
    """w = AX(u) element by element (w_e = D^T G_e D u_e).  u: (E, N^3) or flat,
    G: (E, 6, N^3), D: (N, N) row-major."""
    D = _c(D)
    N = D.shape[0] if N is None else N
    N3 = N ** 3
    u = _c(u).reshape(-1)
    E = u.size // N3
    w = np.zeros(E * N3)
    lib().ora_ax(N, E, u, _c(G).reshape(-1), D, w)
    return w.reshape(E, N3)


class GS:
    """Gather-scatter (dssum) over nodes that share a global id."""

    def __init__(self, gid):
        self.gid = _c(gid, np.int64).reshape(-1)
        self.n = self.gid.size
        self._h = lib().ora_gs_create(self.gid, self.n)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().ora_gs_free(self._h)
            self._h = None

    def dssum(self, v):
        v = np.array(v, dtype=np.float64, copy=True).reshape(-1)
        lib().ora_dssum(self._h, v)
        return v

    def multiplicity(self):
        m = np.zeros(self.n)
        lib().ora_multiplicity(self._h, m)
        return m


def mask(bnd, v):
    v = np.array(v, dtype=np.float64, copy=True).reshape(-1)
    lib().ora_mask(_c(bnd, np.uint8).reshape(-1), v.size, v)
    return v


def jacobi_diag(G, D):
    """Unassembled diagonal of every A_e (closed form; pinned by the
    diagonal of the brute-force dense A_e)."""
    D = _c(D); N = D.shape[0]; N3 = N ** 3
    G = _c(G).reshape(-1); E = G.size // (6 * N3)
    d = np.zeros(E * N3)
    lib().ora_jacobi_diag(N, E, G, D, d)
    return d


def wdot(c, a, b) -> float:
    a = _c(a).reshape(-1)
    return lib().ora_wdot(a.size, _c(c).reshape(-1), a, _c(b).reshape(-1))


def sine_source(x, y, z):
    """f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z), so that -lap u* = f for
    u* = sin(pi x) sin(pi y) sin(pi z), which vanishes on the cube's
    boundary."""
    return 3.0 * np.pi ** 2 * np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def exact_solution(x, y, z):
    return np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


# --------------------------------------------------------------- problem

@dataclass
class Problem:
    brick: object
    N: int
    E: int
    xi: np.ndarray
    w: np.ndarray
    D: np.ndarray
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    G: np.ndarray
    bm: np.ndarray
    jmin: float
    gid: np.ndarray
    bnd: np.ndarray
    gs: GS
    mult: np.ndarray
    c: np.ndarray
    dinv: np.ndarray
    b: np.ndarray

    @property
    def n(self) -> int:
        return self.E * self.N ** 3

    def apply_A(self, p):
        """mask(dssum(AX(p)))."""
        return mask(self.bnd, self.gs.dssum(ax(p, self.G, self.D).reshape(-1)))


def setup(brick, rhs_values=None) -> Problem:
    """Builds everything a solve needs from a workload description:
    GLL, D, coordinates, G, bm, global ids, boundary flags, multiplicity,
    c = 1/m, dinv = 1/dssum(diag) (0 on the boundary), and the load vector
    b = mask(dssum(bm * f)).  ``rhs_values`` overrides f with nodal values
    (the "random" right-hand side)."""
    N = brick.N
    xi, w = gll(N)
    D = deriv(N, xi)
    x, y, z = brick_coords(brick, xi)
    G, bm, jmin = geom(N, D, w, x, y, z)
    gid, bnd = brick_ids(brick)
    gs = GS(gid)
    mult = gs.multiplicity()
    c = 1.0 / mult
    d = gs.dssum(jacobi_diag(G, D))
    dinv = np.where(bnd.astype(bool), 0.0, 1.0 / d)
    if rhs_values is not None:
        f = _c(rhs_values).reshape(-1)
    elif brick.rhs == "sine":
        f = sine_source(x, y, z)
    else:
        raise ValueError("a 'random' right-hand side needs rhs_values")
    b = mask(bnd, gs.dssum(bm.reshape(-1) * f))
    return Problem(brick, N, brick.E, xi, w, D, x, y, z, G, bm, jmin, gid, bnd,
                   gs, mult, c, dinv, b)


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    state: int          # 0 limit reached, 1 converged, 2 breakdown
    relres: float
    hist: np.ndarray


def pcg(P: Problem, b=None, max_iter=1000, rtol=1e-10) -> PCGResult:
    """Jacobi-PCG from x = 0 (ora_pcg)."""
    n = P.n
    b = P.b if b is None else _c(b).reshape(-1)
    x = np.zeros(n); r = np.zeros(n); z = np.zeros(n); p = np.zeros(n); w = np.zeros(n)
    hist = np.zeros(max(max_iter, 1))
    st = C.c_int(0); rel = C.c_double(0)
    it = lib().ora_pcg(P.N, P.E, _c(P.G).reshape(-1), _c(P.D), P.gs._h,
                       _c(P.bnd, np.uint8), _c(P.dinv), _c(P.c), b, x, r, z, p, w,
                       max_iter, rtol, hist.ctypes.data_as(C.c_void_p),
                       C.byref(st), C.byref(rel))
    return PCGResult(x, it, st.value, rel.value, hist[:it].copy())


def pcg_start(P: Problem, b=None):
    """Initial CG state (x, r, z, p, rho) for x = 0."""
    b = P.b if b is None else _c(b).reshape(-1)
    x = np.zeros(P.n); r = b.copy(); z = P.dinv * r; p = z.copy()
    return x, r, z, p, wdot(P.c, r, z)


def pcg_iterate(P: Problem, state, n_iter: int, stop_rr: float = 0.0):
    """Advances (x, r, z, p, rho) by n_iter iterations (copies the state).
    Returns (x, r, z, p, rho, iters_done, flag, hist)."""
    x, r, z, p, rho = [np.array(a, dtype=np.float64, copy=True) if isinstance(a, np.ndarray)
                       else a for a in state]
    w = np.zeros(P.n)
    rho_c = C.c_double(float(rho)); st = C.c_int(0)
    hist = np.zeros(max(n_iter, 1))
    it = lib().ora_pcg_iterate(P.N, P.E, _c(P.G).reshape(-1), _c(P.D), P.gs._h,
                               _c(P.bnd, np.uint8), _c(P.dinv), _c(P.c), x, r, z, p, w,
                               C.byref(rho_c), n_iter, stop_rr,
                               hist.ctypes.data_as(C.c_void_p), C.byref(st))
    return x, r, z, p, rho_c.value, it, st.value, hist[:it].copy()


def ax_flops(N: int, E: int) -> int:
    """Flop count of one AX: E N^3 (12N + 11) (six length-N contractions at
    2N-1 flops, 15 for the geometric step, 2 for the two accumulations);
    pinned by the paper's 203 flops per point and 831488 per element at
    16 nodes per direction (Section II-B, Section III)."""
    return E * N ** 3 * (12 * N + 11)


def ax_f32(u, G, D):
    """AX in IEEE single arithmetic (u, G rounded to float, D rounded to
    float inside).  Pinned against the FP64 AX at single-precision accuracy."""
    D = _c(D); N = D.shape[0]; N3 = N ** 3
    u = np.ascontiguousarray(u, dtype=np.float32).reshape(-1)
    E = u.size // N3
    w = np.zeros(E * N3, dtype=np.float32)
    lib().ora_ax_f32(N, E, u, np.ascontiguousarray(G, dtype=np.float32).reshape(-1), D, w)
    return w.reshape(E, N3)


def dssum_f32(gs: GS, v):
    v = np.array(v, dtype=np.float32, copy=True).reshape(-1)
    lib().ora_dssum_f32(gs._h, v)
    return v


@dataclass
class IRResult:
    x: np.ndarray
    outer: int
    inner_iters: int
    relres: float


def _pcg32(P: Problem, G32, dinv32, r64, inner_rtol, max_iter):
    """Jacobi-PCG on A d = r in single precision: float vectors, float AX
    and dssum, dot products accumulated in double, alpha and beta in double
    applied as floats.  Same step order as ora_pcg_iterate."""
    c = P.c
    bnd = P.bnd.astype(bool)
    r = r64.astype(np.float32)
    d = np.zeros_like(r)
    z = dinv32 * r
    p = z.copy()
    rho = float(np.sum(c * r.astype(np.float64) * z.astype(np.float64)))
    stop = inner_rtol ** 2 * float(np.sum(c * r.astype(np.float64) ** 2))
    for k in range(max_iter):
        w = dssum_f32(P.gs, ax_f32(p, G32, P.D).reshape(-1))
        w[bnd] = 0.0
        pap = float(np.sum(p.astype(np.float64) * w.astype(np.float64) * c))
        alpha = rho / pap
        d += np.float32(alpha) * p
        r -= np.float32(alpha) * w
        rr = float(np.sum(c * r.astype(np.float64) ** 2))
        if rr <= stop:
            return d, k + 1
        z = dinv32 * r
        rho2 = float(np.sum(c * r.astype(np.float64) * z.astype(np.float64)))
        beta = rho2 / rho
        rho = rho2
        p = z + np.float32(beta) * p
    return d, max_iter


def ir_solve(P: Problem, b=None, rtol=1e-10, inner_rtol=1e-5, max_outer=20,
             max_inner=5000) -> IRResult:
    """Iterative refinement (Wilkinson; Moler 1967; Carson & Higham 2018):
    x = 0, r = b; repeat: solve A d = r in single precision to inner_rtol,
    x += d, r = b - A x in double, until ||r||_c <= rtol ||b||_c."""
    b = P.b if b is None else _c(b).reshape(-1)
    G32 = P.G.astype(np.float32)
    dinv32 = P.dinv.astype(np.float32)
    x = np.zeros(P.n)
    r = b.copy()
    bb = wdot(P.c, b, b)
    total = 0
    rel = np.sqrt(wdot(P.c, r, r) / bb) if bb > 0 else 0.0
    outer = 0
    while rel > rtol and outer < max_outer:
        d, it = _pcg32(P, G32, dinv32, r, inner_rtol, max_inner)
        total += it
        outer += 1
        x += d.astype(np.float64)
        r = b - P.apply_A(x)
        rel = np.sqrt(wdot(P.c, r, r) / bb)
    return IRResult(x, outer, total, float(rel))


def num_threads() -> int:
    return lib().ora_num_threads()


def set_num_threads(n: int) -> None:
    lib().ora_set_num_threads(int(n))
