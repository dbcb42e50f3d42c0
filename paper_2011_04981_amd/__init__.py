"""MI355X-native spectral-element Poisson hot path (matrix-free AX, dssum,
Jacobi-PCG) -- Python binding of libnbx.

This module only marshals arguments into the C ABI declared in
include/nbx.h; every step of the computation runs in the library's HIP
kernels.  torch supplies device memory and streams.  If libnbx.so has not
been built the import of any compute entry point fails loudly: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbx.so")

F64, F32, BF16, F16 = 0, 1, 2, 3
SCAL_LEN = 16
NOALLOC_MAX_BLOCKS = 262144   # partial sums nbx_pcg_iterate_noalloc can hold
S_RHO, S_BETA, S_ALPHA, S_PAP, S_RR, S_BB, S_STOP, S_FLAG, S_ITER, S_MAXIT = range(10)

STATUS = {0: "ok", 1: "not converged", -1: "invalid argument", -2: "unsupported",
          -3: "HIP error", -4: "out of memory", -5: "CG breakdown"}


class NbxError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} (status {status})")


_lib = None


class PcgOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("fixed_iters", C.c_int), ("check_every", C.c_int),
                ("use_graph", C.c_int), ("rtol", C.c_double), ("prec", C.c_int),
                ("inner_rtol", C.c_double), ("max_outer", C.c_int),
                ("mixed_mode", C.c_int), ("inner_mfma", C.c_int)]


class PcgResult(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer_iters", C.c_int), ("relres", C.c_double),
                ("true_relres", C.c_double), ("fell_back", C.c_int), ("flag", C.c_int),
                ("seconds", C.c_double)]


def lib():
    """The loaded libnbx (raises if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                           "(python paper_2011_04981_amd/build.py) first")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "nbx_status_str": ([i32], C.c_char_p),
        "nbx_last_hip_error": ([], i32),
        "nbx_version": ([], i32),
        "nbx_copy_f64": ([vp, vp, i64, vp], i32),
        "nbx_stream_f64": ([i32, vp, vp, i64, vp, vp], i32),
        "nbx_gll": ([i32, vp, vp], i32),
        "nbx_deriv": ([i32, vp], i32),
        "nbx_geom_brick": ([i32, i32, i32, i32, vp, vp, vp, vp, vp], i32),
        "nbx_geom": ([vp, i32, i64, vp, vp, vp], i32),
        "nbx_brick_ids": ([i32, i32, i32, i32, vp, vp], i32),
        "nbx_ax": ([i32, vp, vp, vp, i32, i64, vp, vp], i32),
        "nbx_ax_tiled": ([i32, vp, vp, vp, i32, i64, vp, i32, vp], i32),
        "nbx_ax_paired": ([i32, vp, vp, vp, i32, i64, vp, vp], i32),
        "nbx_ax_paired_tiled": ([i32, vp, vp, vp, i32, i64, vp, i32, vp], i32),
        "nbx_ax_set_tile": ([i32, i32, i32], i32),
        "nbx_ax_get_tile": ([i32, i32], i32),
        "nbx_pcg_set_tile": ([i32, i32, i32], i32),
        "nbx_pcg_get_tile": ([i32, i32], i32),
        "nbx_gs_create": ([vp, i64, vp, C.POINTER(vp), vp], i32),
        "nbx_gs_destroy": ([vp], i32),
        "nbx_dssum": ([vp, i32, vp, i32, vp], i32),
        "nbx_gs_multiplicity": ([vp, vp, vp], i32),
        "nbx_jacobi_setup": ([vp, vp, i32, i64, vp, vp, vp], i32),
        "nbx_rhs": ([vp, vp, vp, i64, vp, vp], i32),
        "nbx_sine_source": ([vp, i64, vp, vp], i32),
        "nbx_problem_create": ([vp, vp, i32, i64, vp, C.POINTER(vp), vp], i32),
        "nbx_problem_destroy": ([vp], i32),
        "nbx_problem_dinv": ([vp, vp, vp], i32),
        "nbx_problem_exchange_info": ([vp, vp], i32),
        "nbx_repack_g_aos_to_soa": ([vp, vp, i32, i64, vp], i32),
        "nbx_pair_factors": ([vp, vp, i32, i64, vp], i32),
        "nbx_pcg_iterate": ([vp, vp, vp, vp, vp, vp, i32, vp], i32),
        "nbx_pcg_iterate_noalloc": ([vp, vp, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, i32,
                                     vp], i32),
        "nbx_pcg_default_opts": ([C.POINTER(PcgOpts)], None),
        "nbx_pcg": ([vp, vp, vp, C.POINTER(PcgOpts), C.POINTER(PcgResult), vp], i32),
        "nbx_pcg_batched": ([C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), i32,
                             C.POINTER(PcgOpts), C.POINTER(PcgResult), C.POINTER(dp), vp], i32),
        "nbx_gemm_bf16": ([i32, i32, i32, i32, i32, vp, i32, vp, i32, vp, i32, vp], i32),
        "nbx_mlp_create": ([i32, i32, i32, i32, C.POINTER(vp)], i32),
        "nbx_mlp_destroy": ([vp], i32),
        "nbx_mlp_shape": ([vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i64)], i32),
        "nbx_mlp_set_params": ([vp, vp, vp], i32),
        "nbx_mlp_get_params": ([vp, vp, vp, vp], i32),
        "nbx_mlp_forward": ([vp, vp, i32, vp, vp], i32),
        "nbx_mlp_grad": ([vp, vp, vp, i32, vp, vp], i32),
        "nbx_mlp_train_step": ([vp, vp, vp, i32, C.c_float, vp, vp], i32),
        "nbx_g16_pack": ([i32, vp, i32, i64, vp, vp, vp], i32),
        "nbx_ax_g16": ([i32, vp, vp, vp, vp, i32, i64, vp, vp], i32),
        "nbx_ax_mfma": ([i32, vp, vp, vp, vp, i32, i64, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    _apply_tile_cache(L)
    return L


def _apply_tile_cache(L) -> None:
    """Installs the autotuner's stored tiles (tiles.json next to this file, or
    $NBX_TILE_CACHE) into the library's tile table."""
    import json
    path = os.environ.get("NBX_TILE_CACHE", os.path.join(HERE, "tiles.json"))
    if not os.path.exists(path):
        return
    with open(path) as f:
        rec = json.load(f)
    for pname, rows in rec.get("tiles", {}).items():
        kind, _, pn = pname.rpartition("_")
        prec = {"f64": F64, "f32": F32, "g16": F16}.get(pn)
        setter = {"": L.nbx_ax_set_tile, "pcg": L.nbx_pcg_set_tile}.get(kind)
        if prec is None or setter is None:
            continue
        for N, row in rows.items():
            setter(prec, int(N), int(row["epb"]))


def _check(st: int, what: str) -> int:
    if st < 0:
        raise NbxError(st, what)
    return st


def _torch():
    import torch
    return torch


def _dptr(t, dtype=None, name="tensor"):
    """Device pointer of a contiguous, 16-byte aligned CUDA tensor (checked:
    the kernels read and write 16-byte vectors, so a view at another offset
    is refused)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.data_ptr() % 16:
        raise ValueError(f"{name} must start at a 16-byte aligned address")
    return C.c_void_p(t.data_ptr())


def _need(t, n: int, name: str):
    """The library reads or writes exactly n elements through this tensor:
    refuse anything else before a kernel can run past its end."""
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _hptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def copy_f64(src, dst, stream=None):
    """dst <- src with the library's streaming copy kernel."""
    torch = _torch()
    if src.numel() != dst.numel():
        raise ValueError("size mismatch")
    _check(lib().nbx_copy_f64(_dptr(src, torch.float64), _dptr(dst, torch.float64),
                              src.numel(), _stream(stream)), "nbx_copy_f64")
    return dst


# ----------------------------------------------------------------- set-up

def stream_f64(mode: int, src, dst=None, sink=None, stream=None):
    """Bandwidth references (nbx_stream_f64): mode 0 non-temporal copy
    src -> dst, mode 1 read-only stream over src."""
    torch = _torch()
    n = src.numel()
    if mode == 0:
        _need(dst, n, "dst")
    if mode == 1 and sink is None:
        sink = torch.zeros(1, dtype=torch.float64, device=src.device)
    _check(lib().nbx_stream_f64(mode, _dptr(src, torch.float64, "src"),
                                _dptr(dst, torch.float64, "dst") if mode == 0 else None, n,
                                _dptr(sink, torch.float64, "sink") if mode == 1 else None,
                                _stream(stream)), "nbx_stream_f64")


def gll(N: int):
    xi = np.zeros(N); w = np.zeros(N)
    _check(lib().nbx_gll(N, _hptr(xi), _hptr(w)), "nbx_gll")
    return xi, w


def deriv(N: int) -> np.ndarray:
    D = np.zeros((N, N))
    _check(lib().nbx_deriv(N, _hptr(D)), "nbx_deriv")
    return D


def deriv_device(N: int, device="cuda"):
    return _torch().from_numpy(deriv(N)).to(device)


def geom_brick(ex: int, ey: int, ez: int, N: int, deform=None, with_xyz=False,
               device="cuda", stream=None):
    """(G [E,6,N^3] one plane per factor, bm [E,N^3], xyz [3,E,N^3] or
    None) for a deformed brick, computed on the device."""
    torch = _torch()
    E = ex * ey * ez
    N3 = N ** 3
    G = torch.empty((E, 6, N3), dtype=torch.float64, device=device)
    bm = torch.empty((E, N3), dtype=torch.float64, device=device)
    xyz = torch.empty((3, E, N3), dtype=torch.float64, device=device) if with_xyz else None
    d = np.ascontiguousarray(deform if deform is not None else
                             [[0, 1, 1, 1]] * 3, dtype=np.float64).reshape(12)
    _check(lib().nbx_geom_brick(ex, ey, ez, N, _hptr(d), _dptr(G), _dptr(bm),
                                _dptr(xyz) if xyz is not None else None, _stream(stream)),
           "nbx_geom_brick")
    return G, bm, xyz


def geom(xyz, N: int, stream=None):
    torch = _torch()
    if xyz.dim() != 3 or xyz.shape[0] != 3 or xyz.shape[2] != N ** 3:
        raise ValueError("xyz must be [3, E, N^3]")
    E = xyz.shape[1]
    G = torch.empty((E, 6, N ** 3), dtype=torch.float64, device=xyz.device)
    bm = torch.empty((E, N ** 3), dtype=torch.float64, device=xyz.device)
    _check(lib().nbx_geom(_dptr(xyz, torch.float64, "xyz"), N, E, _dptr(G), _dptr(bm),
                          _stream(stream)), "nbx_geom")
    return G, bm


def _factor_layout(fn: str, src, N: int, out, stream, shape):
    torch = _torch()
    n6 = src.numel()
    if n6 % (6 * N ** 3):
        raise ValueError("the factors must hold 6 values for every node of whole elements")
    E = n6 // (6 * N ** 3)
    out = torch.empty((E, *shape), dtype=torch.float64, device=src.device) \
        if out is None else _need(out, n6, "out")
    _check(getattr(lib(), fn)(_dptr(src, torch.float64, "factors"),
                              _dptr(out, torch.float64, "out"), N, E, _stream(stream)), fn)
    return out


def repack_g_aos_to_soa(g_aos, N: int, out=None, stream=None):
    """Geometric factors in the layout of the operator's g argument,
    g(6, N^3, E) with the factor fastest (a float64 tensor of E*N^3*6 values,
    e.g. shaped [E, N^3, 6]), repacked on the device into one plane per
    factor, [E, 6, N^3], the layout every call takes."""
    return _factor_layout("nbx_repack_g_aos_to_soa", g_aos, N, out, stream, (6, N ** 3))


def pair_factors(g6, N: int, out=None, stream=None):
    """Geometric factors as one plane per factor, [E, 6, N^3] float64,
    repacked on the device into planes of factor pairs [E, 3, N^3, 2], the
    layout of ax_paired (nbx_pair_factors)."""
    return _factor_layout("nbx_pair_factors", g6, N, out, stream, (3, N ** 3, 2))


def brick_ids(ex: int, ey: int, ez: int, N: int):
    n = ex * ey * ez * N ** 3
    gid = np.zeros(n, dtype=np.int64); bnd = np.zeros(n, dtype=np.uint8)
    _check(lib().nbx_brick_ids(ex, ey, ez, N, _hptr(gid), _hptr(bnd)), "nbx_brick_ids")
    return gid, bnd


# --------------------------------------------------------------------- AX

def _ax_call(fn, fn_tiled, u, G, D, N, out, stream, epb, gshape):
    torch = _torch()
    N = D.shape[0] if N is None else N
    E = u.numel() // N ** 3
    _need(u, E * N ** 3, "u")
    _need(D, N * N, "D")
    prec = {torch.float64: F64, torch.float32: F32}.get(u.dtype)
    if prec is None:
        raise TypeError(f"unsupported dtype {u.dtype}")
    if G.dtype != u.dtype:
        raise TypeError("G and u must share a dtype")
    if tuple(G.shape) != (E, *gshape(N)):
        raise ValueError(f"G must be shaped {(E, *gshape(N))}, got {tuple(G.shape)}")
    w = torch.empty_like(u) if out is None else _need(out, u.numel(), "out")
    args = (prec, _dptr(u, name="u"), _dptr(G, name="G"), _dptr(D, torch.float64, "D"), N, E,
            _dptr(w, u.dtype, "w"))
    if epb is None:
        _check(getattr(lib(), fn)(*args, _stream(stream)), fn)
    else:
        _check(getattr(lib(), fn_tiled)(*args, int(epb), _stream(stream)), fn_tiled)
    return w


def ax(u, G, D, N: Optional[int] = None, out=None, stream=None, epb: Optional[int] = None):
    """w = AX(u) (nbx_ax) for u [E, N^3] (float64 or float32), G [E, 6, N^3]
    (one plane per factor) of the same dtype, D [N, N] float64 (device).
    epb forces a tile (elements per workgroup); by default the library's
    tile table decides."""
    return _ax_call("nbx_ax", "nbx_ax_tiled", u, G, D, N, out, stream, epb,
                    lambda N: (6, N ** 3))


def ax_paired(u, Gp, D, N: Optional[int] = None, out=None, stream=None,
              epb: Optional[int] = None):
    """The same operator on factor pairs Gp [E, 3, N^3, 2] (pair_factors'
    output; nbx_ax_paired)."""
    return _ax_call("nbx_ax_paired", "nbx_ax_paired_tiled", u, Gp, D, N, out, stream, epb,
                    lambda N: (3, N ** 3, 2))


def g16_pack(G, N: int, gprec: int, stream=None):
    """From G [E, 6, N^3] float64: (G16 [E, 3, N^3, 2] int16 words, gscale
    [E] float32), the factors in
    16-bit storage (gprec F16 or BF16) with per-element power-of-two
    scales, as factor pairs (g1,g2), (g3,g4), (g5,g6) per node
    (nbx_g16_pack)."""
    torch = _torch()
    E = G.shape[0]
    if tuple(G.shape) != (E, 6, N ** 3):
        raise ValueError(f"G must be shaped (E, 6, {N ** 3})")
    G16 = torch.empty((E, 3, N ** 3, 2), dtype=torch.int16, device=G.device)
    gs = torch.empty(E, dtype=torch.float32, device=G.device)
    _check(lib().nbx_g16_pack(gprec, _dptr(G, torch.float64, "G"), N, E, _dptr(G16),
                              _dptr(gs), _stream(stream)), "nbx_g16_pack")
    return G16, gs


def ax_g16(u, G16, gscale, D, gprec: int, out=None, stream=None):
    """w = AX(u) in FP32 with 16-bit factors (nbx_ax_g16)."""
    torch = _torch()
    N = D.shape[0]
    E = u.numel() // N ** 3
    if u.numel() != E * N ** 3 or G16.numel() != 6 * u.numel() or gscale.numel() != E:
        raise ValueError("u [E, N^3], G16 [E, 3, N^3, 2] and gscale [E] must agree")
    _need(D, N * N, "D")
    w = torch.empty_like(u) if out is None else out
    if w.numel() != u.numel():
        raise ValueError("out must match u")
    _check(lib().nbx_ax_g16(gprec, _dptr(u, torch.float32, "u"), _dptr(G16, torch.int16, "G16"),
                            _dptr(gscale, torch.float32, "gscale"), _dptr(D, torch.float64, "D"),
                            N, E, _dptr(w, torch.float32, "w"), _stream(stream)), "nbx_ax_g16")
    return w


def ax_mfma(u, G, D, gprec: int = F32, gscale=None, out=None, stream=None):
    """w = AX(u) in FP32 on matrix cores (nbx_ax_mfma): G float32
    [E, 6, N^3] for gprec F32, or 16-bit words from g16_pack with gscale."""
    torch = _torch()
    N = D.shape[0]
    E = u.numel() // N ** 3
    _need(u, E * N ** 3, "u")
    _need(D, N * N, "D")
    if gprec == F32:
        if tuple(G.shape) != (E, 6, N ** 3) or G.dtype != torch.float32:
            raise ValueError(f"G must be float32 shaped (E, 6, {N ** 3})")
        gp, sp = _dptr(G, torch.float32, "G"), None
    else:
        if G.numel() != 6 * E * N ** 3 or gscale is None or gscale.numel() != E:
            raise ValueError("G16 [E, 3, N^3, 2] and gscale [E] must match u")
        gp, sp = _dptr(G, torch.int16, "G16"), _dptr(gscale, torch.float32, "gscale")
    w = torch.empty_like(u) if out is None else _need(out, u.numel(), "out")
    _check(lib().nbx_ax_mfma(gprec, _dptr(u, torch.float32, "u"), gp, sp,
                             _dptr(D, torch.float64, "D"), N, E, _dptr(w, torch.float32, "w"),
                             _stream(stream)), "nbx_ax_mfma")
    return w


def set_tile(prec: int, N: int, epb: int) -> None:
    _check(lib().nbx_ax_set_tile(prec, N, epb), "nbx_ax_set_tile")


def get_tile(prec: int, N: int) -> int:
    return _check(lib().nbx_ax_get_tile(prec, N), "nbx_ax_get_tile")


def set_pcg_tile(prec: int, N: int, epb: int) -> None:
    """Tile of the solvers' fused first stage (nbx_pcg_set_tile)."""
    _check(lib().nbx_pcg_set_tile(prec, N, epb), "nbx_pcg_set_tile")


def get_pcg_tile(prec: int, N: int) -> int:
    return _check(lib().nbx_pcg_get_tile(prec, N), "nbx_pcg_get_tile")


# --------------------------------------------------------- gather-scatter

class GS:
    """dssum plan built from host global ids and Dirichlet flags."""

    def __init__(self, gid: np.ndarray, bnd: Optional[np.ndarray] = None):
        gid = np.ascontiguousarray(gid, dtype=np.int64).reshape(-1)
        self.n = gid.size
        b = None if bnd is None else np.ascontiguousarray(bnd, dtype=np.uint8).reshape(-1)
        if b is not None and b.size != self.n:
            raise ValueError("one Dirichlet flag per local node")
        h = C.c_void_p()
        _check(lib().nbx_gs_create(_hptr(gid), self.n, _hptr(b) if b is not None else None,
                                   C.byref(h), _stream(None)), "nbx_gs_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().nbx_gs_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dssum(self, v, mask: bool = True, stream=None):
        torch = _torch()
        prec = {torch.float64: F64, torch.float32: F32}[v.dtype]
        _need(v, self.n, "v")
        _check(lib().nbx_dssum(self._h, prec, _dptr(v), 1 if mask else 0, _stream(stream)),
               "nbx_dssum")
        return v

    def multiplicity(self, device="cuda", stream=None):
        torch = _torch()
        m = torch.empty(self.n, dtype=torch.float64, device=device)
        _check(lib().nbx_gs_multiplicity(self._h, _dptr(m), _stream(stream)),
               "nbx_gs_multiplicity")
        return m


def jacobi_setup(G, D, gs: GS, N: int, stream=None):
    torch = _torch()
    E = G.shape[0]
    if tuple(G.shape) != (E, 6, N ** 3):
        raise ValueError(f"G must be shaped (E, 6, {N ** 3})")
    _need(D, N * N, "D")
    if gs.n != E * N ** 3:
        raise ValueError("the gather-scatter plan does not match G")
    dinv = torch.empty((E, N ** 3), dtype=torch.float64, device=G.device)
    _check(lib().nbx_jacobi_setup(_dptr(G, torch.float64), _dptr(D, torch.float64), N, E,
                                  gs.handle, _dptr(dinv), _stream(stream)), "nbx_jacobi_setup")
    return dinv


def sine_source(xyz, stream=None):
    """f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) at the nodes xyz [3, ...]."""
    torch = _torch()
    n = xyz[0].numel()
    f = torch.empty(xyz.shape[1:], dtype=torch.float64, device=xyz.device)
    _check(lib().nbx_sine_source(_dptr(xyz, torch.float64, "xyz"), n, _dptr(f),
                                 _stream(stream)), "nbx_sine_source")
    return f


def rhs(gs: GS, bm, f, stream=None):
    torch = _torch()
    _need(bm, gs.n, "bm")
    _need(f, gs.n, "f")
    b = torch.empty_like(bm)
    _check(lib().nbx_rhs(gs.handle, _dptr(bm, torch.float64), _dptr(f, torch.float64),
                         bm.numel(), _dptr(b), _stream(stream)), "nbx_rhs")
    return b


# -------------------------------------------------------------------- PCG

def default_opts(**kw) -> PcgOpts:
    o = PcgOpts()
    lib().nbx_pcg_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


@dataclass
class SolveResult:
    status: int
    iters: int
    outer_iters: int
    relres: float
    true_relres: float
    fell_back: int
    flag: int
    seconds: float


class Problem:
    """Binds (D, N, E, gs) and a copy of G [E, 6, N^3]; owns dinv and the
    solver workspace."""

    def __init__(self, G, D, N: int, gs: GS, stream=None):
        torch = _torch()
        self.D, self.N, self.gs = D, N, gs
        self.E = G.shape[0]
        self.n = self.E * N ** 3
        self.device = G.device
        if tuple(G.shape) != (self.E, 6, N ** 3):
            raise ValueError(f"G must be shaped (E, 6, {N ** 3})")
        _need(D, N * N, "D")
        if gs.n != self.n:
            raise ValueError("the gather-scatter plan does not match G")
        h = C.c_void_p()
        _check(lib().nbx_problem_create(_dptr(G, torch.float64), _dptr(D, torch.float64), N,
                                        self.E, gs.handle, C.byref(h), _stream(stream)),
               "nbx_problem_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().nbx_problem_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dinv(self, stream=None):
        torch = _torch()
        out = torch.empty((self.E, self.N ** 3), dtype=torch.float64, device=self.device)
        _check(lib().nbx_problem_dinv(self._h, _dptr(out), _stream(stream)), "nbx_problem_dinv")
        return out

    def exchange_info(self) -> dict:
        """Groups of the full exchange plan and of the solvers' exchange, and
        the offsets of the face pairs the update step sums (x, y, z; only x
        pairs are taken)."""
        out = (C.c_int64 * 5)()
        _check(lib().nbx_problem_exchange_info(self._h, out), "nbx_problem_exchange_info")
        return {"full_groups": out[0], "solver_groups": out[1],
                "pair_offsets": (out[2], out[3], out[4])}

    def pcg(self, b, x=None, stream=None, **opts) -> tuple:
        torch = _torch()
        _need(b, self.n, "b")
        x = torch.empty_like(b) if x is None else _need(x, self.n, "x")
        o = default_opts(**opts)
        r = PcgResult()
        st = lib().nbx_pcg(self._h, _dptr(b, torch.float64, "b"), _dptr(x, torch.float64, "x"),
                           C.byref(o), C.byref(r), _stream(stream))
        if st < 0 and st != -5:
            raise NbxError(st, "nbx_pcg")
        return x, SolveResult(st, r.iters, r.outer_iters, r.relres, r.true_relres,
                              r.fell_back, r.flag, r.seconds)

    def pcg_iterate(self, x, r, z, p, scal, n_iter: int, stream=None):
        torch = _torch()
        for t, nm in ((x, "x"), (r, "r"), (z, "z"), (p, "p")):
            _need(t, self.n, nm)
        _need(scal, SCAL_LEN, "scal")
        _check(lib().nbx_pcg_iterate(self._h, _dptr(x, torch.float64), _dptr(r, torch.float64),
                                     _dptr(z, torch.float64), _dptr(p, torch.float64),
                                     _dptr(scal, torch.float64), n_iter, _stream(stream)),
               "nbx_pcg_iterate")


def pcg_iterate_noalloc(Gp, D, N: int, gs: GS, dinv, x, r, z, p, w, scal, n_iter: int,
                        stream=None):
    """nbx_pcg_iterate_noalloc: FP64 Jacobi-PCG iterations on caller state
    with factor pairs Gp [E, 3, N^3, 2]; the library allocates nothing."""
    torch = _torch()
    E = Gp.shape[0]
    if tuple(Gp.shape) != (E, 3, N ** 3, 2):
        raise ValueError(f"Gp must be shaped (E, 3, {N ** 3}, 2)")
    n = E * N ** 3
    _need(D, N * N, "D")
    for t, nm in ((dinv, "dinv"), (x, "x"), (r, "r"), (z, "z"), (p, "p"), (w, "w")):
        _need(t, n, nm)
    _need(scal, SCAL_LEN, "scal")
    f = torch.float64
    _check(lib().nbx_pcg_iterate_noalloc(_dptr(Gp, f, "Gp"), _dptr(D, f, "D"), N, E, gs.handle,
                                         _dptr(dinv, f, "dinv"), _dptr(x, f, "x"),
                                         _dptr(r, f, "r"), _dptr(z, f, "z"), _dptr(p, f, "p"),
                                         _dptr(w, f, "w"), _dptr(scal, f, "scal"), n_iter,
                                         _stream(stream)), "nbx_pcg_iterate_noalloc")


def ax_flops(N: int, E: int) -> int:
    """E N^3 (12N + 11): the paper's per-point operation count (203 at 16
    nodes per direction, Section III)."""
    return E * N ** 3 * (12 * N + 11)


def ax_bytes(N: int, E: int, itemsize: int = 8) -> int:
    """Algorithmic HBM bytes of one AX: u, six factors and w per node."""
    return E * N ** 3 * 8 * itemsize


@dataclass
class BrickSetup:
    """Device-side set-up of a brick problem: geometry, numbering, the
    gather-scatter plan, the solver problem and the load vector."""
    N: int
    E: int
    D: object
    G: object
    bm: object
    xyz: object
    gs: GS
    problem: Problem
    b: object


def setup_brick(ex: int, ey: int, ez: int, N: int, deform=None, f=None, device="cuda",
                stream=None) -> BrickSetup:
    """Builds a brick problem on the device.  f: nodal source values (torch
    float64 [E, N^3] on the device) or None for the manufactured sine
    source."""
    torch = _torch()
    D = deriv_device(N, device)
    G, bm, xyz = geom_brick(ex, ey, ez, N, deform, with_xyz=True, device=device, stream=stream)
    gid, bnd = brick_ids(ex, ey, ez, N)
    gs = GS(gid, bnd)
    P = Problem(G, D, N, gs, stream=stream)
    if f is None:
        f = sine_source(xyz, stream=stream)
    b = rhs(gs, bm, f, stream=stream)
    return BrickSetup(N, ex * ey * ez, D, G, bm, xyz, gs, P, b)


def pcg_batched(problems, bs, xs=None, stream=None, **opts):
    """Solves independent problems together (nbx_pcg_batched).  Returns
    (xs, [SolveResult], per-solve seconds on the device clock)."""
    torch = _torch()
    n = len(problems)
    if len(bs) != n:
        raise ValueError("one right-hand side per problem")
    for P, b in zip(problems, bs):
        _need(b, P.n, "b")
    xs = [torch.empty_like(b) for b in bs] if xs is None else xs
    if len(xs) != n:
        raise ValueError("one solution vector per problem")
    for P, x in zip(problems, xs):
        _need(x, P.n, "x")
    P_arr = (C.c_void_p * n)(*[p._h.value for p in problems])
    b_arr = (C.c_void_p * n)(*[_dptr(b, torch.float64, "b").value for b in bs])
    x_arr = (C.c_void_p * n)(*[_dptr(x, torch.float64, "x").value for x in xs])
    res = (PcgResult * n)()
    lat = (C.c_double * n)()
    o = default_opts(**opts)
    st = lib().nbx_pcg_batched(P_arr, b_arr, x_arr, n, C.byref(o), res, lat, _stream(stream))
    if st < 0 and st != -5:
        raise NbxError(st, "nbx_pcg_batched")
    out = [SolveResult(st, r.iters, r.outer_iters, r.relres, r.true_relres, r.fell_back,
                       r.flag, r.seconds) for r in res]
    return xs, out, list(lat)


# ------------------------------------------------------- BF16 network

def gemm_bf16(A, B, trans_a=False, trans_b=False, stream=None):
    """C = op(A) op(B) in FP32 from bfloat16 operands (matrix cores)."""
    torch = _torch()
    if A.dtype != torch.bfloat16 or B.dtype != torch.bfloat16:
        raise TypeError("operands must be bfloat16")
    if A.dim() != 2 or B.dim() != 2:
        raise ValueError("operands must be matrices")
    M, K = (A.shape[1], A.shape[0]) if trans_a else (A.shape[0], A.shape[1])
    Kb, N = (B.shape[1], B.shape[0]) if trans_b else (B.shape[0], B.shape[1])
    if K != Kb:
        raise ValueError("inner dimensions differ")
    Cm = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(lib().nbx_gemm_bf16(int(trans_a), int(trans_b), M, N, K, _dptr(A), A.shape[1],
                               _dptr(B), B.shape[1], _dptr(Cm), N, _stream(stream)),
           "nbx_gemm_bf16")
    return Cm


class Mlp:
    """Handle of the element-local network (see include/nbx.h)."""

    def __init__(self, n_in: int, n_hidden: int, n_out: int, max_batch: int):
        h = C.c_void_p()
        _check(lib().nbx_mlp_create(n_in, n_hidden, n_out, max_batch, C.byref(h)),
               "nbx_mlp_create")
        self._h = h
        ip, op, npar = C.c_int(), C.c_int(), C.c_int64()
        _check(lib().nbx_mlp_shape(h, C.byref(ip), C.byref(op), C.byref(npar)), "nbx_mlp_shape")
        self.n_in, self.n_hidden, self.n_out, self.max_batch = n_in, n_hidden, n_out, max_batch
        self.in_pad, self.out_pad, self.n_params = ip.value, op.value, npar.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().nbx_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, stream=None):
        torch = _torch()
        _need(params, self.n_params, "params")
        _check(lib().nbx_mlp_set_params(self._h, _dptr(params, torch.float32), _stream(stream)),
               "nbx_mlp_set_params")

    def get_params(self, grads=False, stream=None):
        torch = _torch()
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        if grads:
            _check(lib().nbx_mlp_get_params(self._h, None, _dptr(out), _stream(stream)),
                   "nbx_mlp_get_params")
        else:
            _check(lib().nbx_mlp_get_params(self._h, _dptr(out), None, _stream(stream)),
                   "nbx_mlp_get_params")
        return out

    def _rows(self, X, T=None):
        if X.dim() != 2 or X.shape[1] != self.in_pad:
            raise ValueError(f"X must be [B, {self.in_pad}]")
        if T is not None and (T.dim() != 2 or tuple(T.shape) != (X.shape[0], self.out_pad)):
            raise ValueError(f"T must be [B, {self.out_pad}]")

    def forward(self, X, stream=None):
        torch = _torch()
        self._rows(X)
        Y = torch.empty((X.shape[0], self.out_pad), dtype=torch.float32, device=X.device)
        _check(lib().nbx_mlp_forward(self._h, _dptr(X, torch.bfloat16), X.shape[0], _dptr(Y),
                                     _stream(stream)), "nbx_mlp_forward")
        return Y

    def grad(self, X, T, stream=None):
        torch = _torch()
        self._rows(X, T)
        loss = torch.empty(1, dtype=torch.float64, device=X.device)
        _check(lib().nbx_mlp_grad(self._h, _dptr(X, torch.bfloat16), _dptr(T, torch.float32),
                                  X.shape[0], _dptr(loss), _stream(stream)), "nbx_mlp_grad")
        return loss

    def train_step(self, X, T, lr: float, stream=None):
        torch = _torch()
        self._rows(X, T)
        loss = torch.empty(1, dtype=torch.float64, device=X.device)
        _check(lib().nbx_mlp_train_step(self._h, _dptr(X, torch.bfloat16),
                                        _dptr(T, torch.float32), X.shape[0], float(lr),
                                        _dptr(loss), _stream(stream)), "nbx_mlp_train_step")
        return loss


_LP_SIGS = {
    "nbx_lpi_create": ([C.c_int, C.c_int, C.c_int, C.POINTER(C.c_void_p)], C.c_int),
    "nbx_lpi_destroy": ([C.c_void_p], C.c_int),
    "nbx_lpi_shape": ([C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int),
                       C.POINTER(C.c_int64)], C.c_int),
    "nbx_lpi_set_params": ([C.c_void_p] * 3, C.c_int),
    "nbx_lpi_get_params": ([C.c_void_p] * 4, C.c_int),
    "nbx_lpi_grad": ([C.c_void_p] * 4 + [C.c_int] + [C.c_void_p] * 2, C.c_int),
    "nbx_lpi_train_step": ([C.c_void_p] * 4 + [C.c_int, C.c_float] + [C.c_void_p] * 2, C.c_int),
    "nbx_lp_create": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p], C.c_int),
    "nbx_lp_destroy": ([C.c_void_p], C.c_int),
    "nbx_lp_refresh": ([C.c_void_p] * 2, C.c_int),
    "nbx_lp_geom_features": ([C.c_void_p] * 3, C.c_int),
    "nbx_lp_apply": ([C.c_void_p] * 4, C.c_int),
    "nbx_lp_samples": ([C.c_void_p] * 4 + [C.c_int] + [C.c_void_p] * 4, C.c_int),
    "nbx_lpi_init_scale": ([C.c_void_p] * 3 + [C.c_int, C.c_void_p], C.c_int),
    "nbx_problem_residual": ([C.c_void_p] * 3, C.c_int),
    "nbx_pcg_learned": ([C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(PcgOpts),
                         C.POINTER(PcgResult), C.c_void_p], C.c_int),
}


def _lp_lib():
    L = lib()
    if not getattr(L, "_lp_sigs", False):
        for name, (args, res) in _LP_SIGS.items():
            getattr(L, name).argtypes = args
            getattr(L, name).restype = res
        L._lp_sigs = True
    return L


FEAT = 64   # width of a feature row (six features, then zeros)


class InteriorModel:
    """The learned element-interior preconditioner's model (nbx_lpi_*): L
    and the gains perceptron, with the training step."""

    def __init__(self, N: int, n_hidden: int = 128, max_batch: int = 1024):
        L = _lp_lib()
        h = C.c_void_p()
        _check(L.nbx_lpi_create(N, n_hidden, max_batch, C.byref(h)), "nbx_lpi_create")
        self._h = h
        ni, nip, npar = C.c_int(), C.c_int(), C.c_int64()
        _check(L.nbx_lpi_shape(h, C.byref(ni), C.byref(nip), C.byref(npar)), "nbx_lpi_shape")
        self.N, self.n_hidden, self.max_batch = N, n_hidden, max_batch
        self.nI, self.nIp, self.n_params = ni.value, nip.value, npar.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().nbx_lpi_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, stream=None):
        torch = _torch()
        _need(params, self.n_params, "params")
        _check(_lp_lib().nbx_lpi_set_params(self._h, _dptr(params, torch.float32),
                                            _stream(stream)), "nbx_lpi_set_params")

    def get_params(self, grads=False, stream=None):
        torch = _torch()
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        p, g = (None, _dptr(out)) if grads else (_dptr(out), None)
        _check(_lp_lib().nbx_lpi_get_params(self._h, p, g, _stream(stream)),
               "nbx_lpi_get_params")
        return out

    def _rows(self, X, T, F):
        B = X.shape[0]
        if X.dim() != 2 or X.shape[1] != self.nIp:
            raise ValueError(f"X must be [B, {self.nIp}]")
        if tuple(T.shape) != (B, self.nIp) or tuple(F.shape) != (B, FEAT):
            raise ValueError(f"T must be [B, {self.nIp}] and F [B, {FEAT}]")
        if B < 64 or B % 64 or B > self.max_batch:
            raise ValueError(f"B must be a multiple of 64 up to {self.max_batch}")
        return B

    def init_scale(self, X, T, stream=None):
        """Gain biases from the least-squares scalar fit of rows (X, T)
        (nbx_lpi_init_scale)."""
        torch = _torch()
        if X.dim() != 2 or X.shape[1] != self.nIp or tuple(T.shape) != tuple(X.shape):
            raise ValueError(f"X and T must be [B, {self.nIp}]")
        _check(_lp_lib().nbx_lpi_init_scale(self._h, _dptr(X, torch.bfloat16),
                                            _dptr(T, torch.float32), X.shape[0],
                                            _stream(stream)), "nbx_lpi_init_scale")

    def grad(self, X, T, F, stream=None):
        torch = _torch()
        B = self._rows(X, T, F)
        loss = torch.empty(1, dtype=torch.float64, device=X.device)
        _check(_lp_lib().nbx_lpi_grad(self._h, _dptr(X, torch.bfloat16),
                                      _dptr(T, torch.float32), _dptr(F, torch.bfloat16), B,
                                      _dptr(loss), _stream(stream)), "nbx_lpi_grad")
        return loss

    def train_step(self, X, T, F, lr: float, stream=None):
        torch = _torch()
        B = self._rows(X, T, F)
        loss = torch.empty(1, dtype=torch.float64, device=X.device)
        _check(_lp_lib().nbx_lpi_train_step(self._h, _dptr(X, torch.bfloat16),
                                            _dptr(T, torch.float32), _dptr(F, torch.bfloat16),
                                            B, float(lr), _dptr(loss), _stream(stream)),
               "nbx_lpi_train_step")
        return loss


class LearnedPrecond:
    """The learned element-interior preconditioner bound to a problem and a
    model (nbx_lp_*): apply, training rows, flexible PCG with the Jacobi
    fallback."""

    def __init__(self, problem: "Problem", model: InteriorModel, stream=None):
        h = C.c_void_p()
        _check(_lp_lib().nbx_lp_create(problem._h, model.handle, C.byref(h), _stream(stream)),
               "nbx_lp_create")
        self._h, self.problem, self.model = h, problem, model

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().nbx_lp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def refresh(self, stream=None):
        """Recomputes the per-element gains after the model changed."""
        _check(_lp_lib().nbx_lp_refresh(self._h, _stream(stream)), "nbx_lp_refresh")

    def geom_features(self, stream=None):
        torch = _torch()
        g = torch.empty((self.problem.E, 8), dtype=torch.float32, device="cuda")
        _check(_lp_lib().nbx_lp_geom_features(self._h, _dptr(g), _stream(stream)),
               "nbx_lp_geom_features")
        return g

    def apply(self, r, stream=None):
        torch = _torch()
        _need(r, self.problem.n, "r")
        z = torch.empty_like(r)
        _check(_lp_lib().nbx_lp_apply(self._h, _dptr(r, torch.float64), _dptr(z),
                                      _stream(stream)), "nbx_lp_apply")
        return z

    def samples(self, v, elems, v0=None, stream=None):
        """(X [n, nIp] bf16, T [n, nIp] f32, F [n, 64] bf16) rows from the
        solver vector v - v0 (v alone if v0 is None) for the element indices
        elems (int32, device)."""
        torch = _torch()
        _need(v, self.problem.n, "v")
        if v0 is not None:
            _need(v0, self.problem.n, "v0")
        n = elems.numel()
        nIp = self.model.nIp
        X = torch.empty((n, nIp), dtype=torch.bfloat16, device="cuda")
        T = torch.empty((n, nIp), dtype=torch.float32, device="cuda")
        F = torch.empty((n, FEAT), dtype=torch.bfloat16, device="cuda")
        _check(_lp_lib().nbx_lp_samples(self._h, _dptr(v, torch.float64),
                                        _dptr(v0, torch.float64, "v0") if v0 is not None
                                        else None,
                                        _dptr(elems, torch.int32), n, _dptr(X), _dptr(T),
                                        _dptr(F), _stream(stream)), "nbx_lp_samples")
        return X, T, F

    def residual(self, stream=None):
        """The recurrence residual left by the problem's last solve."""
        torch = _torch()
        r = torch.empty((self.problem.E, self.problem.N ** 3), dtype=torch.float64,
                        device="cuda")
        _check(_lp_lib().nbx_problem_residual(self.problem._h, _dptr(r), _stream(stream)),
               "nbx_problem_residual")
        return r

    def pcg(self, b, x=None, stream=None, **opts):
        torch = _torch()
        _need(b, self.problem.n, "b")
        x = torch.empty_like(b) if x is None else _need(x, self.problem.n, "x")
        o = default_opts(**opts)
        r = PcgResult()
        st = _lp_lib().nbx_pcg_learned(self._h, _dptr(b, torch.float64),
                                       _dptr(x, torch.float64), C.byref(o), C.byref(r),
                                       _stream(stream))
        if st < 0 and st != -5:
            raise NbxError(st, "nbx_pcg_learned")
        return x, SolveResult(st, r.iters, r.outer_iters, r.relres, r.true_relres,
                              r.fell_back, r.flag, r.seconds)
