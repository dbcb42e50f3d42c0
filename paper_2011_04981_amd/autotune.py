"""Tile autotuner for the AX kernel (elements per workgroup).

Two tables, both indexed by (precision, N):
  * the plain operator (nbx_ax): each tile the library offers (nbx_ax_tiled
    with 1, 2 or 4 elements per workgroup) is timed on an HBM-sized
    synthetic operator; every tile computes identical bits;
  * the solvers' fused first stage (p update, AX, <p,w> partials;
    nbx_pcg_set_tile), whose register and LDS use differ: each tile is timed
    as whole CG iterations on a deformed brick of the same size (FP64 Jacobi
    PCG for "f64", the FP32 inner iterations of the mixed solve for "f32").
The fastest tile is installed and the table can be stored as JSON, which
the package applies when the library loads.

    python -m paper_2011_04981_amd.autotune --save   # writes tiles.json
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
from typing import Dict, Iterable, Optional

from . import (F16, F32, F64, NbxError, ax, ax_g16, g16_pack, get_pcg_tile, get_tile, lib,
               set_pcg_tile, set_tile)

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tiles.json")
# the 16-bit-G kernels (FP16 and BF16 storage, FP32 arithmetic) share one
# table, timed with FP16 storage
PREC_NAME = {F64: "f64", F32: "f32", F16: "g16"}
TILES = (1, 2, 4, 8)


def cache_path() -> str:
    return os.environ.get("NBX_TILE_CACHE", DEFAULT_CACHE)


def time_tiles(prec: int, N: int, nodes: int = 16_000_000, reps: int = 20,
               warmup: int = 10, seed: int = 0) -> Dict[int, float]:
    """Median launch time (seconds) of each tile on E = nodes / N^3 random
    elements.  Tiles whose LDS does not fit are skipped."""
    import torch
    dtype = torch.float64 if prec == F64 else torch.float32
    E = max(64, nodes // N ** 3)
    g = torch.Generator(device="cuda").manual_seed(seed)
    u = torch.rand((E, N ** 3), dtype=dtype, device="cuda", generator=g)
    G = torch.rand((E, 6, N ** 3), dtype=torch.float64 if prec == F16 else dtype,
                   device="cuda", generator=g)
    w = torch.empty_like(u)
    from . import deriv_device
    D = deriv_device(N)
    if prec == F16:
        G16, gsc = g16_pack(G, N, F16)
        old = get_tile(F16, N)

    def run(epb):
        if prec == F16:
            set_tile(F16, N, epb)         # nbx_ax_g16 takes its tile from the table
            ax_g16(u, G16, gsc, D, F16, out=w)
        else:
            ax(u, G, D, out=w, epb=epb)

    out = {}
    for epb in TILES:
        try:
            run(epb)
        except NbxError as e:
            if e.status == -2:
                continue
            raise
        for _ in range(warmup):
            run(epb)
        times = []
        for _ in range(reps):
            s = torch.cuda.Event(enable_timing=True)
            t = torch.cuda.Event(enable_timing=True)
            s.record()
            run(epb)
            t.record()
            t.synchronize()
            times.append(s.elapsed_time(t) * 1e-3)
        out[epb] = statistics.median(times)
    if prec == F16:
        set_tile(F16, N, old)
    return out


def _brick_dims(E: int):
    n = max(1, round(E ** (1 / 3)))
    return n, n, max(1, E // (n * n))


def time_pcg_tiles(prec: int, N: int, nodes: int = 8_000_000, iters: int = 60,
                   seed: int = 0) -> Dict[int, float]:
    """Seconds per CG iteration with each fused-stage tile on a deformed
    brick of about `nodes` local nodes (best of two solves per tile)."""
    import torch
    from . import setup_brick
    ex, ey, ez = _brick_dims(max(8, nodes // N ** 3))
    d = [[0.05, 2, 2, 2]] * 3
    st = setup_brick(ex, ey, ez, N, d)
    out = {}
    old = get_pcg_tile(prec, N)
    for epb in TILES:
        try:
            set_pcg_tile(prec, N, epb)
        except NbxError:
            continue
        best = None
        for _ in range(2):
            try:
                if prec == F64:
                    _, r = st.problem.pcg(st.b, max_iter=iters, fixed_iters=1, check_every=20)
                else:
                    _, r = st.problem.pcg(st.b, rtol=1e-6, max_iter=20 * iters, prec=prec,
                                          check_every=20)
            except NbxError as e:
                if e.status == -2:
                    break
                raise
            per = r.seconds / max(r.iters, 1)
            best = per if best is None else min(best, per)
        if best is not None:
            out[epb] = best
    set_pcg_tile(prec, N, old)
    st.problem.close()
    torch.cuda.synchronize()
    return out


def tune(Ns: Iterable[int] = (6, 8, 10, 12), precs: Iterable[int] = (F64, F32, F16),
         nodes: int = 16_000_000, reps: int = 20, apply: bool = True,
         pcg: bool = True) -> dict:
    """Times every tile for every (precision, N), installs the fastest and
    returns {"f64": {"10": {"epb": 2, "us": {"1": .., "2": .., "4": ..}}},
    "pcg_f64": {...}, ...} (pcg_* rows: microseconds per CG iteration)."""
    table: dict = {}
    for prec in precs:
        for N in Ns:
            t = time_tiles(prec, N, nodes=nodes, reps=reps)
            best = min(t, key=t.get)
            table.setdefault(PREC_NAME[prec], {})[str(N)] = {
                "epb": best, "us": {str(k): round(v * 1e6, 2) for k, v in t.items()}}
            if apply:
                set_tile(prec, N, best)
            if pcg:
                t = time_pcg_tiles(prec, N, nodes=nodes // 2)
                best = min(t, key=t.get)
                table.setdefault("pcg_" + PREC_NAME[prec], {})[str(N)] = {
                    "epb": best, "us": {str(k): round(v * 1e6, 2) for k, v in t.items()}}
                if apply:
                    set_pcg_tile(prec, N, best)
    return table


def apply_table(table: dict) -> int:
    """Installs a stored table; returns the number of entries applied."""
    n = 0
    for pname, rows in table.items():
        kind, _, pn = pname.rpartition("_")
        prec = {v: k for k, v in PREC_NAME.items()}.get(pn)
        setter = {"": set_tile, "pcg": set_pcg_tile}.get(kind)
        if prec is None or setter is None:
            continue
        for N, row in rows.items():
            setter(prec, int(N), int(row["epb"]))
            n += 1
    return n


def save(table: dict, path: Optional[str] = None) -> str:
    path = path or cache_path()
    with open(path, "w") as f:
        json.dump({"arch": "gfx950", "tiles": table}, f, indent=1, sort_keys=True)
    return path


def load(path: Optional[str] = None, apply: bool = True) -> Optional[dict]:
    path = path or cache_path()
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    table = rec.get("tiles", {})
    if apply:
        lib()
        apply_table(table)
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, nargs="*", default=[6, 8, 10, 12])
    ap.add_argument("--nodes", type=int, default=16_000_000)
    ap.add_argument("--save", action="store_true")
    ap.add_argument("--no-pcg", action="store_true", help="skip the fused-stage table")
    a = ap.parse_args()
    table = tune(a.N, nodes=a.nodes, pcg=not a.no_pcg)
    print(json.dumps(table, indent=1))
    if a.save:
        print("saved", save(table))


if __name__ == "__main__":
    main()
