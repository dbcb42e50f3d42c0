"""Tile autotuner for the AX kernel (elements per workgroup).

For every (precision, N) it times each tile the library offers
(nbx_ax_tiled with 1, 2 or 4 elements per workgroup) on an HBM-sized
synthetic operator, keeps the fastest, installs it in the library's tile
table (nbx_ax_set_tile, used by nbx_ax, the solvers and the batched solver)
and can store the table as JSON.  Every tile computes identical bits, so the
choice only affects speed.

    python -m paper_2011_04981_amd.autotune --save   # writes tiles.json
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
from typing import Dict, Iterable, Optional

from . import F32, F64, NbxError, ax, lib, set_tile

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tiles.json")
PREC_NAME = {F64: "f64", F32: "f32"}
TILES = (1, 2, 4)


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
    G = torch.rand((E, 6, N ** 3), dtype=dtype, device="cuda", generator=g)
    w = torch.empty_like(u)
    from . import deriv_device
    D = deriv_device(N)
    out = {}
    for epb in TILES:
        try:
            ax(u, G, D, out=w, epb=epb)
        except NbxError as e:
            if e.status == -2:
                continue
            raise
        for _ in range(warmup):
            ax(u, G, D, out=w, epb=epb)
        times = []
        for _ in range(reps):
            s = torch.cuda.Event(enable_timing=True)
            t = torch.cuda.Event(enable_timing=True)
            s.record()
            ax(u, G, D, out=w, epb=epb)
            t.record()
            t.synchronize()
            times.append(s.elapsed_time(t) * 1e-3)
        out[epb] = statistics.median(times)
    return out


def tune(Ns: Iterable[int] = (6, 8, 10, 12), precs: Iterable[int] = (F64, F32),
         nodes: int = 16_000_000, reps: int = 20, apply: bool = True) -> dict:
    """Times every tile for every (precision, N), installs the fastest and
    returns {"f64": {"10": {"epb": 2, "us": {"1": .., "2": .., "4": ..}}}, ...}."""
    table: dict = {}
    for prec in precs:
        for N in Ns:
            t = time_tiles(prec, N, nodes=nodes, reps=reps)
            best = min(t, key=t.get)
            table.setdefault(PREC_NAME[prec], {})[str(N)] = {
                "epb": best, "us": {str(k): round(v * 1e6, 2) for k, v in t.items()}}
            if apply:
                set_tile(prec, N, best)
    return table


def apply_table(table: dict) -> int:
    """Installs a stored table; returns the number of entries applied."""
    n = 0
    for pname, rows in table.items():
        prec = {v: k for k, v in PREC_NAME.items()}.get(pname)
        if prec is None:
            continue
        for N, row in rows.items():
            set_tile(prec, int(N), int(row["epb"]))
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
    a = ap.parse_args()
    table = tune(a.N, nodes=a.nodes)
    print(json.dumps(table, indent=1))
    if a.save:
        print("saved", save(table))


if __name__ == "__main__":
    main()
