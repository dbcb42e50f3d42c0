"""The tile table and the autotuner's cache on the host (no GPU needed:
the table is host state of the library)."""
import json

import pytest

import paper_2011_04981_amd as nbx
from paper_2011_04981_amd import autotune


def test_apply_and_load_cache(tmp_path):
    old = {(p, N): nbx.get_tile(p, N) for p in (nbx.F64, nbx.F32, nbx.F16)
           for N in (6, 8, 10, 12)}
    try:
        table = {"f64": {"6": {"epb": 1, "us": {}}, "10": {"epb": 4, "us": {}}},
                 "f32": {"8": {"epb": 2, "us": {}}},
                 "g16": {"10": {"epb": 8, "us": {}}}}
        path = autotune.save(table, str(tmp_path / "tiles.json"))
        rec = json.load(open(path))
        assert rec["arch"] == "gfx950"
        loaded = autotune.load(path)
        assert loaded == table
        assert nbx.get_tile(nbx.F64, 6) == 1
        assert nbx.get_tile(nbx.F64, 10) == 4
        assert nbx.get_tile(nbx.F32, 8) == 2
        # one table for both 16-bit storage formats, apart from FP32's
        assert nbx.get_tile(nbx.F16, 10) == 8 and nbx.get_tile(nbx.BF16, 10) == 8
        assert nbx.get_tile(nbx.F32, 10) != 8 or old[(nbx.F32, 10)] == 8
    finally:
        for (p, N), e in old.items():
            nbx.set_tile(p, N, e)


def test_tile_table_rejects_invalid_entries():
    with pytest.raises(nbx.NbxError):
        nbx.set_tile(nbx.F64, 10, 3)
    with pytest.raises(nbx.NbxError):
        nbx.set_tile(nbx.F64, 17, 2)
    with pytest.raises(nbx.NbxError):
        nbx.set_tile(7, 10, 2)                      # not a precision
    # tiles that do not fit: 8 FP64 elements of 10^3 nodes need 192 KB of
    # LDS; 8 elements of 12^2 columns need 1152 threads
    for p, N in ((nbx.F64, 10), (nbx.F32, 12)):
        with pytest.raises(nbx.NbxError) as e:
            nbx.set_tile(p, N, 8)
        assert e.value.status == -2
    old = nbx.get_tile(nbx.F32, 10)
    nbx.set_tile(nbx.F32, 10, 8)                    # 96 KB, 832 threads: fits
    assert nbx.get_tile(nbx.F32, 10) == 8
    nbx.set_tile(nbx.F32, 10, old)
    assert nbx.get_tile(nbx.F64, 10) in (1, 2, 4, 8)


def test_fused_stage_table_is_separate(tmp_path):
    old = {(p, N): (nbx.get_tile(p, N), nbx.get_pcg_tile(p, N))
           for p in (nbx.F64, nbx.F32) for N in (8, 10)}
    try:
        table = {"f64": {"10": {"epb": 1, "us": {}}},
                 "pcg_f64": {"10": {"epb": 2, "us": {}}},
                 "pcg_f32": {"8": {"epb": 4, "us": {}}}}
        path = autotune.save(table, str(tmp_path / "tiles.json"))
        assert autotune.load(path) == table
        assert nbx.get_tile(nbx.F64, 10) == 1 and nbx.get_pcg_tile(nbx.F64, 10) == 2
        assert nbx.get_pcg_tile(nbx.F32, 8) == 4
        nbx.set_pcg_tile(nbx.F64, 10, 4)
        assert nbx.get_tile(nbx.F64, 10) == 1          # the plain table is untouched
        with pytest.raises(nbx.NbxError):
            nbx.set_pcg_tile(7, 10, 2)
    finally:
        for (p, N), (a, b) in old.items():
            nbx.set_tile(p, N, a)
            nbx.set_pcg_tile(p, N, b)


def test_missing_cache_is_ignored(tmp_path):
    assert autotune.load(str(tmp_path / "absent.json")) is None
