"""Pins of the 16-bit geometric-factor storage reference (oracle/g16.py)
against facts of the IEEE formats and of the operator."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from oracle import g16


def _elem(values, N=2):
    """One element's G [1][6][N^3] holding `values` first, zeros after."""
    G = np.zeros((1, 6, N ** 3))
    G.reshape(-1)[:len(values)] = values
    return G


@pytest.mark.parametrize("fmt", g16.FORMATS)
def test_scale_places_max_in_top_binade(fmt):
    G = S.random_factors(30, 4, seed=3) * np.logspace(-9, 3, 30)[:, None, None]
    gs = g16.scales(G, 4)
    m = np.abs(G).reshape(30, -1).max(axis=1)
    q = m / gs
    assert np.all((q >= 2 ** 14) & (q < 2 ** 15))
    assert np.all(np.log2(gs) == np.round(np.log2(gs)))          # powers of two
    assert g16.scales(np.zeros((1, 6, 8)), 2)[0] == 1.0


@pytest.mark.parametrize("fmt", g16.FORMATS)
def test_representable_values_survive(fmt):
    # max 2^14 gives scale 1; small integers and binary fractions with few
    # significant bits are exact in both formats
    vals = [2.0 ** 14, 1.0, -3.0, 0.5, 0.0, 96.0, -0.75, 2.0 ** -6]
    G = _elem(vals)
    w, gs = g16.pack(G, 2, fmt)
    assert gs[0] == 1.0
    np.testing.assert_array_equal(g16.unpack(w, gs, 2, fmt), G)


def test_ties_round_to_even():
    G = _elem([2.0 ** 14, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8])
    d16 = g16.unpack(*g16.pack(G, 2, "f16"), 2, "f16").reshape(-1)[:5]
    db = g16.unpack(*g16.pack(G, 2, "bf16"), 2, "bf16").reshape(-1)[:5]
    # binary16 spacing at 1 is 2^-10: halfway points go to the even neighbour
    assert d16[1] == 1.0 and d16[2] == 1 + 2.0 ** -9
    assert d16[3] == 1 + 2.0 ** -8 and d16[4] == 1 + 3 * 2.0 ** -8
    # bfloat16 spacing at 1 is 2^-7
    assert db[1] == 1.0 and db[3] == 1.0 and db[4] == 1 + 2.0 ** -6
    # bit patterns of 1.0 in each format
    w16, _ = g16.pack(_elem([2.0 ** 14, 1.0]), 2, "f16")
    wb, _ = g16.pack(_elem([2.0 ** 14, 1.0]), 2, "bf16")
    assert w16.reshape(-1)[1] == 0x3C00 and wb.reshape(-1)[1] == 0x3F80


@pytest.mark.parametrize("fmt", g16.FORMATS)
def test_relative_error_within_unit_roundoff(fmt):
    N = 5
    G = S.random_factors(20, N, seed=9)
    d = g16.unpack(*g16.pack(G, N, fmt), N, fmt)
    gs = g16.scales(G, N).astype(np.float64)[:, None, None]
    normal = np.abs(G) / gs >= 2.0 ** -14          # binary16 normal range
    u = g16.unit_roundoff(fmt)
    rel = np.abs(d - G)[normal] / np.abs(G)[normal]
    assert rel.max() <= u * (1 + 2.0 ** -12)       # two roundings: + 2^-24
    assert rel.max() >= 0.25 * u                   # and the format is really used


@pytest.mark.parametrize("fmt", g16.FORMATS)
def test_operator_perturbation_bounded_in_energy(fmt):
    # on an affine brick (diagonal-dominant SPD factor blocks) a relative
    # perturbation u of every factor changes <v, A v> by at most ~u <v, A v>
    b = S.Brick(2, 2, 2, 5, ((0.0, 1, 1, 1),) * 3)
    P = O.setup(b)
    Gd = g16.unpack(*g16.pack(P.G, 5, fmt), 5, fmt)
    v = S.uniform_field(b.E, 5, seed=4)
    e1 = np.sum(v * O.ax(v, P.G, P.D))
    e2 = np.sum(v * O.ax(v, Gd.reshape(P.G.shape), P.D))
    assert abs(e2 - e1) <= 2 * g16.unit_roundoff(fmt) * abs(e1)
