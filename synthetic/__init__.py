"""Seeded synthetic workloads for the spectral-element Poisson path.

This module is shared by the CPU oracle tests and the HIP path.  It holds
workload *descriptions* (brick sizes, polynomial size, the deformation
family's amplitudes and wave numbers, seeds) and raw random draws only.  It
contains none of the method's arithmetic: no quadrature nodes, no
derivative matrices, no geometric factors, no operator.  Each side turns a
description into nodes, coordinates and factors with its own code.

Conventions both sides follow (stated here so that a description is
unambiguous):

* Elements of an ``ex x ey x ez`` brick on the unit cube are numbered
  ``e = a + ex*(b + ey*c)`` for element position ``(a, b, c)``.
* Nodes inside an element are numbered ``i + N*(j + N*k)`` (``i`` fastest),
  the column-major ``u(i,j,k,e)`` layout of the paper's Fortran listing
  (Section II-B, Listing 1).
* A deformation is three terms, one per physical coordinate ``c``:
  ``c = C + A_c * sin(k1 pi X) sin(k2 pi Y) sin(k3 pi Z)`` where ``(X,Y,Z)``
  is the undeformed position; integer wave numbers keep the boundary of the
  unit cube fixed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
from typing import List, Optional, Tuple

import numpy as np

Deform = Tuple[Tuple[float, int, int, int], Tuple[float, int, int, int],
               Tuple[float, int, int, int]]

NO_DEFORM: Deform = ((0.0, 1, 1, 1), (0.0, 1, 1, 1), (0.0, 1, 1, 1))


@dataclass(frozen=True)
class Brick:
    """A structured box mesh of hexahedral elements on [0,1]^3."""
    ex: int
    ey: int
    ez: int
    N: int                        # GLL nodes per direction (degree N-1)
    deform: Deform = NO_DEFORM
    rhs: str = "sine"             # "sine" or "random"
    rhs_seed: int = 0
    name: str = ""

    @property
    def E(self) -> int:
        return self.ex * self.ey * self.ez

    @property
    def n_local(self) -> int:
        return self.E * self.N ** 3

    def deform_array(self) -> np.ndarray:
        """The deformation as a float64 (3, 4) array: rows (A, k1, k2, k3)."""
        return np.array([[float(a), float(k1), float(k2), float(k3)]
                         for (a, k1, k2, k3) in self.deform], dtype=np.float64)

    def is_affine(self) -> bool:
        return all(t[0] == 0.0 for t in self.deform)


# ---------------------------------------------------------------- workloads

def c1_brick() -> Brick:
    """4x4x4 affine brick (E=64), N=10, manufactured sine right-hand side."""
    return Brick(4, 4, 4, 10, NO_DEFORM, "sine", 0, "c1_affine_E64_N10")


def c2_brick(N: int = 10) -> Brick:
    """32x32x32 brick (E=32768) with the sin(2 pi X)sin(2 pi Y)sin(2 pi Z)
    deformation at amplitude 0.05 on every coordinate."""
    d = (0.05, 2, 2, 2)
    return Brick(32, 32, 32, N, (d, d, d), "sine", 0, f"c2_deformed_E32768_N{N}")


def scaled_c2_brick(n: int, N: int = 10) -> Brick:
    """The C2 deformation on an n x n x n brick (small parity cases)."""
    d = (0.05, 2, 2, 2)
    return Brick(n, n, n, N, (d, d, d), "sine", 0, f"deformed_E{n**3}_N{N}")


def _brick_dims(target: float) -> Tuple[int, int, int]:
    """ex >= ey >= ez, ex <= 2*ez, product closest to ``target``."""
    best = None
    for ez in range(1, 64):
        for ey in range(ez, 2 * ez + 1):
            for ex in range(ey, 2 * ez + 1):
                p = ex * ey * ez
                d = abs(math.log(p) - math.log(target))
                if best is None or d < best[0]:
                    best = (d, (ex, ey, ez))
    return best[1]


def c4_problems(count: int = 64, seed0: int = 1000) -> List[Brick]:
    """Independent problems: E log-uniform in [64, 4096], N from {6,8,10,12},
    deformation amplitude U[0, 0.1] (C2's wave numbers), random RHS."""
    out = []
    for p in range(count):
        rng = np.random.default_rng(seed0 + p)
        t = rng.uniform(math.log(64), math.log(4096))
        ex, ey, ez = _brick_dims(math.exp(t))
        N = int(rng.choice([6, 8, 10, 12]))
        a = float(rng.uniform(0.0, 0.1))
        d = (a, 2, 2, 2)
        out.append(Brick(ex, ey, ez, N, (d, d, d), "random", seed0 + p,
                         f"batch{p}_E{ex*ey*ez}_N{N}"))
    return out


def deformation_family(seed: int, amax: float = 0.1) -> Deform:
    """Per-coordinate amplitude U[0, amax] and wave numbers from {1,2,3}^3."""
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(3):
        a = float(rng.uniform(0.0, amax))
        k = rng.integers(1, 4, size=3)
        terms.append((a, int(k[0]), int(k[1]), int(k[2])))
    return tuple(terms)  # type: ignore[return-value]


def c5_train_meshes(count: int = 200, N: int = 10) -> List[Brick]:
    """Training meshes: 32x16x16 bricks (E=8192) with seeded deformations."""
    return [Brick(32, 16, 16, N, deformation_family(s), "random", s,
                  f"train{s}") for s in range(count)]


def c5_eval_meshes(count: int = 2, N: int = 10, n: int = 32) -> List[Brick]:
    """Held-out meshes: n^3 bricks, unseen deformation seeds (>= 10000),
    plus the C2 mapping itself."""
    out = [Brick(n, n, n, N, deformation_family(10000 + s), "random",
                 10000 + s, f"eval{10000+s}") for s in range(count)]
    d = (0.05, 2, 2, 2)
    out.append(Brick(n, n, n, N, (d, d, d), "sine", 0, "eval_c2"))
    return out


# ------------------------------------------------------------ random draws

def uniform_field(E: int, N: int, seed: int = 0) -> np.ndarray:
    """u ~ U[-1, 1] on every local node, shape (E, N^3), float64."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(E, N ** 3))


def random_factors(E: int, N: int, seed: int = 1) -> np.ndarray:
    """Six per-node factors in [E][6][N^3] order forming a symmetric 3x3
    matrix [[g1,g2,g3],[g2,g4,g5],[g3,g5,g6]] that is strictly diagonally
    dominant (diagonal in [2,3], off-diagonal in [-0.5,0.5]), hence SPD."""
    rng = np.random.default_rng(seed)
    G = rng.uniform(-0.5, 0.5, size=(E, 6, N ** 3))
    for f in (0, 3, 5):
        G[:, f, :] = rng.uniform(2.0, 3.0, size=(E, N ** 3))
    return G


def rhs_values(b: Brick) -> np.ndarray:
    """Nodal source values f_l ~ U[-1,1] for a "random" right-hand side,
    shape (E, N^3); the assembled load vector is built from them."""
    rng = np.random.default_rng(b.rhs_seed + 7919)
    return rng.uniform(-1.0, 1.0, size=(b.E, b.N ** 3))


def mlp_init(n_in: int, n_hidden: int, n_out: int, seed: int = 0):
    """He-uniform initial weights for a 3-layer MLP, float64, stored
    row-major as W[out][in]; biases zero."""
    rng = np.random.default_rng(seed)
    def lin(o, i):
        lim = math.sqrt(6.0 / i)
        return rng.uniform(-lim, lim, size=(o, i))
    return {
        "W1": lin(n_hidden, n_in), "b1": np.zeros(n_hidden),
        "W2": lin(n_hidden, n_hidden), "b2": np.zeros(n_hidden),
        "W3": lin(n_out, n_hidden) * 0.1, "b3": np.zeros(n_out),
    }


def mlp_batch(B: int, n_in: int, n_out: int, seed: int = 0):
    """A random regression batch (X, Y) for MLP parity checks."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((B, n_in)), rng.standard_normal((B, n_out)))
