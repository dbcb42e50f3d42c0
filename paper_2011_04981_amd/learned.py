"""Training and evaluation of the learned element-local preconditioner.

Pipeline (all arithmetic in libnbx kernels; torch only holds buffers):
  1. for each training mesh, the FP64 Jacobi-PCG solves A x* = b tightly;
     then it is re-run to a few iteration counts k, and for a random subset
     of elements the pair (features of r_k, target (e_k - dinv r_k) / s_e)
     with e_k = x* - x_k is extracted (nbx_lp_samples);
  2. the network is trained on these rows with Adam (nbx_mlp_train_step,
     BF16 matrix-core forward and backward, FP32 master weights);
  3. on held-out meshes, flexible PCG with the learned preconditioner is
     compared with Jacobi-PCG; it is capped at Jacobi's iteration count and
     falls back to Jacobi when it does not beat it (nbx_pcg_learned).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

from . import (GS, LearnedPrecond, Mlp, Problem, brick_ids, deriv_device, geom_brick, rhs,
               sine_source)

HIDDEN = 128


@dataclass
class MeshProblem:
    N: int
    E: int
    G: object
    bm: object
    b: object
    problem: Problem
    gs: GS


class MeshFactory:
    """Builds problems on bricks, sharing one gather-scatter plan per brick
    shape (the numbering does not depend on the deformation)."""

    def __init__(self):
        self._gs: Dict[Tuple[int, int, int, int], GS] = {}

    def gs(self, ex, ey, ez, N) -> GS:
        key = (ex, ey, ez, N)
        if key not in self._gs:
            gid, bnd = brick_ids(ex, ey, ez, N)
            self._gs[key] = GS(gid, bnd)
        return self._gs[key]

    def build(self, brick, f=None) -> MeshProblem:
        """brick: a synthetic.Brick; f: nodal source values (device) or None
        for the sine source."""
        N = brick.N
        D = deriv_device(N)
        G, bm, xyz = geom_brick(brick.ex, brick.ey, brick.ez, N, brick.deform_array(),
                                with_xyz=f is None)
        gs = self.gs(brick.ex, brick.ey, brick.ez, N)
        P = Problem(G, D, N, gs)
        src = sine_source(xyz) if f is None else f
        return MeshProblem(N, brick.E, G, bm, rhs(gs, bm, src), P, gs)


def pack_params(net: Mlp, init: dict) -> np.ndarray:
    """The FP32 parameter arena of nbx_mlp_set_params from unpadded
    matrices W1[h][n_in], b1, W2[h][h], b2, W3[n_out][h], b3."""
    h, i, o = net.n_hidden, net.in_pad, net.out_pad
    W1 = np.zeros((h, i)); W1[:, :net.n_in] = init["W1"]
    W3 = np.zeros((o, h)); W3[:net.n_out] = init["W3"]
    b3 = np.zeros(o); b3[:net.n_out] = init["b3"]
    return np.concatenate([W1.ravel(), init["b1"], np.ravel(init["W2"]), init["b2"],
                           W3.ravel(), b3]).astype(np.float32)


def new_network(N: int, max_batch: int = 4096, hidden: int = HIDDEN, seed: int = 0) -> Mlp:
    """The element-local network for N nodes per direction (n_in = N^3 + 6,
    n_out = N^3), initialised with synthetic.mlp_init: He-uniform layers,
    last layer scaled by 0.1 so the correction starts small (near Jacobi)."""
    import torch
    import synthetic as S
    N3 = N ** 3
    net = Mlp(N3 + 6, hidden, N3, max_batch)
    arena = pack_params(net, S.mlp_init(N3 + 6, hidden, N3, seed))
    net.set_params(torch.as_tensor(arena).cuda())
    return net


@dataclass
class Samples:
    X: object
    T: object
    rows: int
    meshes: int
    seconds: float


def collect_samples(factory: MeshFactory, bricks, net: Mlp, n_iterates: int = 4,
                    elems_per_iterate: int = 512, seed: int = 0, rhs_kind: str = "mixed",
                    check_every: int = 20) -> Samples:
    """Training rows from FP64 CG runs on the given meshes."""
    import torch
    import synthetic as S
    t0 = time.perf_counter()
    rng = np.random.default_rng(seed)
    Xs, Ts = [], []
    for q, brick in enumerate(bricks):
        use_sine = rhs_kind == "sine" or (rhs_kind == "mixed" and q % 2 == 0)
        f = None if use_sine else torch.as_tensor(S.rhs_values(brick)).cuda()
        mp = factory.build(brick, f)
        lp = LearnedPrecond(mp.problem, net)
        xstar, rs = mp.problem.pcg(mp.b, rtol=1e-12, max_iter=20000, check_every=check_every)
        total = max(rs.iters, 4)
        ks = sorted(set(int(round(v)) for v in np.geomspace(2, 0.8 * total, n_iterates)))
        for k in ks:
            xk, _ = mp.problem.pcg(mp.b, max_iter=k, fixed_iters=1, check_every=check_every)
            rk = lp.residual()
            el = torch.as_tensor(rng.integers(0, mp.E, size=elems_per_iterate), dtype=torch.int32)
            X, T = lp.samples(rk, xstar, xk, el.cuda())
            Xs.append(X); Ts.append(T)
        lp.close()
        mp.problem.close()
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    torch.cuda.synchronize()
    return Samples(X, T, X.shape[0], len(bricks), time.perf_counter() - t0)


def train(net: Mlp, data: Samples, epochs: int = 30, batch: int = 1024, lr: float = 1e-3,
          seed: int = 0) -> List[float]:
    """Minibatch Adam over contiguous row blocks in random order (rows are
    already a random mix of meshes, iterates and elements); cosine decay of
    the learning rate.  Returns the mean loss per epoch."""
    import torch
    rng = np.random.default_rng(seed)
    nb = data.rows // batch
    if nb == 0:
        raise ValueError("fewer samples than one batch")
    losses = []
    step, total = 0, epochs * nb
    for ep in range(epochs):
        acc = []
        for bi in rng.permutation(nb):
            lr_t = lr * 0.5 * (1 + math.cos(math.pi * step / total))
            acc.append(net.train_step(data.X[bi * batch:(bi + 1) * batch],
                                      data.T[bi * batch:(bi + 1) * batch], max(lr_t, 1e-6)))
            step += 1
        losses.append(float(torch.cat(acc).mean()))
    return losses


@dataclass
class EvalResult:
    name: str
    E: int
    jacobi_iters: int
    jacobi_seconds: float
    learned_iters: int
    learned_seconds: float
    fell_back: int
    learned_relres: float
    iteration_ratio: float
    speedup: float


def evaluate(factory: MeshFactory, brick, net: Mlp, rtol: float = 1e-10, reps: int = 2,
             f=None, check_every: int = 20) -> EvalResult:
    """Jacobi-PCG vs learned flexible PCG (capped at Jacobi's count, with
    Jacobi fallback) on one mesh; best of `reps` timings."""
    mp = factory.build(brick, f)
    lp = LearnedPrecond(mp.problem, net)
    jt, lt = [], []
    for _ in range(reps):
        h0 = time.perf_counter()
        _, rj = mp.problem.pcg(mp.b, rtol=rtol, max_iter=20000, check_every=check_every)
        jt.append(time.perf_counter() - h0)
    for _ in range(reps):
        h0 = time.perf_counter()
        _, rl = lp.pcg(mp.b, rtol=rtol, max_iter=rj.iters, check_every=check_every)
        lt.append(time.perf_counter() - h0)
    lp.close()
    mp.problem.close()
    return EvalResult(brick.name, brick.E, rj.iters, min(jt), rl.iters, min(lt), rl.fell_back,
                      rl.true_relres, rl.iters / max(rj.iters, 1), min(jt) / min(lt))
