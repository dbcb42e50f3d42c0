"""Training and evaluation of the learned element-interior preconditioner.

Pipeline (every step of the method runs in libnbx kernels; torch holds
buffers and index lists only):
  1. for each training mesh the FP64 solver produces vectors: a converged
     solution x*, iterates x_k of FP64 Jacobi-PCG at a few iteration counts
     k and their residuals r_k; for a random subset of elements each
     error x* - x_k and each residual r_k gives one training row
     (nbx_lp_samples: X = A_SS v_S / (|v_S| gd), T = v_S / |v_S|, features);
  2. the model (L and the gains perceptron) starts as the least-squares
     scalar map of the rows (nbx_lpi_init_scale) and is trained with Adam
     on them (nbx_lpi_train_step: BF16 matrix-core products, FP32 master
     weights);
  3. a validation brick of the training distribution decides deployment:
     the learned preconditioner is enabled only if its flexible CG needs
     fewer iterations than Jacobi-PCG there, without falling back;
  4. held-out meshes compare learned flexible CG with Jacobi-PCG in
     iterations and wall-clock to the same relative residual.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

from . import (F16, GS, InteriorModel, LearnedPrecond, Problem, brick_ids, deriv_device,
               geom_brick, rhs, sine_source)

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


def initial_arena(model: InteriorModel, seed: int = 0) -> np.ndarray:
    """The parameter arena [L | perceptron] before training: L the identity
    on the nI interior nodes (zero padding), the perceptron's first two
    layers He-uniform draws (synthetic.mlp_init), its last layer and every
    bias zero (nbx_lpi_init_scale then sets the gain biases)."""
    import synthetic as S
    nI, nIp, h = model.nI, model.nIp, model.n_hidden
    L = np.zeros((nIp, nIp))
    L[np.arange(nI), np.arange(nI)] = 1.0
    init = S.mlp_init(6, h, nI, seed)
    W1 = np.zeros((h, 64)); W1[:, :6] = init["W1"]
    parts = [L.ravel(), W1.ravel(), np.zeros(h), np.ravel(init["W2"]), np.zeros(h),
             np.zeros(nIp * h), np.zeros(nIp)]
    arena = np.concatenate(parts).astype(np.float32)
    assert arena.size == model.n_params
    return arena


def new_model(N: int, hidden: int = HIDDEN, max_batch: int = 1024,
              seed: int = 0) -> InteriorModel:
    import torch
    model = InteriorModel(N, hidden, max_batch)
    model.set_params(torch.as_tensor(initial_arena(model, seed)).cuda())
    return model


@dataclass
class Samples:
    X: object
    T: object
    F: object
    rows: int
    meshes: int
    seconds: float


def collect_samples(factory: MeshFactory, bricks, model: InteriorModel,
                    iterates=(8, 32, 128, 512), elems_per_vector: int = 512, seed: int = 0,
                    check_every: int = 20, log=None) -> Samples:
    """Training rows from the FP64 solver on each brick: its solution x*
    (to 1e-11, FP16-stored operator with FP64 reliable updates), and for
    each k in `iterates` below the FP64 solve's count the error x* - x_k
    and the residual r_k of FP64 Jacobi-PCG after k iterations, each on
    elems_per_vector random elements (<= 0: all).  Bricks alternate sine
    and random right-hand sides.  The rows stay in device memory."""
    import torch
    import synthetic as S
    t0 = time.perf_counter()
    rng = np.random.default_rng(seed)
    Xs, Ts, Fs = [], [], []
    for q, brick in enumerate(bricks):
        f = None if q % 2 == 0 else torch.as_tensor(S.rhs_values(brick)).cuda()
        mp = factory.build(brick, f)
        lp = LearnedPrecond(mp.problem, model)
        xstar, rs = mp.problem.pcg(mp.b, rtol=1e-11, max_iter=20000, check_every=check_every,
                                   prec=F16, inner_rtol=0.1)
        for k in iterates:
            if k >= rs.iters:
                continue
            xk, _ = mp.problem.pcg(mp.b, max_iter=k, fixed_iters=1, check_every=check_every)
            rk = lp.residual()
            for v, v0 in ((xstar, xk), (rk, None)):
                if elems_per_vector <= 0 or elems_per_vector >= mp.E:
                    el = torch.arange(mp.E, dtype=torch.int32)
                else:
                    el = torch.as_tensor(rng.choice(mp.E, size=elems_per_vector, replace=False),
                                         dtype=torch.int32)
                X, T, F = lp.samples(v, el.cuda(), v0=v0)
                Xs.append(X); Ts.append(T); Fs.append(F)
        lp.close()
        mp.problem.close()
        if log and (q + 1) % 25 == 0:
            log(f"  samples from {q + 1} meshes, {time.perf_counter() - t0:.1f} s")
    # one global shuffle so that minibatches mix meshes, iterates and
    # elements (a row permutation: data movement only)
    perm = torch.as_tensor(rng.permutation(sum(x.shape[0] for x in Xs))).cuda()
    X = torch.cat(Xs).index_select(0, perm)
    T = torch.cat(Ts).index_select(0, perm)
    F = torch.cat(Fs).index_select(0, perm)
    del Xs, Ts, Fs
    torch.cuda.synchronize()
    return Samples(X, T, F, X.shape[0], len(bricks), time.perf_counter() - t0)


def train(model: InteriorModel, data: Samples, epochs: int = 8, batch: int = 1024,
          lr: float = 1e-3, seed: int = 0) -> List[float]:
    """Minibatch Adam over contiguous row blocks in random order (the rows
    were shuffled once when collected), cosine decay of the learning rate;
    the gains start from the rows' least-squares scalar fit.  Returns the
    mean loss per epoch."""
    import torch
    rng = np.random.default_rng(seed)
    nb = data.rows // batch
    if nb == 0:
        raise ValueError("fewer samples than one batch")
    model.init_scale(data.X[:min(data.rows, 64 * batch)], data.T[:min(data.rows, 64 * batch)])
    losses = []
    step, total = 0, epochs * nb
    for ep in range(epochs):
        acc = []
        for bi in rng.permutation(nb):
            lr_t = lr * 0.5 * (1 + math.cos(math.pi * step / total))
            sl = slice(bi * batch, (bi + 1) * batch)
            acc.append(model.train_step(data.X[sl], data.T[sl], data.F[sl], max(lr_t, 1e-6)))
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
    flexible_iters: int
    learned_relres: float
    iteration_ratio: float
    speedup: float


def evaluate(factory: MeshFactory, brick, model: InteriorModel, rtol: float = 1e-10,
             reps: int = 2, f=None, check_every: int = 20) -> EvalResult:
    """Jacobi-PCG vs learned flexible CG on one mesh, to the same relative
    residual; best of `reps` timings each.  The learned solve has the same
    iteration budget as Jacobi's (20000) and falls back only on breakdown."""
    mp = factory.build(brick, f)
    lp = LearnedPrecond(mp.problem, model)
    jt, lt = [], []
    for _ in range(reps):
        h0 = time.perf_counter()
        _, rj = mp.problem.pcg(mp.b, rtol=rtol, max_iter=20000, check_every=check_every)
        jt.append(time.perf_counter() - h0)
    for _ in range(reps):
        h0 = time.perf_counter()
        _, rl = lp.pcg(mp.b, rtol=rtol, max_iter=20000, check_every=check_every)
        lt.append(time.perf_counter() - h0)
    lp.close()
    mp.problem.close()
    return EvalResult(brick.name, brick.E, rj.iters, min(jt), rl.iters, min(lt), rl.fell_back,
                      rl.outer_iters, rl.true_relres, rl.iters / max(rj.iters, 1),
                      min(jt) / min(lt))


def run_c5(n_train: int = 200, train_dims=(32, 16, 16), N: int = 10, eval_meshes=None,
           epochs: int = 8, batch: int = 1024, lr: float = 1e-3,
           iterates=(8, 32, 128, 512), elems_per_vector: int = 512, rtol: float = 1e-10,
           seed: int = 0, log=print) -> dict:
    """Train on n_train seeded deformed bricks, decide deployment on a
    validation brick of the training distribution (seed 5000), evaluate
    learned flexible CG against Jacobi-PCG on held-out meshes (by default a
    32^3 brick with an unseen deformation, N = 10)."""
    import torch
    import synthetic as S
    fac = MeshFactory()
    bricks = [S.Brick(*train_dims, N, S.deformation_family(s), "random", s, f"train{s}")
              for s in range(n_train)]
    model = new_model(N, max_batch=batch, seed=seed)
    t0 = time.perf_counter()
    data = collect_samples(fac, bricks, model, iterates=iterates,
                           elems_per_vector=elems_per_vector, seed=seed, log=log)
    log(f"samples: {data.rows} rows from {data.meshes} meshes in {data.seconds:.1f} s")
    t1 = time.perf_counter()
    losses = train(model, data, epochs=epochs, batch=batch, lr=lr, seed=seed)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    log(f"training: {epochs} epochs in {t_train:.1f} s, loss {losses[0]:.4g} -> "
        f"{losses[-1]:.4g} (targets have unit norm: mean square {1.0 / model.nI:.4g})")
    rows = data.rows
    del data
    vb = S.Brick(*train_dims, N, S.deformation_family(5000), "random", 5000, "val5000")
    vf = torch.as_tensor(S.rhs_values(vb)).cuda()
    rv = evaluate(fac, vb, model, rtol=rtol, reps=1, f=vf)
    use_learned = rv.learned_iters < rv.jacobi_iters and not rv.fell_back
    log(f"validation: learned {rv.learned_iters} it (fell back {rv.fell_back}), "
        f"Jacobi {rv.jacobi_iters} it -> learned_enabled {use_learned}")
    if eval_meshes is None:
        eval_meshes = [S.Brick(32, 32, 32, N, S.deformation_family(10000), "random", 10000,
                               "eval10000")]
    results = []
    for b in eval_meshes:
        f = torch.as_tensor(S.rhs_values(b)).cuda() if b.rhs == "random" else None
        r = evaluate(fac, b, model, rtol=rtol, reps=2, f=f)
        log(f"eval {b.name} E={b.E}: Jacobi {r.jacobi_iters} it {r.jacobi_seconds:.3f} s, "
            f"learned {r.learned_iters} it {r.learned_seconds:.3f} s "
            f"({r.speedup:.2f}x), fell back {r.fell_back}")
        results.append(r)
    return {
        "train_meshes": n_train, "train_dims": list(train_dims), "N": N,
        "rows": rows, "sample_seconds": round(t1 - t0, 3), "train_seconds": round(t_train, 3),
        "epochs": epochs, "loss_first": losses[0], "loss_last": losses[-1],
        "target_mean_square": 1.0 / model.nI,
        "validation": {"learned_iters": rv.learned_iters, "jacobi_iters": rv.jacobi_iters,
                       "fell_back": rv.fell_back},
        "learned_enabled": bool(use_learned),
        "eval": [r.__dict__ for r in results],
        "fallback_count": int(sum(r.fell_back for r in results)),
    }


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="train and evaluate the learned preconditioner")
    ap.add_argument("--train", type=int, default=200, help="number of training meshes")
    ap.add_argument("--N", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--eval-n", type=int, default=32, help="held-out brick is n^3 elements")
    args = ap.parse_args(argv)
    import synthetic as S
    ev = [S.Brick(args.eval_n, args.eval_n, args.eval_n, args.N, S.deformation_family(10000),
                  "random", 10000, "eval10000")]
    out = run_c5(n_train=args.train, N=args.N, epochs=args.epochs, eval_meshes=ev,
                 log=lambda m: print(m, flush=True))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
