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
    """Training rows from FP64 CG runs on the given meshes: n_iterates
    iterates per mesh (geometrically spaced), elems_per_iterate elements of
    each (<= 0: all).  The rows stay in device memory."""
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
            if elems_per_iterate <= 0 or elems_per_iterate >= mp.E:
                el = torch.arange(mp.E, dtype=torch.int32)       # every element
            else:
                el = torch.as_tensor(rng.choice(mp.E, size=elems_per_iterate, replace=False),
                                     dtype=torch.int32)
            X, T = lp.samples(rk, xstar, xk, el.cuda())
            Xs.append(X); Ts.append(T)
        lp.close()
        mp.problem.close()
    # one global shuffle so that minibatches mix meshes, iterates and
    # elements (a row permutation: data movement only)
    perm = torch.as_tensor(rng.permutation(sum(x.shape[0] for x in Xs))).cuda()
    X = torch.cat(Xs).index_select(0, perm)
    T = torch.cat(Ts).index_select(0, perm)
    del Xs, Ts
    torch.cuda.synchronize()
    return Samples(X, T, X.shape[0], len(bricks), time.perf_counter() - t0)


def train(net: Mlp, data: Samples, epochs: int = 30, batch: int = 1024, lr: float = 1e-3,
          seed: int = 0) -> List[float]:
    """Minibatch Adam over contiguous row blocks in random order (the rows
    were shuffled once when collected); cosine decay of the learning rate.
    Returns the mean loss per epoch."""
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


def set_damping(net: Mlp, trained, a: float):
    """Deploys a * f (last layer scaled by a) from the trained arena."""
    import torch
    h, i, o = net.n_hidden, net.in_pad, net.out_pad
    p = trained.clone()
    w3 = h * i + h + h * h + h
    p[w3:] *= a                                   # W3 and b3
    net.set_params(p)


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
                      rl.outer_iters, rl.true_relres, rl.iters / max(rj.iters, 1), min(jt) / min(lt))


def run_c5(n_train: int = 16, train_dims=(32, 16, 16), N: int = 10, eval_meshes=None,
           epochs: int = 20, batch: int = 1024, lr: float = 1e-3, n_iterates: int = 4,
           elems_per_iterate: int = 0, dampings=(1.0, 0.5, 0.25), rtol: float = 1e-10,
           seed: int = 0, log=print) -> dict:
    """Train on n_train seeded deformed bricks, choose the output damping on
    a validation brick of the training distribution (seed 5000), evaluate
    learned FPCG (with that damping) against Jacobi-PCG on held-out meshes
    (by default one 32^3 brick with an unseen deformation, N=10).
    learned_enabled reports the deployment decision: the learned
    preconditioner is used only if it needed fewer iterations than Jacobi
    on the validation brick without falling back."""
    import torch
    import synthetic as S
    fac = MeshFactory()
    bricks = [S.Brick(*train_dims, N, S.deformation_family(s), "random", s, f"train{s}")
              for s in range(n_train)]
    net = new_network(N, max_batch=4096, seed=seed)
    t0 = time.perf_counter()
    data = collect_samples(fac, bricks, net, n_iterates=n_iterates,
                           elems_per_iterate=elems_per_iterate, seed=seed)
    log(f"samples: {data.rows} rows from {data.meshes} meshes in {data.seconds:.1f} s")
    t1 = time.perf_counter()
    losses = train(net, data, epochs=epochs, batch=batch, lr=lr, seed=seed)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    tvar = float((data.T.double() ** 2).sum(1).mean() / net.n_out)
    log(f"training: {epochs} epochs in {t_train:.1f} s, loss {losses[0]:.4g} -> {losses[-1]:.4g}"
        f" (target mean square {tvar:.4g})")
    rows = data.rows
    del data
    trained = net.get_params()
    vb = S.Brick(*train_dims, N, S.deformation_family(5000), "random", 5000, "val5000")
    vf = torch.as_tensor(S.rhs_values(vb)).cuda()
    val = {}
    for a in dampings:
        set_damping(net, trained, a)
        r = evaluate(fac, vb, net, rtol=rtol, reps=1, f=vf)
        val[a] = (r.learned_iters if not r.fell_back else 10 ** 9, r.jacobi_iters)
        log(f"validation damping {a}: learned {r.learned_iters} it (fell back {r.fell_back} "
            f"after {r.flexible_iters} flexible), Jacobi {r.jacobi_iters} it")
    # the damping with the fewest validation iterations (ties: the larger);
    # the learned preconditioner is deployed only if it beats Jacobi there
    best = min(val, key=lambda a: (val[a][0], -a))
    use_learned = val[best][0] < val[best][1]
    set_damping(net, trained, best)
    if eval_meshes is None:
        eval_meshes = [S.Brick(32, 32, 32, N, S.deformation_family(10000), "random", 10000,
                               "eval10000")]
    results = []
    for b in eval_meshes:
        f = torch.as_tensor(S.rhs_values(b)).cuda() if b.rhs == "random" else None
        r = evaluate(fac, b, net, rtol=rtol, reps=2, f=f)
        log(f"eval {b.name} E={b.E}: Jacobi {r.jacobi_iters} it {r.jacobi_seconds:.3f} s, "
            f"learned {r.learned_iters} it {r.learned_seconds:.3f} s, fell back {r.fell_back} "
            f"after {r.flexible_iters} flexible")
        results.append(r)
    return {
        "train_meshes": n_train, "train_dims": list(train_dims), "N": N,
        "rows": rows, "sample_seconds": round(t1 - t0, 3), "train_seconds": round(t_train, 3),
        "epochs": epochs, "loss_first": losses[0], "loss_last": losses[-1],
        "target_mean_square": tvar,
        "validation": {str(a): {"learned_iters": v[0] if v[0] < 10 ** 9 else None,
                                "jacobi_iters": v[1]} for a, v in val.items()},
        "damping": best, "learned_enabled": bool(use_learned),
        "eval": [r.__dict__ for r in results],
        "fallback_count": int(sum(r.fell_back for r in results)),
    }


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="train and evaluate the learned preconditioner")
    ap.add_argument("--train", type=int, default=16, help="number of training meshes")
    ap.add_argument("--N", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=30)
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
