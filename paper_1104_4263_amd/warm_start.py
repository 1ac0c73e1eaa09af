"""The learned warm start's configured network: training on solutions the block solver
generates, and the stored parameters.

The configured network has 4 levels and 32 base channels on 256 x 256 cells (h = lambda/48).
It is trained on random-field objects of the batched recipe (object i has seed 100 000 + i,
64 equispaced TE incidence angles each), solved by block GMRES(30) to the relative residual
1e-8.  The input is the contrast and the incident field, the target the scattered field
e_tot - e_in, the loss the mean square error (every kernel is the library's own: bf16
matrix-core convolutions with float32 accumulation, Adam).

    python -m paper_1104_4263_amd.warm_start --out DIR [--objects 313] [--epochs 16]

writes DIR/warm_start_l4c32_n256.f32 (raw little-endian float32 parameters, in the library's
order) and DIR/warm_start_l4c32_n256.json (the training record).  The package ships them in
paper_1104_4263_amd/data/."""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
NAME = "warm_start_l4c32_n256"
PARAMS_PATH = os.path.join(HERE, "data", NAME + ".f32")
RECORD_PATH = os.path.join(HERE, "data", NAME + ".json")
LEVELS, BASE, SIDE = 4, 32, 256
N_ANGLES = 64
RESTART, TOL, MAX_ITERS = 30, 1e-8, 20000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_network(max_batch: int = 16, path: str = PARAMS_PATH):
    """The configured network with the stored parameters (FileNotFoundError if absent)."""
    from .api import UNet
    if not os.path.exists(path):
        raise FileNotFoundError(f"no stored warm-start parameters at {path}")
    net = UNet(LEVELS, BASE, SIDE, SIDE, max_batch=max_batch, seed=0)
    p = np.fromfile(path, dtype="<f4")
    if p.size != net.n_params:
        net.close()
        raise ValueError(f"{path} holds {p.size} values, the network has {net.n_params}")
    net.set_params(p)
    return net


def generate(n_objects: int, seed0: int = 100_000, per_call: int = 4):
    """Inputs X [S, 256, 256, 8] and targets T [S, 256, 256, 4] (float32, device) of
    S = 64 n_objects solves, object by object, angle by angle."""
    import torch
    from synth import plane_wave, random_field_object
    from .api import Solver, UNet
    S = n_objects * N_ANGLES
    X = torch.empty(S, SIDE, SIDE, 8, dtype=torch.float32, device="cuda")
    T = torch.empty(S, SIDE, SIDE, 4, dtype=torch.float32, device="cuda")
    g = None
    B1 = None
    iters = []
    for o0 in range(0, n_objects, per_call):
        objs = [random_field_object(SIDE, seed=seed0 + o) for o in range(o0, min(n_objects, o0 + per_call))]
        if g is None:
            g = objs[0][0]
            psis = [2.0 * math.pi * j / N_ANGLES for j in range(N_ANGLES)]
            B1 = torch.from_numpy(np.stack([plane_wave(g, p) for p in psis])).cuda()
        solvers = [Solver.from_grid(g, e) for _, e in objs]
        res, rc = Solver.solve_batch(solvers, [B1] * len(objs), restart=RESTART, max_iters=MAX_ITERS, tol=TOL,
                                     mixed=1, block=2)
        if rc != 0 or any(x["rel_res_true"] > TOL for _, inf in res for x in inf):
            raise RuntimeError(f"training solves of objects {o0}.. did not converge (rc {rc})")
        for k, ((u, inf), (_, e)) in enumerate(zip(res, objs)):
            s0 = (o0 + k) * N_ANGLES
            eps = torch.from_numpy(e[None]).cuda()
            X[s0:s0 + N_ANGLES] = UNet.pack_inputs(eps, B1)
            T[s0:s0 + N_ANGLES] = UNet.pack_targets(u, B1)
            iters.append(float(np.mean([x["iters"] for x in inf])))
        for s in solvers:
            s.close()
        log(f"warm start: generated {min(n_objects, o0 + per_call) * N_ANGLES} / {S} solves")
    return X, T, g, B1, iters


def train(X, T, epochs: int, batch: int = 16, lr: float = 5e-4, lr_final: float = 2.5e-5, seed: int = 1):
    """Adam on shuffled mini-batches, the learning rate decaying by a cosine from lr to
    lr_final; returns the network and the mean loss of each epoch."""
    import torch
    from .api import UNet
    net = UNet(LEVELS, BASE, SIDE, SIDE, max_batch=batch, seed=seed)
    rng = np.random.default_rng(seed)
    S = X.shape[0]
    steps_per_epoch = S // batch
    total = epochs * steps_per_epoch
    step = 0
    means = []
    for ep in range(epochs):
        order = rng.permutation(S)
        losses = []
        for k in range(steps_per_epoch):
            idx = torch.from_numpy(order[k * batch:(k + 1) * batch]).cuda()
            a = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * step / max(total - 1, 1)))
            losses.append(net.train_step(X[idx], T[idx], a))
            step += 1
        means.append(float(np.mean(losses)))
        log(f"warm start: epoch {ep} mean loss {means[-1]:.5f}")
    return net, means


def held_out_errors(net, n_objects: int = 4, seed0: int = 300_000):
    """Relative error of the network's guess and of the incident field against the solution
    on objects the training never saw."""
    import torch
    from synth import plane_wave, random_field_object
    from .api import Solver
    objs = [random_field_object(SIDE, seed=seed0 + o) for o in range(n_objects)]
    g = objs[0][0]
    psis = [2.0 * math.pi * j / N_ANGLES for j in range(N_ANGLES)]
    B1 = torch.from_numpy(np.stack([plane_wave(g, p) for p in psis])).cuda()
    solvers = [Solver.from_grid(g, e) for _, e in objs]
    res, rc = Solver.solve_batch(solvers, [B1] * n_objects, restart=RESTART, max_iters=MAX_ITERS, tol=TOL, mixed=1,
                                 block=2)
    e_net, e_inc = [], []
    for s, (u, _) in zip(solvers, res):
        x0 = net.warm_start(s, B1)
        for r in range(N_ANGLES):
            nu = torch.linalg.vector_norm(u[r]).item()
            e_net.append(torch.linalg.vector_norm(x0[r] - u[r]).item() / nu)
            e_inc.append(torch.linalg.vector_norm(B1[r] - u[r]).item() / nu)
        s.close()
    return {"objects": n_objects, "seeds": [seed0, seed0 + n_objects - 1], "converged": rc == 0,
            "guess_rel_err_median": round(float(np.median(e_net)), 4),
            "incident_rel_err_median": round(float(np.median(e_inc)), 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--objects", type=int, default=313)
    ap.add_argument("--epochs", type=int, default=16)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=5e-4)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    X, T, _, _, iters = generate(args.objects)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    net, means = train(X, T, args.epochs, batch=args.batch, lr=args.lr)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    steps = args.epochs * (X.shape[0] // args.batch)
    del X, T
    torch.cuda.empty_cache()
    held = held_out_errors(net)
    os.makedirs(args.out, exist_ok=True)
    p = net.get_params().numpy().astype("<f4")
    p.tofile(os.path.join(args.out, NAME + ".f32"))
    rec = {"network": {"levels": LEVELS, "base": BASE, "height": SIDE, "width": SIDE, "params": int(p.size)},
           "data": {"objects": args.objects, "seeds": [100_000, 100_000 + args.objects - 1], "angles": N_ANGLES,
                    "solves": args.objects * N_ANGLES, "solver": "block GMRES(30), tol 1e-8, binary16 Gram-Schmidt",
                    "block_steps_mean": round(float(np.mean(iters)), 1), "generate_s": round(gen_s, 1)},
           "training": {"epochs": args.epochs, "batch": args.batch, "lr": [args.lr, 2.5e-5], "schedule": "cosine",
                        "steps": steps, "train_s": round(train_s, 1),
                        "TFLOPs": round(3 * 21.3e9 * args.batch * steps / train_s / 1e12, 1),
                        "epoch_mean_loss": [round(m, 6) for m in means]},
           "held_out": held}
    with open(os.path.join(args.out, NAME + ".json"), "w") as f:
        json.dump(rec, f, indent=1)
    log(json.dumps(rec))
    net.close()


if __name__ == "__main__":
    main()
