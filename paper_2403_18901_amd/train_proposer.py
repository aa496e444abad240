"""Trains the learned decimation proposer for [[144,12,12]] circuit-level
windows on the GPU and writes its FP32 parameters (numpy .npy, no pickle).

  python -m paper_2403_18901_amd.train_proposer --shots 1000000 \\
      --out paper_2403_18901_amd/proposer_144.npy

Shots are spread evenly over noise levels p in [pmin, pmax]; each is decoded
with plain GDG in record mode on its first window, or with --windows all on
one of the windows, spread evenly over them, after the earlier windows are
decoded and committed (12 noisy rounds, W = 3, g = 4, 8 preprocessing
iterations; Alg. 3 on above p = 0.002).
"""
import argparse
import json
import time

import numpy as np
import torch

from gdg_inputs.bb import get_code
from gdg_inputs.dem import circuit_dem

from . import gdg as G
from . import learned as LRN


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shots", type=int, default=1_000_000)
    ap.add_argument("--pmin", type=float, default=0.001)
    ap.add_argument("--pmax", type=float, default=0.005)
    ap.add_argument("--levels", type=int, default=9)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--windows", choices=["first", "all"], default="first")
    ap.add_argument("--out", default=LRN.default_model_path("144"))
    a = ap.parse_args()
    t0 = time.time()
    ps = np.linspace(a.pmin, a.pmax, a.levels)
    per = a.shots // a.levels
    xs, ys = [], []
    for i, p in enumerate(ps):
        dem = circuit_dem(get_code("144"), 12, float(p))
        prm = G.params(alpha=1.0, g=4, pre_iters=8, trunc_factor=2, low_error=int(p <= 0.002))
        n_win = G.n_windows(dem.n_rounds, 3) if a.windows == "all" else 1
        for k in range(n_win):
            x, y = LRN.record(dem, prm, per // n_win, seed=a.seed + i, stream=k, window=k)
            xs.append(x)
            ys.append(y)
            print(f"p={p:.4f} window {k}: {x.shape[0]} candidates, in error "
                  f"{float(y.mean()):.3f}", flush=True)
    x, y = torch.cat(xs), torch.cat(ys)
    n = x.shape[0]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(a.seed)
    perm = torch.randperm(n, device="cuda", generator=gen)
    nv = max(n // 20, 1)
    xv, yv = x[perm[:nv]], y[perm[:nv]]
    xt, yt = x[perm[nv:]].contiguous(), y[perm[nv:]].contiguous()
    t1 = time.time()
    params = LRN.train(xt, yt, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed,
                       log=lambda s: print(s, flush=True))
    torch.cuda.synchronize()
    t2 = time.time()
    z = G.mlp_forward(params, xv.contiguous())
    acc = float(((z > 0).float() == yv).float().mean())
    base = float(max(yv.mean(), 1 - yv.mean()))
    LRN.save(params, a.out)
    print(json.dumps({"candidates": n, "validation": nv, "val_accuracy": acc,
                      "val_majority_class_rate": base, "record_s": t1 - t0, "train_s": t2 - t1,
                      "out": a.out}))


if __name__ == "__main__":
    main()
