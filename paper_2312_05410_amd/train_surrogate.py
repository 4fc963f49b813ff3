"""Train the blended run's U-Net on stepper snapshots and save its weights.

    python -m paper_2312_05410_amd.train_surrogate --epochs 60 --time-limit 900 \
        --out paper_2312_05410_amd/weights/unet_blend_512.npz

Generates the 2000 training pairs (20 staggered 512^2 trajectories x 100
jumps of 100 steps) and two held-out trajectories with the GPU stepper,
trains with Adam (batch 5, lr 1e-4 as in the paper) until the epoch count or
the time limit, prints one line per epoch, and writes the parameters (npz,
one array per named tensor) and the training history (json beside it).
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--time-limit", type=float, default=900.0)
    ap.add_argument("--lr", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--out", default="paper_2312_05410_amd/weights/unet_blend_512.npz")
    ap.add_argument("--init", default="", help="start from these weights (npz)")
    ap.add_argument("--head-gamma", type=float, default=1e-3,
                    help="initial output-head GN scale (the increments over one jump are ~1e-3)")
    a = ap.parse_args(argv)

    import torch

    from . import surrogate as S
    from .unet import UNet, UNetConfig, param_entries
    from .unet_inputs import init_params

    t0 = time.time()
    snaps = S.make_training_set(n=a.n)
    val = S.make_training_set(seed0=S.VAL_SEED, n_traj=2, stagger=20_000, n=a.n)
    print(f"training set {tuple(snaps.shape)} and validation {tuple(val.shape)} in {time.time() - t0:.1f} s",
          flush=True)
    cfg = UNetConfig(height=a.n, width=a.n, max_batch=5)
    if a.init:
        with np.load(a.init, allow_pickle=False) as z:
            params = {k: z[k] for k in z.files}
    else:
        params = init_params([(e[0], e[2]) for e in param_entries(cfg)], a.seed, head_gamma=a.head_gamma)
    net = UNet(cfg, params=params)
    hist = S.train(net, snaps, a.epochs, val=val, lr=a.lr, seed=a.seed, time_limit=a.time_limit)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    np.savez(a.out, **net.param_dict())
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump({"epochs": len(hist), "lr": a.lr, "seed": a.seed, "n": a.n,
                   "history": [h.__dict__ for h in hist]}, f, indent=1)
    print(f"wrote {a.out}", flush=True)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
