"""Train the learned pivot proposer on synthetic sectored Hamiltonians.

Recipe (instance s = 0 .. instances-1, all seeded):
  * n = 1000 * round(10^(5 + U) / 1000) with U ~ U(0, 1), mean nnz/row
    z ~ U{100..200}, sectors of 1000 rows, 70 % in-sector couplings, generator
    seed s; truncation n_t = 1 % of n; FP32 values and basis;
  * the plain solver (bootstrap pivot, b = k = 10, tol 1e-6) gives the lowest
    10 eigenvectors X; the features of H give P_D; the targets are
    sqrt(n) X Q, Q the Procrustes rotation of X onto P_D;
  * Adam (lr 1e-3, betas 0.9 / 0.999) on uniformly sampled batches for a
    number of epochs over all rows; the last 10 % of instances are held out,
    their loss is evaluated 40 times during training and the parameters with
    the lowest held-out loss are kept (early stopping).

Every step runs in libbbl.so's kernels (generation of the synthetic matrices
aside, which is host code in ``synthgen``).  Usage:

  python -m paper_2210_15763_amd.train_pivot --instances 200 --epochs 20 \
      --out paper_2210_15763_amd/weights/pivot_mlp_sectored.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import synthgen  # noqa: E402
import paper_2210_15763_amd as bbl  # noqa: E402

SECTOR = 1000
B = K = 10
TOL = 1e-6


def log(msg):
    print("[train] " + msg, flush=True)


def instance_shape(s: int):
    rng = np.random.default_rng([s, 20])
    u = rng.random()
    n = int(1000 * round(10 ** (5 + u) / 1000))
    z = int(rng.integers(100, 201))
    q = max(1, int(round(0.5263 * (z - 1))))   # draws per row -> ~z stored entries
    return n, z, q


def generate(s: int):
    n, z, q = instance_shape(s)
    return synthgen.generate(n, SECTOR, q, 0.7, s)


def identity_params(torch):
    """Parameters whose output reproduces feature columns 18..27 (sqrt(n) P_D):
    in the residual form, all zero.  The held-out loss of this map is what
    the network has to beat."""
    return torch.zeros(bbl.MLP_PARAMS, dtype=torch.float32, device="cuda")


def build_instance(torch, H, m_max: int):
    """Features (bf16 bits) and float32 targets of one instance, on the device."""
    Hd = bbl.DeviceCSR.from_host(H, "float32")
    n_t = max(20, H.n // 100)
    P, _ = bbl.bootstrap_pivot(Hd, n_t, B, TOL, m_max=m_max)
    r = bbl.block_lanczos(Hd, P, K, TOL, m_max=m_max)
    f = bbl.pivot_features(Hd, n_t, SECTOR, TOL, m_max=m_max)
    T = bbl.procrustes_targets(r.eigvecs, f["p_d"])
    return f["feats"], T, r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--instances", type=int, default=200)
    ap.add_argument("--epochs", type=float, default=20)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--m-max", type=int, default=200)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--data-out", default=None,
                    help="also save the training set (features, targets) to this .npz")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "weights", "pivot_mlp_sectored.npy"))
    args = ap.parse_args()

    import torch
    bbl.load_library()
    n_val = max(1, args.instances // 10)
    n_train = args.instances - n_val
    feats, targs, meta = [], [], []
    t0 = time.time()
    # generate instance s + 1 on the host while the GPU works on instance s
    nxt = {}

    def prefetch(s):
        nxt[s] = generate(s)

    th = threading.Thread(target=prefetch, args=(0,))
    th.start()
    for s in range(args.instances):
        th.join()
        H = nxt.pop(s)
        if s + 1 < args.instances:
            th = threading.Thread(target=prefetch, args=(s + 1,))
            th.start()
        F, T, r = build_instance(torch, H, args.m_max)
        feats.append(F)
        targs.append(T)
        meta.append({"seed": s, "n": H.n, "nnz_per_row": H.nnz / H.n, "iters": r.stats["iters"],
                     "converged": bool(r.converged)})
        log("instance %d/%d n=%d z=%.1f iters=%d converged=%s (%.0f s)" %
            (s + 1, args.instances, H.n, H.nnz / H.n, r.stats["iters"], r.converged,
             time.time() - t0))
        del H
    Ftr = torch.cat(feats[:n_train])
    Ttr = torch.cat(targs[:n_train])
    Fva = torch.cat(feats[n_train:])
    Tva = torch.cat(targs[n_train:])
    del feats, targs
    rows = Ftr.shape[0]
    steps = int(args.epochs * rows / args.batch)
    log("dataset: %d training rows, %d held-out rows; %d steps of %d" %
        (rows, Fva.shape[0], steps, args.batch))
    params = bbl.mlp_init(args.seed)
    tr = bbl.MlpTrainer(params, args.batch, sample_key=synthgen.pivot_key(args.seed + 7))

    def val_loss(p=None):
        tot, cnt = 0.0, 0
        for a in range(0, Fva.shape[0], 1 << 20):
            Fb, Tb = Fva[a:a + (1 << 20)], Tva[a:a + (1 << 20)]
            _, l = bbl.mlp_grad(params if p is None else p, Fb, Tb)
            tot += l.item() * Fb.shape[0]
            cnt += Fb.shape[0]
        return tot / cnt

    ident = val_loss(identity_params(torch))
    hist = [{"step": 0, "val_loss": val_loss()}]
    log("initial held-out loss %.4f; the P_D amplitudes alone: %.4f" % (hist[0]["val_loss"], ident))
    best = (hist[0]["val_loss"], 0, params.clone())
    t1 = time.time()
    report = max(1, steps // 40)
    for i in range(1, steps + 1):
        loss = tr.step(Ftr, Ttr, args.lr)
        if i % report == 0 or i == steps:
            hist.append({"step": i, "batch_loss": loss.item(), "val_loss": val_loss()})
            if hist[-1]["val_loss"] < best[0]:
                best = (hist[-1]["val_loss"], i, params.clone())
            log("step %d/%d batch loss %.4f held-out %.4f (%.1f s)" %
                (i, steps, hist[-1]["batch_loss"], hist[-1]["val_loss"], time.time() - t1))
    log("kept step %d (held-out loss %.4f)" % (best[1], best[0]))
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, best[2].cpu().numpy().astype(np.float32), allow_pickle=False)
    rec = {"instances": args.instances, "held_out": n_val, "epochs": args.epochs,
           "batch": args.batch, "lr": args.lr, "steps": steps, "train_rows": rows,
           "train_seconds": time.time() - t1, "data_seconds": t1 - t0, "history": hist,
           "kept_step": best[1], "kept_val_loss": best[0], "identity_val_loss": ident,
           "instances_meta": meta}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    log("saved %s" % args.out)


if __name__ == "__main__":
    main()
