"""Train the learned corrector on method-generated pairs and evaluate it.

    python -m paper_2006_14794_amd.train_corrector --pairs 200000 --epochs 12 \
        --out paper_2006_14794_amd/corrector_weights.npz

Pairs are 256-point paths in R^8 with Gaussian increments of standard
deviation 0.3 / sqrt(256) (independent x and y), drawn from the seeded
generators of ``workloads.py`` (training seed 14798, held-out seed 14799).
Targets are the plain scheme at dyadic order 3 (``sigkernel_pair``); the
held-out evaluation reports the corrected values' errors against that same
plain solve, next to the order-0 values and the (order 0, order 1)
extrapolation to order 3, and the fallback fraction and final errors of
``Corrector.predict``.  Everything runs on the GPU through libsigkernel.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402  (seeded synthetic inputs, no method arithmetic)

from . import corrector as corr  # noqa: E402
from .api import sigkernel_pair  # noqa: E402


def _sync_time(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t0


def rel_stats(err: np.ndarray) -> dict:
    return {"median": float(np.median(err)), "p90": float(np.percentile(err, 90)),
            "p99": float(np.percentile(err, 99)), "max": float(err.max())}


def evaluate(model: corr.Corrector, n_eval: int, *, kappa: float, tol: float, log=print) -> dict:
    X, Y = workloads.corrector_pairs(workloads.SEED_CORRECTOR_EVAL, n_eval)
    Xc = torch.from_numpy(X.astype(np.float32)).cuda()
    Yc = torch.from_numpy(Y.astype(np.float32)).cuda()
    del X, Y
    k3, t3 = _sync_time(lambda: corr.order3_targets(Xc, Yc))
    log(f"eval: plain order-3 solve of {n_eval} pairs {t3:.2f} s")
    k0, t0 = _sync_time(lambda: sigkernel_pair(Xc, Yc, 0))
    k1, t1 = _sync_time(lambda: sigkernel_pair(Xc, Yc, 1))
    model.predict(Xc[:256], Yc[:256], kappa=kappa, tol=tol)  # warm
    (out, err, fb), tp = _sync_time(lambda: model.predict(Xc, Yc, kappa=kappa, tol=tol))
    (raw, _, _), traw = _sync_time(lambda: model.predict(Xc, Yc, kappa=kappa, tol=1e30))
    k3n = k3.cpu().numpy().astype(np.float64)
    k0n = k0.cpu().numpy().astype(np.float64)
    k1n = k1.cpu().numpy().astype(np.float64)
    rel = lambda v: np.abs(v - k3n) / np.abs(k3n)  # noqa: E731
    extrap = k0n + (k1n - k0n) * (63.0 / 64.0) * (4.0 / 3.0)
    fbn = fb.cpu().numpy()
    m = 255
    cells3 = n_eval * (m << 3) * (m << 3)
    res = {
        "pairs": n_eval,
        "plain_order3": {"seconds": t3, "cells_per_s": cells3 / t3},
        "order0": {"seconds": t0, "rel_err_vs_order3": rel_stats(rel(k0n))},
        "extrapolation_order0_order1": {"seconds": t0 + t1,
                                         "rel_err_vs_order3": rel_stats(rel(extrap))},
        "corrector_no_fallback": {"seconds": traw,
                                  "rel_err_vs_order3": rel_stats(rel(raw.cpu().numpy()))},
        "corrector": {"seconds": tp, "kappa": kappa, "tol": tol,
                      "fallback_fraction": float(fbn.mean()),
                      "rel_err_vs_order3": rel_stats(rel(out.cpu().numpy())),
                      "order3_equivalent_cells_per_s": cells3 / tp,
                      "speedup_vs_plain_order3": t3 / tp},
    }
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=200000)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval-pairs", type=int, default=65536)
    ap.add_argument("--kappa", type=float, default=corr.KAPPA)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--out", default=None, help="weights file (.npz)")
    ap.add_argument("--summary", default=None, help="JSON summary file")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    t_all = time.time()
    X, Y = workloads.corrector_pairs(workloads.SEED_CORRECTOR_TRAIN, args.pairs)
    Xc = torch.from_numpy(X.astype(np.float32)).cuda()
    Yc = torch.from_numpy(Y.astype(np.float32)).cuda()
    del X, Y
    log(f"generated {args.pairs} training pairs ({time.time() - t_all:.1f} s)")
    k3 = torch.empty(args.pairs, dtype=torch.float32, device="cuda")
    t0 = time.time()
    chunk = 16384
    for a in range(0, args.pairs, chunk):
        b = min(args.pairs, a + chunk)
        sigkernel_pair(Xc[a:b], Yc[a:b], 3, out=k3[a:b])
        torch.cuda.synchronize()
        log(f"targets {b}/{args.pairs} ({time.time() - t0:.1f} s)")
    t_labels = time.time() - t0
    model, t_train = _sync_time(lambda: corr.train(Xc, Yc, k3, epochs=args.epochs,
                                                   batch=args.batch, lr=args.lr, seed=args.seed,
                                                   log_every=500, log=log))
    model.meta["label_seconds"] = round(t_labels, 2)
    del Xc, Yc, k3
    torch.cuda.empty_cache()
    if args.out:
        model.save(args.out)
        log(f"saved {args.out}")
    res = {"train": {"pairs": args.pairs, "epochs": args.epochs, "batch": args.batch,
                     "label_seconds": t_labels, "train_seconds": t_train}}
    if args.eval_pairs:
        res["eval"] = evaluate(model, args.eval_pairs, kappa=args.kappa, tol=args.tol, log=log)
    line = json.dumps(res)
    print(line, flush=True)
    if args.summary:
        with open(args.summary, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
