"""Training and evaluation of the refinement surrogate (orchestration over the C-ABI).

Data: 256^3 periodic random-wave tangles (512 waves, |n| in [4, 8], one seed per field) generated
on the GPU; every pierced cell is refined by the plain method (Sec. 3.3.3), and the converged
single-core samples become (features, target = sample - first estimate) rows on the device.
Training: Adam on shuffled minibatches (the permutations are drawn on the host and passed in),
learning rate decaying as a cosine from lr to lr / 20. The confidence head learns whether the
network's point lies within conf_tol (0.25 cell) of the refined sample on every axis, i.e. close
enough for the one Newton step of the inference path to land on the same core. Evaluation: a fresh-seed field, plain
refinement against surrogate + fallback on the same listed cells, with kernel times from HIP
events and the position error of every surrogate sample measured against the plain result.

    python -m paper_1911_12070_amd.surrogate train --out weights.bin [--fields 150] [--epochs 12]
    python -m paper_1911_12070_amd.surrogate eval --weights weights.bin
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import (KIND_MLP, KIND_POLISH, KIND_REFINE, MLP_MAX_STEP, MLP_NHID, MLP_NPARAMS, SAMPLE_SURROGATE,
               AdamParams, Extractor, dims, samples_to_numpy, vx_mlp_create, vx_mlp_dataset, vx_mlp_destroy,
               vx_mlp_infer, vx_mlp_load, vx_mlp_reserve, vx_mlp_save, vx_mlp_train_step, vx_profile_enable,
               vx_profile_read)

BAD = 8 | 16 | 32 | 64  # NONZERO_MIN, NOT_CONVERGED, NO_FACES, BAD_CELL


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_dataset(ex: Extractor, tangles, n_cap: int):
    """Device arrays (features bf16 [n_cap][128], targets f32 [n_cap][3]) and the row count."""
    torch = ex.torch
    dev = f"cuda:{ex.device}"
    feat = torch.empty((n_cap, 128), dtype=torch.bfloat16, device=dev)
    target = torch.empty((n_cap, 3), dtype=torch.float32, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    for f, t in enumerate(tangles):
        psi = ex.gen_tangle(t)
        nz, ny, nx = psi.shape
        out = ex.alloc_winding(psi.shape, face_cap=nx * ny * nz // 32, cell_cap=nx * ny * nz // 32, wind=False)
        ex.winding(psi, 7, out)
        smp = ex.refine(psi, out, 7)
        cap = out["cells"].numel()
        vx_mlp_dataset(ex.h, dims(nx, ny, nz, 7), psi, out["cells"], out["cdesc"], smp, out["counts"][1:], cap,
                       feat, target, n_out, n_cap)
        if f % 10 == 9 or f == len(tangles) - 1:
            torch.cuda.synchronize()
            _log(f"[surrogate] dataset: {f + 1} fields, {int(n_out.cpu())} rows")
    torch.cuda.synchronize()
    n = min(int(n_out.cpu()), n_cap)
    return feat, target, n


def train(ex: Extractor, feat, target, n: int, init_params, epochs: int = 12, batch: int = 8192, lr: float = 2e-3,
          conf_lambda: float = 0.1, conf_tol: float = 0.25, seed: int = 0, log_every: int = 200):
    """Trains a new network from init_params (flat float32, library layout); returns the vx_mlp handle, the
    loss history, the training time and the number of steps."""
    torch = ex.torch
    dev = f"cuda:{ex.device}"
    m = vx_mlp_create(ex.h, init_params, batch)
    rng = np.random.default_rng(seed)
    steps_per_epoch = n // batch
    total = max(1, epochs * steps_per_epoch)
    loss = torch.zeros(2, dtype=torch.float32, device=dev)
    hist = []
    step = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(dev)
        for b in range(steps_per_epoch):
            a = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * step / total)))
            prm = AdamParams(a, 0.9, 0.999, 1e-8, conf_lambda, conf_tol)
            vx_mlp_train_step(ex.h, m, feat, target, perm[b * batch:(b + 1) * batch], batch, prm, loss)
            step += 1
            if step == 1 or step % log_every == 0 or step == total:
                l = loss.cpu().numpy()
                hist.append((step, float(l[0]), float(l[1])))
                _log(f"[surrogate] epoch {ep} step {step}/{total}: mse {l[0]:.3e} conf {l[1]:.3e} "
                     f"({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return m, hist, time.perf_counter() - t0, step


def evaluate(ex: Extractor, m, tangle, threshold: float = 0.9, reps: int = 10, max_step: float = MLP_MAX_STEP):
    """Plain refinement vs surrogate + fallback on every pierced cell of one field."""
    torch = ex.torch
    psi = ex.gen_tangle(tangle)
    nz, ny, nx = psi.shape
    d = dims(nx, ny, nz, 7)
    n_all = nx * ny * nz
    out = ex.alloc_winding(psi.shape, face_cap=n_all // 16, cell_cap=n_all // 16, wind=False)
    ex.winding(psi, 7, out)
    torch.cuda.synchronize()
    nc = int(out["counts"][1].cpu())
    cap = out["cells"].numel()
    vx_mlp_reserve(ex.h, m, cap)
    plain = ex.alloc_samples(cap)
    sur = ex.alloc_samples(cap)
    # warm up both paths, then time them alternately (one call of each per round, so that a drift of
    # the clock or of the memory system over the run affects both alike): kernel time from HIP events,
    # median over the rounds, and wall clock per call
    ex.refine(psi, out, 7, plain)
    vx_mlp_infer(ex.h, m, d, psi, out["cells"], out["cdesc"], out["counts"][1:], cap, threshold, sur,
                 max_step=max_step)
    torch.cuda.synchronize()
    t_plain, t_net, t_pol, t_fb, w_plain, w_sur = [], [], [], [], [], []
    for _ in range(reps):
        vx_profile_enable(ex.h, True)
        t0 = time.perf_counter()
        ex.refine(psi, out, 7, plain)
        torch.cuda.synchronize()
        w_plain.append(time.perf_counter() - t0)
        ms, k = vx_profile_read(ex.h, KIND_REFINE)
        t_plain.append(ms / max(k, 1))
        vx_profile_enable(ex.h, True)
        t0 = time.perf_counter()
        vx_mlp_infer(ex.h, m, d, psi, out["cells"], out["cdesc"], out["counts"][1:], cap, threshold, sur,
                     max_step=max_step)
        torch.cuda.synchronize()
        w_sur.append(time.perf_counter() - t0)
        t_net.append(vx_profile_read(ex.h, KIND_MLP)[0])
        t_pol.append(vx_profile_read(ex.h, KIND_POLISH)[0])
        t_fb.append(vx_profile_read(ex.h, KIND_REFINE)[0])
    vx_profile_enable(ex.h, False)
    med = lambda v: float(np.median(v))
    plain_ms = med(t_plain)
    net_ms, pol_ms, fb_ms = med(t_net), med(t_pol), med(t_fb)
    sur_ms = med([a + b + c for a, b, c in zip(t_net, t_pol, t_fb)])
    plain_wall, sur_wall = med(w_plain), med(w_sur)
    a = samples_to_numpy(plain, nc)
    b = samples_to_numpy(sur, nc)
    assert np.array_equal(a["cell"], b["cell"])
    used = (b["status"] & SAMPLE_SURROGATE) != 0
    ok = (a["status"] & BAD) == 0
    err = np.abs(b["off"].astype(np.float64) - a["off"].astype(np.float64)).max(axis=1)
    e_sur = err[used & ok]
    e_all = err[ok]
    # matrix-core work of the network per cell (two hidden layers and the head, multiply-adds x 2)
    flop = 2 * (128 * MLP_NHID + MLP_NHID * MLP_NHID + MLP_NHID * 4)
    net_s = net_ms * 1e-3
    return {
        "field": f"{nx}x{ny}x{nz}",
        "cells": nc,
        "threshold": threshold,
        "max_step": max_step,
        "surrogate_fraction": float(used.mean()),
        "fallback_fraction": float(1.0 - used.mean()),
        "median_err_surrogate_cells": float(np.median(e_sur)) if len(e_sur) else None,
        "p90_err_surrogate_cells": float(np.percentile(e_sur, 90)) if len(e_sur) else None,
        "p99_err_surrogate_cells": float(np.percentile(e_sur, 99)) if len(e_sur) else None,
        "max_err_surrogate_cells": float(e_sur.max()) if len(e_sur) else None,
        "surrogate_cells_above_0.02": int((e_sur > 0.02).sum()),
        "surrogate_cells_above_1e-3": int((e_sur > 1e-3).sum()),
        "median_err_all_cells": float(np.median(e_all)),
        "p99_err_all_cells": float(np.percentile(e_all, 99)),
        "max_err_all_cells": float(e_all.max()),
        "plain_kernel_ms": plain_ms,
        "surrogate_kernel_ms": sur_ms,
        "surrogate_net_ms": net_ms,
        "surrogate_polish_ms": pol_ms,
        "surrogate_fallback_ms": fb_ms,
        "plain_samples_per_s": nc / (plain_ms * 1e-3),
        "surrogate_samples_per_s": nc / (sur_ms * 1e-3),
        "plain_wall_ms": plain_wall * 1e3,
        "surrogate_wall_ms": sur_wall * 1e3,
        "speedup_kernel": plain_ms / sur_ms,
        "network_hidden_width": MLP_NHID,
        "network_flop_per_cell": flop,
        "network_tflops": flop * nc / net_s / 1e12,
        "network_frac_of_bf16_peak": flop * nc / net_s / 2.5e15,
    }


def main(argv=None):
    import vxinputs
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--out", required=True)
    tr.add_argument("--fields", type=int, default=150)
    tr.add_argument("--epochs", type=int, default=12)
    tr.add_argument("--batch", type=int, default=8192)
    tr.add_argument("--lr", type=float, default=2e-3)
    tr.add_argument("--seed", type=int, default=0)
    tr.add_argument("--eval", action="store_true", help="evaluate on the fresh-seed 512^3 field afterwards")
    ev = sub.add_parser("eval")
    ev.add_argument("--weights", required=True)
    ev.add_argument("--threshold", type=float, default=0.9)
    args = ap.parse_args(argv)
    ex = Extractor(0)
    if args.cmd == "train":
        tangles = vxinputs.surrogate_train_tangles(1000, args.fields)
        feat, target, n = build_dataset(ex, tangles, n_cap=80_000 * args.fields)
        m, hist, secs, steps = train(ex, feat, target, n, vxinputs.mlp_pack(vxinputs.mlp_init(args.seed)), args.epochs, args.batch,
                                     args.lr, seed=args.seed)
        vx_mlp_save(ex.h, m, args.out)
        res = {"rows": n, "steps": steps, "train_s": secs, "final_mse": hist[-1][1] if hist else None,
               "final_conf_loss": hist[-1][2] if hist else None}
        if args.eval:
            res["eval"] = evaluate(ex, m, vxinputs.tangle_512())
        print(json.dumps(res))
        vx_mlp_destroy(ex.h, m)
    else:
        m = vx_mlp_create(ex.h, np.zeros(MLP_NPARAMS, np.float32), 64)
        vx_mlp_load(ex.h, m, args.weights)
        print(json.dumps(evaluate(ex, m, vxinputs.tangle_512(), args.threshold)))
        vx_mlp_destroy(ex.h, m)
    ex.close()


if __name__ == "__main__":
    main()
