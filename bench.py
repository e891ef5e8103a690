"""Benchmark of the vortex-core hot path on one MI355X.

Workload: the 1024^3 periodic random-wave tangle (4096 waves, |n| in [8, 24], seed 3; a synthetic
stand-in for the paper's 2048^3 turbulence data), generated on the GPU before timing. One step =
winding + compaction of the whole grid (packed field + pierced face/cell lists) followed by the
refinement of every pierced cell, all in the library's HIP kernels, inputs resident in HBM.

Prints one JSON line. `roofline` describes the dominant kernel (winding + compaction): algorithmic
bytes per launch (8 B psi read + 1 B packed write per node, plus the list entries) over its average
duration measured with HIP events on the launch stream inside the timed region. `cpu_baseline` is
the CPU oracle (plain C) timed on a 256^3 block of the same field's bytes, on one host thread and on
all of them (median of 5 runs each), with the host's CPU model and thread count.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline]

With --workload series_64 it measures batching instead: 64 frames of uneven size (128^3 to 384^3,
one 1024-wave tangle advanced in time, 1.32e9 cells in all), winding + compaction + refinement of
every frame in one HIP graph launch per step (z-chunk depths and the resident workgroups per CU of
the winding and the refinement autotuned before timing).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "cells/s + core samples/s, %HBM peak; surrogate vs plain at ≤0.02-cell error"


def kernel_hash() -> str:
    with open(os.path.join(ROOT, "paper_1911_12070_amd", "csrc", "vx_wind.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_record(grid: int):
    """HBM bytes per launch of the winding kernel from the committed rocprofv3 counter runs
    (`key = value` lines), if they were taken on the current kernel source and grid."""
    path = os.path.join(ROOT, "profiles", "wind_bits_k_tangle_1024_traffic.txt")
    rec = {}
    try:
        with open(path) as fh:
            for line in fh:
                if "=" in line and not line.lstrip().startswith("#"):
                    k, v = line.split("=", 1)
                    rec[k.strip()] = v.strip()
    except OSError:
        return None
    if rec.get("kernel_sha") != kernel_hash() or rec.get("grid") != str(grid):
        return None
    try:
        return float(rec["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_info():
    """CPU model and the number of host threads this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return model, n


def cpu_baseline(block, label: str, runs: int = 5):
    """The CPU oracle (plain C, FP64 refinement) on `block`, a cube of psi bytes copied back from the
    GPU, taken as a periodic grid (the per-node work is the same as inside the big grid): winding +
    pierced lists (z-slabs of 16 planes) and the refinement of every pierced cell (contiguous chunks of
    the list), once on one thread and once on every host thread, median of `runs` runs each."""
    import numpy as np

    import oracle

    model, nthreads = host_info()
    nodes = int(block.size)

    def once(threads):
        a = time.perf_counter()
        C, D = [], []
        for k0, k1, pk, cd in oracle.winding_slabs(block, 7, threads=threads, slab=16):
            _, _, c, d = oracle.lists_from_packed(pk, cd, k0 * block.shape[1] * block.shape[2])
            C.append(c)
            D.append(d)
        cells, cdesc = np.concatenate(C), np.concatenate(D)
        b = time.perf_counter()
        oracle.refine(block, cells, cdesc, threads=threads)
        c = time.perf_counter()
        return b - a, c - b, len(cells)

    res = {}
    for key, th in (("one_thread", 1), ("all_threads", nthreads)):
        runs_ = [once(th) for _ in range(runs)]
        tw = float(np.median([r[0] for r in runs_]))
        tr = float(np.median([r[1] for r in runs_]))
        tt = float(np.median([r[0] + r[1] for r in runs_]))
        ncell = runs_[0][2]
        res[key] = {"threads": th, "cells_per_s": nodes / tt, "winding_cells_per_s": nodes / tw,
                    "refine_samples_per_s": ncell / tr if tr > 0 else None, "median_step_s": tt}
    allc = res["all_threads"]
    return {
        "value": allc["cells_per_s"],
        "unit": "cells/s",
        "cores": nthreads,
        "kind": "oracle",
        "sample": f"{label} ({nodes} cells, {ncell} pierced) taken as a periodic grid; winding + pierced lists + "
                  f"FP64 refinement of every pierced cell; median of {runs} runs on {nthreads} threads "
                  f"(and on one thread: one_thread)",
        "cpu_model": model,
        "nproc": nthreads,
        "winding_cells_per_s": allc["winding_cells_per_s"],
        "refine_samples_per_s": allc["refine_samples_per_s"],
        "one_thread": res["one_thread"],
    }


def bench_surrogate(ex):
    """Surrogate path (committed trained network, fallback below confidence 0.9) against the plain
    refinement on every pierced cell of the fresh-seed 512^3 tangle (2048 waves, |n| in [6,16],
    seed 5); kernel times from HIP events, position errors against the plain result."""
    import numpy as np

    import vxinputs
    from paper_1911_12070_amd import MLP_NPARAMS, vx_mlp_create, vx_mlp_destroy, vx_mlp_load
    from paper_1911_12070_amd.surrogate import evaluate
    path = os.path.join(ROOT, "paper_1911_12070_amd", "weights", "surrogate_c2.bin")
    if not os.path.exists(path):
        return None
    print("[bench] surrogate vs plain refinement on the 512^3 tangle", file=sys.stderr, flush=True)
    m = vx_mlp_create(ex.h, np.zeros(MLP_NPARAMS, np.float32), 64)
    vx_mlp_load(ex.h, m, path)
    r = evaluate(ex, m, vxinputs.tangle_512(), 0.9)
    vx_mlp_destroy(ex.h, m)
    r["workload"] = "tangle_512: 512^3 periodic random-wave tangle, 2048 waves, |n| in [6,16], seed 5 (unseen)"
    return r


def bench_pipeline(ex, psi, steps: int, warmup: int, cap: int, wl: str, N: int):
    """The same frames as a stream: the winding of frame k runs on one stream while frame k-1 is
    refined on another (FramePipeline; same kernels, same results). Timed from the first winding
    to the last refinement of `steps` frames, pipeline fill and drain included."""
    import torch

    from paper_1911_12070_amd import KIND_REFINE, KIND_WIND, FramePipeline, vx_profile_enable, vx_profile_read
    print("[bench] frame pipeline (winding of frame k beside the refinement of frame k-1)", file=sys.stderr,
          flush=True)
    pipe = FramePipeline(ex, psi.shape, cap, cap)
    for _ in range(max(warmup, 2)):
        pipe.push(psi)
    pipe.sync()
    torch.cuda.synchronize()
    vx_profile_enable(ex.h, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.push(psi)
    pipe.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    wind_ms, nw = vx_profile_read(ex.h, KIND_WIND)
    ref_ms, nr = vx_profile_read(ex.h, KIND_REFINE)
    vx_profile_enable(ex.h, False)
    del pipe
    torch.cuda.empty_cache()
    return {
        "value": N ** 3 * steps / elapsed,
        "unit": "cells/s",
        "frames": steps,
        "ms_per_frame": 1e3 * elapsed / steps,
        "kernel_ms_while_overlapped": {"wind_compact": wind_ms / max(nw, 1), "refine": ref_ms / max(nr, 1)},
        "workload": f"{wl} as a stream of frames: winding of frame k on one HIP stream beside the refinement "
                    "of frame k-1 on another, two alternating output buffer sets",
    }


def bench_node_circulation(ex, wind, steps: int):
    """Node-centred circulation (vx_node_circulation) on the benchmark's packed field: per-node byte
    field and vortex-node list; kernel time from HIP events; algorithmic bytes 1 read + 1 written per
    node plus 8 per listed vortex node."""
    import torch

    from paper_1911_12070_amd import KIND_NODE, dims, vx_node_circulation, vx_profile_enable, vx_profile_read
    nz, ny, nx = wind.shape
    node = torch.empty_like(wind)
    lst = torch.empty(1 << 26, dtype=torch.int64, device=wind.device)
    count = torch.zeros(1, dtype=torch.int64, device=wind.device)
    d = dims(nx, ny, nz, 7)
    for _ in range(2):
        vx_node_circulation(ex.h, d, wind, count, node, lst)
    torch.cuda.synchronize()
    vx_profile_enable(ex.h, True)
    for _ in range(steps):
        vx_node_circulation(ex.h, d, wind, count, node, lst)
    ms, k = vx_profile_read(ex.h, KIND_NODE)
    vx_profile_enable(ex.h, False)
    ms /= max(k, 1)
    nv = int(count.cpu())
    nodes = nx * ny * nz
    alg = 2 * nodes + 8 * nv + 8
    del node, lst
    torch.cuda.empty_cache()
    # the library takes the wide-row kernel when rows are whole 16-node words (torch buffers are
    # 256-byte aligned)
    kname = "node_circ_wide_k" if nx % 16 == 0 else "node_circ_k"
    return {"kernel": kname, "kernel_ms": ms, "vortex_nodes": nv, "algorithmic_bytes_per_launch": alg,
            "achieved_GBs": alg / (ms * 1e-3) / 1e9, "frac_of_hbm_peak": alg / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "nodes_per_s": nodes / (ms * 1e-3)}


def bench_vectorisation(ex, psi, out, nf: int, nc: int, box_k: int = 4):
    """The consumers of the benchmark's lists: dual graph and line classes, box-mean samples with graph
    reduction (host C++), their refinement from the box-mean seeds (GPU), Catmull-Rom curves (host),
    and the density error metric e at the box means, the refined samples and the curve points (GPU
    density kernels). Wall times of the host steps, HIP-event times of the GPU ones."""
    import numpy as np
    import torch

    from paper_1911_12070_amd import (KIND_REFINE, dims, samples_to_numpy, vx_curves, vx_density, vx_graph_lines,
                                      vx_mean_density, vx_profile_enable, vx_profile_read, vx_reduce, vx_refine)
    print("[bench] vectorisation consumers", file=sys.stderr, flush=True)
    nz, ny, nx = psi.shape
    d = dims(nx, ny, nz, 7)
    cells = out["cells"][:nc].cpu().numpy().view(np.uint64)
    cdesc = out["cdesc"][:nc].cpu().numpy().view(np.uint16)
    t0 = time.perf_counter()
    comp, deg, types, st = vx_graph_lines(d, cells, cdesc)
    t1 = time.perf_counter()
    R = vx_reduce(d, cells, cdesc, box_k, 5)
    t2 = time.perf_counter()
    m = len(R["seed_cell"])
    dev = psi.device
    sc = torch.from_numpy(R["seed_cell"].view(np.int64)).to(dev)
    sd = torch.from_numpy(R["seed_desc"].view(np.int16)).to(dev)
    so = torch.from_numpy(R["seed_off"]).to(dev)
    cnt = torch.tensor([m], dtype=torch.int64, device=dev)
    smp = torch.empty((m, 8), dtype=torch.int32, device=dev)
    vx_refine(ex.h, d, psi, sc, sd, cnt, smp, seed=so, cap=m)
    torch.cuda.synchronize()
    vx_profile_enable(ex.h, True)
    for _ in range(5):
        vx_refine(ex.h, d, psi, sc, sd, cnt, smp, seed=so, cap=m)
    ref_ms, k = vx_profile_read(ex.h, KIND_REFINE)
    vx_profile_enable(ex.h, False)
    s = samples_to_numpy(smp, m)
    c = R["seed_cell"].astype(np.int64)
    xstar = np.stack([c % nx, (c // nx) % ny, c // (nx * ny)], 1).astype(np.float64) + s["off"].astype(np.float64)
    t3 = time.perf_counter()
    C = vx_curves(d, xstar, R["edges"], 8)
    t4 = time.perf_counter()
    rbar = torch.zeros(1, dtype=torch.float64, device=dev)
    vx_mean_density(ex.h, d, psi, rbar)
    rbar = float(rbar.cpu())
    e = {}
    for tag, pts in (("box_means", R["pos"]), ("refined_samples", xstar), ("curve_points", C["points"])):
        p = torch.from_numpy(np.ascontiguousarray(pts)).to(dev)
        rho = torch.empty(len(pts), dtype=torch.float32, device=dev)
        vx_density(ex.h, d, psi, p, rho)
        e[tag] = float(rho.double().sum().cpu()) / (rbar * len(pts))
    ok = (s["status"] & (8 | 16)) == 0
    return {
        "box_k": box_k,
        "graph": {"lines": st["ncomp"], "by_type": st["ntype"], "branch_cells": st["nbranch"], "host_s": t1 - t0},
        "reduction": {"cells": nc, "samples": m, "passes": R["passes"], "host_s": t2 - t1},
        "seeded_refinement": {"kernel_ms": ref_ms / max(k, 1), "converged_fraction": float(ok.mean())},
        "curves": {"count": len(C["length"]), "closed": int(C["closed"].sum()), "points": len(C["points"]),
                   "total_length_cells": C["total_length"], "host_s": t4 - t3},
        "error_metric_e": e,
        "mean_density": rbar,
    }


def calib_copy():
    """Kernels of known traffic: their FETCH_SIZE / WRITE_SIZE readings calibrate the counters
    (fill: writes 1 GiB; sum: reads 1 GiB)."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    src.fill_(1.0)
    torch.cuda.synchronize()
    total = float(src.sum())
    torch.cuda.synchronize()
    del src, total


def bench_series(args):
    import numpy as np
    import torch

    import vxinputs
    from paper_1911_12070_amd import (KIND_REFINE, KIND_WIND, Batch, Extractor, samples_to_numpy,
                                      vx_profile_enable, vx_profile_read)

    series = vxinputs.series_64()
    ex = Extractor(0)
    print("[bench] generating 64 frames on the GPU", file=sys.stderr, flush=True)
    tangles = [series.frame(f) for f in range(64)]
    psis = [ex.gen_tangle(t) for t in tangles]
    batch = Batch(ex, [(p, 7) for p in psis])
    stream = torch.cuda.current_stream()
    print("[bench] autotuning z-chunk depths", file=sys.stderr, flush=True)
    batch.autotune(None, stream)
    tuned = {t.dims[0]: batch.zchunk(f) for f, t in enumerate(tangles)}
    refine_wg = batch.refine_wg()
    wind_wg = batch.wind_wg()
    for _ in range(args.warmup):
        batch.launch(stream)
    torch.cuda.synchronize()
    counts = [tuple(int(v) for v in o["counts"].cpu()) for o in batch.outs]
    for (nf, nc), o in zip(counts, batch.outs):
        if nf > o["faces"].numel() or nc > o["cells"].numel():
            raise RuntimeError("list capacity too small")
    if args.calib_copy:
        calib_copy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.launch(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # per-kernel durations from eager launches of the same kernels (HIP events on the stream)
    vx_profile_enable(ex.h, True)
    for _ in range(5):
        batch.launch(stream, graph=False)
    wind_ms, nw = vx_profile_read(ex.h, KIND_WIND)
    ref_ms, nr = vx_profile_read(ex.h, KIND_REFINE)
    vx_profile_enable(ex.h, False)
    wind_avg, ref_avg = wind_ms / max(nw, 1), ref_ms / max(nr, 1)
    cells = sum(int(np.prod(t.dims)) for t in tangles)
    nf_all = sum(c[0] for c in counts)
    nc_all = sum(c[1] for c in counts)
    alg_bytes = cells * 9 + nf_all * 9 + nc_all * 10 + 64 * 16
    achieved = alg_bytes / (wind_avg * 1e-3) / 1e9
    ok = np.concatenate([(samples_to_numpy(o["samples"], c[1])["status"] & (8 | 16 | 32)) == 0
                         for o, c in zip(batch.outs, counts)])
    res = {
        "metric": METRIC,
        "value": cells * args.steps / elapsed,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "series_64: 64 frames, sizes drawn from {128,192,256,384}^3 (seed 4), one 1024-wave "
                        "tangle (|n| in [4,12]) advanced by exp(-i |n|^2 t / 2), t = 0.05 f; winding + compaction "
                        "+ refinement of every frame in one HIP graph launch",
            "cells": cells,
            "frames_per_size": {str(k): series.sizes.count(k) for k in sorted(set(series.sizes))},
            "zchunk_per_size": {str(k): v for k, v in sorted(tuned.items())},
            "winding_workgroups_per_cu": wind_wg,
            "refine_workgroups_per_cu": refine_wg,
            "pierced_faces": nf_all,
            "pierced_cells": nc_all,
        },
        "samples_per_s": nc_all * args.steps / elapsed,
        "kernel_ms": {"wind_batch": wind_avg, "refine_batch": ref_avg},
        "refine_converged_fraction": float(ok.mean()) if len(ok) else None,
        "roofline": {
            "bound": "hbm",
            "kernel": "wind_batch_k",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": None,
            "algorithmic_bytes_per_launch": alg_bytes,
        },
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        f256 = next(f for f, t in enumerate(tangles) if t.dims[0] == 256)
        res["cpu_baseline"] = cpu_baseline(psis[f256].cpu().numpy(), "one whole 256^3 frame of the series")
    batch.close()
    ex.close()
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["tangle_1024", "series_64"], default="tangle_1024")
    ap.add_argument("--grid", type=int, default=1024)
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import vxinputs
    from paper_1911_12070_amd import (KIND_REFINE, KIND_WIND, Extractor, samples_to_numpy, vx_profile_enable,
                                      vx_profile_read)

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.workload == "series_64":
        return bench_series(args)

    N = args.grid
    if N == 1024:
        tangle = vxinputs.tangle_1024()
        wl = "tangle_1024"
    else:
        tangle = vxinputs.make_tangle((N, N, N), 4096, (8, 24), 3)
        wl = f"tangle_{N}"
    ex = Extractor(0)
    ex.config(args.zchunk)
    print(f"[bench] generating {N}^3 field on the GPU", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    psi = ex.gen_tangle(tangle)
    torch.cuda.synchronize()
    print(f"[bench] generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    cap = 1 << 24
    out = ex.alloc_winding(psi.shape, face_cap=cap, cell_cap=cap, wind=True)
    samples = ex.alloc_samples(cap)
    stream = torch.cuda.current_stream()

    def step():
        ex.winding(psi, 7, out, stream)
        ex.refine(psi, out, 7, samples, None, None, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    nf, nc = (int(v) for v in out["counts"].cpu())
    if nf > cap or nc > cap:
        raise RuntimeError(f"list capacity {cap} too small: {nf} faces, {nc} cells")

    if args.calib_copy:
        calib_copy()

    vx_profile_enable(ex.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    wind_ms, nw = vx_profile_read(ex.h, KIND_WIND)
    ref_ms, nr = vx_profile_read(ex.h, KIND_REFINE)
    vx_profile_enable(ex.h, False)

    cells = N ** 3
    ms_step = 1e3 * elapsed / args.steps
    wind_avg_ms = wind_ms / max(nw, 1)
    ref_avg_ms = ref_ms / max(nr, 1)
    alg_bytes = cells * (8 + 1) + nf * (8 + 1) + nc * (8 + 2) + 2 * 8
    achieved = alg_bytes / (wind_avg_ms * 1e-3) / 1e9
    trf = traffic_record(N)

    s = samples_to_numpy(samples[: min(nc, 1 << 20)])
    st = s["status"]
    ok = (st & (8 | 16 | 32)) == 0

    res = {
        "metric": METRIC,
        "value": cells * args.steps / elapsed,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{wl}: {N}^3 periodic random-wave tangle, 4096 waves, |n| in [8,24], seed 3; "
                        "winding + compaction + refinement of every pierced cell",
            "grid": [N, N, N],
            "pierced_faces": nf,
            "pierced_cells": nc,
        },
        "samples_per_s": nc * args.steps / elapsed,
        "refine_samples_per_s_kernel": nc / (ref_avg_ms * 1e-3) if ref_avg_ms > 0 else None,
        "kernel_ms": {"wind_compact": wind_avg_ms, "refine": ref_avg_ms},
        "refine_converged_fraction": float(ok.mean()) if len(ok) else None,
        "roofline": {
            "bound": "hbm",
            "kernel": "wind_bits_k",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": trf,
            "algorithmic_bytes_per_launch": alg_bytes,
        },
    }
    res["node_circulation"] = bench_node_circulation(ex, out["wind"], args.steps)
    res["vectorisation"] = bench_vectorisation(ex, psi, out, nf, nc)
    del out, samples
    torch.cuda.empty_cache()
    res["pipelined"] = bench_pipeline(ex, psi, args.steps, args.warmup, cap, wl, N)
    B = min(256, N)
    block = psi[:B, :B, :B].cpu().numpy() if not args.no_cpu_baseline else None
    del psi
    torch.cuda.empty_cache()
    res["surrogate"] = bench_surrogate(ex)
    if block is not None:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(block, f"the {B}^3 corner block of the benchmark field")
    ex.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
