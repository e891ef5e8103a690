"""Whole-field parity on every benchmark configuration, in the launch configuration bench.py times.

For each configuration the GPU generates psi, runs the winding + compaction and the refinement,
and the oracle then processes the very psi bytes the GPU read (copied back): every byte of the
packed field, the complete sorted face and cell lists, and every refined sample are compared --
windings and lists bit for bit, samples against the FP64 refinement to 1e-4 cell. The error
statistics of the FP32 refinement are reported per configuration (max, p99, median, the samples
above 1e-4 with the condition number of their in-plane Jacobian, status disagreements):
  C1  32^3 line + ring, noise 1e-3            C2  256^3 tangle, 512 waves
  C3  1024^3 tangle, 4096 waves (bench.py's)  C4  the 64-frame series, batched in one graph launch
  C5  512^3 tangle, 2048 waves (the surrogate's evaluation field; the surrogate path is reported
      against the oracle as well)
Exact invariants that need no oracle are checked on every packed field too.
"""
import numpy as np
import pytest

import vxinputs
from gpu_util import log
from whole_parity import COND_LIMIT, TOL, assert_samples, explain, sample_parity, winding_parity

pytestmark = pytest.mark.gpu

def field_invariants(packed):
    """Exact invariants of a periodic packed field (torch uint8 tensor (nz, ny, nx) on the GPU).
    Returns (pierced faces, pierced cells)."""
    import torch
    p = packed.to(torch.int16)

    def w(shift):
        v = (p >> shift) & 3
        return torch.where(v == 3, -1, v).to(torch.int8)
    wx, wy, wz = w(0), w(2), w(4)
    assert int(((p >> 7) & 1).sum()) == 0, "bit 7 set"
    for a in range(3):
        assert int((((p >> (2 * a)) & 3) == 2).sum()) == 0, "winding code 2 (|w| > 1)"
    net = (torch.roll(wx, -1, 2) - wx).to(torch.int16) + (torch.roll(wy, -1, 1) - wy) + (torch.roll(wz, -1, 0) - wz)
    assert int((net != 0).sum()) == 0, "a cell has nonzero net winding"
    assert int(wz.to(torch.int64).sum(dim=(1, 2)).abs().max()) == 0
    assert int(wy.to(torch.int64).sum(dim=(0, 2)).abs().max()) == 0
    assert int(wx.to(torch.int64).sum(dim=(0, 1)).abs().max()) == 0
    anyf = (wx != 0) | (torch.roll(wx, -1, 2) != 0) | (wy != 0) | (torch.roll(wy, -1, 1) != 0) | (wz != 0) | \
        (torch.roll(wz, -1, 0) != 0)
    assert bool(torch.equal(anyf, ((p >> 6) & 1).bool())), "pierced-cell bit disagrees with the faces"
    nf = int((wx != 0).sum()) + int((wy != 0).sum()) + int((wz != 0).sum())
    return nf, int(anyf.sum())


def run_single(ex, psi, periodic, tag, cap, invariants=True):
    """Winding + refinement as bench.py runs them; whole-field parity; returns the stats."""
    import torch
    from paper_1911_12070_amd import samples_to_numpy
    out = ex.alloc_winding(psi.shape, face_cap=cap, cell_cap=cap, wind=True)
    ex.winding(psi, periodic, out)
    smp = ex.alloc_samples(cap)
    ex.refine(psi, out, periodic, smp)
    torch.cuda.synchronize()
    nf, nc = (int(v) for v in out["counts"].cpu())
    log(f"{tag}: {nf} pierced faces, {nc} pierced cells")
    if invariants and periodic == 7:
        assert (nf, nc) == field_invariants(out["wind"])
    psi_h = psi.cpu().numpy()
    packed_g = out["wind"].cpu().numpy()
    cells, cdesc = winding_parity(psi_h, packed_g, out, periodic, tag)
    del packed_g
    g = samples_to_numpy(smp, nc)
    stats, err, ok, R = sample_parity(psi_h, cells, cdesc, g, periodic, tag)
    g = g[np.argsort(g["cell"], kind="stable")]
    assert_samples(stats, err, ok, R, g, psi_h, cells, cdesc, lambda idx: explain(psi_h, cells, cdesc, g, R, idx))
    return out, psi_h, cells, cdesc, R


def test_c1_line_ring_32():
    from paper_1911_12070_amd import Extractor
    ex = Extractor(0)
    try:
        psi = ex.gen_line_ring(vxinputs.line_ring_32())
        run_single(ex, psi, 7, "C1 line_ring_32", 1 << 15)
    finally:
        ex.close()


def test_c2_tangle_256():
    from paper_1911_12070_amd import Extractor
    ex = Extractor(0)
    try:
        psi = ex.gen_tangle(vxinputs.tangle_256())
        run_single(ex, psi, 7, "C2 tangle_256", 1 << 20)
    finally:
        ex.close()


def test_c3_tangle_1024():
    from paper_1911_12070_amd import Extractor
    ex = Extractor(0)
    try:
        log("C3: generating the 1024^3 tangle on the GPU")
        psi = ex.gen_tangle(vxinputs.tangle_1024())
        run_single(ex, psi, 7, "C3 tangle_1024", 1 << 24)
    finally:
        ex.close()


def test_c5_tangle_512_plain_and_surrogate():
    import os

    import torch
    from paper_1911_12070_amd import (MLP_NPARAMS, SAMPLE_SURROGATE, Extractor, dims, samples_to_numpy, vx_mlp_create,
                                      vx_mlp_destroy, vx_mlp_infer, vx_mlp_load, vx_mlp_reserve)
    ex = Extractor(0)
    try:
        psi = ex.gen_tangle(vxinputs.tangle_512())
        cap = 1 << 21
        out, psi_h, cells, cdesc, R = run_single(ex, psi, 7, "C5 tangle_512", cap)
        nc = len(cells)
        weights = os.path.join(os.path.dirname(__file__), "..", "paper_1911_12070_amd", "weights", "surrogate_c2.bin")
        m = vx_mlp_create(ex.h, np.zeros(MLP_NPARAMS, np.float32), 64)
        vx_mlp_reserve(ex.h, m, cap)
        vx_mlp_load(ex.h, m, weights)
        sur = ex.alloc_samples(cap)
        vx_mlp_infer(ex.h, m, dims(512, 512, 512, 7), psi, out["cells"], out["cdesc"], out["counts"][1:], cap, 0.9,
                     sur)
        torch.cuda.synchronize()
        vx_mlp_destroy(ex.h, m)
        s = samples_to_numpy(sur, nc)
        s = s[np.argsort(s["cell"], kind="stable")]
        assert np.array_equal(s["cell"], cells)
        used = (s["status"] & SAMPLE_SURROGATE) != 0
        ok = (R.status & (8 | 16 | 32)) == 0
        err = np.abs(s["off"].astype(np.float64) - R.x).max(axis=1)
        e_sur = err[used & ok]
        log(f"C5 surrogate path vs the FP64 oracle: {used.mean():.4f} of the cells from the network; "
            f"median {np.median(e_sur):.2e}, p99 {np.percentile(e_sur, 99):.2e}, max {e_sur.max():.2e} cell; "
            f"all cells: median {np.median(err[ok]):.2e}, max {err[ok].max():.2e}")
        assert np.median(err[ok]) <= 0.02 and np.median(e_sur) <= 0.02
        # the plain refinement's samples (fallback) within TOL of the oracle, as on the plain path
        fb = ~used & ok & (R.cond <= COND_LIMIT) & ((s["status"] & (8 | 16)) == 0)
        assert (err[fb] <= TOL).all()
    finally:
        ex.close()


def test_c4_series_64_batched():
    import torch
    from paper_1911_12070_amd import Batch, Extractor, samples_to_numpy
    series = vxinputs.series_64()
    ex = Extractor(0)
    try:
        log(f"C4: generating 64 frames (sizes {sorted(set(series.sizes))}) on the GPU")
        tangles = [series.frame(f) for f in range(64)]
        psis = [ex.gen_tangle(t) for t in tangles]
        batch = Batch(ex, [(p, 7) for p in psis])
        stream = torch.cuda.current_stream()
        batch.autotune(None, stream)
        batch.launch(stream)
        torch.cuda.synchronize()
        errs, oks, conds, total, div = [], [], [], 0, 0
        for f in range(64):
            o = batch.outs[f]
            nf, nc = (int(v) for v in o["counts"].cpu())
            assert (nf, nc) == field_invariants(o["wind"]), f"frame {f}"
            psi_h = psis[f].cpu().numpy()
            tag = f"C4 frame {f} ({tangles[f].dims[0]}^3)"
            cells, cdesc = winding_parity(psi_h, o["wind"].cpu().numpy(), o, 7, tag)
            g = samples_to_numpy(o["samples"], nc)
            stats, err, ok, R = sample_parity(psi_h, cells, cdesc, g, 7, tag, report=False)
            g = g[np.argsort(g["cell"], kind="stable")]
            div += assert_samples(stats, err, ok, R, g, psi_h, cells, cdesc,
                                  lambda idx: explain(psi_h, cells, cdesc, g, R, idx))
            errs.append(err[ok])
            conds.append(R.cond[ok])
            total += nc
        e = np.concatenate(errs)
        c = np.concatenate(conds)
        above = e > TOL
        import json
        import os
        summary = {"config": "C4 series_64 (all frames)", "samples": total, "oracle_converged": int(len(e)),
                   "max_err": float(e.max()), "p99_err": float(np.percentile(e, 99)), "median_err": float(np.median(e)),
                   "above_tol": int(above.sum()), "tol": TOL, "above_tol_cond": sorted(float(v) for v in c[above])[:50],
                   "path_divergences": div}
        log("PARITY " + json.dumps(summary))
        path = os.environ.get("VX_PARITY_OUT")
        if path:
            with open(path, "a") as fh:
                fh.write(json.dumps(summary) + "\n")
        batch.close()
    finally:
        ex.close()
